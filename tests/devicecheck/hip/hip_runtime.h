// CPU emulation of the HIP device model for the device-code check (tests/devicecheck):
// a kernel launch runs its workgroups one after another, each workgroup as one host
// thread per lane.  __syncthreads is a workgroup barrier, DPP quad permutes exchange
// values inside a quad of lanes and __shfl_xor inside a 64-lane wave, each through a
// barrier, so every exchange needs all participating lanes to arrive (a lane that never
// arrives is reported as divergence after a timeout).  Device memory is host memory.
// Not a GPU build: it lets the sanitizers watch every load and store of the kernels.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>

#ifndef __clang__
typedef unsigned short __bf16;  // the network headers name the type; no network kernel is built here
#endif

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define EMU_DYNAMIC_SHARED extern
#define __align__(n)  // the LDS definition in emu.cpp carries the alignment

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
extern thread_local dim3 threadIdx, blockIdx;
extern dim3 blockDim, gridDim;
constexpr size_t kEmuLdsBytes = 160 * 1024;
// the dynamic LDS of the kernels (declared inside the kernels of namespace mppi)
namespace mppi {
extern unsigned char lds_raw[kEmuLdsBytes];
}

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1 };
typedef void* hipStream_t;
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t)
{
    std::memmove(d, s, n);
    return hipSuccess;
}
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k) { return hipMemcpyAsync(d, s, n, k, 0); }
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t)
{
    std::memset(d, v, n);
    return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
// launches run to completion when issued, so streams and events only keep issue order
typedef void* hipEvent_t;
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2 };
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = (void*)2; return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = (void*)1; return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t* e) { *e = (void*)1; return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 1.f; return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "emulation"; }
hipError_t hipGetLastError();
// pointer attributes: every buffer here is reported as device memory (the start-state
// finiteness check then falls to the device code)
enum hipMemoryType { hipMemoryTypeUnregistered = 0, hipMemoryTypeHost = 1, hipMemoryTypeDevice = 2,
                     hipMemoryTypeManaged = 3 };
struct hipPointerAttribute_t {
    hipMemoryType type;
    int device;
    void* devicePointer;
    void* hostPointer;
    int isManaged;
    unsigned allocationFlags;
};
inline hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void* p)
{
    *a = hipPointerAttribute_t{};
    a->type = hipMemoryTypeDevice;
    a->devicePointer = const_cast<void*>(p);
    return hipSuccess;
}

// one emulated device of two compute units (the persistent batch grid is blocks_per_cu x 2)
enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount };
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) { *v = 2; return hipSuccess; }
// pinned host memory is plain host memory here
enum { hipHostMallocDefault = 0 };
inline hipError_t hipHostMalloc(void** p, size_t n, unsigned)
{
    *p = std::malloc(n ? n : 1);
    return *p ? hipSuccess : hipErrorInvalidValue;
}
inline hipError_t hipHostFree(void* p) { std::free(p); return hipSuccess; }
// stream capture records the launches issued while it is open; a graph launch replays them
struct EmuGraph {
    std::vector<std::function<void()>> ops;
};
typedef EmuGraph* hipGraph_t;
typedef EmuGraph* hipGraphExec_t;
enum hipStreamCaptureMode { hipStreamCaptureModeThreadLocal };
extern EmuGraph* g_emu_capture;
inline hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode)
{
    if (g_emu_capture) return hipErrorInvalidValue;
    g_emu_capture = new EmuGraph;
    return hipSuccess;
}
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g)
{
    *g = g_emu_capture;
    g_emu_capture = nullptr;
    return *g ? hipSuccess : hipErrorInvalidValue;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, void*, void*, size_t)
{
    *e = new EmuGraph(*g);
    return hipSuccess;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t)
{
    for (auto& op : e->ops) op();
    return hipSuccess;
}
inline hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t e) { delete e; return hipSuccess; }

// ---- device built-ins --------------------------------------------------------------
void __syncthreads();
inline void __threadfence() { __atomic_thread_fence(__ATOMIC_SEQ_CST); }
int emu_quad_exchange(int v, int src_lane);
uint64_t emu_wave_exchange(uint64_t v, int src_lane);
// quad_perm control (the only DPP form the kernels use): lane i of a quad reads lane
// (ctrl >> 2i) & 3
inline int __builtin_amdgcn_update_dpp(int, int v, int ctrl, int row_mask, int bank_mask, bool)
{
    if (ctrl > 0xFF || row_mask != 0xF || bank_mask != 0xF) {
        std::fprintf(stderr, "emulation: unsupported DPP control 0x%x\n", ctrl);
        std::abort();
    }
    return emu_quad_exchange(v, (ctrl >> (2 * (threadIdx.x & 3))) & 3);
}
template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64)
{
    static_assert(sizeof(T) <= 8, "shuffle of up to 8 bytes");
    if (width != 64) std::abort();
    uint64_t b = 0;
    std::memcpy(&b, &v, sizeof(T));
    b = emu_wave_exchange(b, (int)((threadIdx.x & 63) ^ (unsigned)mask));
    T r;
    std::memcpy(&r, &b, sizeof(T));
    return r;
}
inline int __builtin_amdgcn_readfirstlane(int v) { return v; }  // the batch kernels: wave-uniform values
// wave vote: the mask of the lanes whose predicate holds (a butterfly of exchanges, so every
// lane of the wave must arrive)
inline unsigned long long __builtin_amdgcn_ballot_w64(bool p)
{
    uint64_t m = p ? (1ull << (threadIdx.x & 63)) : 0ull;
    for (int o = 1; o < 64; o <<= 1) m |= emu_wave_exchange(m, (int)((threadIdx.x & 63) ^ (unsigned)o));
    return m;
}
inline int atomicAdd(int* p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline uint32_t __umulhi(uint32_t a, uint32_t b) { return (uint32_t)(((uint64_t)a * b) >> 32); }
inline float __int_as_float(int i) { float f; std::memcpy(&f, &i, 4); return f; }
// the fast exponential (the hardware's base-2 exponential on the GPU); the host's expf here
inline float __expf(float x) { return std::exp(x); }
inline int __float_as_int(float f) { int i; std::memcpy(&i, &f, 4); return i; }
inline int __double2loint(double d) { int64_t i; std::memcpy(&i, &d, 8); return (int)(i & 0xffffffff); }
inline int __double2hiint(double d) { int64_t i; std::memcpy(&i, &d, 8); return (int)(i >> 32); }
inline double __hiloint2double(int hi, int lo)
{
    const int64_t i = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    double d;
    std::memcpy(&d, &i, 8);
    return d;
}
inline void sincospif(float x, float* s, float* c) { *s = sinf((float)M_PI * x); *c = cosf((float)M_PI * x); }
inline void sincospi(double x, double* s, double* c) { *s = sin(M_PI * x); *c = cos(M_PI * x); }
using std::max;
using std::min;

// ---- launch: workgroups in sequence, one host thread per lane -----------------------
void emu_run_grid(dim3 grid, dim3 block, size_t lds, const std::function<void()>& body);
template <typename K, typename... A>
void emu_launch(K kernel, dim3 grid, dim3 block, size_t lds, A... args)
{
    std::function<void()> run = [=]() { emu_run_grid(grid, block, lds, [=]() { kernel(args...); }); };
    if (g_emu_capture) g_emu_capture->ops.push_back(run);
    else run();
}
#define hipLaunchKernelGGL(kernel, grid, block, lds, stream, ...) emu_launch(kernel, grid, block, lds, __VA_ARGS__)

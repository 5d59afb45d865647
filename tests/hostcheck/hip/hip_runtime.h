// CPU stand-in of the HIP runtime for the host range check (tests/hostcheck): device
// memory is host memory the driver registers, copies and fills check their ranges and
// run, events and streams are no-ops, and a graph replays the launches it captured.
// Not a GPU build.
#pragma once
#include "flop_count_stub.h"

#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>

#ifndef __clang__
typedef unsigned short __bf16;
#endif

bool range_check(const void* p, size_t bytes, const char* what);

enum { hipSuccess = 0, hipErrorInvalidValue = 1 };
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
enum { hipHostMallocDefault = 0, hipStreamNonBlocking = 1, hipEventDisableTiming = 2, hipStreamCaptureModeThreadLocal = 1,
       hipDeviceAttributeMultiprocessorCount = 3 };
typedef void* hipEvent_t;
typedef void* hipGraph_t;
typedef void* hipGraphExec_t;

inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t)
{
    if (k != hipMemcpyHostToDevice) range_check(s, n, "copy source");
    if (k != hipMemcpyDeviceToHost) range_check(d, n, "copy destination");
    std::memcpy(d, s, n);
    return hipSuccess;
}
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k) { return hipMemcpyAsync(d, s, n, k, 0); }
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t)
{
    range_check(d, n, "fill");
    std::memset(d, v, n);
    return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "stand-in"; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipHostMalloc(void** p, size_t n, int)
{
    *p = std::aligned_alloc(256, (n + 255) / 256 * 256);
    return *p ? hipSuccess : hipErrorInvalidValue;
}
inline hipError_t hipHostFree(void* p)
{
    std::free(p);
    return hipSuccess;
}
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, int) { *e = (void*)1; return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t* e) { *e = (void*)1; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 1.f; return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, int) { *s = (void*)2; return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipDeviceGetAttribute(int* v, int, int) { *v = 256; return hipSuccess; }

// graph capture: the stand-in launchers record what they were given; a graph launch
// re-checks those launches against the current contents of the (host) device memory
void capture_begin();
void capture_replay();
inline hipError_t hipStreamBeginCapture(hipStream_t, int) { capture_begin(); return hipSuccess; }
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) { *g = (void*)3; return hipSuccess; }
inline hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t, void*, void*, size_t) { *e = (void*)4; return hipSuccess; }
inline hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { capture_replay(); return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
inline hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }

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

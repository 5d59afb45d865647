// Runtime of the CPU emulation of the HIP device model (see hip/hip_runtime.h): grids,
// workgroup barriers, quad and wave exchanges, and stand-ins for the network launchers
// (the checks here run no network kernel).
#include <errno.h>
#include <pthread.h>
#include <time.h>

#include <vector>

#include "hip/hip_runtime.h"
#include "mlp_launch.h"

#if defined(__has_feature)
#if __has_feature(memory_sanitizer)
#define EMU_MSAN 1
#include <sanitizer/msan_interface.h>
#endif
#endif
#ifndef EMU_MSAN
#define EMU_MSAN 0
#endif

thread_local dim3 threadIdx, blockIdx;
dim3 blockDim, gridDim;
EmuGraph* g_emu_capture = nullptr;
namespace mppi {
alignas(16) unsigned char lds_raw[kEmuLdsBytes];
}
using mppi::lds_raw;

hipError_t hipGetLastError() { return hipSuccess; }

namespace {

struct Barrier {
    pthread_mutex_t m = PTHREAD_MUTEX_INITIALIZER;
    pthread_cond_t c = PTHREAD_COND_INITIALIZER;
    int count = 0, waiting = 0;
    unsigned gen = 0;
    void wait(const char* what)
    {
        pthread_mutex_lock(&m);
        const unsigned g = gen;
        if (++waiting == count) {
            waiting = 0;
            ++gen;
            pthread_cond_broadcast(&c);
        } else {
            timespec dl;
            clock_gettime(CLOCK_REALTIME, &dl);
            dl.tv_sec += 120;
            while (g == gen)
                if (pthread_cond_timedwait(&c, &m, &dl) == ETIMEDOUT) {
                    std::fprintf(stderr, "emulation: lanes missing at %s (block %u, lane %u)\n", what, blockIdx.x,
                                 threadIdx.x);
                    std::abort();
                }
        }
        pthread_mutex_unlock(&m);
    }
};

Barrier g_block;
std::vector<Barrier> g_quad, g_wave;
std::vector<int> g_quad_slot;
std::vector<uint64_t> g_wave_slot;

struct Lane {
    unsigned tid;
    dim3 bid;
    const std::function<void()>* body;
};

void* lane_main(void* arg)
{
    const Lane* l = static_cast<const Lane*>(arg);
    threadIdx = dim3(l->tid % blockDim.x, (l->tid / blockDim.x) % blockDim.y, l->tid / (blockDim.x * blockDim.y));
    blockIdx = l->bid;
    (*l->body)();
    return nullptr;
}

unsigned linear_tid() { return threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z); }

}  // namespace

void __syncthreads() { g_block.wait("__syncthreads"); }

int emu_quad_exchange(int v, int src)
{
    const unsigned t = linear_tid(), q = t >> 2;
    g_quad_slot[t] = v;
    g_quad[q].wait("DPP quad permute");
    const int r = g_quad_slot[4 * q + src];
    g_quad[q].wait("DPP quad permute");
    return r;
}

uint64_t emu_wave_exchange(uint64_t v, int src)
{
    const unsigned t = linear_tid(), w = t >> 6;
    g_wave_slot[t] = v;
    g_wave[w].wait("wave shuffle");
    const uint64_t r = g_wave_slot[64 * w + src];
    g_wave[w].wait("wave shuffle");
    return r;
}

void emu_run_grid(dim3 grid, dim3 block, size_t lds, const std::function<void()>& body)
{
    if (lds > kEmuLdsBytes) {
        std::fprintf(stderr, "emulation: %zu bytes of dynamic LDS requested\n", lds);
        std::abort();
    }
    const unsigned n = block.x * block.y * block.z;
    blockDim = block;
    gridDim = grid;
    g_block.count = (int)n;
    g_quad.assign((n + 3) / 4, Barrier());
    g_wave.assign((n + 63) / 64, Barrier());
    for (unsigned q = 0; q < g_quad.size(); ++q) g_quad[q].count = (int)std::min(4u, n - 4 * q);
    for (unsigned w = 0; w < g_wave.size(); ++w) g_wave[w].count = (int)std::min(64u, n - 64 * w);
    g_quad_slot.assign(n, 0);
    g_wave_slot.assign(n, 0);
    std::vector<pthread_t> th(n);
    std::vector<Lane> lanes(n);
    pthread_attr_t attr;
    pthread_attr_init(&attr);
    pthread_attr_setstacksize(&attr, 8u << 20);
    for (unsigned bz = 0; bz < grid.z; ++bz)
        for (unsigned by = 0; by < grid.y; ++by)
            for (unsigned bx = 0; bx < grid.x; ++bx) {
                // LDS starts undefined in every workgroup: poisoned for the memory sanitizer,
                // a NaN pattern otherwise
#if EMU_MSAN
                __msan_poison(lds_raw, lds);
#else
                std::memset(lds_raw, 0xff, lds);
#endif
                for (unsigned t = 0; t < n; ++t) {
                    lanes[t] = Lane{t, dim3(bx, by, bz), &body};
                    if (pthread_create(&th[t], &attr, lane_main, &lanes[t])) {
                        std::fprintf(stderr, "emulation: thread creation failed\n");
                        std::abort();
                    }
                }
                for (unsigned t = 0; t < n; ++t) pthread_join(th[t], nullptr);
            }
    pthread_attr_destroy(&attr);
}

// the checks run no network kernel: the network launchers refuse
namespace mlp {
hipError_t launch_gemm(int, const GemmArgs&, int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_prep(const PrepArgs&, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_loss(const LossArgs&, hipStream_t) { return hipErrorInvalidValue; }
int loss_rows_per_block() { return 32; }
hipError_t launch_reduce(const ReduceArgs&, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_adam(const AdamArgs&, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_reduce_adam(const ReduceArgs&, const AdamArgs&, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_head(const HeadArgs&, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_loss_sum(const float*, int, float, float*, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_pairs(const PairsArgs&, hipStream_t) { return hipErrorInvalidValue; }
}  // namespace mlp

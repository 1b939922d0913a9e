// Device-side building blocks shared by the PTP kernels: control-block
// layout, the grid-wide barrier of the persistent kernels, block scans and
// the workspace carve.  Internal to the HIP library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptp {

constexpr int kBlock = 256;                 // threads per workgroup (4 waves)
constexpr int kWave = 64;

// ---- control block (int32 words in device memory) ----------------------
// Hot words sit on their own 128-byte lines.
enum CtrlWord : int {
    C_STATUS = 0,        // validation / fault bits (ST_*)
    C_RHO = 1,           // number of toplesets
    C_REACH = 2,         // number of reachable vertices
    C_ITERS = 3,         // K of the last run
    C_RUNSTAT = 4,       // 0 ok, 1 cap reached (ENOCONV)
    C_UPD_LO = 5,        // vertex updates, low / high 32 bits
    C_UPD_HI = 6,
    C_ABORT = 7,         // a barrier timed out
    C_BAR_PREP = 32,     // barrier counter of the BFS kernel
    C_BAR_RUN = 64,      // barrier counter of the relaxation kernel
    C_FLAGS = 96,        // 3 rotating "not converged" words, one line each
    C_WORDS = 256
};

enum StatusBits : int {
    ST_BAD_FACE = 1,
    ST_BAD_COORD = 2,
    ST_BAD_SOURCE = 4,
    ST_DUP_SOURCE = 8,
    ST_BARRIER_TIMEOUT = 16,
};

// ---- grid barrier ------------------------------------------------------
// Every workgroup of a cooperative launch increments one counter; the
// barrier of epoch e completes when it reaches e * nblocks.  Agent-scope
// release before and acquire after make every store before the barrier
// visible to every load after it, across XCDs.  A wall-clock limit turns a
// barrier that can never complete into an abort flag instead of a hang.
struct GridBarrier {
    unsigned* counter;
    int* abort_flag;
    unsigned nblocks;
    unsigned epoch;

    __device__ bool sync() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0) {
            epoch += 1;
            const unsigned target = epoch * nblocks;
            __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const long long t0 = wall_clock64();
            while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(1);
                if (wall_clock64() - t0 > 400000000ll) {   // seconds at the 100 MHz clock
                    __hip_atomic_fetch_or(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        return __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    }
};

__device__ inline int load_agent(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- block-wide scans (kBlock threads) ----------------------------------
// Exclusive prefix of `v` over the workgroup; *total receives the sum.
template <typename T>
__device__ inline T block_exclusive_scan(T v, T* total) {
    __shared__ T warp_sums[kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    T x = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        T y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    if (lane == kWave - 1) warp_sums[wid] = x;
    __syncthreads();
    T wbase = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) {
        T s = warp_sums[w];
        if (w < wid) wbase += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return wbase + x - v;
}

template <typename T>
__device__ inline T block_sum(T v) {
    T tot;
    (void)block_exclusive_scan(v, &tot);
    return tot;
}

}  // namespace ptp

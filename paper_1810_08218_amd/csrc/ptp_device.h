// Device-side building blocks shared by the PTP kernels: control-block
// layout, coherent memory access, the grid barrier of the persistent
// kernels and block scans.  Internal to the HIP library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptp {

constexpr int kBlock = 256;                 // threads per workgroup (4 waves)
constexpr int kWave = 64;
constexpr int kLine = 32;                   // ints per 128-byte line

// ---- control block (int32 words in device memory) ----------------------
enum CtrlWord : int {
    C_STATUS = 0,        // validation / fault bits (ST_*)
    C_RHO = 1,           // number of toplesets
    C_REACH = 2,         // number of reachable vertices
    C_ITERS = 3,         // K of the last run
    C_RUNSTAT = 4,       // 0 ok, 1 cap reached (ENOCONV)
    C_UPD_LO = 5,        // vertex updates, low / high 32 bits
    C_UPD_HI = 6,
    C_ABORT = 7,         // a barrier timed out
    C_FPS_KEY = 8,       // words 8, 9: farthest point sampling argmax key (64 bits)
    C_QHEAD = 12,        // words 12..14: next entry of each mesh queue of the relaxation
    C_WORDS = 64
};

enum StatusBits : int {
    ST_BAD_FACE = 1,
    ST_BAD_COORD = 2,
    ST_BAD_SOURCE = 4,
    ST_DUP_SOURCE = 8,
    ST_FPS_EMPTY = 16,   // farthest point sampling found no vertex to add
};

// ---- coherent access ---------------------------------------------------
// Each XCD has its own L2; plain stores may sit there unseen by the other
// XCDs.  Data that one workgroup writes and another reads inside the same
// persistent kernel (distances, labels, levels, frontier bitmaps, counters)
// is therefore only touched with agent-scope accesses, which are coherent
// across XCDs without L2 write-back or invalidation.  Read-only data (mesh,
// incidence, offsets) keeps ordinary cached loads.
template <typename T>
__device__ inline T ld_c(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ inline void st_c(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Store for data shared inside a group.  When every workgroup of the group
// runs on one XCD (`local`), a plain store suffices: it writes through the
// CU's L1 into the XCD's L2, where the readers' coherent loads find it; an
// agent-scope store has to travel to memory, which costs several times more
// when it follows coherent loads of the same lines.  Otherwise agent scope.
template <typename T>
__device__ inline void st_g(T* p, T v, bool local) {
    if (local) *p = v;
    else st_c(p, v);
}

// Index of the XCD (accelerator complex die) this workgroup runs on.
__device__ inline unsigned xcc_id() {
    unsigned x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
    return x & 0xfu;
}
// Wait until this wave's outstanding memory operations have completed.  Also
// a compiler barrier: no access moves across it.
__device__ inline void wait_memory() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Workgroup barrier that orders LDS only: each wave waits for its own LDS
// operations, not for its outstanding global stores (__syncthreads waits for
// those too, a full memory round trip when they are scattered).
__device__ inline void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// OR of `v` (bits 0 and 1) over the workgroup: ballots per wave, one LDS
// word per wave, one LDS-only barrier.  `slots` holds two sets of one word
// per wave, used in turn (`par` flips on every call), so that a wave writing
// the words of the next call cannot overwrite those another wave is still
// reading (it can only get there after the next call's barrier, which every
// wave reaches after its reads).
__device__ inline unsigned block_or(unsigned v, unsigned* slots, unsigned& par) {
    constexpr int kWaves = kBlock / kWave;
    unsigned* set = slots + par * kWaves;
    par ^= 1u;
    const unsigned long long b0 = __ballot((v & 1u) != 0);
    const unsigned long long b1 = __ballot((v & 2u) != 0);
    if ((threadIdx.x & (kWave - 1)) == 0) set[threadIdx.x / kWave] = (b0 ? 1u : 0u) | (b1 ? 2u : 0u);
    lds_barrier();
    unsigned r = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) r |= set[w];
    return r;
}

// ---- group barrier -----------------------------------------------------
// Flag-array barrier among the gsize workgroups of a group of a cooperative
// launch.  Every workgroup publishes (epoch << 1 | bit) in its own 128-byte
// line and then polls every line of the group (one line per thread), so a
// barrier costs one store-to-load hop; the OR of the bits (the "not
// converged" vote of the PTP iteration, a duplicate source in the BFS) comes
// out the same in every workgroup.  The lines of consecutive epochs
// alternate between two banks: a workgroup may already publish epoch e + 1
// while a slower one still reads epoch e, but it cannot reach e + 2 before
// every workgroup has published e + 1, that is, finished reading e.  No
// counter is contended.  A wall-clock limit turns a barrier that can never
// complete into an abort flag instead of a hang: the workgroups whose wait
// times out raise the flag and leave; the flag is not read on the way (every
// workgroup of a stuck group times out by itself), which saves a memory
// round trip per barrier.  The votes inside the workgroup go through LDS
// words and LDS-only barriers (block_or), not through __syncthreads_or /
// __syncthreads_and, which cost several times more.
//
// Ordering: each wave waits for its own coherent stores to complete before
// the workgroup publishes; loads after the barrier are coherent loads issued
// after every flag was observed.  A group of one workgroup needs only that
// wait and the block barrier (its coherent accesses meet in L2).
struct FlagBarrier {
    unsigned* bank0;     // [gsize * kLine], zero at launch: even epochs
    unsigned* bank1;     // [gsize * kLine], zero at launch: odd epochs
    int* abort_flag;
    unsigned gsize, rank;
    unsigned epoch;
    bool local = false;  // the whole group runs on one XCD: plain flag stores
    unsigned* slots = nullptr;   // LDS: 2 * kBlock / kWave words (block_or)
    unsigned par = 0;

    static constexpr long long kTimeoutTicks = 400000000ll;   // seconds at 100 MHz

    // Wait until the line at p holds an epoch >= want.  The clock is read
    // every 64 polls only, the first time after 64 (a read costs a scalar
    // memory round trip, which would delay the next poll).
    __device__ bool spin_ge(const unsigned* p, unsigned want, unsigned* seen) {
        long long t0 = 0;
        unsigned v;
        for (unsigned n = 1; ((v = ld_c(p)) >> 1) < want; ++n) {
            __builtin_amdgcn_s_sleep(1);
            if ((n & 63u) == 0) {
                const long long t = wall_clock64();
                if (n == 64) {
                    t0 = t;
                } else if (t - t0 > kTimeoutTicks) {
                    __hip_atomic_fetch_or(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    *seen = 0;
                    return false;
                }
            }
        }
        *seen = v;
        return true;
    }

    // Returns false when the barrier timed out (the kernel must exit);
    // *any receives the OR of `bit` over the group.
    __device__ bool sync(unsigned bit, unsigned* any) {
        const unsigned tid = threadIdx.x;
        wait_memory();
        bit = block_or(bit ? 1u : 0u, slots, par);
        if (gsize == 1) {            // a group of one workgroup: the block barrier suffices
            *any = bit;
            return true;
        }
        epoch += 1;
        unsigned* lines = (epoch & 1u) ? bank1 : bank0;
        if (tid == 0) st_g(lines + (size_t)rank * kLine, (epoch << 1) | bit, local);
        unsigned acc = 0;
        for (unsigned x = tid; x < gsize; x += blockDim.x) {
            unsigned v;
            if (!spin_ge(lines + (size_t)x * kLine, epoch, &v)) {
                acc |= 2u;
                break;
            }
            acc |= v & 1u;
        }
        const unsigned r = block_or(acc, slots, par);
        *any = r & 1u;
        return (r & 2u) == 0;   // a timed-out wait raised the abort flag itself
    }
};

// Mesh of a flat element index: the largest b with prefix[b] <= x
// (prefix[0] = 0, prefix[B] = total; empty meshes are skipped).
__device__ inline int mesh_of(const int* prefix, int B, long long x) {
    int lo = 0, hi = B;          // invariant: prefix[lo] <= x < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((long long)prefix[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// mesh_of by one whole wave (every lane calls it and gets the result): each
// round the 64 lanes test 64 evenly spaced prefix entries of the remaining
// range and a ballot keeps the last one at or below x, so 512 meshes take two
// dependent loads instead of nine.
__device__ inline int mesh_of_wave(const int* prefix, int B, long long x) {
    const int lane = threadIdx.x & (kWave - 1);
    int lo = 0, len = B;         // invariant: prefix[lo] <= x < prefix[lo + len]
    while (len > 1) {
        const int step = (len + kWave - 1) / kWave;
        const int i = lo + lane * step;
        const bool le = i < lo + len && (long long)prefix[i] <= x;
        const unsigned long long m = __ballot(le);      // lane 0 always set
        const int last = 63 - __clzll((long long)m);
        const int nlo = lo + last * step;
        len = min(step, lo + len - nlo);
        lo = nlo;
    }
    return lo;
}

// Element loops over the concatenation take tiles of kTile consecutive
// elements per workgroup.  The mesh of a tile's first element is found once
// (binary search over the prefix) and each thread advances it across the
// few mesh boundaries inside the tile, so an element costs no search of its
// own.  f(x, b) gets the element and its mesh.
constexpr int kTileItems = 8;
constexpr int kTile = kTileItems * kBlock;

template <class Fn>
__device__ inline void for_tiles(const int* prefix, int B, long long total, Fn f) {
    __shared__ int tile_mesh;
    const long long ntiles = (total + kTile - 1) / kTile;
    for (long long t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const long long base = t * kTile;
        if (threadIdx.x < kWave) {
            const int b0 = mesh_of_wave(prefix, B, base);
            if (threadIdx.x == 0) tile_mesh = b0;
        }
        __syncthreads();
        int b = tile_mesh;
        __syncthreads();        // tile_mesh is rewritten for the next tile
        for (int q = 0; q < kTileItems; ++q) {
            const long long x = base + (long long)q * kBlock + threadIdx.x;
            if (x >= total) break;
            while ((long long)prefix[b + 1] <= x) ++b;
            f(x, b);
        }
    }
}

// The meshes of this thread's elements of tile t (element base + q kBlock +
// threadIdx.x of the tile, q < kTileItems) into bq[q], for loops that load
// all their elements before using any (so that the loads overlap).  When the
// tile lies inside one mesh, the usual case, no thread reads the prefix.
__device__ inline void tile_meshes(const int* prefix, int B, long long total, long long t, int* bq) {
    __shared__ int tile_b, tile_whole;
    const long long base = t * kTile;
    if (threadIdx.x < kWave) {
        const int b0 = mesh_of_wave(prefix, B, base);
        const long long end = base + kTile < total ? base + kTile : total;
        if (threadIdx.x == 0) {
            tile_b = b0;
            tile_whole = (long long)prefix[b0 + 1] >= end;
        }
    }
    __syncthreads();
    int b = tile_b;
    const bool whole = tile_whole != 0;
    __syncthreads();        // both are rewritten for the next tile
#pragma unroll
    for (int q = 0; q < kTileItems; ++q) {
        const long long x = base + (long long)q * kBlock + threadIdx.x;
        if (!whole && x < total)
            while ((long long)prefix[b + 1] <= x) ++b;
        bq[q] = b;
    }
}

// ---- block-wide scans --------------------------------------------------
// Inclusive prefix sum over the 64 lanes of a wave with DPP moves: shifts by
// 1, 2, 4, 8 inside each row of 16 lanes (lanes shifted in from outside the
// row add 0), then the last lane of row 0 / 2 added to rows 1 / 3 and the
// last lane of row 1 to rows 2 and 3.  (A shuffle through the LDS crossbar
// per step costs several times more.)
__device__ inline int wave_inclusive_sum(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 -> rows 1, 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 -> rows 2, 3
    return x;
}

// Exclusive prefix of `v` over a workgroup of NT threads; *total receives
// the sum.  LDS_ONLY: its barriers order LDS only (see lds_barrier).
template <int NT, typename T, bool LDS_ONLY = false>
__device__ inline T block_exclusive_scan_n(T v, T* total) {
    __shared__ T warp_sums[NT / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    T x = wave_inclusive_sum(v);
    if (lane == kWave - 1) warp_sums[wid] = x;
    if (LDS_ONLY) lds_barrier();
    else __syncthreads();
    T wbase = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / kWave; ++w) {
        T s = warp_sums[w];
        if (w < wid) wbase += s;
        tot += s;
    }
    if (LDS_ONLY) lds_barrier();
    else __syncthreads();
    *total = tot;
    return wbase + x - v;
}

template <typename T>
__device__ inline T block_exclusive_scan(T v, T* total) {
    return block_exclusive_scan_n<kBlock>(v, total);
}

template <typename T>
__device__ inline T block_sum(T v) {
    T tot;
    (void)block_exclusive_scan(v, &tot);
    return tot;
}

}  // namespace ptp

// Preparation of a mesh for PTP on the device:
//   validation (problem statement, Sec. 3.1),
//   vertex -> triangle incidence,
//   toplesets V_r by a level-synchronous BFS from S (Sec. 4.1), emitted in the
//   canonical order (topleset, then ascending caller id),
//   reorder of coordinates and incidence into that order (Sec. 4.3), with
//   every triangle stored at each of its corners as the opposite edge
//   ("wedge") in new positions.
#include "ptp_device.h"
#include "ptp_kernels.h"

namespace ptp {

namespace {

constexpr int kScanItems = 16;                      // per thread
constexpr int kScanTile = kBlock * kScanItems;      // per workgroup
constexpr int kListCap = 4096;                      // BFS LDS batch

__device__ inline bool gated(const int* ctrl) { return ld_c(ctrl + C_STATUS) != 0; }

__global__ __launch_bounds__(kBlock) void k_fill(int* p, long long len, int val) {
    for (long long x = blockIdx.x * (long long)kBlock + threadIdx.x; x < len;
         x += (long long)gridDim.x * kBlock)
        p[x] = val;
}

__global__ __launch_bounds__(kBlock) void k_validate(const float* V, int n, const int* F, int f,
                                                     const int* S, int m, int* ctrl) {
    int bad = 0;
    const long long gsz = (long long)gridDim.x * kBlock;
    const long long g0 = blockIdx.x * (long long)kBlock + threadIdx.x;
    for (long long x = g0; x < 3ll * f; x += gsz) {
        int v = F[x];
        if (v < 0 || v >= n) bad |= ST_BAD_FACE;
    }
    for (long long x = g0; x < 3ll * n; x += gsz) {
        float c = V[x];
        if (!(fabsf(c) <= 3.0e38f)) bad |= ST_BAD_COORD;
    }
    for (long long x = g0; x < m; x += gsz) {
        int s = S[x];
        if (s < 0 || s >= n) bad |= ST_BAD_SOURCE;
    }
    if (bad) atomicOr(ctrl + C_STATUS, bad);
}

// degree of each caller vertex, counted into row[v + 1]
__global__ __launch_bounds__(kBlock) void k_count(const int* F, int f, int* row, const int* ctrl) {
    if (gated(ctrl)) return;
    const long long gsz = (long long)gridDim.x * kBlock;
    for (long long x = blockIdx.x * (long long)kBlock + threadIdx.x; x < 3ll * f; x += gsz)
        atomicAdd(row + F[x] + 1, 1);
}

__global__ __launch_bounds__(kBlock) void k_fill_incidence(const int* F, int f, const int* row,
                                                           int* cursor, int* corner, const int* ctrl) {
    if (gated(ctrl)) return;
    const long long gsz = (long long)gridDim.x * kBlock;
    for (long long x = blockIdx.x * (long long)kBlock + threadIdx.x; x < 3ll * f; x += gsz) {
        int v = F[x];
        int slot = atomicAdd(cursor + v, 1);
        corner[row[v] + slot] = (int)x;
    }
}

// ---- in-place inclusive scan of a[0..len) (three passes) ----------------
__device__ inline int tile_load_scan(int* a, long long len, long long base, int* tile_sum,
                                     int* vals) {
    __shared__ int buf[kScanTile];
    for (int q = 0; q < kScanItems; ++q) {
        long long x = base + q * kBlock + threadIdx.x;
        buf[q * kBlock + threadIdx.x] = x < len ? a[x] : 0;
    }
    __syncthreads();
    int s = 0;
    for (int q = 0; q < kScanItems; ++q) {
        vals[q] = buf[threadIdx.x * kScanItems + q];
        s += vals[q];
    }
    __syncthreads();
    int tot;
    int pre = block_exclusive_scan(s, &tot);
    *tile_sum = tot;
    return pre;
}

__global__ __launch_bounds__(kBlock) void k_scan_partial(int* a, long long len, int* bsum,
                                                         const int* ctrl) {
    if (gated(ctrl)) return;
    int vals[kScanItems];
    int tot;
    (void)tile_load_scan(a, len, (long long)blockIdx.x * kScanTile, &tot, vals);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_scan_bsums(int* bsum, int nb, const int* ctrl) {
    if (gated(ctrl)) return;
    int carry = 0;
    for (int base = 0; base < nb; base += kBlock) {
        int x = base + threadIdx.x;
        int v = x < nb ? bsum[x] : 0;
        int tot;
        int pre = block_exclusive_scan(v, &tot);
        if (x < nb) bsum[x] = carry + pre;
        carry += tot;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(int* a, long long len, const int* bsum,
                                                       const int* ctrl) {
    if (gated(ctrl)) return;
    __shared__ int out[kScanTile];
    int vals[kScanItems];
    int tot;
    const long long base = (long long)blockIdx.x * kScanTile;
    int run = tile_load_scan(a, len, base, &tot, vals) + bsum[blockIdx.x];
    for (int q = 0; q < kScanItems; ++q) {
        run += vals[q];
        out[threadIdx.x * kScanItems + q] = run;
    }
    __syncthreads();
    for (int q = 0; q < kScanItems; ++q) {
        long long x = base + q * kBlock + threadIdx.x;
        if (x < len) a[x] = out[q * kBlock + threadIdx.x];
    }
}

hipError_t scan_inplace(int* a, long long len, int* tmp, const int* ctrl, hipStream_t st) {
    if (len <= 0) return hipSuccess;
    int nb = (int)((len + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(k_scan_partial, dim3(nb), dim3(kBlock), 0, st, a, len, tmp, ctrl);
    hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(kBlock), 0, st, tmp, nb, ctrl);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kBlock), 0, st, a, len, tmp, ctrl);
    return hipGetLastError();
}

// ---- BFS toplesets (persistent, cooperative launch) ---------------------
struct BfsArgs {
    int n, m, nwords, cw;
    const int* F;
    const int* S;
    const int* row;
    const int* corner;
    int* level;
    int* perm;
    int* iperm;
    int* offsets;
    unsigned* bits;
    int* cnt;
    int* ctrl;
    unsigned* bar;
};

__device__ inline int other1(int c) { return c == 2 ? 0 : c + 1; }
__device__ inline int other2(int c) { return c == 0 ? 2 : c - 1; }

// The bitmap of V_r is split into G equal chunks of words, one per
// workgroup.  Per level r, each workgroup
//   1. reads the chunk counts of V_r (made by the discoveries of level r-1),
//      giving |V_r| and the start of its chunk inside V_r;
//   2. writes its chunk's vertices, in ascending id order, to perm (this is
//      the canonical order: level, then id), clears the chunk;
//   3. expands those vertices: each unvisited neighbour gets level r+1 (one
//      CAS decides the discoverer), its bit in the next bitmap and a count in
//      the next chunk counts.
// One grid barrier per level.  A level with no vertex ends the loop: rho = r.
// level, bits and cnt are shared between workgroups: coherent access only.
__global__ __launch_bounds__(kBlock) void k_bfs(BfsArgs a) {
    if (gated(a.ctrl)) return;
    const int G = gridDim.x, w = blockIdx.x, tid = threadIdx.x;
    FlagBarrier gb{a.bar, a.bar + (size_t)G * kLine, a.ctrl + C_ABORT, 0};
    unsigned any = 0;
    const long long gsz = (long long)G * kBlock;
    const long long g0 = (long long)w * kBlock + tid;
    unsigned* bits0 = a.bits;
    unsigned* bits1 = a.bits + a.nwords;
    for (long long v = g0; v < a.n; v += gsz) st_c(a.level + v, -1);
    for (long long x = g0; x < 2ll * a.nwords; x += gsz) st_c(a.bits + x, 0u);
    for (long long x = g0; x < 4ll * G; x += gsz) st_c(a.cnt + x, 0);
    if (!gb.sync(0, &any)) return;
    unsigned dup = 0;
    for (long long s = g0; s < a.m; s += gsz) {
        int v = a.S[s];
        if (atomicCAS(a.level + v, -1, 0) != -1) {
            dup = 1;
        } else {
            atomicOr(bits0 + (v >> 5), 1u << (v & 31));
            atomicAdd(a.cnt + (v >> 5) / a.cw, 1);
        }
    }
    if (!gb.sync(dup, &any)) return;
    if (any) {
        if (w == 0 && tid == 0) atomicOr(a.ctrl + C_STATUS, ST_DUP_SOURCE);
        return;
    }

    __shared__ int list[kListCap];
    const int wbeg = min(w * a.cw, a.nwords);
    const int wend = min(wbeg + a.cw, a.nwords);
    const int q = (wend - wbeg + kBlock - 1) / kBlock;
    const int my0 = min(wbeg + tid * q, wend);
    const int my1 = min(my0 + q, wend);
    int base = 0;
    int r = 0;
    for (;; ++r) {
        const int* cr = a.cnt + (r % 3) * G;
        int part = 0, partpre = 0;
        for (int x = tid; x < G; x += kBlock) {
            int c = ld_c(cr + x);
            part += c;
            if (x < w) partpre += c;
        }
        const int total = block_sum(part);
        const int chunk_pre = block_sum(partpre);
        if (total == 0) break;
        if (w == 0 && tid == 0) a.offsets[r] = base;
        if (tid == 0) st_c(a.cnt + ((r + 2) % 3) * G + w, 0);
        unsigned* cur = (r & 1) ? bits1 : bits0;
        unsigned* nxt = (r & 1) ? bits0 : bits1;
        int* cn = a.cnt + ((r + 1) % 3) * G;

        int pc = 0;
        for (int x = my0; x < my1; ++x) pc += __popc(ld_c(cur + x));
        int tot_w;
        const int pre = block_exclusive_scan(pc, &tot_w);
        for (int done = 0; done < tot_w; done += kListCap) {
            int rank = pre;
            for (int x = my0; x < my1 && rank < done + kListCap; ++x) {
                unsigned word = ld_c(cur + x);
                while (word) {
                    int b = __ffs(word) - 1;
                    word &= word - 1;
                    int u = x * 32 + b;
                    if (rank >= done && rank < done + kListCap) {
                        list[rank - done] = u;
                        int pos = base + chunk_pre + rank;
                        a.perm[pos] = u;
                        a.iperm[u] = pos;
                    }
                    ++rank;
                }
            }
            __syncthreads();
            const int cntl = min(kListCap, tot_w - done);
            const int lvl = r + 1;
            for (int t = tid; t < cntl; t += kBlock) {
                const int u = list[t];
                for (int e = a.row[u]; e < a.row[u + 1]; ++e) {
                    const int cx = a.corner[e];
                    const int tri = cx / 3, c = cx - 3 * tri;
                    const int nb[2] = {a.F[3 * tri + other1(c)], a.F[3 * tri + other2(c)]};
                    for (int z = 0; z < 2; ++z) {
                        const int x = nb[z];
                        if (ld_c(a.level + x) < 0 && atomicCAS(a.level + x, -1, lvl) == -1) {
                            atomicOr(nxt + (x >> 5), 1u << (x & 31));
                            atomicAdd(cn + (x >> 5) / a.cw, 1);
                        }
                    }
                }
            }
            __syncthreads();
        }
        for (int x = my0; x < my1; ++x) st_c(cur + x, 0u);
        base += total;
        if (!gb.sync(0, &any)) return;
    }
    const int rho = r;
    const int reach = base;
    if (w == 0 && tid == 0) a.offsets[rho] = reach;

    // unreachable vertices follow, in ascending id order
    const int cv = (a.n + G - 1) / G;
    const int vb = min(w * cv, a.n), ve = min(vb + cv, a.n);
    const int qv = (ve - vb + kBlock - 1) / kBlock;
    const int v0 = min(vb + tid * qv, ve), v1 = min(v0 + qv, ve);
    int pc = 0;
    for (int v = v0; v < v1; ++v) pc += ld_c(a.level + v) < 0;
    int tot_w;
    int pre = block_exclusive_scan(pc, &tot_w);
    if (tid == 0) st_c(a.cnt + 3 * G + w, tot_w);
    if (!gb.sync(0, &any)) return;
    int partpre = 0;
    for (int x = tid; x < w; x += kBlock) partpre += ld_c(a.cnt + 3 * G + x);
    const int chunk_pre = block_sum(partpre);
    int pos = reach + chunk_pre + pre;
    for (int v = v0; v < v1; ++v)
        if (ld_c(a.level + v) < 0) {
            a.perm[pos] = v;
            a.iperm[v] = pos;
            ++pos;
        }
    if (w == 0 && tid == 0) {
        a.ctrl[C_RHO] = rho;
        a.ctrl[C_REACH] = reach;
    }
}

__global__ void k_zero_lines(unsigned* p, long long len) {
    for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < len;
         x += (long long)gridDim.x * blockDim.x)
        p[x] = 0u;
}

// degree of each position, into rowN[p + 1]
__global__ __launch_bounds__(kBlock) void k_degree_new(const int* perm, const int* rowO, int n,
                                                       int* rowN, const int* ctrl) {
    if (gated(ctrl)) return;
    const long long gsz = (long long)gridDim.x * kBlock;
    for (long long p = blockIdx.x * (long long)kBlock + threadIdx.x; p < n; p += gsz) {
        int v = perm[p];
        rowN[p + 1] = rowO[v + 1] - rowO[v];
        if (p == 0) rowN[0] = 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_reorder(const float* V, const int* F, const int* perm,
                                                    const int* iperm, const int* rowO,
                                                    const int* corner, const int* rowN, int n,
                                                    float4* xyz, int2* wedge, const int* ctrl) {
    if (gated(ctrl)) return;
    const long long gsz = (long long)gridDim.x * kBlock;
    for (long long p = blockIdx.x * (long long)kBlock + threadIdx.x; p < n; p += gsz) {
        const int v = perm[p];
        xyz[p] = make_float4(V[3ll * v], V[3ll * v + 1], V[3ll * v + 2], 0.f);
        const int b = rowO[v], e = rowO[v + 1];
        int o = rowN[p];
        for (int x = b; x < e; ++x, ++o) {
            const int cx = corner[x];
            const int tri = cx / 3, c = cx - 3 * tri;
            wedge[o] = make_int2(iperm[F[3 * tri + other1(c)]], iperm[F[3 * tri + other2(c)]]);
        }
    }
}

int grid_for(long long work) {
    long long g = (work + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (int)g;
}

}  // namespace

hipError_t launch_prepare(const Work& w, int n, int f, int m, const float* V, const int* F,
                          const int* S, int g_bfs, hipStream_t st) {
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(kBlock), 0, st, w.ctrl, (long long)C_WORDS, 0);
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n + 1)), dim3(kBlock), 0, st, w.rowO, (long long)n + 1, 0);
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kBlock), 0, st, w.cursor, (long long)n, 0);
    long long vwork = 3ll * (f > n ? f : n);
    hipLaunchKernelGGL(k_validate, dim3(grid_for(vwork)), dim3(kBlock), 0, st, V, n, F, f, S, m, w.ctrl);
    hipLaunchKernelGGL(k_count, dim3(grid_for(3ll * f)), dim3(kBlock), 0, st, F, f, w.rowO, w.ctrl);
    hipError_t e = scan_inplace(w.rowO + 1, n, w.scan_tmp, w.ctrl, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fill_incidence, dim3(grid_for(3ll * f)), dim3(kBlock), 0, st, F, f, w.rowO,
                       w.cursor, w.faceO, w.ctrl);
    e = hipGetLastError();
    if (e != hipSuccess) return e;

    BfsArgs a;
    a.n = n;
    a.m = m;
    a.nwords = (n + 31) / 32;
    a.cw = (a.nwords + g_bfs - 1) / g_bfs;
    if (a.cw < 1) a.cw = 1;
    a.F = F;
    a.S = S;
    a.row = w.rowO;
    a.corner = w.faceO;
    a.level = w.level;
    a.perm = w.perm;
    a.iperm = w.iperm;
    a.offsets = w.offsets;
    a.bits = w.bits;
    a.cnt = w.cnt;
    a.ctrl = w.ctrl;
    a.bar = w.bar;
    launch_barrier_reset(w, g_bfs, st);
    void* args[] = {&a};
    e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_bfs), dim3(g_bfs), dim3(kBlock),
                                   args, 0, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_degree_new, dim3(grid_for(n)), dim3(kBlock), 0, st, w.perm, w.rowO, n,
                       w.rowN, w.ctrl);
    e = scan_inplace(w.rowN + 1, n, w.scan_tmp, w.ctrl, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reorder, dim3(grid_for(n)), dim3(kBlock), 0, st, V, F, w.perm, w.iperm,
                       w.rowO, w.faceO, w.rowN, n, w.xyz, w.wedge, w.ctrl);
    return hipGetLastError();
}

void launch_barrier_reset(const Work& w, int g, hipStream_t st) {
    const long long len = (long long)(g + 1) * kLine;
    hipLaunchKernelGGL(k_zero_lines, dim3((unsigned)((len + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                       w.bar, len);
}

int max_coop_blocks_bfs(int cus) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_bfs, kBlock, 0) != hipSuccess || nb < 1)
        nb = 1;
    return nb * cus;
}

}  // namespace ptp

// Preparation of a batch of meshes for PTP on the device:
//   validation (problem statement, Sec. 3.1),
//   vertex -> triangle incidence over the concatenation, every triangle stored
//   at each of its corners as the opposite edge ("wedge"),
//   toplesets V_r of each mesh by a level-synchronous BFS from its sources
//   (Sec. 4.1), emitted in the canonical order (topleset, then ascending id),
//   reorder of coordinates and incidence into that order (Sec. 4.3), and the
//   incidence as fans of neighbours (each neighbour named once) for the
//   relaxation.
#include "ptp_device.h"
#include "ptp_kernels.h"

namespace ptp {

namespace {

constexpr int kScanItems = 16;                      // per thread
constexpr int kScanTile = kBlock * kScanItems;      // per workgroup
constexpr int kListCap = 4096;                      // BFS LDS batch

__device__ inline bool gated(const int* ctrl) { return ld_c(ctrl + C_STATUS) != 0; }
__device__ inline int other1(int c) { return c == 2 ? 0 : c + 1; }
__device__ inline int other2(int c) { return c == 0 ? 2 : c - 1; }

__global__ __launch_bounds__(kBlock) void k_fill(int* p, long long len, int val) {
    for (long long x = blockIdx.x * (long long)kBlock + threadIdx.x; x < len;
         x += (long long)gridDim.x * kBlock)
        p[x] = val;
}

__global__ __launch_bounds__(kBlock) void k_zero_lines(unsigned* p, long long len) {
    for (long long x = blockIdx.x * (long long)kBlock + threadIdx.x; x < len;
         x += (long long)gridDim.x * kBlock)
        p[x] = 0u;
}

// Coordinates must be finite, sources lie in their mesh (face ids are
// checked by k_count).  Bad meshes are flagged in their state and in the
// batch word.
// Loops run over the internal (concatenated) index spaces and read the
// caller's rows.
__global__ __launch_bounds__(kBlock) void k_validate(const float* __restrict__ V, const int* __restrict__ F,
                                                     const int* __restrict__ S, const MeshDesc* mesh, int B,
                                                     const int* vo, const int* fo3, const int* so, long long N,
                                                     long long F3, long long Stot, MeshState* state, int* ctrl) {
    int bad = 0;
    // coordinates: every element of a tile loaded, then checked (the face
    // corners are checked by k_count, which reads them anyway)
    for (long long t = blockIdx.x; t < (N + kTile - 1) / kTile; t += gridDim.x) {
        int bq[kTileItems];
        long long at[kTileItems];
        float c[kTileItems][3];
        tile_meshes(vo, B, N, t, bq);
#pragma unroll
        for (int q = 0; q < kTileItems; ++q)
            at[q] = 3 * ((long long)mesh[bq[q]].v_in + (t * kTile + (long long)q * kBlock + threadIdx.x - vo[bq[q]]));
        const bool full = t * kTile + kTile <= N;
#pragma unroll
        for (int q = 0; q < kTileItems; ++q) {
            const bool ok = full || t * kTile + (long long)q * kBlock + threadIdx.x < N;
#pragma unroll
            for (int k = 0; k < 3; ++k) c[q][k] = ok ? V[at[q] + k] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < kTileItems; ++q)
            if (!(fabsf(c[q][0]) <= 3.0e38f) || !(fabsf(c[q][1]) <= 3.0e38f) || !(fabsf(c[q][2]) <= 3.0e38f)) {
                atomicOr(&state[bq[q]].status, ST_BAD_COORD);
                bad |= ST_BAD_COORD;
            }
    }
    for_tiles(so, B, Stot, [&](long long x, int b) {
        const int s = S[mesh[b].s_in + (x - so[b])];
        if (s < 0 || s >= mesh[b].n) {
            atomicOr(&state[b].status, ST_BAD_SOURCE);
            bad |= ST_BAD_SOURCE;
        }
    });
    if (bad) atomicOr(ctrl + C_STATUS, bad);
}

// Corner loops of the incidence build: a tile of kTile corners (consecutive
// faces) usually touches a narrow range of vertex ids, so their counts are
// gathered in LDS first and each distinct vertex costs one global atomic
// instead of one per corner (a vertex appears in about six corners, mostly of
// nearby faces).  Tiles whose id range exceeds kAgg fall back to per-corner
// global atomics.
constexpr int kAgg = 4096;

constexpr int kBadCorner = -2;

struct TileCorners {
    int vid[kTileItems];   // global vertex id of each of this thread's corners, -1 past the end,
                           // kBadCorner for an id outside the corner's mesh
    int b[kTileItems];     // the corner's mesh
    long long t3[kTileItems];   // caller row of the corner's face
    int c[kTileItems];     // corner inside the face
    int vo[kTileItems];    // vertex offset of the corner's mesh
};

// Loads this thread's corners of tile t and returns the tile's id range
// [*lo, *hi] (block-wide; lo > hi when the tile is empty).  The corners'
// meshes are found first, then every corner is loaded before any is used.
// kCheck: ids outside the corner's mesh become kBadCorner (else they are
// known to be valid).
template <bool kCheck>
__device__ inline void load_tile_corners(const int* F, const MeshDesc* mesh, int B, const int* fo3, long long F3,
                                         long long t, TileCorners& tc, int* lo, int* hi, int* red) {
    const long long base = t * kTile;
    int bq[kTileItems], nq[kTileItems];
    tile_meshes(fo3, B, F3, t, bq);
#pragma unroll
    for (int q = 0; q < kTileItems; ++q) {
        const long long x = base + (long long)q * kBlock + threadIdx.x;
        const int b = bq[q];
        const long long lc = x - fo3[b];
        tc.t3[q] = 3 * (long long)mesh[b].f_in + (lc - lc % 3);
        tc.c[q] = (int)(lc % 3);
        tc.vo[q] = mesh[b].v_off;
        tc.b[q] = b;
        nq[q] = kCheck ? mesh[b].n : 0x7fffffff;
    }
    int f[kTileItems];
    if (base + kTile <= F3) {       // a full tile: no guards, so the loads issue together
#pragma unroll
        for (int q = 0; q < kTileItems; ++q) f[q] = F[tc.t3[q] + tc.c[q]];
    } else {
#pragma unroll
        for (int q = 0; q < kTileItems; ++q) f[q] = base + (long long)q * kBlock + threadIdx.x < F3 ? F[tc.t3[q] + tc.c[q]] : -1;
    }
#pragma unroll
    for (int q = 0; q < kTileItems; ++q) {
        const bool past = base + (long long)q * kBlock + threadIdx.x >= F3;
        tc.vid[q] = past ? -1 : (!kCheck || (f[q] >= 0 && f[q] < nq[q])) ? tc.vo[q] + f[q] : kBadCorner;
    }
    int mn = 0x7fffffff, mx = -1;
#pragma unroll
    for (int q = 0; q < kTileItems; ++q)
        if (tc.vid[q] >= 0) {
            mn = min(mn, tc.vid[q]);
            mx = max(mx, tc.vid[q]);
        }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        mn = min(mn, __shfl_xor(mn, o, kWave));
        mx = max(mx, __shfl_xor(mx, o, kWave));
    }
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        red[w] = mn;
        red[4 + w] = mx;
    }
    __syncthreads();
    mn = min(min(red[0], red[1]), min(red[2], red[3]));
    mx = max(max(red[4], red[5]), max(red[6], red[7]));
    *lo = mn;
    *hi = mx;
    __syncthreads();        // red is rewritten by the next tile
}

// Degree of each internal vertex, counted into row[v + 1]; a face id outside
// its mesh flags the mesh (ST_BAD_FACE) and is not counted (the passes after
// this one are gated on the flag).
__global__ __launch_bounds__(kBlock) void k_count(const int* F, const MeshDesc* mesh, int B,
                                                  const int* fo3, long long F3, int* row,
                                                  MeshState* state, int* ctrl) {
    if (gated(ctrl)) return;
    __shared__ int cnt[kAgg];
    __shared__ int red[8];
    const long long ntiles = (F3 + kTile - 1) / kTile;
    int bad = 0;
    for (long long t = blockIdx.x; t < ntiles; t += gridDim.x) {
        TileCorners tc;
        int lo, hi;
        load_tile_corners<true>(F, mesh, B, fo3, F3, t, tc, &lo, &hi, red);
#pragma unroll
        for (int q = 0; q < kTileItems; ++q)
            if (tc.vid[q] == kBadCorner) {
                atomicOr(&state[tc.b[q]].status, ST_BAD_FACE);
                bad = ST_BAD_FACE;
            }
        if (hi - lo >= kAgg) {
#pragma unroll
            for (int q = 0; q < kTileItems; ++q)
                if (tc.vid[q] >= 0) atomicAdd(row + tc.vid[q] + 1, 1);
            continue;
        }
        const int range = hi - lo + 1;
        for (int i = threadIdx.x; i < range; i += kBlock) cnt[i] = 0;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kTileItems; ++q)
            if (tc.vid[q] >= 0) atomicAdd(cnt + (tc.vid[q] - lo), 1);
        __syncthreads();
        for (int i = threadIdx.x; i < range; i += kBlock)
            if (cnt[i]) atomicAdd(row + lo + i + 1, cnt[i]);
        __syncthreads();
    }
    if (bad) atomicOr(ctrl + C_STATUS, bad);
}

__global__ __launch_bounds__(kBlock) void k_fill_incidence(const int* F, const MeshDesc* mesh, int B,
                                                           const int* fo3, long long F3,
                                                           const int* row, int* cursor,
                                                           int2* wedgeO, const int* ctrl) {
    if (gated(ctrl)) return;
    __shared__ int cnt[kAgg];
    __shared__ int red[8];
    const long long ntiles = (F3 + kTile - 1) / kTile;
    for (long long t = blockIdx.x; t < ntiles; t += gridDim.x) {
        TileCorners tc;
        int lo, hi;
        load_tile_corners<false>(F, mesh, B, fo3, F3, t, tc, &lo, &hi, red);
        int slot[kTileItems];
        const bool agg = hi - lo < kAgg;
        if (agg) {
            const int range = hi - lo + 1;
            for (int i = threadIdx.x; i < range; i += kBlock) cnt[i] = 0;
            __syncthreads();
#pragma unroll
            for (int q = 0; q < kTileItems; ++q)
                slot[q] = tc.vid[q] >= 0 ? atomicAdd(cnt + (tc.vid[q] - lo), 1) : 0;
            __syncthreads();
            // each vertex's slots in this tile follow the ones taken before
            for (int i = threadIdx.x; i < range; i += kBlock)
                if (cnt[i]) cnt[i] = atomicAdd(cursor + lo + i, cnt[i]);
            __syncthreads();
        }
        if (agg && t * kTile + kTile <= F3) {
            // a full tile: every corner's incidence row and wedge loaded, then stored
            int at[kTileItems];
            int2 wd[kTileItems];
#pragma unroll
            for (int q = 0; q < kTileItems; ++q) {
                const int v = tc.vid[q], c = tc.c[q];
                at[q] = row[v] + cnt[v - lo] + slot[q];
                wd[q] = make_int2(tc.vo[q] + F[tc.t3[q] + other1(c)], tc.vo[q] + F[tc.t3[q] + other2(c)]);
            }
#pragma unroll
            for (int q = 0; q < kTileItems; ++q) wedgeO[at[q]] = wd[q];
        } else {
#pragma unroll
            for (int q = 0; q < kTileItems; ++q) {
                const int v = tc.vid[q];
                if (v < 0) continue;
                const int s = agg ? cnt[v - lo] + slot[q] : atomicAdd(cursor + v, 1);
                const int c = tc.c[q];
                wedgeO[row[v] + s] =
                    make_int2(tc.vo[q] + F[tc.t3[q] + other1(c)], tc.vo[q] + F[tc.t3[q] + other2(c)]);
            }
        }
        if (agg) __syncthreads();       // cnt is rewritten by the next tile
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

// ---- BFS toplesets (persistent, cooperative launch, groups of workgroups) --
struct BfsArgs {
    int G;                 // workgroups of the launch
    const MeshDesc* mesh;
    MeshState* state;
    const WgInfo* wg;
    const int* glist;      // per group: starts [ngroups + 1], then mesh ids
    const int* S;
    const int* row;
    const int2* wedgeO;
    const int* ellO;       // neighbour rows, global ids
    int* level;
    int* perm;
    int* iperm;
    int* offsets;
    unsigned* bits;
    int* cnt;
    int* ctrl;
    unsigned* bar;
};

constexpr int kExpandG = 6;    // wedges loaded together per expanded vertex

// One group handles one mesh at a time.  The mesh's bitmap of V_r is split
// into gsize equal chunks of words, one per workgroup of the group.  Per
// level r, each workgroup
//   1. reads the chunk counts of V_r (made by the discoveries of level r-1),
//      giving |V_r| and the start of its chunk inside V_r;
//   2. writes its chunk's vertices, in ascending id order, to perm (this is
//      the canonical order: level, then id), clears the chunk;
//   3. expands those vertices: each unvisited neighbour gets level r+1 (one
//      CAS decides the discoverer), its bit in the next bitmap and a count in
//      the next chunk counts.
// One group barrier per level.  A level with no vertex ends the loop: rho = r.
// level, bits and cnt are shared between workgroups: coherent access only.
__global__ __launch_bounds__(kBlock) void k_bfs(BfsArgs a) {
    if (gated(a.ctrl)) return;
    const WgInfo me = a.wg[blockIdx.x];
    if (me.group < 0) return;                 // an unused launch slot
    const int gs = me.gsize, w = me.rank, tid = threadIdx.x;
    __shared__ unsigned bar_slots[2 * kBlock / kWave];
    FlagBarrier gb{a.bar + (size_t)me.first * kLine, a.bar + (size_t)(a.G + me.first) * kLine,
                   a.ctrl + C_ABORT, (unsigned)gs, (unsigned)w, 0};
    gb.slots = bar_slots;
    unsigned any = 0;
    const long long gsz = (long long)gs * kBlock;
    const long long g0 = (long long)w * kBlock + tid;
    int* cntg = a.cnt + 4 * me.first;
    __shared__ int list[kListCap];

    const int* lst = a.glist + a.glist[me.group];
    const int nlst = a.glist[me.group + 1] - a.glist[me.group];
    for (int li = 0; li < nlst; ++li) {
        const int b = lst[li];
        const MeshDesc d = a.mesh[b];
        const int n = d.n, vo = d.v_off;
        const int nwords = (n + 31) / 32;
        const int cw = max(1, (nwords + gs - 1) / gs);
        unsigned* bits0 = a.bits + 2ll * d.w_off;
        unsigned* bits1 = bits0 + nwords;
        int* offs = a.offsets + vo + b;
        for (long long v = g0; v < n; v += gsz) st_c(a.level + vo + v, -1);
        for (long long x = g0; x < 2ll * nwords; x += gsz) st_c(bits0 + x, 0u);
        for (long long x = g0; x < 4ll * gs; x += gsz) st_c(cntg + x, 0);
        if (!gb.sync(0, &any)) return;
        unsigned dup = 0;
        for (long long s = g0; s < d.m; s += gsz) {
            const int v = a.S[d.s_in + s];
            if (atomicCAS(a.level + vo + v, -1, 0) != -1) {
                dup = 1;
            } else {
                atomicOr(bits0 + (v >> 5), 1u << (v & 31));
                atomicAdd(cntg + (v >> 5) / cw, 1);
            }
        }
        if (!gb.sync(dup, &any)) return;
        if (any) {
            if (w == 0 && tid == 0) {
                atomicOr(&a.state[b].status, ST_DUP_SOURCE);
                atomicOr(a.ctrl + C_STATUS, ST_DUP_SOURCE);
            }
            continue;   // every workgroup of the group skips this mesh
        }

        const int wbeg = min(w * cw, nwords);
        const int wend = min(wbeg + cw, nwords);
        const int q = (wend - wbeg + kBlock - 1) / kBlock;
        const int my0 = min(wbeg + tid * q, wend);
        const int my1 = min(my0 + q, wend);
        int base = 0;
        int r = 0;
        for (;; ++r) {
            const int* cr = cntg + (r % 3) * gs;
            int part = 0, partpre = 0;
            for (int x = tid; x < gs; x += kBlock) {
                const int c = ld_c(cr + x);
                part += c;
                if (x < w) partpre += c;
            }
            int total, chunk_pre;
            (void)block_exclusive_scan_n<kBlock, int, true>(part, &total);
            (void)block_exclusive_scan_n<kBlock, int, true>(partpre, &chunk_pre);
            if (total == 0) break;
            if (w == 0 && tid == 0) offs[r] = base;
            if (tid == 0) st_c(cntg + ((r + 2) % 3) * gs + w, 0);
            unsigned* cur = (r & 1) ? bits1 : bits0;
            unsigned* nxt = (r & 1) ? bits0 : bits1;
            int* cn = cntg + ((r + 1) % 3) * gs;

            int pc = 0;
            for (int x = my0; x < my1; ++x) pc += __popc(ld_c(cur + x));
            int tot_w;
            const int pre = block_exclusive_scan_n<kBlock, int, true>(pc, &tot_w);
            for (int done = 0; done < tot_w; done += kListCap) {
                int rank = pre;
                for (int x = my0; x < my1 && rank < done + kListCap; ++x) {
                    unsigned word = ld_c(cur + x);
                    while (word) {
                        const int bt = __ffs(word) - 1;
                        word &= word - 1;
                        if (rank >= done && rank < done + kListCap) list[rank - done] = x * 32 + bt;
                        ++rank;
                    }
                }
                lds_barrier();
                const int cntl = min(kListCap, tot_w - done);
                const int lvl = r + 1;
                for (int t = tid; t < cntl; t += kBlock) {      // the chunk's slice of the order
                    const int pos = base + chunk_pre + done + t;
                    a.perm[vo + pos] = vo + list[t];
                    a.iperm[vo + list[t]] = vo + pos;
                }
                for (int t = tid; t < cntl; t += kBlock) {
                    const int u = vo + list[t];
                    // the neighbour row, then the neighbours' levels
                    // (independent loads), then a CAS for the unvisited ones
                    const int4* er = reinterpret_cast<const int4*>(a.ellO + (size_t)kEll * u);
                    const int4 r0 = er[0], r1 = er[1];
                    const int ev[kEll] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
                    if (ev[kEll - 1] != kEllMore) {
                        int lv[kEll];
#pragma unroll
                        for (int q = 0; q < kEll; ++q) lv[q] = ld_c(a.level + (ev[q] >= 0 ? ev[q] : u));
#pragma unroll
                        for (int q = 0; q < kEll; ++q) {
                            const int x = ev[q];
                            if (x >= 0 && lv[q] < 0 && atomicCAS(a.level + x, -1, lvl) == -1) {
                                const int xl = x - vo;
                                atomicOr(nxt + (xl >> 5), 1u << (xl & 31));
                                atomicAdd(cn + (xl >> 5) / cw, 1);
                            }
                        }
                        continue;
                    }
                    const int e0 = a.row[u], e1 = a.row[u + 1];
                    for (int eb = e0; eb < e1; eb += kExpandG) {
                        // wedges, then their neighbours' levels (independent
                        // loads), then a CAS for the unvisited ones
                        const int cnt = min(kExpandG, e1 - eb);
                        int2 nb[kExpandG];
                        int lv[2 * kExpandG];
#pragma unroll
                        for (int q = 0; q < kExpandG; ++q) nb[q] = q < cnt ? a.wedgeO[eb + q] : make_int2(u, u);
#pragma unroll
                        for (int q = 0; q < kExpandG; ++q) {
                            lv[2 * q] = ld_c(a.level + nb[q].x);
                            lv[2 * q + 1] = ld_c(a.level + nb[q].y);
                        }
#pragma unroll
                        for (int q = 0; q < 2 * kExpandG; ++q) {
                            const int x = (q & 1) ? nb[q >> 1].y : nb[q >> 1].x;
                            if (lv[q] < 0 && atomicCAS(a.level + x, -1, lvl) == -1) {
                                const int xl = x - vo;
                                atomicOr(nxt + (xl >> 5), 1u << (xl & 31));
                                atomicAdd(cn + (xl >> 5) / cw, 1);
                            }
                        }
                    }
                }
                lds_barrier();
            }
            for (int x = my0; x < my1; ++x) st_c(cur + x, 0u);
            base += total;
            if (!gb.sync(0, &any)) return;
        }
        const int rho = r;
        const int reach = base;
        if (w == 0 && tid == 0) offs[rho] = reach;

        // unreachable vertices of the mesh follow, in ascending id order
        const int cv = (n + gs - 1) / gs;
        const int vb = min(w * cv, n), ve = min(vb + cv, n);
        const int qv = (ve - vb + kBlock - 1) / kBlock;
        const int v0 = min(vb + tid * qv, ve), v1 = min(v0 + qv, ve);
        int pc = 0;
        for (int v = v0; v < v1; ++v) pc += ld_c(a.level + vo + v) < 0;
        int tot_w;
        const int pre = block_exclusive_scan(pc, &tot_w);
        if (tid == 0) st_c(cntg + 3 * gs + w, tot_w);
        if (!gb.sync(0, &any)) return;
        int partpre = 0;
        for (int x = tid; x < w; x += kBlock) partpre += ld_c(cntg + 3 * gs + x);
        const int chunk_pre = block_sum(partpre);
        int pos = reach + chunk_pre + pre;
        for (int v = v0; v < v1; ++v)
            if (ld_c(a.level + vo + v) < 0) {
                a.perm[vo + pos] = vo + v;
                a.iperm[vo + v] = vo + pos;
                ++pos;
            }
        if (w == 0 && tid == 0) {
            a.state[b].rho = rho;
            a.state[b].reach = reach;
        }
        if (!gb.sync(0, &any)) return;   // the group's counters are reused by its next mesh
    }
}

// ---- BFS of one mesh in one workgroup, bitmaps in LDS --------------------
// For a mesh whose two n-bit bitmaps fit in LDS, one workgroup of
// kLdsBlock threads runs the whole BFS with block barriers only: `vis`
// marks discovered vertices, `nxt` holds the next topleset.  Per level the
// set bits of `nxt` are compacted in ascending id order (the canonical
// order: level, then id) straight into perm / iperm / level, and the level's
// vertices (kept in an LDS list, or read back from perm beyond its capacity)
// are expanded with LDS atomics deciding the discoverer.  Same outputs as
// k_bfs for the meshes it is given.
constexpr int kLdsBlock = 1024;
constexpr int kLdsList = 4096;
constexpr int kExpand = 8;     // wedges loaded together per expanded vertex

// Inputs and outputs of the reorder into topleset order.
struct ReorderArgs {
    const float* V;
    const MeshDesc* mesh;
    const int* vo;
    const int* iperm;
    const int* rowO;
    const int* fanO;
    const int* fanlen;
    const int2* wedgeO;    // the incidence (the reorder inside the BFS launch builds the fans)
    int2* fanrow;
    float4* xyz;
    int* fan;
    int* fan6;
};

struct BfsLdsArgs {
    const int* lmesh;      // mesh ids, one per workgroup: the n_big large ones first
    int n_big;
    unsigned* bits;        // frontier bitmaps in global memory (large meshes)
    const MeshDesc* mesh;
    MeshState* state;
    const int* S;
    const int* row;        // rowO
    const int2* wedgeO;    // global ids
    const int* ellO;       // neighbour rows, global ids
    int* level;
    int* perm;
    int* iperm;
    int* offsets;
    int* ctrl;
    int fuse;              // reorder inside this launch (bfs_reorder_tail)
    int n_one;             // workgroups of the launch
    int B;                 // meshes of the batch
    int* rq;               // queues of the reorder
    ReorderArgs ro;
};

__device__ __forceinline__ bool bfs_lds(const BfsLdsArgs& a) {
    extern __shared__ unsigned lds[];
    const int tid = threadIdx.x;
    const int b = a.lmesh[blockIdx.x];
    const MeshDesc d = a.mesh[b];
    const int n = d.n, vo = d.v_off;
    const int W = (n + 31) / 32;
    unsigned* vis = lds;
    unsigned* nxt = lds + W;
    int* wpre = reinterpret_cast<int*>(lds + 2 * W);          // [W + 1]
    int* list = reinterpret_cast<int*>(lds + 3 * W + 1);
    int* offs = a.offsets + vo + b;
    for (int x = tid; x < 2 * W; x += kLdsBlock) lds[x] = 0u;
    __syncthreads();
    unsigned dup = 0;
    for (int s = tid; s < d.m; s += kLdsBlock) {
        const int v = a.S[d.s_in + s];
        const unsigned bit = 1u << (v & 31);
        if (atomicOr(vis + (v >> 5), bit) & bit) dup = 1;
        else atomicOr(nxt + (v >> 5), bit);
    }
    if (__syncthreads_or(dup)) {
        if (tid == 0) {
            atomicOr(&a.state[b].status, ST_DUP_SOURCE);
            atomicOr(a.ctrl + C_STATUS, ST_DUP_SOURCE);
        }
        return false;
    }
    const int q = (W + kLdsBlock - 1) / kLdsBlock;
    const int my0 = min(tid * q, W), my1 = min(my0 + q, W);
    int base = 0, r = 0;
    for (;; ++r) {
        int pc = 0;
        for (int x = my0; x < my1; ++x) pc += __popc(nxt[x]);
        int total;
        int run = block_exclusive_scan_n<kLdsBlock, int, true>(pc, &total);
        if (total == 0) break;
        if (tid == 0) offs[r] = base;
        // rank of the first vertex of every word (ascending id order)
        for (int x = my0; x < my1; ++x) {
            wpre[x] = run;
            run += __popc(nxt[x]);
        }
        if (tid == 0) wpre[W] = total;
        lds_barrier();
        // vertex of rank t: the word holding it by binary search over the
        // word ranks, then the matching set bit; one vertex per thread, so a
        // dense run of ids costs no more than a sparse one
        for (int t = tid; t < total; t += kLdsBlock) {
            int lo = 0, hi = W;                 // wpre[lo] <= t < wpre[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (wpre[mid] <= t) lo = mid;
                else hi = mid;
            }
            unsigned w = nxt[lo];
            int k = t - wpre[lo], bit = 0;
            for (int step = 16; step >= 1; step >>= 1) {   // k-th set bit of w
                const unsigned low = w & ((1u << step) - 1u);
                const int c = __popc(low);
                if (k >= c) {
                    k -= c;
                    w >>= step;
                    bit += step;
                } else {
                    w = low;
                }
            }
            const int u = lo * 32 + bit;
            if (t < kLdsList) list[t] = u;
            a.perm[vo + base + t] = vo + u;
            a.iperm[vo + u] = vo + base + t;
            a.level[vo + u] = r;
        }
        if (total > kLdsList) wait_memory();   // perm is read back below
        lds_barrier();                          // perm / iperm / level stores need not land
        for (int x = my0; x < my1; ++x) nxt[x] = 0u;
        lds_barrier();
        for (int t = tid; t < total; t += kLdsBlock) {
            const int u = t < kLdsList ? list[t] : ld_c(a.perm + vo + base + t) - vo;
            // the neighbour row in one round trip (two 16-byte loads)
            const int4* er = reinterpret_cast<const int4*>(a.ellO + (size_t)kEll * (vo + u));
            const int4 r0 = er[0], r1 = er[1];
            const int ev[kEll] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
            if (ev[kEll - 1] != kEllMore) {
#pragma unroll
                for (int q = 0; q < kEll; ++q) {
                    if (ev[q] < 0) continue;
                    const int x = ev[q] - vo;
                    const unsigned bit = 1u << (x & 31);
                    if (!(vis[x >> 5] & bit) && !(atomicOr(vis + (x >> 5), bit) & bit))
                        atomicOr(nxt + (x >> 5), bit);
                }
                continue;
            }
            const int e0 = a.row[vo + u], e1 = a.row[vo + u + 1];
            for (int eb = e0; eb < e1; eb += kExpand) {
                // the wedges' loads first (independent), then the LDS marks
                const int cnt = min(kExpand, e1 - eb);
                int2 nb[kExpand];
#pragma unroll
                for (int q = 0; q < kExpand; ++q) nb[q] = q < cnt ? a.wedgeO[eb + q] : make_int2(vo + u, vo + u);
#pragma unroll
                for (int q = 0; q < kExpand; ++q) {
                    const int xs[2] = {nb[q].x - vo, nb[q].y - vo};
                    for (int z = 0; z < 2; ++z) {
                        const int x = xs[z];
                        const unsigned bit = 1u << (x & 31);
                        if (!(vis[x >> 5] & bit) && !(atomicOr(vis + (x >> 5), bit) & bit))
                            atomicOr(nxt + (x >> 5), bit);
                    }
                }
            }
        }
        lds_barrier();
        base += total;
    }
    const int rho = r, reach = base;
    // unreachable vertices follow in ascending id order, level -1
    int pc = 0;
    for (int x = my0; x < my1; ++x) {
        unsigned word = ~vis[x];
        if (x == W - 1 && (n & 31)) word &= (1u << (n & 31)) - 1u;
        pc += __popc(word);
    }
    int total;
    int rank = block_exclusive_scan_n<kLdsBlock, int, true>(pc, &total);
    for (int x = my0; x < my1; ++x) {
        unsigned word = ~vis[x];
        if (x == W - 1 && (n & 31)) word &= (1u << (n & 31)) - 1u;
        while (word) {
            const int u = x * 32 + __ffs(word) - 1;
            word &= word - 1;
            const int pos = reach + rank;
            a.perm[vo + pos] = vo + u;
            a.iperm[vo + u] = vo + pos;
            a.level[vo + u] = -1;
            ++rank;
        }
    }
    if (tid == 0) {
        offs[rho] = reach;
        a.state[b].rho = rho;
        a.state[b].reach = reach;
    }
    return true;
}

// ---- BFS of one larger mesh in one workgroup -----------------------------
// For a mesh whose visited bitmap fits in LDS but whose topleset bitmaps and
// rank table do not.  The expansion marks new vertices in the visited bitmap
// and the words it touches in a summary bitmap, both in LDS; the vertices of
// the previous levels are a bitmap `done` in global memory (this workgroup's
// share of the frontier bitmaps, served from L2).  Per level the touched
// words are staged in ascending order in rounds of kBigWl; a staged word's
// new topleset is visited & ~done, and done takes the visited word (one load
// and one store per staged word, by one thread: no global atomics, which
// serialise on the words a level shares).  Each vertex is then found by a
// binary search over the ranks (one vertex per thread), emitted in canonical
// order, and expanded with LDS atomics only.
constexpr int kBigWl = 2048;

__device__ inline int kth_bit(unsigned w, int k) {
    int bit = 0;
    for (int step = 16; step >= 1; step >>= 1) {
        const unsigned low = w & ((1u << step) - 1u);
        const int c = __popc(low);
        if (k >= c) {
            k -= c;
            w >>= step;
            bit += step;
        } else {
            w = low;
        }
    }
    return bit;
}

// Expansion of vertex u (mesh-local) of a level of bfs_big from its
// neighbour row (r0, r1): each neighbour not yet visited is marked visited
// and its word in the summary (LDS atomics only); a row that ends in
// kEllMore is expanded from the vertex's wedges instead.
__device__ inline void bfs_big_expand(const BfsLdsArgs& a, int vo, int u, int4 r0, int4 r1, unsigned* vis,
                                      unsigned* summ) {
    auto visit = [&](int x) {
        const unsigned bit = 1u << (x & 31);
        if (!(vis[x >> 5] & bit) && !(atomicOr(vis + (x >> 5), bit) & bit))
            atomicOr(summ + (x >> 10), 1u << ((x >> 5) & 31));
    };
    const int ev[kEll] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
    if (ev[kEll - 1] != kEllMore) {
#pragma unroll
        for (int q = 0; q < kEll; ++q)
            if (ev[q] >= 0) visit(ev[q] - vo);
        return;
    }
    const int e0 = a.row[vo + u], e1 = a.row[vo + u + 1];
    for (int eb = e0; eb < e1; eb += kExpand) {
        const int cnt = min(kExpand, e1 - eb);
        int2 nb[kExpand];
#pragma unroll
        for (int q = 0; q < kExpand; ++q) nb[q] = q < cnt ? a.wedgeO[eb + q] : make_int2(vo + u, vo + u);
#pragma unroll
        for (int q = 0; q < kExpand; ++q) {
            visit(nb[q].x - vo);
            visit(nb[q].y - vo);
        }
    }
}

__device__ __forceinline__ bool bfs_big(const BfsLdsArgs& a) {
    extern __shared__ unsigned lds[];
    const int tid = threadIdx.x;
    const int b = a.lmesh[blockIdx.x];
    const MeshDesc d = a.mesh[b];
    const int n = d.n, vo = d.v_off;
    const int W = (n + 31) / 32, SW = (W + 31) / 32;
    unsigned* vis = lds;                                         // [W]
    unsigned* summ = lds + W;                                    // [SW]
    int* wl = reinterpret_cast<int*>(summ + SW);                 // [kBigWl]
    int* wpre = wl + kBigWl;                                     // [kBigWl + 1]
    unsigned* wv = reinterpret_cast<unsigned*>(wpre + kBigWl + 1);   // [kBigWl]
    unsigned* done = a.bits + 2ll * d.w_off;                     // [W], global
    int* offs = a.offsets + vo + b;
    for (int x = tid; x < W; x += kLdsBlock) {
        vis[x] = 0u;
        done[x] = 0u;
    }
    for (int x = tid; x < SW; x += kLdsBlock) summ[x] = 0u;
    wait_memory();                                               // cleared before the atomics
    __syncthreads();
    unsigned dup = 0;
    for (int s = tid; s < d.m; s += kLdsBlock) {
        const int v = a.S[d.s_in + s];
        const unsigned bit = 1u << (v & 31);
        if (atomicOr(vis + (v >> 5), bit) & bit) dup = 1;
        else atomicOr(summ + (v >> 10), 1u << ((v >> 5) & 31));
    }
    wait_memory();
    if (__syncthreads_or(dup)) {
        if (tid == 0) {
            atomicOr(&a.state[b].status, ST_DUP_SOURCE);
            atomicOr(a.ctrl + C_STATUS, ST_DUP_SOURCE);
        }
        return false;
    }
    const int sq = (SW + kLdsBlock - 1) / kLdsBlock;
    const int s0 = min(tid * sq, SW), s1 = min(s0 + sq, SW);
    int base = 0, r = 0;
    for (;; ++r) {
        int nw = 0;
        for (int x = s0; x < s1; ++x) nw += __popc(summ[x]);
        int totw;
        const int wbase = block_exclusive_scan_n<kLdsBlock, int, true>(nw, &totw);
        if (totw == 0) break;
        if (tid == 0) offs[r] = base;
        int total = 0;
        // a level staged in one round keeps each thread's vertices (at most
        // two) in registers for its expansion
        const bool one_round = totw <= kBigWl;
        int um0 = -1, um1 = -1;
        for (int w0 = 0; w0 < totw; w0 += kBigWl) {
            const int cnt = min(kBigWl, totw - w0);
            int k = wbase;
            for (int x = s0; x < s1 && k < w0 + kBigWl; ++x) {
                unsigned sm = summ[x];
                while (sm) {
                    const int w = x * 32 + __ffs(sm) - 1;
                    sm &= sm - 1;
                    if (k >= w0 && k < w0 + kBigWl) wl[k - w0] = w;
                    ++k;
                }
            }
            lds_barrier();
            // the staged words' new vertices: visited, not done (coherent
            // loads: the stores of done completed before the level's barrier)
            unsigned v0 = 0u, v1 = 0u;
            if (tid < cnt) {
                const unsigned vw = vis[wl[tid]];
                v0 = vw & ~ld_c(done + wl[tid]);
                done[wl[tid]] = vw;
            }
            if (tid + kLdsBlock < cnt) {
                const unsigned vw = vis[wl[tid + kLdsBlock]];
                v1 = vw & ~ld_c(done + wl[tid + kLdsBlock]);
                done[wl[tid + kLdsBlock]] = vw;
            }
            int t0, t1 = 0;
            const int p0 = block_exclusive_scan_n<kLdsBlock, int, true>(__popc(v0), &t0);
            const int p1 = cnt > kLdsBlock ? block_exclusive_scan_n<kLdsBlock, int, true>(__popc(v1), &t1) : 0;
            const int tv = t0 + t1;
            // a round of at most 2 kBigWl + 1 vertices: each staged word's
            // thread writes its vertices into a list in rank order (over wpre
            // and wv, which this form does not use); larger rounds find each
            // vertex by a binary search over the words' ranks
            const bool listed = tv <= 2 * kBigWl + 1;
            int* ul = wpre;
            if (listed) {
                if (tid < cnt) {
                    const int wb = wl[tid] * 32;
                    int k = p0;
                    for (unsigned m = v0; m; m &= m - 1) ul[k++] = wb + __ffs(m) - 1;
                }
                if (tid + kLdsBlock < cnt) {
                    const int wb = wl[tid + kLdsBlock] * 32;
                    int k = t0 + p1;
                    for (unsigned m = v1; m; m &= m - 1) ul[k++] = wb + __ffs(m) - 1;
                }
            } else {
                if (tid < cnt) {
                    wpre[tid] = p0;
                    wv[tid] = v0;
                }
                if (tid + kLdsBlock < cnt) {
                    wpre[tid + kLdsBlock] = t0 + p1;
                    wv[tid + kLdsBlock] = v1;
                }
                if (tid == 0) wpre[cnt] = tv;
            }
            lds_barrier();
            for (int t = tid; t < tv; t += kLdsBlock) {
                int u;
                if (listed) {
                    u = ul[t];
                } else {
                    int lo = 0, hi = cnt;           // wpre[lo] <= t < wpre[hi]
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (wpre[mid] <= t) lo = mid;
                        else hi = mid;
                    }
                    u = wl[lo] * 32 + kth_bit(wv[lo], t - wpre[lo]);
                }
                const int pos = base + total + t;
                a.perm[vo + pos] = vo + u;
                a.iperm[vo + u] = vo + pos;
                a.level[vo + u] = r;
                if (t == tid) um0 = u;
                else if (t == tid + kLdsBlock) um1 = u;
            }
            total += tv;
            lds_barrier();                          // the stage is rewritten by the next round
        }
        // the summary collects the next level's words; the level's stores of
        // done and perm complete before the next level reads them
        for (int x = s0; x < s1; ++x) summ[x] = 0u;
        wait_memory();
        __syncthreads();
        if (one_round && total <= 2 * kLdsBlock) {
            // both neighbour rows loaded before either is expanded
            int4 ra0 = make_int4(-1, -1, -1, -1), rb0 = ra0, ra1 = ra0, rb1 = ra0;
            if (um0 >= 0) {
                const int4* er = reinterpret_cast<const int4*>(a.ellO + (size_t)kEll * (vo + um0));
                ra0 = er[0];
                rb0 = er[1];
            }
            if (um1 >= 0) {
                const int4* er = reinterpret_cast<const int4*>(a.ellO + (size_t)kEll * (vo + um1));
                ra1 = er[0];
                rb1 = er[1];
            }
            if (um0 >= 0) bfs_big_expand(a, vo, um0, ra0, rb0, vis, summ);
            if (um1 >= 0) bfs_big_expand(a, vo, um1, ra1, rb1, vis, summ);
        } else {
            for (int t = tid; t < total; t += kLdsBlock) {
                const int u = ld_c(a.perm + vo + base + t) - vo;
                const int4* er = reinterpret_cast<const int4*>(a.ellO + (size_t)kEll * (vo + u));
                bfs_big_expand(a, vo, u, er[0], er[1], vis, summ);
            }
        }
        __syncthreads();                            // the expansion's LDS atomics completed
        base += total;
    }
    const int rho = r, reach = base;
    // unreachable vertices follow in ascending id order, level -1
    const int q = (W + kLdsBlock - 1) / kLdsBlock;
    const int my0 = min(tid * q, W), my1 = min(my0 + q, W);
    int pc = 0;
    for (int x = my0; x < my1; ++x) {
        unsigned word = ~vis[x];
        if (x == W - 1 && (n & 31)) word &= (1u << (n & 31)) - 1u;
        pc += __popc(word);
    }
    int total;
    int rank = block_exclusive_scan_n<kLdsBlock, int, true>(pc, &total);
    for (int x = my0; x < my1; ++x) {
        unsigned word = ~vis[x];
        if (x == W - 1 && (n & 31)) word &= (1u << (n & 31)) - 1u;
        while (word) {
            const int u = x * 32 + __ffs(word) - 1;
            word &= word - 1;
            const int pos = reach + rank;
            a.perm[vo + pos] = vo + u;
            a.iperm[vo + u] = vo + pos;
            a.level[vo + u] = -1;
            ++rank;
        }
    }
    if (tid == 0) {
        offs[rho] = reach;
        a.state[b].rho = rho;
        a.state[b].reach = reach;
    }
    return true;
}

constexpr int kFanStage = 8;       // wedges of a vertex staged in LDS for its fan build

// The chains of one vertex's wedges wd(0..c) (see kFanStart): a chain starts
// at a wedge that no unused wedge leads into (the lowest unused one if every
// unused wedge has a predecessor: a closed fan), and follows (a, b) -> (b, c)
// while an unused wedge continues it.  Entry q goes to emit(q, value);
// returns the number of entries.  Every wedge is used exactly once, as a
// consecutive pair of one chain or as the closing pair.
template <class Get, class Emit>
__device__ __forceinline__ int build_fan(Get wd, int c, Emit emit) {
    if (c > kFanChainMax) {
        for (int q = 0; q < c; ++q) {
            const int2 t = wd(q);
            emit(2 * q, t.x | kFanStart);
            emit(2 * q + 1, t.y);
        }
        return 2 * c;
    }
    unsigned left = c == 32 ? ~0u : (1u << c) - 1u;
    int len = 0;
    while (left) {
        int s = __ffs(left) - 1;
        for (unsigned m = left; m; m &= m - 1) {
            const int i = __ffs(m) - 1;
            const int ai = wd(i).x;
            bool pred = false;
            for (unsigned m2 = left; m2 && !pred; m2 &= m2 - 1) {
                const int j = __ffs(m2) - 1;
                pred = j != i && wd(j).y == ai;
            }
            if (!pred) {
                s = i;
                break;
            }
        }
        left &= ~(1u << s);
        const int first = wd(s).x;
        const bool whole = len == 0;
        emit(len++, first | kFanStart);
        int cur = wd(s).y;
        emit(len++, cur);
        for (;;) {
            int nx = -1;
            for (unsigned m = left; m; m &= m - 1) {
                const int j = __ffs(m) - 1;
                if (wd(j).x == cur) {
                    nx = j;
                    break;
                }
            }
            if (nx < 0) break;
            left &= ~(1u << nx);
            cur = wd(nx).y;
            if (whole && !left && cur == first) {     // one closed chain: no repeat
                emit(0, first | kFanStart | kFanClosed);
                break;
            }
            emit(len++, cur);
        }
    }
    return len;
}

// Coordinates and fans in topleset order: the position of each vertex takes
// its coordinates and a copy of its fan with every neighbour id turned into
// that neighbour's position (flags kept): the first kFan6 entries in its
// fixed-size record, the whole fan in the row form as well when it is longer
// (at twice the vertex's incidence offset, the room fanO gives it, so no scan
// over the positions is needed; fanrow holds its start and end).
// The loops run over vertex ids, so
// the fans are read in storage order and the neighbours' positions are
// looked up around the vertex's own id (meshes number neighbours closely);
// only the writes scatter, one row per vertex.  A thread takes kReItems
// vertices at a time through three rounds of loads (position, coordinates and
// fan offset; fan row and the first kReFan fan entries; the neighbours'
// positions), each round issued for all of them before any result is used.
constexpr int kReItems = 4;
constexpr int kReFan = 8;
static_assert(kReFan >= kFan6, "the fan records are filled from the entries in registers");

// The vertices v[i] (internal ids, -1 for none) of meshes bq[i].
__device__ inline void reorder_items(const float* __restrict__ V, const MeshDesc* mesh, const int* vo,
                                     const int* __restrict__ iperm, const int* __restrict__ rowO,
                                     const int* __restrict__ fanO, const int* __restrict__ fanlen,
                                     int2* __restrict__ fanrow, float4* __restrict__ xyz, int* __restrict__ fan,
                                     int* __restrict__ fan6, const long long* v, const int* bq) {
    auto pos = [&](long long x) { return iperm[x]; };
    int p[kReItems], r0[kReItems], len[kReItems], e[kReItems][kReFan];
    float c[kReItems][3];
#pragma unroll
    for (int i = 0; i < kReItems; ++i) {
        p[i] = 0;
        r0[i] = 0;
        len[i] = 0;
        c[i][0] = c[i][1] = c[i][2] = 0.f;
        if (v[i] >= 0) {
            const int b = bq[i];
            const float* cp = V + 3 * ((long long)mesh[b].v_in + (v[i] - vo[b]));
            p[i] = pos(v[i]);
            c[i][0] = cp[0];
            c[i][1] = cp[1];
            c[i][2] = cp[2];
            r0[i] = rowO[v[i]];
            len[i] = fanlen[v[i]];
        }
    }
#pragma unroll
    for (int i = 0; i < kReItems; ++i) {
#pragma unroll
        for (int q = 0; q < kReFan; ++q) e[i][q] = q < len[i] ? fanO[2 * (long long)r0[i] + q] : 0;
    }
#pragma unroll
    for (int i = 0; i < kReItems; ++i)
#pragma unroll
        for (int q = 0; q < kReFan; ++q)
            if (q < len[i]) e[i][q] = pos(e[i][q] & kFanId) | (e[i][q] & ~kFanId);
#pragma unroll
    for (int i = 0; i < kReItems; ++i) {
        if (v[i] < 0) continue;
        xyz[p[i]] = make_float4(c[i][0], c[i][1], c[i][2], 0.f);
        const int fr = 2 * r0[i];     // the row's start: twice the incidence offset, as in fanO
        if (len[i] > kFan6) {         // a longer fan: also in the row form
            fanrow[p[i]] = make_int2(fr, fr + len[i]);
#pragma unroll
            for (int q = 0; q < kReFan; ++q)
                if (q < len[i]) fan[fr + q] = e[i][q];
        }
        // the fixed-size record of the first kFan6 entries
        int rec[kFan6];
        const int first = len[i] > 0 ? e[i][0] : p[i];
#pragma unroll
        for (int q = 0; q < kFan6; ++q)
            rec[q] = q < len[i] ? e[i][q] : (q == 0 ? p[i] : (first & kFanId) | kFan6Pad);
        if (len[i] > kFan6) rec[0] |= kFan6Pad;
        int2* r6 = reinterpret_cast<int2*>(fan6 + (size_t)kFan6 * p[i]);
        r6[0] = make_int2(rec[0], rec[1]);
        r6[1] = make_int2(rec[2], rec[3]);
        r6[2] = make_int2(rec[4], rec[5]);
        for (int q = kReFan; q < len[i]; ++q) {
            const int x = fanO[2 * (long long)r0[i] + q];
            fan[fr + q] = pos(x & kFanId) | (x & ~kFanId);
        }
    }
}

// The reorder inside the BFS launch, which builds each vertex's fan from its
// wedges itself (before the BFS only the BFS rows are built then): the
// wedges of a vertex with at most kFanStage of them are staged in the
// thread's LDS column wd_s, the first kReFan fan entries go to its column
// row_s, later ones (raw ids) straight to the vertex's row in fan, converted
// once this thread's stores have landed.  The vertices v[i] (-1 for none)
// belong to mesh b; positions are read with coherent loads (written in the
// same launch).
__device__ __forceinline__ void reorder_items_build(const ReorderArgs& r, const long long* v, int b, int2* wd_s,
                                           int* row_s) {
    const int tid = threadIdx.x;
    auto pos = [&](long long x) { return ld_c(r.iperm + x); };
    int p[kReItems], r0[kReItems], c[kReItems], len[kReItems], e[kReItems][kReFan];
    float x3[kReItems][3];
    const long long vin = (long long)r.mesh[b].v_in - r.vo[b];
#pragma unroll
    for (int i = 0; i < kReItems; ++i) {
        p[i] = 0;
        r0[i] = 0;
        c[i] = 0;
        x3[i][0] = x3[i][1] = x3[i][2] = 0.f;
        if (v[i] >= 0) {
            const float* cp = r.V + 3 * (vin + v[i]);
            p[i] = pos(v[i]);
            x3[i][0] = cp[0];
            x3[i][1] = cp[1];
            x3[i][2] = cp[2];
            r0[i] = r.rowO[v[i]];
            c[i] = r.rowO[v[i] + 1] - r0[i];
        }
    }
    // one fan at a time through the thread's LDS columns; the next vertex's
    // wedges are loaded while this one is built
    int2 wn[kFanStage];
#pragma unroll
    for (int q = 0; q < kFanStage; ++q)
        wn[q] = q < c[0] && c[0] <= kFanStage ? r.wedgeO[r0[0] + q] : make_int2(0, 0);
#pragma unroll
    for (int i = 0; i < kReItems; ++i) {
#pragma unroll
        for (int q = 0; q < kFanStage; ++q)
            if (q < c[i] && c[i] <= kFanStage) wd_s[q * kLdsBlock + tid] = wn[q];
        if (i + 1 < kReItems) {
#pragma unroll
            for (int q = 0; q < kFanStage; ++q)
                wn[q] = q < c[i + 1] && c[i + 1] <= kFanStage ? r.wedgeO[r0[i + 1] + q] : make_int2(0, 0);
        }
        len[i] = 0;
        if (v[i] >= 0) {
            int* out = r.fan + 2 * (long long)r0[i];
            auto emit = [&](int q, int x) {
                if (q < kReFan) row_s[q * kLdsBlock + tid] = x;
                else out[q] = x;
            };
            if (c[i] <= kFanStage)
                len[i] = build_fan([&](int q) { return wd_s[q * kLdsBlock + tid]; }, c[i], emit);
            else
                len[i] = build_fan([&](int q) { return r.wedgeO[r0[i] + q]; }, c[i], emit);
        }
#pragma unroll
        for (int q = 0; q < kReFan; ++q) e[i][q] = q < len[i] ? row_s[q * kLdsBlock + tid] : 0;
    }
#pragma unroll
    for (int i = 0; i < kReItems; ++i)
#pragma unroll
        for (int q = 0; q < kReFan; ++q)
            if (q < len[i]) e[i][q] = pos(e[i][q] & kFanId) | (e[i][q] & ~kFanId);
    wait_memory();      // the raw entries past kReFan have landed before they are read back
#pragma unroll
    for (int i = 0; i < kReItems; ++i) {
        if (v[i] < 0) continue;
        r.xyz[p[i]] = make_float4(x3[i][0], x3[i][1], x3[i][2], 0.f);
        const int fr = 2 * r0[i];
        if (len[i] > kFan6) {
            r.fanrow[p[i]] = make_int2(fr, fr + len[i]);
#pragma unroll
            for (int q = 0; q < kReFan; ++q)
                if (q < len[i]) r.fan[fr + q] = e[i][q];
            for (int q = kReFan; q < len[i]; ++q) {
                const int x = r.fan[fr + q];
                r.fan[fr + q] = pos(x & kFanId) | (x & ~kFanId);
            }
        }
        int rec[kFan6];
        const int first = len[i] > 0 ? e[i][0] : p[i];
#pragma unroll
        for (int q = 0; q < kFan6; ++q)
            rec[q] = q < len[i] ? e[i][q] : (q == 0 ? p[i] : (first & kFanId) | kFan6Pad);
        if (len[i] > kFan6) rec[0] |= kFan6Pad;
        int2* r6 = reinterpret_cast<int2*>(r.fan6 + (size_t)kFan6 * p[i]);
        r6[0] = make_int2(rec[0], rec[1]);
        r6[1] = make_int2(rec[2], rec[3]);
        r6[2] = make_int2(rec[4], rec[5]);
    }
}

__global__ __launch_bounds__(kBlock) void k_reorder(ReorderArgs r, int B, long long N, const int* ctrl) {
    if (gated(ctrl)) return;
    for (long long t = blockIdx.x; t < (N + kTile - 1) / kTile; t += gridDim.x) {
        int bq[kTileItems];
        tile_meshes(r.vo, B, N, t, bq);
#pragma unroll
        for (int h = 0; h < kTileItems; h += kReItems) {
            long long v[kReItems];
#pragma unroll
            for (int i = 0; i < kReItems; ++i) {
                v[i] = t * kTile + (long long)(h + i) * kBlock + threadIdx.x;
                if (v[i] >= N) v[i] = -1;
            }
            reorder_items(r.V, r.mesh, r.vo, r.iperm, r.rowO, r.fanO, r.fanlen, r.fanrow, r.xyz, r.fan,
                                 r.fan6, v, bq + h);
        }
    }
}

// The reorder of a batch inside its one-workgroup BFS launch (see kRqWords).
// The mesh's positions are in this XCD's L2 once every thread's stores have
// completed; the mesh then goes into this XCD's queue (a coherent store,
// completed before the workgroup counts itself finished).  The last
// kShareLast meshes to finish (the deepest, whose reorder ends the launch)
// go instead into a queue every XCD reads, after a release fence has
// written this XCD's L2 back to memory.  Thread 0 claims chunks of kReChunk
// vertices from its XCD's queue, then from the shared one; with none left
// it waits, but only while some BFS is still running and every workgroup of
// the launch has started (so a waiting workgroup never holds the place of one
// that has yet to run), and leaves otherwise.  The positions are read with
// coherent loads, which see what another CU of this XCD wrote or what a
// fence wrote back.
constexpr int kReChunk = kReItems * kLdsBlock;
constexpr int kShareLast = 16;
constexpr int kFuseMinMeshes = 256;     // one workgroup per CU of the device
// LDS of the reorder inside the BFS launch: per thread kFanStage staged
// wedges and kReFan fan entries
constexpr size_t kTailLds = (sizeof(int2) * kFanStage + sizeof(int) * kReFan) * kLdsBlock;

// The reorder runs inside the one-workgroup BFS when every mesh takes it and
// the finished workgroups can cover the device.
bool fuse_reorder(int g_prep, int n_one) { return g_prep == 0 && n_one >= kFuseMinMeshes; }

__device__ __forceinline__ void bfs_reorder_tail(const BfsLdsArgs& a, bool ok) {
    __shared__ int job[2];
    const int tid = threadIdx.x;
    const int x = (int)(xcc_id() & 7u);
    int* own = a.rq + kRqWords + x * a.B;
    int* shared = a.rq + kRqWords + 8 * a.B;
    int* claimed = a.rq + kRqWords + 9 * a.B;
    wait_memory();
    __syncthreads();
    if (tid == 0) {
        if (ok) {
            if (atomicAdd(a.rq + RQ_FINISHING, 1) >= a.n_one - kShareLast) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");     // this XCD's L2 to memory
                const int s = atomicAdd(a.rq + RQ_SHARED, 1);
                st_c(shared + s, a.lmesh[blockIdx.x] + 1);
            } else {
                const int s = atomicAdd(a.rq + RQ_SLOTS + x, 1);
                st_c(own + s, a.lmesh[blockIdx.x] + 1);
            }
            wait_memory();
        }
        atomicAdd(a.rq + RQ_FINISHED, 1);
    }
    int cur0 = 0, cur1 = 0;    // thread 0: per queue, the next slot that may have chunks left
    for (;;) {
        if (tid == 0) {
            int b = -1, c = 0;
            const long long t0 = wall_clock64();
            for (;;) {
                const int fin = ld_c(a.rq + RQ_FINISHED);
                bool drained = true;     // every slot taken so far is published and fully claimed
                auto claim = [&](int* slots, int taken, int& cur) {
                    while (b < 0 && cur < taken) {
                        const int mb = ld_c(slots + cur);
                        if (mb == 0) {           // taken, not yet published
                            drained = false;
                            return;
                        }
                        const int nc = (a.mesh[mb - 1].n + kReChunk - 1) / kReChunk;
                        const int k = atomicAdd(claimed + mb - 1, 1);
                        if (k < nc) {
                            b = mb - 1;
                            c = k;
                            return;
                        }
                        ++cur;
                    }
                };
                claim(own, ld_c(a.rq + RQ_SLOTS + x), cur0);
                if (b < 0) claim(shared, ld_c(a.rq + RQ_SHARED), cur1);
                if (b >= 0) break;
                // nothing to claim: leave when every BFS has finished (all
                // published meshes are claimed) or when waiting is not safe
                if (drained && (fin >= a.n_one || ld_c(a.rq + RQ_STARTED) < a.n_one)) break;
                if (wall_clock64() - t0 > FlagBarrier::kTimeoutTicks) {     // cannot happen: fail, not hang
                    __hip_atomic_fetch_or(a.ctrl + C_ABORT, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(32);
            }
            job[0] = b;
            job[1] = c;
        }
        __syncthreads();
        const int b = job[0], c = job[1];
        __syncthreads();
        if (b < 0) return;
        const long long v0 = a.mesh[b].v_off + (long long)c * kReChunk, v1 = a.mesh[b].v_off + a.mesh[b].n;
        long long v[kReItems];
#pragma unroll
        for (int i = 0; i < kReItems; ++i) {
            v[i] = v0 + (long long)i * kLdsBlock + tid;
            if (v[i] >= v1) v[i] = -1;
        }
        extern __shared__ unsigned lds[];     // free once the BFS is done: at least kTailLds bytes
        int2* wd_s = reinterpret_cast<int2*>(lds);
        reorder_items_build(a.ro, v, b, wd_s, reinterpret_cast<int*>(wd_s + kFanStage * kLdsBlock));
    }
}

// One workgroup per mesh: the larger meshes (first n_big blocks) with the
// frontier in global memory, the others with every bitmap in LDS.
__global__ __launch_bounds__(kLdsBlock) void k_bfs_one(BfsLdsArgs a) {
    if (gated(a.ctrl)) return;
    if (a.fuse && threadIdx.x == 0) atomicAdd(a.rq + RQ_STARTED, 1);
    const bool ok = (int)blockIdx.x < a.n_big ? bfs_big(a) : bfs_lds(a);
    if (a.fuse) bfs_reorder_tail(a, ok);
}

// Fans by vertex id.  A vertex's wedges (loaded together and staged in LDS,
// one column per thread, when there are at most kFanStage; 24 KB of LDS per
// workgroup leave room for six workgroups per CU) are chained into fanO at
// twice the vertex's incidence offset (a fan has at most two entries per
// triangle), the length goes to fanlen, and the BFS neighbour row to ellO:
// the fan's ids (each neighbour named once per chain) padded with -1, or
// kEllMore in the last entry when the fan has more than kEll entries (the
// BFS then expands the vertex from its wedges).
__global__ __launch_bounds__(kBlock) void k_fan_global(const int* rowO, const int2* wedgeO, long long N,
                                                       int* fanO, int* fanlen, int* ellO, const int* ctrl) {
    if (gated(ctrl)) return;
    __shared__ int2 wd_s[kFanStage * kBlock];
    __shared__ int row_s[kEll * kBlock];       // the first kEll fan entries, for the BFS row
    const int tid = threadIdx.x;
    const long long gsz = (long long)gridDim.x * kBlock;
    long long v = blockIdx.x * (long long)kBlock + tid;
    int r0 = 0, c = 0;
    if (v < N) {
        r0 = rowO[v];
        c = rowO[v + 1] - r0;
    }
    for (; v < N; v += gsz) {
        // the next vertex's incidence row is loaded while this one is built
        const long long vn = v + gsz;
        int r0n = 0, cn = 0;
        if (vn < N) {
            r0n = rowO[vn];
            cn = rowO[vn + 1] - r0n;
        }
        int* out = fanO + 2 * (long long)r0;
        auto emit = [&](int q, int x) {
            out[q] = x;
            if (q < kEll) row_s[q * kBlock + tid] = x;
        };
        int len;
        if (c <= kFanStage) {
            int2 w[kFanStage];
#pragma unroll
            for (int q = 0; q < kFanStage; ++q) w[q] = q < c ? wedgeO[r0 + q] : make_int2(0, 0);
#pragma unroll
            for (int q = 0; q < kFanStage; ++q)
                if (q < c) wd_s[q * kBlock + tid] = w[q];
            len = build_fan([&](int q) { return wd_s[q * kBlock + tid]; }, c, emit);
        } else {
            len = build_fan([&](int q) { return wedgeO[r0 + q]; }, c, emit);
        }
        fanlen[v] = len;
        int nb[kEll];
#pragma unroll
        for (int q = 0; q < kEll; ++q) nb[q] = q < len ? (row_s[q * kBlock + tid] & kFanId) : -1;
        if (len > kEll) nb[kEll - 1] = kEllMore;
        int4* er = reinterpret_cast<int4*>(ellO + kEll * v);
        er[0] = make_int4(nb[0], nb[1], nb[2], nb[3]);
        er[1] = make_int4(nb[4], nb[5], nb[6], nb[7]);
        r0 = r0n;
        c = cn;
    }
}

// The BFS rows alone (the fans are then built by the reorder inside the BFS
// launch): each vertex's distinct neighbours, the ends of its wedges, padded
// with -1, or kEllMore in the last entry when it has more than kEll of them
// or more than kEll wedges (the BFS then expands it from its wedges).  The
// neighbours are a set to the BFS, so their order does not matter.
__global__ __launch_bounds__(kBlock) void k_ell_rows(const int* rowO, const int2* wedgeO, long long N, int* ellO,
                                                     const int* ctrl) {
    if (gated(ctrl)) return;
    const long long gsz = (long long)gridDim.x * kBlock;
    for (long long v = blockIdx.x * (long long)kBlock + threadIdx.x; v < N; v += gsz) {
        const int r0 = rowO[v], c = rowO[v + 1] - r0;
        int nb[kEll];
#pragma unroll
        for (int q = 0; q < kEll; ++q) nb[q] = -1;
        if (c > kEll) {
            nb[kEll - 1] = kEllMore;
        } else {
            int x[2 * kEll];
#pragma unroll
            for (int q = 0; q < kEll; ++q) {
                const int2 w = q < c ? wedgeO[r0 + q] : make_int2(-1, -1);
                x[2 * q] = w.x;
                x[2 * q + 1] = w.y;
            }
            // rank of each first occurrence among the first occurrences
            int rank = 0;
#pragma unroll
            for (int j = 0; j < 2 * kEll; ++j) {
                bool first = x[j] >= 0;
#pragma unroll
                for (int k = 0; k < j; ++k) first = first && x[k] != x[j];
#pragma unroll
                for (int q = 0; q < kEll; ++q)
                    if (first && rank == q) nb[q] = x[j];
                rank += first ? 1 : 0;
            }
            if (rank > kEll) nb[kEll - 1] = kEllMore;
        }
        int4* er = reinterpret_cast<int4*>(ellO + kEll * v);
        er[0] = make_int4(nb[0], nb[1], nb[2], nb[3]);
        er[1] = make_int4(nb[4], nb[5], nb[6], nb[7]);
    }
}

int tile_grid(long long total) {
    const long long t = (total + kTile - 1) / kTile;
    return (int)(t < 1 ? 1 : (t > 8192 ? 8192 : t));
}

int grid_for(long long work) {
    long long g = (work + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (int)g;
}

}  // namespace

void launch_barrier_reset(const Work& w, int lines, hipStream_t st) {
    const long long len = (long long)lines * kLine;
    hipLaunchKernelGGL(k_zero_lines, dim3(grid_for(len)), dim3(kBlock), 0, st, w.bar, len);
}

hipError_t launch_prepare(const Work& w, const Sizes& z, const float* V, const int* F,
                          const int* S, int g_prep, int n_one, int n_big, hipStream_t st) {
    const long long N = z.N, F3 = 3 * z.F;
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(kBlock), 0, st, w.ctrl, (long long)C_WORDS, 0);
    hipLaunchKernelGGL(k_fill, dim3(grid_for(N + 1)), dim3(kBlock), 0, st, w.rowO, N + 1, 0);
    hipLaunchKernelGGL(k_fill, dim3(grid_for(N)), dim3(kBlock), 0, st, w.cursor, N, 0);
    hipLaunchKernelGGL(k_validate, dim3(grid_for(N)), dim3(kBlock), 0, st, V, F, S,
                       w.mesh, z.B, w.vo, w.fo3, w.so, N, F3, z.S, w.state, w.ctrl);
    hipLaunchKernelGGL(k_count, dim3(tile_grid(F3)), dim3(kBlock), 0, st, F, w.mesh, z.B, w.fo3, F3,
                       w.rowO, w.state, w.ctrl);
    hipError_t e = scan_inplace(w.rowO + 1, N, w.scan_tmp, w.ctrl, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fill_incidence, dim3(tile_grid(F3)), dim3(kBlock), 0, st, F, w.mesh, z.B,
                       w.fo3, F3, w.rowO, w.cursor, w.wedgeO, w.ctrl);
    if (fuse_reorder(g_prep, n_one))     // the fans are built by the reorder inside the BFS launch
        hipLaunchKernelGGL(k_ell_rows, dim3(grid_for(N)), dim3(kBlock), 0, st, w.rowO, w.wedgeO, N, w.ellO, w.ctrl);
    else
        hipLaunchKernelGGL(k_fan_global, dim3(grid_for(N)), dim3(kBlock), 0, st, w.rowO, w.wedgeO, N, w.fanO,
                           w.fanlen, w.ellO, w.ctrl);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_prepare_bfs(w, z, V, S, g_prep, n_one, n_big, st);
}

// Toplesets by BFS from the current sources, then the reorder of coordinates
// and fans into topleset order.  The incidence and the fans by vertex id
// (rowO, wedgeO, ellO, fanO, fanlen) must already be built; they do not
// depend on the sources.
hipError_t launch_prepare_bfs(const Work& w, const Sizes& z, const float* V, const int* S, int g_prep,
                              int n_one, int n_big, hipStream_t st) {
    const long long N = z.N;
    hipError_t e;
    BfsArgs a;
    a.G = g_prep;
    a.mesh = w.mesh;
    a.state = w.state;
    a.wg = w.wg_prep;
    a.glist = w.glist_prep;
    a.S = S;
    a.row = w.rowO;
    a.wedgeO = w.wedgeO;
    a.ellO = w.ellO;
    a.level = w.level;
    a.perm = w.perm;
    a.iperm = w.iperm;
    a.offsets = w.offsets;
    a.bits = w.bits;
    a.cnt = w.cnt;
    a.ctrl = w.ctrl;
    a.bar = w.bar;
    ReorderArgs ro;
    ro.V = V;
    ro.mesh = w.mesh;
    ro.vo = w.vo;
    ro.iperm = w.iperm;
    ro.rowO = w.rowO;
    ro.fanO = w.fanO;
    ro.fanlen = w.fanlen;
    ro.wedgeO = w.wedgeO;
    ro.fanrow = w.fanrow;
    ro.xyz = w.xyz;
    ro.fan = w.fan;
    ro.fan6 = w.fan6;
    const bool fuse = fuse_reorder(g_prep, n_one);
    if (n_one > 0) {
        BfsLdsArgs l;
        l.lmesh = w.lds_mesh;
        l.n_big = n_big;
        l.bits = w.bits;
        l.mesh = w.mesh;
        l.state = w.state;
        l.S = S;
        l.row = w.rowO;
        l.wedgeO = w.wedgeO;
        l.ellO = w.ellO;
        l.level = w.level;
        l.perm = w.perm;
        l.iperm = w.iperm;
        l.offsets = w.offsets;
        l.ctrl = w.ctrl;
        l.fuse = fuse ? 1 : 0;
        l.n_one = n_one;
        l.B = z.B;
        l.rq = w.rq;
        l.ro = ro;
        if (fuse)
            hipLaunchKernelGGL(k_fill, dim3(grid_for(kRqWords + 10ll * z.B)), dim3(kBlock), 0, st, w.rq,
                               kRqWords + 10ll * z.B, 0);
        size_t bytes = bfs_one_bytes(z.lds_words, z.big_words);
        if (fuse && bytes < kTailLds) bytes = kTailLds;
        hipLaunchKernelGGL(k_bfs_one, dim3(n_one), dim3(kLdsBlock), bytes, st, l);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (g_prep > 0) {
        launch_barrier_reset(w, 2 * g_prep, st);
        void* args[] = {&a};
        e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_bfs), dim3(g_prep), dim3(kBlock),
                                       args, 0, st);
        if (e != hipSuccess) return e;
    }
    if (!fuse) hipLaunchKernelGGL(k_reorder, dim3(grid_for(N)), dim3(kBlock), 0, st, ro, z.B, N, w.ctrl);
    return hipGetLastError();
}

// Dynamic LDS of the one-workgroup BFS launch: three words per 32 vertices
// and the emission list for the largest mesh with every bitmap in LDS; one
// word per 32 vertices, one per 1,024 and the round stage for the largest
// mesh with its frontier in global memory.
size_t bfs_one_bytes(long long lds_words, long long big_words) {
    const size_t lds = lds_words > 0 ? sizeof(unsigned) * (size_t)(3 * lds_words + 1) + sizeof(int) * kLdsList : 0;
    const size_t big =
        big_words > 0 ? sizeof(unsigned) * (size_t)(big_words + (big_words + 31) / 32 + 3 * kBigWl + 1) : 0;
    return lds > big ? lds : big;
}

// Largest meshes (vertices) the two one-workgroup BFS paths take on this
// device (0 if none); raises the kernel's dynamic LDS limit to what the
// device allows.
void bfs_one_limits(int device, int* lds_max, int* big_max) {
    *lds_max = *big_max = 0;
    int smem = 0;
    if (hipDeviceGetAttribute(&smem, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) return;
    const long long avail = (long long)smem - 1024;                 // static LDS of the kernel
    if (avail <= (long long)sizeof(int) * (3 * kBigWl + 64)) return;
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bfs_one), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)avail) != hipSuccess)
        return;
    const long long a_lds = avail - (long long)sizeof(int) * kLdsList - 4;
    *lds_max = a_lds > 0 ? (int)(a_lds / 12) * 32 : 0;                   // three words per 32 vertices
    const long long a_big = avail - (long long)sizeof(unsigned) * (3 * kBigWl + 2);
    // W + ceil(W / 32) words with W = n / 32 vertices' words: about 33 words per 1,024 vertices
    *big_max = (int)std::min<long long>(a_big / 4 * 32 / 33 * 32, 1ll << 29);
}

int max_coop_blocks_bfs(int cus) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_bfs, kBlock, 0) != hipSuccess || nb < 1)
        nb = 1;
    return nb * cus;
}

}  // namespace ptp

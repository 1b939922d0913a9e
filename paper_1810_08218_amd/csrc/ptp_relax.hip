// The PTP iteration (Sec. 4.2) as one persistent, cooperative kernel over a
// batch of meshes; per mesh:
//   init (d = +inf, d(S) = 0, labels),
//   for k = 1, 2, ...: Jacobi update of the band B_{i_k}^{j_k} from the
//     previous map with the planar update (Sec. 3.2) in increment form,
//     relative-change test of the band's first topleset (Eq. lower_band),
//     band ends advanced on the device (Eq. upper_band / lower_band),
//   unpermute of distances and labels to the caller's order.
// Two other controllers share the loop: the fixed half band
// [floor((k+1)/2), k] of the complexity analysis (Sec. 6) and plain Jacobi
// over every topleset until no value changes (the fixed point the iteration
// approximates).  The arithmetic is float32, or float64 (Sec. 5.1 runs both)
// in the `double` instantiation.
// One group barrier per iteration; the controller state (i, j, k) is kept in
// registers, identical in every workgroup of the group, and the only datum
// exchanged per iteration besides the distances is the "not converged" vote,
// carried by the barrier.
#include "ptp_device.h"
#include <algorithm>

#include "ptp_kernels.h"

namespace ptp {

namespace {

constexpr float kInf = __builtin_huge_valf();
template <typename R>
__device__ constexpr R inf_of() { return (R)__builtin_huge_val(); }

template <typename R>
__device__ inline R dot3(R ax, R ay, R az, R bx, R by, R bz) {
    return ax * bx + ay * by + az * bz;
}

// Square root and reciprocal.  float: the hardware instructions (v_sqrt_f32 /
// v_rcp_f32, about 1 ulp): the update needs relative accuracy near 1e-7, not
// correct rounding, and the IEEE sequences are several times longer on the
// critical path.  double: the correctly rounded operations.
__device__ inline float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double fsqrt(double x) { return __builtin_sqrt(x); }
__device__ inline double frcp(double x) { return 1.0 / x; }

// Planar update of x0 from (x1, d1), (x2, d2).
//
// With e_i = x_i - x0, a = e1.e1, b = e1.e2, c = e2.e2, det = |e1 x e2|^2,
// A = |x1 - x2|^2, delta = d2 - d1, the plane front through (x1, d1), (x2, d2)
// with unit in-plane gradient gives x0 the value d1 + q where
//     A q^2 - 2 delta (a - b) q + a delta^2 - det = 0,
// whose larger root is q = (delta (a - b) + sqrt(det (A - delta^2))) / A.
// Working with q = p - d1 keeps every term at the scale of the triangle, so
// float32 does not lose the digits that the textbook form in p cancels.
// The root is used when the front reaches x0 through the opposite edge
// (Q X^T n < 0, both components):  q (c - b) + b delta > 0  and
// q (a - b) > a delta; otherwise the edge updates d_i + |e_i| give the value.
// Label: edge update -> its vertex; planar value -> its smaller input.
//
// Written without branches: every term is computed and the result selected,
// so the updates of a vertex's triangles interleave instead of running one
// after the other.  An infinite input needs no case of its own: its edge
// update is infinite and the discriminant is -inf or NaN, so the finite edge
// update is selected (both infinite: +inf).
template <typename R, bool LABELS>
__device__ inline R local_update(float4 x0, float4 x1, float4 x2, R d1, R d2, int l1, int l2, int& lab) {
    const R e1x = (R)x1.x - (R)x0.x, e1y = (R)x1.y - (R)x0.y, e1z = (R)x1.z - (R)x0.z;
    const R e2x = (R)x2.x - (R)x0.x, e2y = (R)x2.y - (R)x0.y, e2z = (R)x2.z - (R)x0.z;
    const R a = dot3(e1x, e1y, e1z, e1x, e1y, e1z);
    const R c = dot3(e2x, e2y, e2z, e2x, e2y, e2z);
    const R p1 = d1 + fsqrt(a), p2 = d2 + fsqrt(c);
    const R pe = p2 < p1 ? p2 : p1;
    const R b = dot3(e1x, e1y, e1z, e2x, e2y, e2z);
    const R cx = e1y * e2z - e1z * e2y;
    const R cy = e1z * e2x - e1x * e2z;
    const R cz = e1x * e2y - e1y * e2x;
    const R det = dot3(cx, cy, cz, cx, cy, cz);
    const R fx = (R)x1.x - (R)x2.x, fy = (R)x1.y - (R)x2.y, fz = (R)x1.z - (R)x2.z;
    const R A = dot3(fx, fy, fz, fx, fy, fz);
    const R delta = d2 - d1;
    const R disc = det * (A - delta * delta);
    const R q = (delta * (a - b) + fsqrt(disc)) * frcp(A);
    const bool planar = det > (R)1e-12 * a * c && disc >= (R)0 && q * (c - b) + b * delta > (R)0 &&
                        q * (a - b) > a * delta;
    if (LABELS) {
        const int lmin = min(l1, l2);
        const int le = p1 < p2 ? l1 : (p2 < p1 ? l2 : lmin);
        const int lp = d1 < d2 ? l1 : (d2 < d1 ? l2 : lmin);
        lab = planar ? lp : le;
    }
    return planar ? d1 + q : pe;
}

struct RelaxArgs {
    int G;                 // workgroups of the launch
    int kmax_fixed, window;
    int band_rule;         // BandRule
    int certify;           // warm start: certify the bound first (else trusted)
    float tol;
    const MeshDesc* mesh;
    MeshState* state;
    const WgInfo* wg;
    const int* queue;      // mesh queues: class starts [4], class of each group [ngroups], lists
    int ngroups;
    const int* S;
    const float* upper;    // warm start: caller-order upper bound, or null
    int* xpost;            // [G] XCD of each workgroup (scratch)
    const int* perm;
    const int* iperm;
    const int* offsets;
    const int2* fanrow;    // (start, end) of the longer fans' rows in fan
    const int* fan;
    const float4* xyz;
    float* dist;           // [2N]
    unsigned long long* dl;   // [2N] (distance, label) pairs, with labels; doubles in the f64 run
    int* retire;
    int* ctrl;
    unsigned* bar;
    int* mark;             // [N] per position: 1 + the last iteration in which a fan neighbour changed
    const int* fan6;       // [6N] fixed-size fan records by position
    long long N;
    float* out_d;
    double* out_d64;
};

// Fan entries held in registers per band vertex (closed fans of degree <= 6
// and open ones of degree <= 5 in one go; longer fans continue in chunks).
constexpr int kChunk = 6;
constexpr int kCertifyRounds = 4096;   // cap on the certification closure

// The iteration state of a position: its distance (float, or double in the
// float64 run), exchanged between workgroups with coherent loads.
//
// Skipping unchanged work.  A band vertex that was updated in the previous
// iteration and none of whose neighbours changed there keeps its value
// without evaluating its triangles: the update is a function of the
// neighbours' values alone, so it would give the result the previous
// iteration already folded in (d_k = min(d_{k-1}, U(d_{k-1})) with
// U(d_{k-1}) = U(d_{k-2}) >= d_{k-1}).  A position whose value changes in
// iteration k stamps k + 1 on its own mark and on those of its fan entries
// (its neighbours); a band position of the previous band whose mark is below
// k is skipped without touching its distance: it did not change in the
// previous iteration, so this iteration's buffer, written two iterations
// ago, already holds its value.  Such a position is finite (its topleset
// entered the band after the one before it, whose values were finite) and
// unchanged, hence converged.  The results are bit-identical to evaluating
// the whole band.
template <typename R>
__device__ inline R ld_s(const R* s, int id) {
    return ld_c(s + id);
}

// Planar update of x0 from one triangle, folded into the minimum `best`
// (which does not depend on the order in which the triangles come).
template <typename R>
__device__ inline void fold_update(const float4 x0, const float4 x1, const float4 x2, R d1, R d2, R& best,
                                   bool valid = true) {
    int l = 0;
    const R u = local_update<R, false>(x0, x1, x2, d1, d2, 0, 0, l);
    best = valid && u < best ? u : best;
}

// The triangles of the first C entries of a fan of L entries (e: entries
// with flags, entries past L repeat entry 0; d / x: their distances and
// coordinates).  Slot q (1 <= q <= C) is the pair (entry q-1,
// entry q) for q < L unless entry q opens a chain, and the closing pair
// (entry L-1, entry 0) for q = L on a closed fan.
template <typename R, int C>
__device__ inline void eval_fan_first(const float4 x0, const int* e, const R* d, const float4* x, int L,
                                      R& best) {
    const bool closed = (e[0] & kFanClosed) != 0;
#pragma unroll
    for (int q = 1; q <= C; ++q) {
        const int q2 = q < C ? q : 0;
        const bool valid = q < C ? (q < L ? (e[q] & kFanStart) == 0 : (q == L && closed)) : (L == C && closed);
        fold_update<R>(x0, x[q - 1], x[q2], d[q - 1], d[q2], best, valid);
    }
}

// The rest of a fan longer than C entries: chunks of C entries overlapping
// by one, then the closing pair with entry 0 (d0 / xf) on a closed fan.
template <typename R, int C>
__device__ inline void eval_fan_rest(const RelaxArgs& a, int v, const float4 x0, int f0, int L, bool closed,
                                     R d0, float4 xf, const R* sold, R& best) {
    for (int base = C - 1; base < L - 1; base += C - 1) {
        const int cnt = min(C, L - base);
        int e[C];
        R d[C];
        float4 x[C];
#pragma unroll
        for (int q = 0; q < C; ++q) e[q] = q < cnt ? a.fan[f0 + base + q] : v;
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int id = e[q] & kFanId;
            d[q] = ld_s(sold, id);
            x[q] = a.xyz[id];
        }
#pragma unroll
        for (int q = 1; q < C; ++q)
            fold_update<R>(x0, x[q - 1], x[q], d[q - 1], d[q], best, q < cnt && (e[q] & kFanStart) == 0);
        if (closed && base + cnt == L) {      // entry L - 1, loaded again (rare path)
            const int id = a.fan[f0 + L - 1] & kFanId;
            const R dl = ld_s(sold, id);
            const float4 xl = a.xyz[id];
            fold_update<R>(x0, xl, xf, dl, d0, best);
        }
    }
}

// The fan record of position v (global), loaded as three 8-byte words.
__device__ inline void load_fan6(const RelaxArgs& a, int v, int* e) {
    const int2* r = reinterpret_cast<const int2*>(a.fan6 + (size_t)kFan6 * v);
    const int2 x0 = r[0], x1 = r[1], x2 = r[2];
    e[0] = x0.x;
    e[1] = x0.y;
    e[2] = x1.x;
    e[3] = x1.y;
    e[4] = x2.x;
    e[5] = x2.y;
}

// Length of the fan whose record is e (and the start of its row, needed for
// fans longer than the record, read from the row form then).
__device__ inline void fan6_length(const RelaxArgs& a, int v, const int* e, int& L, int& f0) {
    f0 = 0;
    if (!(e[0] & kFanStart)) {
        L = 0;
    } else if (e[0] & kFan6Pad) {
        const int2 r = a.fanrow[v];
        f0 = r.x;
        L = r.y - r.x;
    } else {
        L = 1;
#pragma unroll
        for (int q = 1; q < kFan6; ++q) L += (e[q] & kFan6Pad) ? 0 : 1;
    }
}


// Distances and coordinates of the first C fan entries.
template <typename R, int C>
__device__ inline void gather_fan(const RelaxArgs& a, const int* e, const R* sold, R* d, float4* x) {
#pragma unroll
    for (int q = 0; q < C; ++q) {
        const int id = e[q] & kFanId;
        d[q] = ld_s(sold, id);
        x[q] = a.xyz[id];
    }
}

// Smallest planar update of position v over all its incident triangles.
template <typename R, int C>
__device__ inline void best_update(const RelaxArgs& a, int v, const float4 x0, const R* sold, R& best) {
    static_assert(C == kFan6, "fans are read from the fixed-size records");
    best = inf_of<R>();
    int e[C];
    R d[C];
    float4 x[C];
    load_fan6(a, v, e);
    gather_fan<R, C>(a, e, sold, d, x);
    int L, f0;
    fan6_length(a, v, e, L, f0);
    eval_fan_first<R, C>(x0, e, d, x, L, best);
    if (L > C) eval_fan_rest<R, C>(a, v, x0, f0, L, (e[0] & kFanClosed) != 0, d[0], x[0], sold, best);
}

// Convergence of one position between two iterations (Eq. lower_band): a
// value that was +inf is not converged, an unchanged one is (no 0/0 at
// coincident vertices), otherwise |dn - dv| / dv < tol.  The Jacobi rule runs
// it with tol = 0: "finite and unchanged" (once its band holds every
// topleset, each reachable value is finite, so this is "unchanged").
__device__ inline float absr(float x) { return fabsf(x); }
__device__ inline double absr(double x) { return fabs(x); }

template <typename R>
__device__ inline bool converged(R dv, R dn, float tol) {
    return dv < inf_of<R>() && (dn == dv || absr(dn - dv) / dv < (R)tol);
}

// Marks a changed position v and its fan entries (its neighbours: a vertex is
// in the fan of each of its neighbours) for iteration k1.
template <int C>
__device__ inline void mark_fan(const RelaxArgs& a, int v, const int* e, int f0, int L, int k1, bool local) {
    st_g(a.mark + v, k1, local);
#pragma unroll
    for (int q = 0; q < C; ++q)
        if (q < L) st_g(a.mark + (e[q] & kFanId), k1, local);
    for (int q = C; q < L; ++q) st_g(a.mark + (a.fan[f0 + q] & kFanId), k1, local);
}

// Band positions p0, p0 + gsz, ... (< be) of one thread, in batches of
// kBatch.  The marks of a batch are loaded together (coalesced across the
// group's threads).  A position updated in the previous iteration (below
// bprev) and not marked for this one (mark < k) keeps its value (see ld_s).
// The other positions are evaluated, software-pipelined: while the neighbour
// data of one are in flight, the fan record of the next is loaded (read by
// position: no fan row in front of it).  A position whose value changes
// marks itself and its neighbours for the next iteration.  Returns the "not
// converged" vote of the positions below tb; *evals counts the evaluated
// positions.
constexpr int kBatch = 8;

template <typename R, int C>
__device__ inline unsigned relax_band_marked(const RelaxArgs& a, int vo, int p0, int be, int tb, int gsz,
                                             int bprev, int k, const R* sold, R* snew,
                                             bool local, int* evals) {
    static_assert(C == kFan6, "the band loop reads the fixed-size fan records");
    unsigned notconv = 0;
    for (int pb = p0; pb < be; pb += kBatch * gsz) {
        int mk[kBatch];
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int p = pb + i * gsz;
            mk[i] = p < be && p < bprev ? ld_c(a.mark + vo + p) : k;
        }
        unsigned todo = 0;
#pragma unroll
        for (int i = 0; i < kBatch; ++i)
            if (pb + i * gsz < be && mk[i] >= k) todo |= 1u << i;
        if (!todo) continue;
        int p = pb + (__ffs(todo) - 1) * gsz;
        todo &= todo - 1;
        int e[C];
        load_fan6(a, vo + p, e);
        int pn = -1;
        if (todo) {
            pn = pb + (__ffs(todo) - 1) * gsz;
            todo &= todo - 1;
        }
        for (;;) {
            const int v = vo + p;
            const float4 x0 = a.xyz[v];
            const R dv = ld_s(sold, v);
            R d[C];
            float4 x[C];
            gather_fan<R, C>(a, e, sold, d, x);
            // the next position's fan record
            int en[C];
            if (pn >= 0) load_fan6(a, vo + pn, en);
            int pnn = -1;
            if (todo) {
                pnn = pb + (__ffs(todo) - 1) * gsz;
                todo &= todo - 1;
            }
            int L, f0;
            fan6_length(a, v, e, L, f0);
            R best = inf_of<R>();
            eval_fan_first<R, C>(x0, e, d, x, L, best);
            if (L > C) eval_fan_rest<R, C>(a, v, x0, f0, L, (e[0] & kFanClosed) != 0, d[0], x[0], sold, best);
            ++*evals;
            const R dn = best < dv ? best : dv;
            const bool changed = dn != dv;
            st_g(snew + v, dn, local);
            if (changed) mark_fan<C>(a, v, e, f0, L, k + 1, local);
            if (p < tb) notconv |= converged<R>(dv, dn, a.tol) ? 0u : 1u;
            if (pn < 0) break;
            p = pn;
            pn = pnn;
#pragma unroll
            for (int q = 0; q < C; ++q) e[q] = en[q];
        }
    }
    return notconv;
}

// One certification sweep over positions p, p + gsz, ... (< end) of one
// thread, pipelined like the band loop (the next position's fan record is
// loaded while the neighbour data of the current one are in flight): a bound
// below the planar update from the neighbours' bounds is withdrawn (+inf),
// in place.  Returns whether this thread withdrew any; counts them into
// *rejected.
template <int C>
__device__ inline unsigned certify_pipelined(const RelaxArgs& a, int vo, long long p, long long end,
                                             long long gsz, float* d, bool local, int* rejected) {
    static_assert(C == kFan6, "fans are read from the fixed-size records");
    unsigned changed = 0;
    if (p >= end) return 0;
    int e[C];
    load_fan6(a, vo + (int)p, e);
    for (;;) {
        const int v = vo + (int)p;
        const float4 x0 = a.xyz[v];
        const float wv = ld_c(d + v);
        float dd[C];
        float4 x[C];
        gather_fan<float, C>(a, e, d, dd, x);
        const long long pn = p + gsz;
        int en[C];
        if (pn < end) load_fan6(a, vo + (int)pn, en);
        if (wv < kInf) {
            int L, f0;
            fan6_length(a, v, e, L, f0);
            float best = kInf;
            eval_fan_first<float, C>(x0, e, dd, x, L, best);
            if (L > C) eval_fan_rest<float, C>(a, v, x0, f0, L, (e[0] & kFanClosed) != 0, dd[0], x[0], d, best);
            if (wv < best) {
                st_g(d + v, kInf, local);
                changed = 1;
                ++*rejected;
            }
        }
        if (pn >= end) break;
        p = pn;
#pragma unroll
        for (int q = 0; q < C; ++q) e[q] = en[q];
    }
    return changed;
}

// The smallest position >= c that group thread g (of gsz) owns, c >= 0, in
// 32-bit arithmetic (positions stay below 2^29, groups below 2^18 threads).
__device__ inline int first_owned(int c, int g, int gsz) {
    int r = g - c % gsz;
    if (r < 0) r += gsz;
    return c + r;
}

// Topleset starts staged in LDS for meshes with at most this many toplesets
// (read four times per iteration on the critical path).
constexpr int kOffsLds = 4096;

// Groups of consecutive workgroups run the whole iteration of one mesh at a
// time, with a barrier of their own.  Per iteration k every thread of the
// group takes band vertices in a strided loop; position p of the mesh is
// always handled by group thread p mod (gsize * 256), whatever the band, so a
// vertex stays on one CU across iterations and its incidence and coordinates
// stay in that CU's caches.  For each vertex it first gathers up to kChunk
// wedges, then every neighbour distance and coordinate of those wedges at
// once (independent loads), then evaluates the planar updates.  Distances
// are exchanged between workgroups through coherent loads and stores.
// R = double: the same iteration in float64 (no warm start or cache).
// RULES: the band rule is read at run time (fixed half band, Jacobi);
// otherwise it is the paper's, fixed at compile time, which keeps the band
// loop's registers for the common case.
// The float kernels of the paper's rule without the register cache (the
// batch) are held to 128 VGPRs, four workgroups per CU: the band loop waits
// on memory, and a fourth wave per SIMD hides more of it than the registers
// it costs (only per-mesh values spill).
constexpr int relax_waves(bool f32, bool cache, bool rules) { return f32 && !cache && !rules ? 4 : 1; }

template <typename R, bool WARM, bool CACHE, bool RULES = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(relax_waves(sizeof(R) == 4, CACHE, RULES))))
void k_relax(RelaxArgs a) {
    static_assert(sizeof(R) == 4 || (!WARM && !CACHE), "float64 runs plain only");
    const WgInfo me = a.wg[blockIdx.x];
    if (me.group < 0) return;                 // an unused launch slot
    const int gs = me.gsize;
    __shared__ unsigned bar_slots[2 * kBlock / kWave];
    __shared__ int s_offs[kOffsLds];
    FlagBarrier gb{a.bar + (size_t)me.first * kLine, a.bar + (size_t)(a.G + me.first) * kLine,
                   a.ctrl + C_ABORT, (unsigned)gs, (unsigned)me.rank, 0};
    gb.slots = bar_slots;
    unsigned any = 0;
    const int gsz32 = gs * kBlock;
    const int g032 = me.rank * kBlock + (int)threadIdx.x;
    const long long gsz = (long long)gs * kBlock;
    const long long g0 = (long long)me.rank * kBlock + threadIdx.x;
    const bool leader = me.rank == 0 && threadIdx.x == 0;
    const R kInfR = inf_of<R>();
    float* dA = a.dist;
    float* dB = a.dist + a.N;
    // the iteration state: the float double buffer, or the float64 run's
    // doubles in the 8-byte view of the same memory
    R* sA;
    R* sB;
    if constexpr (sizeof(R) == 8) {
        sA = reinterpret_cast<R*>(a.dl);
        sB = reinterpret_cast<R*>(a.dl + a.N);
    } else {
        sA = dA;
        sB = dB;
    }
    const int rule = RULES ? a.band_rule : (int)BAND_PAPER;
    const bool jacobi = rule == BAND_JACOBI;

    // A group whose workgroups all run on one XCD exchanges its data through
    // that XCD's L2 with plain stores.  Every workgroup posts its XCD, the
    // group syncs, and each compares all posts, so all agree on the mode.
    bool local = true;
    if (gs > 1) {
        if (threadIdx.x == 0) st_c(a.xpost + me.first + me.rank, (int)xcc_id());
        if (!gb.sync(0, &any)) return;
        const int x0 = ld_c(a.xpost + me.first);
        int same = 1;
        for (int x = threadIdx.x; x < gs; x += kBlock) same &= ld_c(a.xpost + me.first + x) == x0;
        local = __syncthreads_and(same) != 0;
    }
    gb.local = local;

    // Meshes are taken from queues at run time: the group's leader takes the
    // next mesh of its class's queue (ordered by decreasing estimated time),
    // or of a smaller class once that is empty, and posts it in the group's
    // slot; a group's last read of the slot precedes its next barrier, which
    // the leader passes before it posts again.
    const int* qs = a.queue;
    const int cls = qs[4 + me.group];
    const int* qlist = qs + 4 + a.ngroups;
    int* slot = a.xpost + a.G + me.group;
    for (;;) {
        if (leader) {
            int bn = -1;
            for (int c = cls; c >= 0 && bn < 0; --c) {
                const int i = atomicAdd(a.ctrl + C_QHEAD + c, 1);
                if (i < qs[c + 1] - qs[c]) bn = qlist[qs[c] + i];
            }
            st_c(slot, bn);
        }
        if (!gb.sync(0, &any)) return;
        const int b = ld_c(slot);
        if (b < 0) break;
        const MeshDesc md = a.mesh[b];
        const int n = md.n, vo = md.v_off;
        const int rho = a.state[b].rho;
        const int* offs = a.offsets + vo + b;    // topleset starts, local positions
        int* retire = a.retire + vo;
        // iteration cap: the caller's, else the rule's default
        const int kmax = a.kmax_fixed > 0 ? a.kmax_fixed : (jacobi ? 64 * rho + 256 : 4 * rho + 16);
        // the fixed half band finalises V_r by iteration 2r - 1 (Sec. 6
        // lemma), so it stops after 2 rho - 3 iterations
        const int kfix = max(1, 2 * rho - 3);
        const int m0 = offs[1];                  // |V_0|: the sources occupy [0, m0)
        if (leader) {
            a.state[b].t_begin = wall_clock64();
            a.state[b].wgs = gs;
        }
        // every read of s_offs of the previous mesh came before its last barrier
        const bool offs_lds = rho < kOffsLds;
        if (offs_lds)
            for (int r = threadIdx.x; r <= rho; r += kBlock) s_offs[r] = offs[r];

        const int reach = a.state[b].reach;
        for (long long p = g0; p < n; p += gsz) {
            st_g(a.mark + vo + p, 0, local);
            R d = p < m0 ? (R)0 : kInfR;
            if (WARM && p >= m0 && p < reach) {      // warm start: the caller's bound
                const int v = a.perm[vo + p];
                const float w = a.upper[md.out_off + (v - vo)];
                d = w >= 0.f ? (R)w : kInfR;             // NaN or negative: no bound
            }
            st_g(sA + vo + p, d, local);
            st_g(sB + vo + p, d, local);
        }
        for (long long r = g0; r < rho; r += gsz) st_g(retire + r, r == 0 ? 0 : -1, local);
        if (!gb.sync(0, &any)) return;

        if (WARM && a.certify) {
            // Certification of the warm start: a vertex whose bound lies below
            // the planar update from its neighbours' bounds (w < U(w)) loses its
            // bound (+inf); repeated until no vertex changes.  The result is a
            // supersolution (w >= U(w), w(S) = 0), hence above the fixed point,
            // so the min-relaxation from it descends to the same fixed point.
            // The closure is unique, so the order of the in-place updates does
            // not matter.
            const long long firstc = first_owned(m0, g032, gsz32);
            int rejected = 0, round = 0;
            for (;; ++round) {
                const unsigned changed =
                    certify_pipelined<kChunk>(a, vo, firstc, reach, gsz, dA, local, &rejected);
                if (!gb.sync(changed, &any)) return;
                if (!any) break;
                if (round == kCertifyRounds) {           // no closure in time: no bound
                    for (long long pp = firstc; pp < reach; pp += gsz) st_g(dA + vo + pp, kInf, local);
                    if (!gb.sync(0, &any)) return;
                    rejected = 0;
                    if (leader) rejected = reach - m0;
                    break;
                }
            }
            if (rejected) atomicAdd(&a.state[b].cert_rejected, rejected);
            if (leader) a.state[b].cert_rounds = round + 1;
            for (long long pp = firstc; pp < reach; pp += gsz) st_g(dB + vo + pp, ld_c(dA + vo + pp), local);
            if (!gb.sync(0, &any)) return;
        }

        int i = 1, lo_prev = 1, k = 0, runstat = 0;
        long long upd = 0;
        int bprev = 0;        // end of the previous iteration's band (none before the first)
        // whether the previous iteration kept the marks (the register-cached
        // loop neither reads nor writes them)
        bool marks_kept = false;
        int evals = 0;        // this thread's evaluated positions
        // CACHE: the fan of the vertex this thread handled last.  While the
        // band is no wider than the group's threads, a band vertex keeps its
        // thread for every iteration it spends in the band, so after its first
        // update only the neighbour distances and coordinates are loaded.
        // (Costs registers, hence occupancy: used for single meshes.)
        constexpr int kCache = kChunk;
        int cv = -1, cL = 0;
        float4 cx0 = make_float4(0.f, 0.f, 0.f, 0.f);
        int ce[kCache];
        while (i < rho) {
            if (k >= kmax) {
                runstat = 1;
                break;
            }
            ++k;
            const int j = min(k, rho - 1);                       // Eq. upper_band
            int lo = i;
            if (rule == BAND_FIXED_HALF) lo = max(1, (k + 1) >> 1);
            if (a.window > 0) lo = max(lo, j - a.window + 1);
            const R* sold = (k & 1) ? sA : sB;
            R* snew = (k & 1) ? sB : sA;
            const int cb = offs_lds ? s_offs[lo_prev] : offs[lo_prev];   // retired since last iteration: copy
            const int bb = offs_lds ? s_offs[lo] : offs[lo];             // band
            const int be = offs_lds ? s_offs[j + 1] : offs[j + 1];
            // tested positions: V_lo (relative change), the whole band (Jacobi)
            const int tb = jacobi ? be : (offs_lds ? s_offs[lo + 1] : offs[lo + 1]);
            unsigned notconv = 0;
            const long long first = first_owned(cb, g032, gsz32);
            // pipelined unless the register cache serves (one position per
            // thread)
            const bool pipe = !(CACHE && be - cb <= gsz);
            if (pipe) {
                for (long long pp = first; pp < bb; pp += gsz)
                    st_g(snew + vo + pp, ld_s(sold, vo + (int)pp), local);
                const long long firstb = first_owned(bb, g032, gsz32);
                notconv |= relax_band_marked<R, kChunk>(a, vo, (int)firstb, be, tb, gsz32, marks_kept ? bprev : 0, k,
                                                        sold, snew, local, &evals);
                cv = -1;
            }
            for (long long pp = pipe ? be : first; pp < be; pp += gsz) {
                const int v = vo + (int)pp;
                if (pp < bb) {
                    st_g(snew + v, ld_s(sold, v), local);
                    continue;
                }
                const bool cached = CACHE && be - cb <= gsz;   // one position per thread
                if (cached && v != cv) {        // a vertex new to this thread
                    cx0 = a.xyz[v];
                    load_fan6(a, v, ce);
                    int f0;
                    fan6_length(a, v, ce, cL, f0);
                    cv = cL <= kCache ? v : -1;
                }
                // every band vertex is evaluated here (at most one per thread):
                // the neighbours' loads need not wait for a mark, and no marks
                // are stored (the next pipelined iteration evaluates its whole band)
                const R dv = ld_s(sold, v);
                R best = kInfR;
                if (cached && cv == v) {
                    R d[kCache];
                    float4 x[kCache];
                    gather_fan<R, kCache>(a, ce, sold, d, x);
                    eval_fan_first<R, kCache>(cx0, ce, d, x, cL, best);
                } else {
                    const float4 x0 = cached ? cx0 : a.xyz[v];
                    best_update<R, kChunk>(a, v, x0, sold, best);
                }
                ++evals;
                const R dn = best < dv ? best : dv;
                st_g(snew + v, dn, local);
                if (pp < tb) notconv |= converged<R>(dv, dn, a.tol) ? 0u : 1u;
            }
            upd += be - bb;
            bprev = be;
            marks_kept = pipe;
            if (!gb.sync(notconv, &any)) return;
            if (leader)
                for (int r = i; r < lo; ++r) st_g(retire + r, k - 1, local);   // pushed out of the band
            if (rule == BAND_FIXED_HALF) {
                // the toplesets below the next iteration's band are final;
                // after the last iteration every topleset is
                const int inew = k >= kfix ? rho : max(lo, (k + 2) >> 1);
                if (leader)
                    for (int r = lo; r < inew; ++r) st_g(retire + r, k, local);
                i = inew;
            } else if (jacobi) {
                // fixed point: no value of the (full) band changed
                if (!any && j == rho - 1) {
                    if (leader)
                        for (int r = lo; r < rho; ++r) st_g(retire + r, k, local);
                    i = rho;
                } else {
                    i = lo;
                }
            } else if (!any && k > lo) {
                // Eq. lower_band.  V_lo may retire only after its second update
                // (k > lo): from +inf that is automatic, and a warm start keeps
                // the same causality, so the band never runs ahead of the front.
                if (leader) st_g(retire + lo, k, local);
                i = lo + 1;
            } else {
                i = lo;
            }
            lo_prev = lo;
        }
        const R* sfin = (k & 1) ? sB : sA;
        for (long long p = g0; p < n; p += gsz) {
            const int v = a.perm[vo + p];
            const R df = ld_s(sfin, vo + (int)p);
            if (sizeof(R) == 8) a.out_d64[md.out_off + (v - vo)] = (double)df;
            else a.out_d[md.out_off + (v - vo)] = (float)df;
        }
        // evaluated positions: a wave sum, one atomic per wave
        long long ev = evals;
        for (int o = kWave / 2; o > 0; o >>= 1) ev += __shfl_xor(ev, o, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0 && ev) atomicAdd(&a.state[b].evaluated, (unsigned long long)ev);
        if (leader) {
            a.state[b].iters = k;
            a.state[b].runstat = runstat;
            a.state[b].updates = upd;
            a.state[b].t_end = wall_clock64();
        }
    }
}

__global__ void k_run_reset(int* ctrl, MeshState* state, int B) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl[C_ABORT] = 0;
        for (int c = 0; c < 3; ++c) ctrl[C_QHEAD + c] = 0;
    }
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
        state[b].iters = 0;
        state[b].runstat = 0;
        state[b].updates = 0;
        state[b].cert_rounds = 0;
        state[b].cert_rejected = 0;
        state[b].t_begin = 0;
        state[b].t_end = 0;
        state[b].wgs = 0;
        state[b].evaluated = 0;
    }
}

// ---- Voronoi labels of the final map ---------------------------------------
// The label of a vertex is the index in S of the source at the root of its
// chain of parents.  The parent is the vertex its final value comes from
// under its best triangle: over the fan's triangles the smallest (update,
// giver id), the giver of a planar value being its smaller input and that of
// an edge update the edge's other end (equal candidates: the smaller id),
// among givers that come before the vertex in (distance, id) order, so that
// the parents form a forest rooted at the sources.  Ids are the caller's
// vertex ids, so the result does not depend on the internal order.  `parent`
// and `root` receive parent positions (a source its own, -1 for an
// unreachable vertex or one without a giver); pointer jumping then turns
// `root` into roots.
__global__ __launch_bounds__(kBlock) void k_parents(const MeshDesc* mesh, const MeshState* state, int B,
                                                    const int* vo_prefix, long long N, const int* perm,
                                                    const int* level, const int2* fanrow, const int* fan,
                                                    const int* fan6,
                                                    const float4* xyz, const float* dist, int* parent,
                                                    int* root) {
    for_tiles(vo_prefix, B, N, [&](long long p, int b) {
        const int vo = mesh[b].v_off;
        // the mesh's final distances: the buffer its last iteration wrote
        const float* d = dist + ((state[b].iters & 1) ? N : 0);
        const int vid = perm[p] - vo;
        if (level[vo + vid] == 0) {
            parent[p] = (int)p;
            root[p] = (int)p;
            return;
        }
        const float dv = fabsf(d[p]);
        int bq = -1;
        if (dv < kInf) {
            const float4 x0 = xyz[p];
            float bu = kInf;
            int bg = 0x7fffffff;
            auto tri = [&](int q1, int q2) {
                const float d1 = fabsf(d[q1]), d2 = fabsf(d[q2]);
                const int i1 = perm[q1] - vo, i2 = perm[q2] - vo;
                int g = 0;
                const float u = local_update<float, true>(x0, xyz[q1], xyz[q2], d1, d2, i1, i2, g);
                if (!(u < kInf)) return;
                const float dg = g == i1 ? d1 : d2;
                if (!(dg < dv || (dg == dv && g < vid))) return;
                if (u < bu || (u == bu && g < bg)) {
                    bu = u;
                    bg = g;
                    bq = g == i1 ? q1 : q2;
                }
            };
            // the fan: its fixed-size record, or the row form for a longer fan
            const int2* r6 = reinterpret_cast<const int2*>(fan6 + (size_t)kFan6 * p);
            const int2 w0 = r6[0], w1 = r6[1], w2 = r6[2];
            const int rec[kFan6] = {w0.x, w0.y, w1.x, w1.y, w2.x, w2.y};
            const bool longf = (rec[0] & kFanStart) && (rec[0] & kFan6Pad);
            int L = 0, f0 = 0;
            if (longf) {
                const int2 r = fanrow[p];
                f0 = r.x;
                L = r.y - r.x;
            } else if (rec[0] & kFanStart) {
                L = 1;
                for (int q = 1; q < kFan6; ++q) L += (rec[q] & kFan6Pad) ? 0 : 1;
            }
            int first = -1, prev = -1;
            for (int q = 0; q < L; ++q) {
                const int e = longf ? fan[f0 + q] : rec[q];
                const int id = e & kFanId;
                if (q == 0) first = id;
                else if (!(e & kFanStart)) tri(prev, id);
                prev = id;
            }
            if (L > 1 && (rec[0] & kFanClosed)) tri(prev, first);
        }
        parent[p] = bq;
        root[p] = bq;
    });
}

// One round of pointer jumping: every vertex moves its pointer to its
// pointer's pointer.  Pointers only ever move towards the roots, so reading a
// neighbour's pointer before or after its update this round is equally
// right; a chain of length c is resolved after ceil(log2 c) rounds.
__global__ __launch_bounds__(kBlock) void k_jump(long long N, int* root) {
    const long long gsz = (long long)gridDim.x * kBlock;
    for (long long p = blockIdx.x * (long long)kBlock + threadIdx.x; p < N; p += gsz) {
        const int r = root[p];
        if (r < 0) continue;
        const int rr = root[r];
        if (rr != r) root[p] = rr;
    }
}

// Index in S of the source at each source position.
__global__ __launch_bounds__(kBlock) void k_source_index(const MeshDesc* mesh, int B, const int* so,
                                                         long long Stot, const int* S, const int* iperm,
                                                         int* srcidx) {
    for_tiles(so, B, Stot, [&](long long x, int b) {
        const int s = (int)(x - so[b]);
        srcidx[iperm[mesh[b].v_off + S[mesh[b].s_in + s]]] = s;
    });
}

__global__ __launch_bounds__(kBlock) void k_label_out(const MeshDesc* mesh, int B, const int* vo_prefix,
                                                      long long N, const int* perm, const int* root,
                                                      const int* srcidx, int* out_l) {
    for_tiles(vo_prefix, B, N, [&](long long p, int b) {
        const int r = root[p];
        out_l[mesh[b].out_off + (perm[p] - mesh[b].v_off)] = r >= 0 ? srcidx[r] : -1;
    });
}

__global__ __launch_bounds__(kBlock) void k_parent_out(const MeshDesc* mesh, int B, const int* vo_prefix,
                                                       long long N, const int* perm, const int* parent,
                                                       int* out) {
    for_tiles(vo_prefix, B, N, [&](long long p, int b) {
        const int vo = mesh[b].v_off, q = parent[p];
        out[mesh[b].out_off + (perm[p] - vo)] = q >= 0 ? perm[q] - vo : -1;
    });
}

template <typename R, bool WARM, bool CACHE, bool RULES = false>
const void* relax_fn() {
    return reinterpret_cast<const void*>(&k_relax<R, WARM, CACHE, RULES>);
}

int tile_grid(long long total) {
    const long long t = (total + kTile - 1) / kTile;
    return (int)std::max<long long>(1, std::min<long long>(8192, t));
}

}  // namespace

hipError_t launch_run(const Work& w, const RunParams& p, bool labels, bool cache, bool f64, int g_run,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_run_reset, dim3((p.B + 255) / 256), dim3(256), 0, st, w.ctrl, w.state, p.B);
    launch_barrier_reset(w, 2 * g_run, st);
    RelaxArgs a;
    a.G = g_run;
    a.kmax_fixed = p.kmax_fixed;
    a.window = p.window;
    a.band_rule = p.band_rule;
    a.certify = p.certify ? 1 : 0;
    a.tol = p.band_rule == BAND_JACOBI ? 0.f : p.tol;
    a.mesh = w.mesh;
    a.state = w.state;
    a.wg = f64 ? w.wg_run64 : w.wg_run;
    a.queue = f64 ? w.glist_run64 : w.glist_run;
    a.ngroups = p.ngroups;
    a.S = p.S;
    a.upper = p.upper;
    a.xpost = w.cnt;
    a.perm = w.perm;
    a.iperm = w.iperm;
    a.offsets = w.offsets;
    a.fanrow = w.fanrow;
    a.fan = w.fan;
    a.xyz = w.xyz;
    a.dist = w.dist;
    a.dl = w.dl;
    a.retire = w.retire;
    a.ctrl = w.ctrl;
    a.bar = w.bar;
    a.mark = w.mark;
    a.fan6 = w.fan6;
    a.N = p.N;
    a.out_d = p.out_d;
    a.out_d64 = p.out_d64;
    void* args[] = {&a};
    const void* fn;
    const bool rules = p.band_rule != BAND_PAPER;
    if (f64)
        fn = rules ? relax_fn<double, false, false, true>() : relax_fn<double, false, false>();
    else if (rules)       // the other band rules: uncached, read at run time
        fn = p.upper ? relax_fn<float, true, false, true>() : relax_fn<float, false, false, true>();
    else if (p.upper)
        fn = cache ? relax_fn<float, true, true>() : relax_fn<float, true, false>();
    else
        fn = cache ? relax_fn<float, false, true>() : relax_fn<float, false, false>();
    hipError_t e = hipLaunchCooperativeKernel(fn, dim3(g_run), dim3(kBlock), args, 0, st);
    if (e != hipSuccess || !labels) return e;
    // labels of the final map: parents (kept in the fill cursors of the
    // prepare, free by now), pointer jumping, then the caller's order; root
    // and source index live in the upper half of the distance region (the
    // float run uses its lower half)
    int* root = reinterpret_cast<int*>(w.dist + 2 * p.N);
    int* srcidx = reinterpret_cast<int*>(w.dist + 3 * p.N);
    const int gN = tile_grid(p.N);
    hipLaunchKernelGGL(k_source_index, dim3(tile_grid(p.Stot)), dim3(kBlock), 0, st, w.mesh, p.B, w.so, p.Stot,
                       p.S, w.iperm, srcidx);
    hipLaunchKernelGGL(k_parents, dim3(gN), dim3(kBlock), 0, st, w.mesh, w.state, p.B, w.vo, p.N, w.perm,
                       w.level, w.fanrow, w.fan, w.fan6, w.xyz, w.dist, w.cursor, root);
    for (int r = 0; r < p.jump_rounds; ++r)
        hipLaunchKernelGGL(k_jump, dim3(gN), dim3(kBlock), 0, st, p.N, root);
    hipLaunchKernelGGL(k_label_out, dim3(gN), dim3(kBlock), 0, st, w.mesh, p.B, w.vo, p.N, w.perm, root, srcidx,
                       p.out_l);
    return hipGetLastError();
}

hipError_t launch_parents_out(const Work& w, int B, long long N, int* out, hipStream_t st) {
    hipLaunchKernelGGL(k_parent_out, dim3(tile_grid(N)), dim3(kBlock), 0, st, w.mesh, B, w.vo, N, w.perm,
                       w.cursor, out);
    return hipGetLastError();
}

namespace {
int blocks_per_cu(const void* fn) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kBlock, 0) != hipSuccess) return 0;
    return nb;
}
}  // namespace

// Co-resident workgroups of the relaxation kernels a plan may launch (the
// plain and the warm-start one; with `cache`, the register-caching variants;
// with `rules`, the run-time-rule variants).
int max_coop_blocks_run(int cus, bool cache, bool rules) {
    int nb;
    if (rules)
        nb = std::min(blocks_per_cu(relax_fn<float, false, false, true>()),
                      blocks_per_cu(relax_fn<float, true, false, true>()));
    else
        nb = std::min(blocks_per_cu(cache ? relax_fn<float, false, true>() : relax_fn<float, false, false>()),
                      blocks_per_cu(cache ? relax_fn<float, true, true>() : relax_fn<float, true, false>()));
    return std::max(nb, 1) * cus;
}

int max_coop_blocks_run64(int cus, bool rules) {
    return std::max(blocks_per_cu(rules ? relax_fn<double, false, false, true>()
                                        : relax_fn<double, false, false>()),
                    1) * cus;
}

}  // namespace ptp

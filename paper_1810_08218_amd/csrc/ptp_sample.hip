// Applications of the distance maps (paper Sec. 5.3): farthest point
// sampling, which grows the source set by the vertex farthest from it, and a
// Lloyd step on the geodesic Voronoi cells towards a centroidal Voronoi
// tessellation (named as an application of the method in Sec. 7).
#include "ptp_device.h"

#include "ptp_kernels.h"

namespace ptp {

namespace {

// ---- farthest point sampling -------------------------------------------
// The farthest vertex of a caller-order map: the largest finite positive
// distance, the smallest vertex id on a tie.  For d >= 0 the bits of a float
// order like its value, so the key (bits(d) << 32) | ~id has its maximum at
// the wanted vertex and one 64-bit atomic maximum per workgroup decides it
// independently of scheduling.
__device__ inline unsigned long long far_key(float d, int v) {
    if (!(d > 0.f) || !(d < __builtin_huge_valf())) return 0ull;
    return ((unsigned long long)__float_as_uint(d) << 32) | (unsigned)(~v);
}

__global__ __launch_bounds__(kBlock) void k_fps_max(const float* dist, int n, unsigned long long* key,
                                                    const int* ctrl) {
    if (ld_c(ctrl + C_STATUS) != 0) return;
    __shared__ unsigned long long red[kBlock / kWave];
    unsigned long long best = 0;
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock)
        best = max(best, far_key(dist[v], v));
    for (int o = kWave / 2; o > 0; o >>= 1) best = max(best, __shfl_xor(best, o));
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / kWave; ++w) best = max(best, red[w]);
        if (best) atomicMax(key, best);
    }
}

// Append the farthest vertex to S at `slot` (slot < 0: record the step
// statistics only), grow the mesh's source count, reset the key.
__global__ void k_fps_commit(unsigned long long* key, int* S, MeshDesc* mesh, const MeshState* state,
                             int slot, float* radius, long long* step_stats, int* ctrl) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (ld_c(ctrl + C_STATUS) != 0) return;
    if (step_stats) {
        step_stats[0] = state[0].iters;
        step_stats[1] = state[0].updates;
    }
    if (slot < 0) return;
    const unsigned long long k = *key;
    *key = 0ull;
    if (k == 0ull) {            // every reachable vertex is a source already
        atomicOr(ctrl + C_STATUS, ST_FPS_EMPTY);
        return;
    }
    const int v = (int)~(unsigned)(k & 0xffffffffull);
    S[mesh[0].s_in + slot] = v;
    if (radius) *radius = __uint_as_float((unsigned)(k >> 32));
    mesh[0].m = slot + 1;
}

// ---- Lloyd step ----------------------------------------------------------
// Cell c gathers, over the faces, a third of each face's area for every
// corner labelled c (the barycentric area of the vertex) and that area times
// the corner's position.  Block (c, chunk) covers one chunk of the faces in
// index order; each thread sums in float64, the block reduces in a fixed
// order, so the result does not depend on scheduling.
__device__ inline void block_sum4(double* v, double* red) {
    // red: [4][kBlock]
    for (int q = 0; q < 4; ++q) red[q * kBlock + threadIdx.x] = v[q];
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int q = 0; q < 4; ++q) red[q * kBlock + threadIdx.x] += red[q * kBlock + threadIdx.x + o];
        __syncthreads();
    }
    for (int q = 0; q < 4; ++q) v[q] = red[q * kBlock];
}

__global__ __launch_bounds__(kBlock) void k_lloyd_moments(const float* V, const int* F, int nf, const int* label,
                                                          double* part) {
    __shared__ double red[4 * kBlock];
    const int c = blockIdx.x, chunk = blockIdx.y;
    const long long per = ((long long)nf + kCvtChunks - 1) / kCvtChunks;
    const long long t0 = (long long)chunk * per, t1 = min((long long)nf, t0 + per);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (long long t = t0 + threadIdx.x; t < t1; t += kBlock) {
        const int v[3] = {F[3 * t], F[3 * t + 1], F[3 * t + 2]};
        const int l0 = label[v[0]], l1 = label[v[1]], l2 = label[v[2]];
        if (l0 != c && l1 != c && l2 != c) continue;
        double x[3][3];
        for (int q = 0; q < 3; ++q)
            for (int r = 0; r < 3; ++r) x[q][r] = (double)V[3 * (long long)v[q] + r];
        const double ax = x[1][0] - x[0][0], ay = x[1][1] - x[0][1], az = x[1][2] - x[0][2];
        const double bx = x[2][0] - x[0][0], by = x[2][1] - x[0][1], bz = x[2][2] - x[0][2];
        const double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
        const double third = 0.5 * __builtin_sqrt(cx * cx + cy * cy + cz * cz) / 3.0;
        const int l[3] = {l0, l1, l2};
        for (int q = 0; q < 3; ++q)
            if (l[q] == c) {
                acc[0] += third;
                acc[1] += third * x[q][0];
                acc[2] += third * x[q][1];
                acc[3] += third * x[q][2];
            }
    }
    block_sum4(acc, red);
    if (threadIdx.x == 0)
        for (int q = 0; q < 4; ++q) part[((size_t)c * kCvtChunks + chunk) * 6 + q] = acc[q];
}

// Centroid of each cell (the generator's position for an empty cell):
// centroid[c] = (x, y, z, area).
__global__ void k_lloyd_centroid(const double* part, const float* V, const int* S_in, int m,
                                 double* centroid) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m) return;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < kCvtChunks; ++k)
        for (int q = 0; q < 4; ++q) s[q] += part[((size_t)c * kCvtChunks + k) * 6 + q];
    double* o = centroid + 4 * (size_t)c;
    if (s[0] > 0.0) {
        o[0] = s[1] / s[0];
        o[1] = s[2] / s[0];
        o[2] = s[3] / s[0];
    } else {
        for (int q = 0; q < 3; ++q) o[q] = (double)V[3 * (long long)S_in[c] + q];
    }
    o[3] = s[0];
}

// Nearest vertex of cell c to its centroid: block (c, chunk) scans one chunk
// of the vertices; (squared distance, id) minima reduced in a fixed order.
__global__ __launch_bounds__(kBlock) void k_lloyd_nearest(const float* V, int nv, const int* label,
                                                          const double* centroid, double* part) {
    __shared__ double rd[kBlock];
    __shared__ int rv[kBlock];
    const int c = blockIdx.x, chunk = blockIdx.y;
    const long long per = ((long long)nv + kCvtChunks - 1) / kCvtChunks;
    const long long v0 = (long long)chunk * per, v1 = min((long long)nv, v0 + per);
    const double* g = centroid + 4 * (size_t)c;
    double bd = __builtin_huge_val();
    int bv = 0x7fffffff;
    for (long long v = v0 + threadIdx.x; v < v1; v += kBlock) {
        if (label[v] != c) continue;
        const double ex = (double)V[3 * v] - g[0], ey = (double)V[3 * v + 1] - g[1],
                     ez = (double)V[3 * v + 2] - g[2];
        const double q = ex * ex + ey * ey + ez * ez;
        if (q < bd || (q == bd && (int)v < bv)) {
            bd = q;
            bv = (int)v;
        }
    }
    rd[threadIdx.x] = bd;
    rv[threadIdx.x] = bv;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const double d2 = rd[threadIdx.x + o];
            const int v2 = rv[threadIdx.x + o];
            if (d2 < rd[threadIdx.x] || (d2 == rd[threadIdx.x] && v2 < rv[threadIdx.x])) {
                rd[threadIdx.x] = d2;
                rv[threadIdx.x] = v2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[((size_t)c * kCvtChunks + chunk) * 6 + 4] = rd[0];
        part[((size_t)c * kCvtChunks + chunk) * 6 + 5] = (double)rv[0];
    }
}

__global__ void k_lloyd_pick(const double* part, const int* S_in, int m, int* S_out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m) return;
    double bd = __builtin_huge_val();
    int bv = 0x7fffffff;
    for (int k = 0; k < kCvtChunks; ++k) {
        const double d2 = part[((size_t)c * kCvtChunks + k) * 6 + 4];
        const int v2 = (int)part[((size_t)c * kCvtChunks + k) * 6 + 5];
        if (d2 < bd || (d2 == bd && v2 < bv)) {
            bd = d2;
            bv = v2;
        }
    }
    S_out[c] = bv == 0x7fffffff ? S_in[c] : bv;
}

}  // namespace

hipError_t launch_fps_pick(const Work& w, const float* dist, int n, int* S, int slot, float* radius,
                           long long* step_stats, hipStream_t st) {
    unsigned long long* key = reinterpret_cast<unsigned long long*>(w.ctrl + C_FPS_KEY);
    if (slot >= 0) {
        const int grid = (int)std::min<long long>(1024, ((long long)n + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_fps_max, dim3(grid), dim3(kBlock), 0, st, dist, n, key, w.ctrl);
    }
    hipLaunchKernelGGL(k_fps_commit, dim3(1), dim3(64), 0, st, key, S, w.mesh, w.state, slot, radius,
                       step_stats, w.ctrl);
    return hipGetLastError();
}

hipError_t launch_lloyd(const Work& w, const float* V, const int* F, int nv, int nf, const int* label,
                        const int* S_in, int m, int* S_out, double* centroid, hipStream_t st) {
    hipLaunchKernelGGL(k_lloyd_moments, dim3(m, kCvtChunks), dim3(kBlock), 0, st, V, F, nf, label, w.cvt);
    hipLaunchKernelGGL(k_lloyd_centroid, dim3((m + 63) / 64), dim3(64), 0, st, w.cvt, V, S_in, m, centroid);
    hipLaunchKernelGGL(k_lloyd_nearest, dim3(m, kCvtChunks), dim3(kBlock), 0, st, V, nv, label, centroid,
                       w.cvt);
    hipLaunchKernelGGL(k_lloyd_pick, dim3((m + 63) / 64), dim3(64), 0, st, w.cvt, S_in, m, S_out);
    return hipGetLastError();
}

}  // namespace ptp

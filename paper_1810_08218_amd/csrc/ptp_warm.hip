// Learned warm start: per-vertex features, the MLP (inference and training),
// Adam.  The certification of the predicted upper bound and the PTP run from
// it live in the relaxation kernel.
//
// Features of vertex v of a prepared mesh (l = mean edge length of the mesh,
// the mean of |x_v - x_a| over every vertex v and incident triangle (v, a, b)):
//   f1 = Euclidean distance to the nearest source,
//   f2 = BFS hop count (the topleset index) times l,
//   f3 = signed discrete mean curvature: with the cotangent Laplacian
//        K(v) = (1 / 2A) sum_{(v,a,b)} cot(angle at b)(x_a - x_v) + cot(angle at a)(x_b - x_v),
//        A = a third of the incident triangle areas, H = |K| / 2 taken with the
//        sign of K . n_v (n_v = sum of the incident face normals).
// The network sees x = (f1 / l, f2 / l, f3 l) / (64, 64, 1).
#include "ptp_device.h"
#include "ptp_kernels.h"
#include "ptp_mlp.h"

#include <algorithm>

namespace ptp {

namespace {

constexpr float kInf = __builtin_huge_valf();
__device__ inline float len3(float x, float y, float z) { return sqrtf(x * x + y * y + z * z); }

__global__ void k_zero_u64(unsigned long long* p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0ull;
}

// The mean edge length of each mesh is a sum of |x_v - x_a| over every
// (vertex, incident triangle) pair, taken in fixed point so that it does not
// depend on the order of the atomics: first the largest term of each mesh
// (a maximum is order-free), then the terms scaled to 2^31 / max, which keeps
// a sum of up to 2^31 terms inside 64 bits.
// One atomic per wave where the wave's positions all lie in one mesh (nearly
// always), otherwise one per lane: a single counter per mesh hit by every
// vertex would serialise the kernel.
__device__ inline bool wave_uniform(int b) {
    const int b0 = __shfl(b, 0, kWave);
    return __all(b == b0);
}

__global__ __launch_bounds__(kBlock) void k_edge_max(const float4* xyz, const int* row, const int2* wedge,
                                                     const int* perm, const int* iperm, const int* vo, int B,
                                                     long long N,
                                                     unsigned long long* emax) {
    const long long gsz = (long long)gridDim.x * kBlock;
    const long long span = (N + gsz - 1) / gsz * gsz;          // every lane runs the same trips
    for (long long p = blockIdx.x * (long long)kBlock + threadIdx.x; p < span; p += gsz) {
        const bool in = p < N;
        const int b = in ? mesh_of(vo, B, p) : -1;
        float mx = 0.f;
        if (in) {
            const float4 x = xyz[p];
            const int v = perm[p];
            for (int e = row[v]; e < row[v + 1]; ++e) {
                const float4 a = xyz[iperm[wedge[e].x]];
                mx = fmaxf(mx, len3(a.x - x.x, a.y - x.y, a.z - x.z));
            }
        }
        if (wave_uniform(b)) {
            for (int m = 1; m < kWave; m <<= 1) mx = fmaxf(mx, __shfl_xor(mx, m, kWave));
            if ((threadIdx.x & (kWave - 1)) == 0 && b >= 0 && mx > 0.f)
                atomicMax(emax + b, (unsigned long long)__float_as_uint(mx));
        } else if (in && mx > 0.f) {
            atomicMax(emax + b, (unsigned long long)__float_as_uint(mx));
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_edge_sum(const float4* xyz, const int* row, const int2* wedge,
                                                     const int* perm, const int* iperm, const int* vo, int B,
                                                     long long N,
                                                     const unsigned long long* emax,
                                                     unsigned long long* acc) {
    const long long gsz = (long long)gridDim.x * kBlock;
    const long long span = (N + gsz - 1) / gsz * gsz;
    for (long long p = blockIdx.x * (long long)kBlock + threadIdx.x; p < span; p += gsz) {
        const bool in = p < N;
        const int b = in ? mesh_of(vo, B, p) : -1;
        unsigned long long s = 0;
        if (in) {
            const float mx = __uint_as_float((unsigned)emax[b]);
            if (mx > 0.f) {
                const double scale = 2147483648.0 / (double)mx;
                const float4 x = xyz[p];
                const int v = perm[p];
                for (int e = row[v]; e < row[v + 1]; ++e) {
                    const float4 a = xyz[iperm[wedge[e].x]];
                    s += (unsigned long long)llrint((double)len3(a.x - x.x, a.y - x.y, a.z - x.z) * scale);
                }
            }
        }
        // integer sums do not depend on the order of the additions
        if (wave_uniform(b)) {
            for (int m = 1; m < kWave; m <<= 1) s += __shfl_xor(s, m, kWave);
            if ((threadIdx.x & (kWave - 1)) == 0 && b >= 0 && s) atomicAdd(acc + b, s);
        } else if (in && s) {
            atomicAdd(acc + b, s);
        }
    }
}

__global__ void k_edge_mean(const unsigned long long* acc, const unsigned long long* emax, const int* row,
                            const MeshDesc* mesh, int B, MeshState* state) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
        const int vo = mesh[b].v_off;
        const long long cnt = (long long)row[vo + mesh[b].n] - row[vo];
        const double mx = (double)__uint_as_float((unsigned)emax[b]);
        const double l = cnt > 0 && mx > 0 ? (double)acc[b] / 2147483648.0 * mx / (double)cnt : 1.0;
        state[b].mean_edge = (float)(l > 0 ? l : 1.0);
    }
}

// One incident triangle (v, a, b) of a vertex at x: the unnormalised face
// normal q = (a - x) x (b - x), twice its area, and its term of the
// cotangent Laplacian, cot(angle at b)(a - x) + cot(angle at a)(b - x)
// (zero for a degenerate triangle).
struct WedgeGeo {
    float3 q, k;
    float dbl;
};

__device__ inline WedgeGeo wedge_geo(const float4 x, const float4 a, const float4 c) {
    WedgeGeo g;
    const float ax = a.x - x.x, ay = a.y - x.y, az = a.z - x.z;   // v -> a
    const float cx = c.x - x.x, cy = c.y - x.y, cz = c.z - x.z;   // v -> b
    g.q = make_float3(ay * cz - az * cy, az * cx - ax * cz, ax * cy - ay * cx);
    g.dbl = len3(g.q.x, g.q.y, g.q.z);
    g.k = make_float3(0.f, 0.f, 0.f);
    if (g.dbl > 0.f) {
        // angle at a: between (v - a) and (b - a); at b: between (v - b) and (a - b)
        const float cot_a = ((-ax) * (cx - ax) + (-ay) * (cy - ay) + (-az) * (cz - az)) / g.dbl;
        const float cot_b = ((-cx) * (ax - cx) + (-cy) * (ay - cy) + (-cz) * (az - cz)) / g.dbl;
        g.k = make_float3(cot_b * ax + cot_a * cx, cot_b * ay + cot_a * cy, cot_b * az + cot_a * cz);
    }
    return g;
}

// Network inputs (x0, x1, x2) and the scale l per internal position; w = -1
// marks positions with no feature (unreachable vertices).
__global__ __launch_bounds__(kBlock) void k_features(const float4* xyz, const int* row, const int2* wedge,
                                                     const int* perm, const int* iperm, const int* level,
                                                     const int* vo,
                                                     const MeshDesc* mesh, const MeshState* state, int B,
                                                     long long N, float4* feat) {
    const long long gsz = (long long)gridDim.x * kBlock;
    for (long long p = blockIdx.x * (long long)kBlock + threadIdx.x; p < N; p += gsz) {
        const int b = mesh_of(vo, B, p);
        const int v0 = mesh[b].v_off;
        const float l = state[b].mean_edge;
        const int hop = level[perm[p]];   // by global vertex id
        if (hop < 0) {
            feat[p] = make_float4(0.f, 0.f, 0.f, -1.f);
            continue;
        }
        const float4 x = xyz[p];
        float f1 = kInf;
        for (int i = 0; i < mesh[b].m; ++i) {           // sources occupy the first m positions
            const float4 s = xyz[v0 + i];
            f1 = fminf(f1, len3(x.x - s.x, x.y - s.y, x.z - s.z));
        }
        // The incidence order of a vertex's triangles is not fixed (it comes
        // from atomics), so the sums are taken in fixed point: a first pass
        // finds the largest magnitude, the second adds integers scaled to it.
        const int v = perm[p];
        const int e0 = row[v], e1 = row[v + 1];
        float mk = 0.f, mq = 0.f;
        for (int e = e0; e < e1; ++e) {
            const WedgeGeo g = wedge_geo(x, xyz[iperm[wedge[e].x]], xyz[iperm[wedge[e].y]]);
            mk = fmaxf(mk, fmaxf(fabsf(g.k.x), fmaxf(fabsf(g.k.y), fabsf(g.k.z))));
            mq = fmaxf(mq, fmaxf(g.dbl, fmaxf(fabsf(g.q.x), fmaxf(fabsf(g.q.y), fabsf(g.q.z)))));
        }
        const double deg = (double)max(1, e1 - e0);
        const double sk = mk > 0.f ? 4611686018427387904.0 / ((double)mk * deg) : 0.0;   // 2^62
        const double sq = mq > 0.f ? 4611686018427387904.0 / ((double)mq * deg) : 0.0;
        long long Kx = 0, Ky = 0, Kz = 0, Nx = 0, Ny = 0, Nz = 0, A = 0;
        for (int e = e0; e < e1; ++e) {
            const WedgeGeo g = wedge_geo(x, xyz[iperm[wedge[e].x]], xyz[iperm[wedge[e].y]]);
            Kx += llrint((double)g.k.x * sk);
            Ky += llrint((double)g.k.y * sk);
            Kz += llrint((double)g.k.z * sk);
            Nx += llrint((double)g.q.x * sq);
            Ny += llrint((double)g.q.y * sq);
            Nz += llrint((double)g.q.z * sq);
            A += llrint((double)g.dbl * sq);
        }
        float H = 0.f;
        if (A > 0 && sk > 0.0) {
            const double area = (double)A / sq / 6.0;      // a third of the incident areas
            const double kx = (double)Kx / sk / (2.0 * area);
            const double ky = (double)Ky / sk / (2.0 * area);
            const double kz = (double)Kz / sk / (2.0 * area);
            H = (float)(0.5 * sqrt(kx * kx + ky * ky + kz * kz));
            if (kx * (double)Nx + ky * (double)Ny + kz * (double)Nz < 0.0) H = -H;
        }
        feat[p] = make_float4(f1 / l * kInScale, (float)hop * kInScale, H * l, l);
    }
}

// The network inputs in the caller's order (training data): X[v][3] and the
// scale l; unreachable vertices get X = 0 and scale -1.
__global__ __launch_bounds__(kBlock) void k_export_features(const float4* feat, const int* perm,
                                                            const int* vo, const MeshDesc* mesh, int B,
                                                            long long N, float* X, float* scale) {
    const long long gsz = (long long)gridDim.x * kBlock;
    for (long long p = blockIdx.x * (long long)kBlock + threadIdx.x; p < N; p += gsz) {
        const int b = mesh_of(vo, B, p);
        const float4 f = feat[p];
        const long long o = mesh[b].out_off + (perm[p] - mesh[b].v_off);
        X[3 * o + 0] = f.x;
        X[3 * o + 1] = f.y;
        X[3 * o + 2] = f.z;
        scale[o] = f.w;
    }
}

// Per-wave LDS for the 32-vertex tile: inputs, and bf16 transposes.
struct TileLds {
    float x[32][3];
    unsigned short h1[32][kH];
    unsigned short dz[32][kH];
};

// Upper bound from the network, written in the caller's order:
// w = inflate * 64 l softplus(o); sources 0; unreachable +inf.
__global__ __launch_bounds__(kBlock) void k_predict(const float* params, const float4* feat, const int* perm,
                                                    const int* vo, const MeshDesc* mesh, int B, long long N,
                                                    float inflate, float* upper) {
    __shared__ float P[kParams];
    __shared__ TileLds T[kBlock / kWave];
    for (int i = threadIdx.x; i < kParams; i += kBlock) P[i] = params[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    bf16x8 w2b[2][4];
    load_w2(P, lane, w2b);
    const long long ntiles = (N + 31) / 32;
    const long long iters = (ntiles + (long long)gridDim.x * 4 - 1) / ((long long)gridDim.x * 4);
    for (long long it = 0; it < iters; ++it) {
        const long long tile = it * gridDim.x * 4 + blockIdx.x * 4 + wv;
        const long long base = tile * 32;
        if (lane < 32) {
            const long long p = base + lane;
            float4 f = p < N ? feat[p] : make_float4(0.f, 0.f, 0.f, -1.f);
            T[wv].x[lane][0] = f.x;
            T[wv].x[lane][1] = f.y;
            T[wv].x[lane][2] = f.z;
        }
        __syncthreads();
        TileFwd t;
        bf16x8 a[2][2];
        tile_forward(P, w2b, T[wv].x, lane, t, a);
        if ((lane & 15) == 0)
            for (int mt = 0; mt < 2; ++mt)
                for (int i = 0; i < 4; ++i) {
                    const long long p = base + 16 * mt + 4 * (lane >> 4) + i;
                    if (p >= N) continue;
                    const float4 f = feat[p];
                    const int v = perm[p];
                    const int b = mesh_of(vo, B, v);
                    const int local_pos = (int)(p - mesh[b].v_off);
                    float w;
                    if (f.w < 0.f) w = kInf;                          // unreachable
                    else if (local_pos < mesh[b].m) w = 0.f;          // a source
                    else w = inflate * kOutScale * f.w * softplus(t.o[mt][i]);
                    upper[mesh[b].out_off + (v - mesh[b].v_off)] = w;
                }
        __syncthreads();
    }
}

// Network output d^ = 64 s softplus(o) for given inputs x[n][3] and scales s[n].
__global__ __launch_bounds__(kBlock) void k_mlp_apply(const float* params, const float* X, const float* S,
                                                      long long n, float* out) {
    __shared__ float P[kParams];
    __shared__ TileLds T[kBlock / kWave];
    for (int i = threadIdx.x; i < kParams; i += kBlock) P[i] = params[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    bf16x8 w2b[2][4];
    load_w2(P, lane, w2b);
    const long long ntiles = (n + 31) / 32;
    const long long iters = (ntiles + (long long)gridDim.x * 4 - 1) / ((long long)gridDim.x * 4);
    for (long long it = 0; it < iters; ++it) {
        const long long base = (it * gridDim.x * 4 + blockIdx.x * 4 + wv) * 32;
        if (lane < 32)
            for (int c = 0; c < 3; ++c)
                T[wv].x[lane][c] = base + lane < n ? X[3 * (base + lane) + c] : 0.f;
        __syncthreads();
        TileFwd t;
        bf16x8 a[2][2];
        tile_forward(P, w2b, T[wv].x, lane, t, a);
        if ((lane & 15) == 0)
            for (int mt = 0; mt < 2; ++mt)
                for (int i = 0; i < 4; ++i) {
                    const long long r = base + 16 * mt + 4 * (lane >> 4) + i;
                    if (r < n) out[r] = kOutScale * S[r] * softplus(t.o[mt][i]);
                }
        __syncthreads();
    }
}

// Fused forward + backward of the loss
//   L = (1/n) sum_v ((d^_v - d_v) / max(d_v, s_v))^2,   d^ = 64 s softplus(o),
// for inputs X[n][3], scales S[n], targets D[n].  Each wave writes its
// partial gradient (kParams values) and loss to part[wave][kParams + 1];
// k_reduce_grad sums the waves in a fixed order.
__global__ __launch_bounds__(kBlock) void k_mlp_grad(const float* params, const float* X, const float* S,
                                                     const float* D, long long n, float* part) {
    __shared__ float P[kParams];
    __shared__ TileLds T[kBlock / kWave];
    for (int i = threadIdx.x; i < kParams; i += kBlock) P[i] = params[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = lane & 15, rb = lane >> 4;
    bf16x8 w2b[2][4], w2t[2][4];
    load_w2(P, lane, w2b);
    load_w2t(P, lane, w2t);
    float w3r[4];
    for (int nt = 0; nt < 4; ++nt) w3r[nt] = bf16_round(P[kOffW3 + 16 * nt + col]);
    const float inv_n = 1.f / (float)n;

    f32x4 gW2[4][4];
    for (int at = 0; at < 4; ++at)
        for (int bt = 0; bt < 4; ++bt) gW2[at][bt] = f32x4{0.f, 0.f, 0.f, 0.f};
    float gW3[4] = {0, 0, 0, 0}, gB2[4] = {0, 0, 0, 0}, gB1[4] = {0, 0, 0, 0};
    float gW1[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    float gB3 = 0.f, loss = 0.f;

    const long long ntiles = (n + 31) / 32;
    const long long iters = (ntiles + (long long)gridDim.x * 4 - 1) / ((long long)gridDim.x * 4);
    for (long long it = 0; it < iters; ++it) {
        const long long base = (it * gridDim.x * 4 + blockIdx.x * 4 + wv) * 32;
        if (lane < 32)
            for (int c = 0; c < 3; ++c)
                T[wv].x[lane][c] = base + lane < n ? X[3 * (base + lane) + c] : 0.f;
        __syncthreads();
        TileFwd t;
        bf16x8 a[2][2];
        tile_forward(P, w2b, T[wv].x, lane, t, a);
        // d L / d o per row (identical in the 16 lanes of a row group)
        float go[2][4];
        for (int mt = 0; mt < 2; ++mt)
            for (int i = 0; i < 4; ++i) {
                const long long r = base + 16 * mt + 4 * rb + i;
                go[mt][i] = 0.f;
                if (r < n) {
                    const float o = t.o[mt][i];
                    const float s = S[r], d = D[r];
                    const float den = fmaxf(d, s);
                    const float e = (kOutScale * s * softplus(o) - d) / den;
                    if (col == 0) loss += e * e;
                    go[mt][i] = 2.f * e / den * kOutScale * s * sigmoid(o) * inv_n;
                    if (col == 0) gB3 += go[mt][i];
                }
            }
        // layer 3 and dz2
        f32x4 dz2[2][4];
        for (int mt = 0; mt < 2; ++mt)
            for (int nt = 0; nt < 4; ++nt)
                for (int i = 0; i < 4; ++i) {
                    const float z = t.z2[mt][nt][i];
                    gW3[nt] += go[mt][i] * gelu(z);
                    const float dz = go[mt][i] * w3r[nt] * gelu_grad(z);
                    dz2[mt][nt][i] = dz;
                    gB2[nt] += dz;
                }
        // transposes through LDS: h1 (from the A operand) and dz2 (D layout)
        for (int mt = 0; mt < 2; ++mt)
            for (int ks = 0; ks < 2; ++ks)
                for (int j = 0; j < 8; ++j)
                    T[wv].h1[16 * mt + col][a_hidden(lane, ks, j)] = (unsigned short)a[mt][ks][j];
        for (int mt = 0; mt < 2; ++mt)
            for (int nt = 0; nt < 4; ++nt)
                for (int i = 0; i < 4; ++i)
                    T[wv].dz[16 * mt + 4 * rb + i][16 * nt + col] = bf16_bits(dz2[mt][nt][i]);
        __syncthreads();
        // dW2 += h1^T dz2  (K = the 32 vertices of the tile)
        for (int at = 0; at < 4; ++at) {
            bf16x8 A;
            for (int j = 0; j < 8; ++j) A[j] = (short)T[wv].h1[8 * rb + j][16 * at + col];
            for (int bt = 0; bt < 4; ++bt) {
                bf16x8 Bo;
                for (int j = 0; j < 8; ++j) Bo[j] = (short)T[wv].dz[8 * rb + j][16 * bt + col];
                gW2[at][bt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bo, gW2[at][bt], 0, 0, 0);
            }
        }
        // dh1 = dz2 W2^T, then dz1 = dh1 gelu'(z1)
        for (int mt = 0; mt < 2; ++mt) {
            bf16x8 A[2];
            for (int ks = 0; ks < 2; ++ks)
                for (int j = 0; j < 8; ++j)
                    A[ks][j] = (short)T[wv].dz[16 * mt + col][a_hidden(lane, ks, j)];
            for (int nt = 0; nt < 4; ++nt) {
                f32x4 dh = {0.f, 0.f, 0.f, 0.f};
                dh = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], w2t[0][nt], dh, 0, 0, 0);
                dh = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], w2t[1][nt], dh, 0, 0, 0);
                const int h = 16 * nt + col;
                for (int i = 0; i < 4; ++i) {
                    const float* x = T[wv].x[16 * mt + 4 * rb + i];
                    const float dz1 = dh[i] * gelu_grad(z1_of(P, x, h));
                    gB1[nt] += dz1;
                    gW1[0][nt] += x[0] * dz1;
                    gW1[1][nt] += x[1] * dz1;
                    gW1[2][nt] += x[2] * dz1;
                }
            }
        }
        __syncthreads();
    }
    // reduce over the four row groups of the wave (lanes col, col+16, +32, +48)
    for (int nt = 0; nt < 4; ++nt) {
        for (int m = 16; m < 64; m <<= 1) {
            gW3[nt] += __shfl_xor(gW3[nt], m, 64);
            gB2[nt] += __shfl_xor(gB2[nt], m, 64);
            gB1[nt] += __shfl_xor(gB1[nt], m, 64);
            for (int c = 0; c < 3; ++c) gW1[c][nt] += __shfl_xor(gW1[c][nt], m, 64);
        }
    }
    for (int m = 1; m < 64; m <<= 1) {
        gB3 += __shfl_xor(gB3, m, 64);
        loss += __shfl_xor(loss, m, 64);
    }
    float* out = part + (size_t)(blockIdx.x * 4 + wv) * (kParams + 1);
    for (int at = 0; at < 4; ++at)
        for (int bt = 0; bt < 4; ++bt)
            for (int i = 0; i < 4; ++i)
                out[kOffW2 + (16 * at + 4 * rb + i) * kH + 16 * bt + col] = gW2[at][bt][i];
    if (rb == 0)
        for (int nt = 0; nt < 4; ++nt) {
            const int h = 16 * nt + col;
            out[kOffW3 + h] = gW3[nt];
            out[kOffB2 + h] = gB2[nt];
            out[kOffB1 + h] = gB1[nt];
            for (int c = 0; c < 3; ++c) out[kOffW1 + c * kH + h] = gW1[c][nt];
        }
    if (lane == 0) {
        out[kOffB3] = gB3;
        out[kParams] = loss * inv_n;
    }
}

__global__ __launch_bounds__(kBlock) void k_reduce_grad(const float* part, int nparts, float* grad,
                                                        float* loss) {
    for (int c = blockIdx.x * kBlock + threadIdx.x; c <= kParams; c += gridDim.x * kBlock) {
        float s = 0.f;
        for (int w = 0; w < nparts; ++w) s += part[(size_t)w * (kParams + 1) + c];
        if (c < kParams) grad[c] = s;
        else if (loss) *loss = s;
    }
}

// Adam with bias correction on the float32 master parameters.
__global__ __launch_bounds__(kBlock) void k_adam(float* params, const float* grad, float* m, float* v,
                                                 float lr, float b1, float b2, float eps, float c1,
                                                 float c2) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < kParams; i += gridDim.x * kBlock) {
        const float g = grad[i];
        const float mi = b1 * m[i] + (1.f - b1) * g;
        const float vi = b2 * v[i] + (1.f - b2) * g * g;
        m[i] = mi;
        v[i] = vi;
        params[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

}  // namespace

constexpr int kMlpGrid = 256;     // workgroups of the training kernel (1024 waves)

size_t mlp_scratch_bytes() { return sizeof(float) * (size_t)kMlpGrid * 4 * (kParams + 1); }

hipError_t launch_features(const Work& w, const Sizes& z, hipStream_t st) {
    const int grid = (int)std::min<long long>(8192, (z.N + kBlock - 1) / kBlock + 1);
    unsigned long long* acc = w.edge_acc;           // [B] sums, then [B] maxima
    unsigned long long* emax = w.edge_acc + z.B;
    hipLaunchKernelGGL(k_zero_u64, dim3((2 * z.B + 255) / 256), dim3(256), 0, st, acc, 2 * z.B);
    hipLaunchKernelGGL(k_edge_max, dim3(grid), dim3(kBlock), 0, st, w.xyz, w.rowO, w.wedgeO, w.perm, w.iperm,
                       w.vo, z.B, z.N, emax);
    hipLaunchKernelGGL(k_edge_sum, dim3(grid), dim3(kBlock), 0, st, w.xyz, w.rowO, w.wedgeO, w.perm, w.iperm,
                       w.vo, z.B, z.N, emax, acc);
    hipLaunchKernelGGL(k_edge_mean, dim3((z.B + 255) / 256), dim3(256), 0, st, acc, emax, w.rowO, w.mesh,
                       z.B, w.state);
    hipLaunchKernelGGL(k_features, dim3(grid), dim3(kBlock), 0, st, w.xyz, w.rowO, w.wedgeO, w.perm, w.iperm,
                       w.level, w.vo, w.mesh, w.state, z.B, z.N, w.feat);
    return hipGetLastError();
}

hipError_t launch_export_features(const Work& w, const Sizes& z, float* X, float* scale, hipStream_t st) {
    const int grid = (int)std::min<long long>(8192, (z.N + kBlock - 1) / kBlock + 1);
    hipLaunchKernelGGL(k_export_features, dim3(grid), dim3(kBlock), 0, st, w.feat, w.perm, w.vo, w.mesh, z.B,
                       z.N, X, scale);
    return hipGetLastError();
}

hipError_t launch_predict(const Work& w, const Sizes& z, const float* params, float inflate, float* upper,
                          hipStream_t st) {
    const long long ntiles = (z.N + 31) / 32;
    const int grid = (int)std::max<long long>(1, std::min<long long>(1024, (ntiles + 3) / 4));
    hipLaunchKernelGGL(k_predict, dim3(grid), dim3(kBlock), 0, st, params, w.feat, w.perm, w.vo, w.mesh, z.B,
                       z.N, inflate, upper);
    return hipGetLastError();
}

hipError_t launch_mlp_apply(const float* params, const float* X, const float* S, long long n, float* out,
                            hipStream_t st) {
    const long long ntiles = (n + 31) / 32;
    const int grid = (int)std::max<long long>(1, std::min<long long>(1024, (ntiles + 3) / 4));
    hipLaunchKernelGGL(k_mlp_apply, dim3(grid), dim3(kBlock), 0, st, params, X, S, n, out);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* params, const float* X, const float* S, const float* D, long long n,
                           float* scratch, float* grad, float* loss, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_grad, dim3(kMlpGrid), dim3(kBlock), 0, st, params, X, S, D, n, scratch);
    hipLaunchKernelGGL(k_reduce_grad, dim3((kParams + kBlock) / kBlock), dim3(kBlock), 0, st, scratch,
                       kMlpGrid * 4, grad, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float* params, const float* grad, float* m, float* v, int t, float lr, float b1,
                       float b2, float eps, hipStream_t st) {
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((kParams + kBlock - 1) / kBlock), dim3(kBlock), 0, st, params, grad, m, v,
                       lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace ptp

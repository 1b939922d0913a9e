// The warm-start network, on one wave: 3 -> 64 -> 64 -> 1 with exact-erf
// GELU, weights rounded to bfloat16, float32 accumulation.
//
//   x   = (f1 / l, hop, f3 * l) / (64, 64, 1)      l = mean edge length
//   h1  = gelu(x W1 + b1)            float32 VALU (K = 3 is too thin for MFMA;
//                                    the inputs stay float32)
//   h2  = gelu(h1 W2 + b2)           bf16 MFMA 16x16x32, float32 accumulate
//   o   = h2 . W3 + b3               float32 VALU + cross-lane sum
//   d^  = 64 l softplus(o)
//
// Parameters: one float32 vector, [W1 (3x64, input-major) | b1 (64) |
// W2 (64x64, input-major) | b2 (64) | W3 (64) | b3 (1)] = 4481 values; the
// weight matrices are rounded to bfloat16 (nearest even) when loaded.
//
// A wave handles tiles of 32 vertices (two 16-row MFMA tiles).  MFMA lane
// layout of v_mfma_f32_16x16x32_bf16 (checked on the device): lane l holds
// A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16], j = 0..7, and
// D[4 (l / 16) + i][l % 16], i = 0..3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptp {

constexpr int kH = 64;
constexpr int kParams = 3 * kH + kH + kH * kH + kH + kH + 1;   // 4481
constexpr int kOffW1 = 0, kOffB1 = 192, kOffW2 = 256, kOffB2 = 4352, kOffW3 = 4416, kOffB3 = 4480;
constexpr float kInScale = 1.f / 64.f;   // input scale of f1 / l and hop
constexpr float kOutScale = 64.f;        // output scale of softplus(o)

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline unsigned short bf16_bits(float x) {     // round to nearest even
    unsigned u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf16_round(float x) { return __uint_as_float((unsigned)bf16_bits(x) << 16); }

__device__ inline float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
    return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}
__device__ inline float softplus(float o) { return o > 20.f ? o : log1pf(expf(o)); }
__device__ inline float sigmoid(float o) { return 1.f / (1.f + expf(-o)); }

// Layer-1 pre-activation of hidden unit h for input x (one fixed order of
// operations, shared by the forward and the backward).
__device__ inline float z1_of(const float* P, const float* x, int h) {
    float z = P[kOffB1 + h];
    z += x[0] * bf16_round(P[kOffW1 + 0 * kH + h]);
    z += x[1] * bf16_round(P[kOffW1 + 1 * kH + h]);
    z += x[2] * bf16_round(P[kOffW1 + 2 * kH + h]);
    return z;
}

// Hidden unit index used by lane l in the layer-2 A operand, K-step ks,
// element j:  32 ks + 8 (l / 16) + j.
__device__ inline int a_hidden(int lane, int ks, int j) { return 32 * ks + 8 * (lane >> 4) + j; }

// Load the bf16 B operands of layer 2 (constant over tiles): W2[k][n] with
// k = 32 ks + 8 (l / 16) + j, n = 16 nt + l % 16.
__device__ inline void load_w2(const float* P, int lane, bf16x8 w2b[2][4]) {
    for (int ks = 0; ks < 2; ++ks)
        for (int nt = 0; nt < 4; ++nt) {
            bf16x8 b;
            for (int j = 0; j < 8; ++j) {
                const int k = 32 * ks + 8 * (lane >> 4) + j;
                const int n = 16 * nt + (lane & 15);
                b[j] = (short)bf16_bits(P[kOffW2 + k * kH + n]);
            }
            w2b[ks][nt] = b;
        }
}

// Forward for a 32-vertex tile.  x[v][3] for the tile's vertices is read by
// each lane for its rows.  Outputs, per lane, the layer-2 pre-activations
// z2[mt][nt][i] (rows 16 mt + 4 (l / 16) + i, column 16 nt + l % 16) and the
// per-row output o (valid in every lane for rows 16 mt + 4 (l / 16) + i).
struct TileFwd {
    f32x4 z2[2][4];
    float o[2][4];
};

__device__ inline void tile_forward(const float* P, const bf16x8 w2b[2][4], const float (*xt)[3],
                                    int lane, TileFwd& t, bf16x8 a_out[2][2]) {
    // layer 1 in the A layout of layer 2: lane holds h1 for row (l % 16) of
    // each 16-row tile and hidden units a_hidden(l, ks, 0..7)
    for (int mt = 0; mt < 2; ++mt) {
        const float* x = xt[16 * mt + (lane & 15)];
        for (int ks = 0; ks < 2; ++ks) {
            bf16x8 a;
            for (int j = 0; j < 8; ++j) {
                a[j] = (short)bf16_bits(gelu(z1_of(P, x, a_hidden(lane, ks, j))));
            }
            a_out[mt][ks] = a;
        }
    }
    for (int mt = 0; mt < 2; ++mt)
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_out[mt][0], w2b[0][nt], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_out[mt][1], w2b[1][nt], acc, 0, 0, 0);
            const float bb = P[kOffB2 + 16 * nt + (lane & 15)];
            for (int i = 0; i < 4; ++i) acc[i] += bb;
            t.z2[mt][nt] = acc;
        }
    // layer 3: per row, sum over the 64 columns (4 per lane, 16 lanes)
    for (int mt = 0; mt < 2; ++mt)
        for (int i = 0; i < 4; ++i) {
            float s = 0.f;
            for (int nt = 0; nt < 4; ++nt) {
                const int h = 16 * nt + (lane & 15);
                s += gelu(t.z2[mt][nt][i]) * bf16_round(P[kOffW3 + h]);
            }
            for (int m = 1; m < 16; m <<= 1) s += __shfl_xor(s, m, 64);
            t.o[mt][i] = s + P[kOffB3];
        }
}

// B operands of W2 transposed (for dh1 = dz2 W2^T): element (k = hidden out,
// n = hidden in) = W2[n][k].
__device__ inline void load_w2t(const float* P, int lane, bf16x8 w2t[2][4]) {
    for (int ks = 0; ks < 2; ++ks)
        for (int nt = 0; nt < 4; ++nt) {
            bf16x8 b;
            for (int j = 0; j < 8; ++j) {
                const int k = 32 * ks + 8 * (lane >> 4) + j;
                const int n = 16 * nt + (lane & 15);
                b[j] = (short)bf16_bits(P[kOffW2 + n * kH + k]);
            }
            w2t[ks][nt] = b;
        }
}

}  // namespace ptp

// pb_mlp.h -- the learned con2prim guess: MLP 5 -> 64 -> 64 -> 1 (ReLU) with
// bfloat16 weights and activations and FP32 accumulation, evaluated on the
// matrix cores by one whole wave for its 64 cells.
//
// Rounding points (round to nearest even): the standardised features, the
// weights, and the post-activation outputs of both hidden layers are bf16;
// products accumulate in FP32; biases are FP32; the output stays FP32.
// Inputs are standardised as (x - mean) * rn(1/std) in binary32.
//
// Matrix-core mapping.  Neurons are rows, the wave's cells are columns, in
// four column tiles nt of 16 cells.  For the 16x16 FP32-output MFMAs lane l
// holds D[4(l/16)+i][l%16] (i = 0..3), so the D tile of 16 hidden units is
// already in the B-operand layout of the next layer (hidden unit = K index).
//  * layer 1: v_mfma_f32_16x16x16_bf16, K = 5 padded to 16, the bias as the
//    accumulator input;
//  * layer 2: v_mfma_f32_16x16x32_bf16 over two K tiles of 32.  The B operand
//    of K tile kt is the lane's two packed D tiles 2kt and 2kt+1, so lane
//    group g, element i (0..7) carries hidden unit
//        u(kt, g, i) = 32 kt + 16 (i / 4) + 4 g + i % 4;
//    the A operands are stored with their K index permuted the same way
//    (a contraction does not depend on the order of its K index as long as
//    both operands use the same one);
//  * layer 3: the same instruction with w3 replicated over the 16 rows, the
//    bias b3 as accumulator input: every row of the result holds the output.
// ReLU runs on the packed bf16 pair (an int16 maximum with 0: bf16 values of
// either sign order like int16 where it matters, -0 maps to +0), after the
// round-to-nearest-even conversion, which commutes with it.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/patchhip.h"
#include "pb_c2p.h"

namespace pb {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef short s16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

constexpr int kMlpIn = 5, kMlpHid = 64;
// FP32 master parameter offsets (the order of the C ABI)
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kMlpHid * kMlpIn, kOffW2 = kOffB1 + kMlpHid,
              kOffB2 = kOffW2 + kMlpHid * kMlpHid, kOffW3 = kOffB2 + kMlpHid, kOffB3 = kOffW3 + kMlpHid,
              kMlpNParam = kOffB3 + 1;
// the normalisation block: x_mean[5], x_std[5], y_mean, y_std
constexpr int kMlpNNorm = 12;

// hidden unit carried by lane group g, element i of K tile kt (see above)
__host__ __device__ constexpr int mlp_kperm(int kt, int g, int i) { return 32 * kt + 16 * (i / 4) + 4 * g + i % 4; }

// Everything inference needs, in operand order; a work-group copies it to
// LDS and every lane picks its operands from there.
struct MlpPack {
    bf16x4_t w1[4][64];      // [m tile][lane]: W1[16 mt + l%16][4 (l/16) + i], zero for k >= 5
    bf16x8_t w2[4][2][64];   // [m tile][K tile][lane]: W2[16 mt + l%16][u(kt, l/16, i)]
    bf16x8_t w3[2][64];      // [K tile][lane]: w3[u(kt, l/16, i)]
    float b1[64], b2[64];
    float xm[5], xi[5];      // feature mean and rn(1/std)
    float ym, ys, b3, pad;
};
static_assert(sizeof(MlpPack) % 16 == 0, "MlpPack is copied in 16-byte words");

struct MlpDev {
    const MlpPack *pack;  // inference blob
    const float *par;     // FP32 master parameters
    const float *norm;    // normalisation block
};

// round to nearest even to bfloat16 (gfx950 converts in hardware,
// v_cvt_pk_bf16_f32, under the default round-to-nearest-even mode)
__device__ __forceinline__ unsigned short bf16_rne(float f)
{
    return __builtin_bit_cast(unsigned short, (__bf16)f);
}

__device__ __forceinline__ float bf16_val(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// two floats -> packed bf16 pair (low half = a)
__device__ __forceinline__ unsigned pack_bf16(float a, float b)
{
    return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2_t){a, b}, bf16x2_t));
}

// the same followed by ReLU on both halves
__device__ __forceinline__ unsigned pack_relu(float a, float b)
{
    s16x2_t v = __builtin_bit_cast(s16x2_t, pack_bf16(a, b));
    v = __builtin_elementwise_max(v, (s16x2_t){0, 0});
    return __builtin_bit_cast(unsigned, v);
}

// Scale-free features of a conserved state (p/E depends only on D/E and
// |S|/E).  The last one measures the internal energy directly:
// E^2 - D^2 - |S|^2 = tau (tau + 2D) - |S|^2, positive for admissible
// states, is where the pressure of a cold, fast cell hides.  The two
// differences that cancel (E - s and that one) are formed in FP64, the
// ratios and logarithms in FP32 (the network reads bf16 inputs).
__device__ __forceinline__ void mlp_features(const C2pIn &in, float *x)
{
    const float iE = __builtin_amdgcn_rcpf((float)in.E);
    const float t = (float)(in.tau * (in.tau + 2.0 * in.D) - in.s2);
    x[0] = __logf((float)in.D * iE);
    x[1] = (float)in.s * iE;
    x[2] = __logf((float)(in.E - in.s) * iE);
    x[3] = __logf((float)in.tau * iE);
    x[4] = __logf(t * iE * iE);
}

// Whole-wave call (every lane of the wave must call it; lanes without a cell
// pass admissible dummy features).  P: the inference blob (in LDS for the
// solver passes); x: this lane's raw features.  Returns the network output
// (standardised log(p/E)).  The cells go through in two halves of two column
// tiles; within a half the layers run one after the other, so each weight
// tile is live only for its layer.
__device__ __forceinline__ float mlp_yhat(const MlpPack &P, const float *xm, const float *xi, const float *x)
{
    const int l = threadIdx.x & 63, g = l >> 4, j = l & 15;
    float z[kMlpIn];
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) z[k] = (x[k] - xm[k]) * xi[k];
    const unsigned p01 = pack_bf16(z[0], z[1]), p23 = pack_bf16(z[2], z[3]), p4 = pack_bf16(z[4], 0.f);
    float y = 0.f;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        // layer 1: h1[t] holds hidden units 16 mt + 4g + i of cell 16 nt + j, nt = 2 half + t
        unsigned h1[2][8];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x4_t w1 = P.w1[mt][l];
            const f32x4_t b1 = *reinterpret_cast<const f32x4_t *>(&P.b1[16 * mt + 4 * g]);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                // B operand: features 4g..4g+3 of cell 16 nt + j
                const int src = 16 * (2 * half + t) + j;
                const unsigned a01 = __shfl(p01, src, 64), a23 = __shfl(p23, src, 64), a4 = __shfl(p4, src, 64);
                const unsigned lo = g == 0 ? a01 : (g == 1 ? a4 : 0u), hi = g == 0 ? a23 : 0u;
                const bf16x4_t bx = __builtin_bit_cast(bf16x4_t, (u32x2_t){lo, hi});
                const f32x4_t d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1, bx, b1, 0, 0, 0);
                h1[t][2 * mt] = pack_relu(d[0], d[1]);
                h1[t][2 * mt + 1] = pack_relu(d[2], d[3]);
            }
        }
        __builtin_amdgcn_sched_barrier(0);   // bound the live range of each layer's tiles
        // layer 2 (K tiles of 32 in the permuted order: the lane's packed tiles)
        unsigned h2[2][8];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x8_t wa = P.w2[mt][0][l], wb = P.w2[mt][1][l];
            const f32x4_t b2 = *reinterpret_cast<const f32x4_t *>(&P.b2[16 * mt + 4 * g]);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const bf16x8_t k0 = __builtin_bit_cast(bf16x8_t, (u32x4_t){h1[t][0], h1[t][1], h1[t][2], h1[t][3]});
                const bf16x8_t k1 = __builtin_bit_cast(bf16x8_t, (u32x4_t){h1[t][4], h1[t][5], h1[t][6], h1[t][7]});
                f32x4_t d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, k0, b2, 0, 0, 0);
                d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb, k1, d, 0, 0, 0);
                h2[t][2 * mt] = pack_relu(d[0], d[1]);
                h2[t][2 * mt + 1] = pack_relu(d[2], d[3]);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        // layer 3: every row of the result is the output of cell 16 nt + j;
        // lane l's own cell sits in tile l / 16
        const bf16x8_t w3a = P.w3[0][l], w3b = P.w3[1][l];
        const float b3 = P.b3;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const bf16x8_t q0 = __builtin_bit_cast(bf16x8_t, (u32x4_t){h2[t][0], h2[t][1], h2[t][2], h2[t][3]});
            const bf16x8_t q1 = __builtin_bit_cast(bf16x8_t, (u32x4_t){h2[t][4], h2[t][5], h2[t][6], h2[t][7]});
            f32x4_t d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3a, q0, (f32x4_t){b3, b3, b3, b3}, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3b, q1, d, 0, 0, 0);
            if (g == 2 * half + t) y = d[0];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    return y;
}

// Whole-wave call.  The learned pressure guess E exp(y_mean + y_std yhat)
// (the solver replaces a guess outside its bracket by the plain guess).
__device__ __forceinline__ double mlp_guess(const MlpPack &P, const float *xm, const float *xi, float ym, float ys,
                                            const C2pIn &in)
{
    float x[kMlpIn];
    if (in.ok) {
        mlp_features(in, x);
    } else {
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) x[k] = xm[k];
    }
    const float yhat = mlp_yhat(P, xm, xi, x);
    return in.E * (double)__expf(fmaf(ys, yhat, ym));
}

}  // namespace pb

struct pb_mlp;
namespace pb {
// device view of an MLP (pointers into its device buffer)
pb_status mlp_device_view(const pb_mlp *m, MlpDev *out);
}  // namespace pb

// pb_mlp.h -- the learned con2prim guess: MLP 5 -> 64 -> 64 -> 1 (ReLU) with
// bfloat16 weights and activations and FP32 accumulation, evaluated on the
// matrix cores by one whole wave for its 64 cells.
//
// Rounding points (round to nearest even): the standardised features, the
// weights, and the post-activation outputs of both hidden layers are bf16;
// products accumulate in FP32; biases are FP32; the output stays FP32.
//
// MFMA mapping (v_mfma_f32_16x16x16_bf16): a 16x16 tile of D = A.B with
// lane l holding A[l%16][4(l/16)+i], B[4(l/16)+i][l%16] and D[4(l/16)+i][l%16]
// (i = 0..3).  With neurons as rows and cells as columns, the D layout of
// layer 1 (rows = hidden units) is exactly the B layout layer 2 needs for
// the K-tile of the same 16 hidden units, so the layers chain in registers.
// Layer 3 is a dot product of each cell's 64 hidden values with w3: every
// lane sums its 16 rows, two butterfly shuffles finish the sum.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/patchhip.h"
#include "pb_c2p.h"

namespace pb {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kMlpIn = 5, kMlpHid = 64;
// FP32 master parameter offsets (the order of the C ABI)
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kMlpHid * kMlpIn, kOffW2 = kOffB1 + kMlpHid,
              kOffB2 = kOffW2 + kMlpHid * kMlpHid, kOffW3 = kOffB2 + kMlpHid, kOffB3 = kOffW3 + kMlpHid,
              kMlpNParam = kOffB3 + 1;
// device scalars: b3 is the master value above; the normalisation block
// holds x_mean[5], x_std[5], y_mean, y_std
constexpr int kMlpNNorm = 12;

struct MlpDev {
    const bf16x4_t *w1;   // [4 m-tiles][64 lanes]: A operands of layer 1 (K = 5 padded to 16)
    const bf16x4_t *w2;   // [4 m-tiles][4 k-tiles][64 lanes]: A operands of layer 2
    const float *par;     // FP32 master parameters (biases and w3 read from here)
    const float *norm;    // normalisation block
};

// round to nearest even to bfloat16 (gfx950 converts in hardware,
// v_cvt_pk_bf16_f32, under the default round-to-nearest-even mode)
__device__ __forceinline__ unsigned short bf16_rne(float f)
{
    return __builtin_bit_cast(unsigned short, (__bf16)f);
}

__device__ __forceinline__ float bf16_val(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// Scale-free features of a conserved state (p/E depends only on D/E and
// |S|/E).  The last one measures the internal energy directly:
// E^2 - D^2 - |S|^2 = tau (tau + 2D) - |S|^2, positive for admissible
// states, is where the pressure of a cold, fast cell hides.
// The ratios (and the cancelling difference) are formed in FP64, the
// logarithms in FP32: the network reads bf16 inputs.
__device__ __forceinline__ void mlp_features(const C2pIn &in, float *x)
{
    const double iE = 1.0 / in.E;
    const double sE = sqrt(in.s2) * iE;
    x[0] = __logf((float)(in.D * iE));
    x[1] = (float)sE;
    x[2] = __logf((float)(1.0 - sE));
    x[3] = __logf((float)(in.tau * iE));
    x[4] = __logf((float)((in.tau * (in.tau + 2.0 * in.D) - in.s2) * iE * iE));
}

// standardised, bf16-rounded features
__device__ __forceinline__ void mlp_inputs(const float *norm, const float *x, unsigned short *xb)
{
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) xb[k] = bf16_rne((x[k] - norm[k]) / norm[5 + k]);
}

// The parameters one lane needs, held in registers so that a wave can push
// several groups of 64 cells through the network with one load: the layer-1
// and layer-2 A operands of its lane, and the biases and w3 of the 16 hidden
// rows its lane group owns.
struct MlpRegs {
    bf16x4_t w1[4];
    bf16x4_t w2[16];
    float b1[4][4], b2[4][4], w3[4][4];
    float b3;
};

__device__ __forceinline__ void mlp_load(const MlpDev &m, MlpRegs &r)
{
    const int l = threadIdx.x & 63, g = l >> 4;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) r.w1[mt] = m.w1[mt * 64 + l];
#pragma unroll
    for (int t = 0; t < 16; ++t) r.w2[t] = m.w2[t * 64 + l];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = mt * 16 + g * 4 + i;
            r.b1[mt][i] = m.par[kOffB1 + row];
            r.b2[mt][i] = m.par[kOffB2 + row];
            r.w3[mt][i] = bf16_val(bf16_rne(m.par[kOffW3 + row]));
        }
    r.b3 = m.par[kOffB3];
}

// Whole-wave call (every lane of the wave must call it; lanes without a cell
// pass admissible dummy features).  x: this lane's raw features.  Returns the
// network output yhat (standardised log(p/E)).
__device__ __forceinline__ float mlp_yhat(const MlpRegs &r, const float *norm, const float *x)
{
    const int l = threadIdx.x & 63, g = l >> 4, j = l & 15;
    unsigned short xb[kMlpIn];
    mlp_inputs(norm, x, xb);
    const int pk01 = (int)xb[0] | ((int)xb[1] << 16);
    const int pk23 = (int)xb[2] | ((int)xb[3] << 16);
    const int pk4 = (int)xb[4];

    float part[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        // B operand of layer 1: features of cell nt*16 + j, k = 4g..4g+3
        const int src = nt * 16 + j;
        const int a01 = __shfl(pk01, src, 64), a23 = __shfl(pk23, src, 64), a4 = __shfl(pk4, src, 64);
        bf16x4_t bx;
        if (g == 0) {
            bx[0] = (short)(a01 & 0xffff); bx[1] = (short)(a01 >> 16);
            bx[2] = (short)(a23 & 0xffff); bx[3] = (short)(a23 >> 16);
        } else if (g == 1) {
            bx[0] = (short)(a4 & 0xffff); bx[1] = 0; bx[2] = 0; bx[3] = 0;
        } else {
            bx[0] = 0; bx[1] = 0; bx[2] = 0; bx[3] = 0;
        }
        bf16x4_t hb[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const f32x4_t z = {0.f, 0.f, 0.f, 0.f};
            const f32x4_t h = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(r.w1[mt], bx, z, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) hb[mt][i] = (short)bf16_rne(fmaxf(h[i] + r.b1[mt][i], 0.f));
        }
        float acc = 0.f;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x4_t d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kt = 0; kt < 4; ++kt)
                d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(r.w2[mt * 4 + kt], hb[kt], d, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float h2 = bf16_val(bf16_rne(fmaxf(d[i] + r.b2[mt][i], 0.f)));
                acc = fmaf(r.w3[mt][i], h2, acc);
            }
        }
        acc += __shfl_xor(acc, 16, 64);
        acc += __shfl_xor(acc, 32, 64);
        part[nt] = acc;
    }
    return r.b3 + (g == 0 ? part[0] : g == 1 ? part[1] : g == 2 ? part[2] : part[3]);
}

__device__ __forceinline__ float mlp_yhat(const MlpDev &m, const float *x)
{
    MlpRegs r;
    mlp_load(m, r);
    return mlp_yhat(r, m.norm, x);
}

// Whole-wave call.  The learned pressure guess E exp(y_mean + y_std yhat)
// (the solver replaces a guess outside its bracket by the plain guess).
__device__ __forceinline__ double mlp_guess(const MlpRegs &r, const float *norm, const C2pIn &in)
{
    float x[kMlpIn];
    if (in.ok) {
        mlp_features(in, x);
    } else {
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) x[k] = norm[k];
    }
    const float yhat = mlp_yhat(r, norm, x);
    return in.E * (double)__expf(norm[10] + norm[11] * yhat);
}

}  // namespace pb

struct pb_mlp;
namespace pb {
// device view of an MLP (pointers into its device buffer)
pb_status mlp_device_view(const pb_mlp *m, MlpDev *out);
}  // namespace pb

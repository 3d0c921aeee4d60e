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

__device__ __forceinline__ unsigned short bf16_rne(float f)
{
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)0x7fc0;  // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float bf16_val(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// Scale-free features of a conserved state (p/E depends only on D/E and
// |S|/E).  The last one measures the internal energy directly:
// E^2 - D^2 - |S|^2 = tau (tau + 2D) - |S|^2, positive for admissible
// states, is where the pressure of a cold, fast cell hides.
__device__ __forceinline__ void mlp_features(const C2pIn &in, float *x)
{
    const double iE = 1.0 / in.E;
    const double sE = sqrt(in.s2) * iE;
    x[0] = (float)log(in.D * iE);
    x[1] = (float)sE;
    x[2] = (float)log(1.0 - sE);
    x[3] = (float)log(in.tau * iE);
    x[4] = (float)log((in.tau * (in.tau + 2.0 * in.D) - in.s2) * iE * iE);
}

// standardised, bf16-rounded features
__device__ __forceinline__ void mlp_inputs(const float *norm, const float *x, unsigned short *xb)
{
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) xb[k] = bf16_rne((x[k] - norm[k]) / norm[5 + k]);
}

// Whole-wave call (every lane of the wave must call it; lanes without a cell
// pass admissible dummy features).  x: this lane's raw features.  Returns the
// network output yhat (standardised log(p/E)).
__device__ __forceinline__ float mlp_yhat(const MlpDev &m, const float *x)
{
    const int l = threadIdx.x & 63, g = l >> 4, j = l & 15;
    unsigned short xb[kMlpIn];
    mlp_inputs(m.norm, x, xb);
    const int pk01 = (int)xb[0] | ((int)xb[1] << 16);
    const int pk23 = (int)xb[2] | ((int)xb[3] << 16);
    const int pk4 = (int)xb[4];

    bf16x4_t w1[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) w1[mt] = m.w1[mt * 64 + l];
    float b1r[4][4], b2r[4][4], w3r[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = mt * 16 + g * 4 + i;
            b1r[mt][i] = m.par[kOffB1 + row];
            b2r[mt][i] = m.par[kOffB2 + row];
            w3r[mt][i] = bf16_val(bf16_rne(m.par[kOffW3 + row]));
        }

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
            const f32x4_t h = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1[mt], bx, z, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) hb[mt][i] = (short)bf16_rne(fmaxf(h[i] + b1r[mt][i], 0.f));
        }
        float acc = 0.f;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x4_t d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kt = 0; kt < 4; ++kt)
                d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(m.w2[(mt * 4 + kt) * 64 + l], hb[kt], d, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float h2 = bf16_val(bf16_rne(fmaxf(d[i] + b2r[mt][i], 0.f)));
                acc = fmaf(w3r[mt][i], h2, acc);
            }
        }
        acc += __shfl_xor(acc, 16, 64);
        acc += __shfl_xor(acc, 32, 64);
        part[nt] = acc;
    }
    return m.par[kOffB3] + (g == 0 ? part[0] : g == 1 ? part[1] : g == 2 ? part[2] : part[3]);
}

// Whole-wave call.  The learned pressure guess E exp(y_mean + y_std yhat)
// (the solver replaces a guess outside its bracket by the plain guess).
__device__ __forceinline__ double mlp_guess(const MlpDev &m, const double *qv, const C2pIn &in)
{
    (void)qv;
    float x[kMlpIn];
    if (in.ok) {
        mlp_features(in, x);
    } else {
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) x[k] = m.norm[k];
    }
    const float yhat = mlp_yhat(m, x);
    return in.E * exp((double)m.norm[10] + (double)m.norm[11] * (double)yhat);
}

}  // namespace pb

struct pb_mlp;
namespace pb {
// device view of an MLP (pointers into its device buffer)
pb_status mlp_device_view(const pb_mlp *m, MlpDev *out);
}  // namespace pb

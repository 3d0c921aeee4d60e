// pb_mlp.hip -- the learned con2prim guess network: parameter storage,
// bf16 operand refresh, the standalone forward pass, and training (forward +
// backward + weight gradients + Adam) with the library's own kernels.
//
// Training arithmetic mirrors the inference rounding points: the forward
// pass uses the bf16 weights, bf16 standardised inputs and bf16 hidden
// activations with FP32 accumulation; the backward pass runs in FP32 through
// the same bf16 values (the rounding is treated as the identity, the usual
// straight-through rule) with ReLU masks h > 0.  Loss: mean squared error of
// the standardised target.  Gradients are reduced deterministically
// (per-chunk partial sums, then a fixed-order sum), so a training run is
// bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "pb_common.h"
#include "pb_mlp.h"

namespace pb {
constexpr int kTrainWavesMax = 256;   // partial-gradient rows (waves of one training call)
constexpr int kPartStride = 4672;     // floats per partial row: kMlpNParam + the loss, padded to 64
static_assert(kPartStride >= kMlpNParam + 1 && kPartStride % 64 == 0, "partial row");
constexpr int kStatBlocks = 256;      // work-groups of the statistics passes
// training-only operands: W2 transposed, with its K index (the output units)
// in the permuted order of the forward pass's D tiles (see pb_mlp.h), so the
// backward product W2^T dh2 reads dh2 straight from those tiles
struct MlpTrainPack {
    bf16x8_t w2t[4][2][64];   // [m tile of input units][K tile][lane]: W2[u(kt, l/16, i)][16 mt + l%16]
};
}  // namespace pb

struct pb_mlp {
    char *dev = nullptr;        // one device allocation holding everything below
    float *par = nullptr;       // FP32 master parameters [kMlpNParam]
    float *madam = nullptr;     // Adam first moments
    float *vadam = nullptr;     // Adam second moments
    float *norm = nullptr;      // [kMlpNNorm]
    pb::MlpPack *pack = nullptr;         // inference operands (bf16, lane-swizzled), see pb_mlp.h
    pb::MlpTrainPack *tpack = nullptr;   // backward operands
    float *grad = nullptr;      // [kMlpNParam] gradient of the last train step
    float *loss = nullptr;      // [1]
    float *part = nullptr;      // partial gradients [kTrainWavesMax][kPartStride] (training scratch)
    double *stats = nullptr;    // normalisation statistics scratch
};

namespace pb {

namespace {

constexpr int kT = 256;

// the inference blob from the FP32 masters and the normalisation block
// (layout of pb_mlp.h)
__global__ __launch_bounds__(256) void mlp_refresh_kernel(const float *__restrict__ par, const float *__restrict__ norm,
                                                          MlpPack *__restrict__ P, MlpTrainPack *__restrict__ TP)
{
    const int t = threadIdx.x;
    for (int idx = t; idx < 4 * 2 * 64; idx += blockDim.x) {
        const int mt = idx / 128, kt = (idx / 64) % 2, l = idx % 64, g = l / 16, j = l % 16, col = 16 * mt + j;
        bf16x8_t v;
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = (__bf16)par[kOffW2 + mlp_kperm(kt, g, i) * kMlpHid + col];
        TP->w2t[mt][kt][l] = v;
    }
    for (int idx = t; idx < 4 * 64; idx += blockDim.x) {
        const int mt = idx / 64, l = idx % 64, g = l / 16, j = l % 16, row = 16 * mt + j;
        bf16x4_t v;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 4 * g + i;
            v[i] = (short)(k < kMlpIn ? bf16_rne(par[kOffW1 + row * kMlpIn + k]) : 0);
        }
        P->w1[mt][l] = v;
    }
    for (int idx = t; idx < 4 * 2 * 64; idx += blockDim.x) {
        const int mt = idx / 128, kt = (idx / 64) % 2, l = idx % 64, g = l / 16, j = l % 16, row = 16 * mt + j;
        bf16x8_t v;
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = (__bf16)par[kOffW2 + row * kMlpHid + mlp_kperm(kt, g, i)];
        P->w2[mt][kt][l] = v;
    }
    for (int idx = t; idx < 2 * 64; idx += blockDim.x) {
        const int kt = idx / 64, l = idx % 64, g = l / 16;
        bf16x8_t v;
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = (__bf16)par[kOffW3 + mlp_kperm(kt, g, i)];
        P->w3[kt][l] = v;
    }
    for (int i = t; i < kMlpHid; i += blockDim.x) {
        P->b1[i] = par[kOffB1 + i];
        P->b2[i] = par[kOffB2 + i];
    }
    if (t < kMlpIn) {
        P->xm[t] = norm[t];
        P->xi[t] = 1.0f / norm[5 + t];
    }
    if (t == 0) {
        P->ym = norm[10];
        P->ys = norm[11];
        P->b3 = par[kOffB3];
        P->pad = 0.f;
    }
}

// standalone forward: x [n][5] raw features -> y [n] (network output)
__global__ __launch_bounds__(kT, 4) void mlp_forward_kernel(MlpDev m, const float *__restrict__ x, float *__restrict__ y,
                                                         long long n)
{
    const long long i = (long long)blockIdx.x * kT + threadIdx.x;
    float xm[kMlpIn], xi[kMlpIn], xr[kMlpIn];
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) {
        xm[k] = m.pack->xm[k];
        xi[k] = m.pack->xi[k];
        xr[k] = i < n ? x[i * kMlpIn + k] : xm[k];
    }
    const float yh = mlp_yhat(*m.pack, xm, xi, xr);   // whole wave
    if (i < n) y[i] = yh;
}

// ---------------------------------------------------------------- training
//
// One wave per chunk of 64 rows (samples are the columns of the 16x16 tiles,
// hidden units the rows, as in inference).  Forward: the inference layers on
// the matrix cores, keeping the bf16 hidden activations h1, h2 (D tiles).
// Backward (the bf16 rounding treated as the identity, ReLU masks h > 0):
//   dy   = 2 (y - t) / n,
//   dh2  = dy w3 (h2 > 0)                 (VALU, in the D tiles),
//   dh1  = (W2^T dh2) (h1 > 0)             (matrix cores: dh2's D tiles are
//          the B operand in the permuted K order, W2^T the A operand),
//   gW2  = dh2 h1^T, gW1 = dh1 xb^T        (matrix cores, K = the 64 samples:
//          dh2, dh1, h1 and xb are staged transposed in LDS),
//   gw3 = h2 dy, gb2 = sum dh2, gb1 = sum dh1, gb3 = sum dy  (FP32 VALU).
// Products on the matrix cores take bf16 operands (dh1 and dh2 rounded to
// nearest even), accumulate in FP32.  Each wave adds its chunk's gradient
// into its own row of the partial buffer (the row is written by that wave
// only, chunk after chunk); the reduction sums the rows in a fixed order, so
// gradients are bitwise reproducible.
constexpr int kLd = 72;               // LDS row stride (bf16) of the transposed staging (16-byte pad)

// row map of a training call: identity (rows row0 + i) or the epoch's
// permutation of [0, n_perm) (see perm_index)
struct RowMap {
    long long row0;     // first position of the batch
    long long n_perm;   // > 0: permuted positions
    unsigned long long key;
    int half_bits;      // Feistel half width (2 half_bits >= bits of n_perm - 1)
};

// SplitMix64 finaliser (Steele, Lea & Flood 2014)
__host__ __device__ __forceinline__ unsigned long long mix64(unsigned long long z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// A seeded bijection of [0, n): a balanced four-round Feistel network on
// 2 h bits (round function: the SplitMix64 finaliser of key, round and the
// right half) with cycle walking into [0, n) (Black & Rogaway, "Ciphers with
// arbitrary finite domains", CT-RSA 2002).  2^(2h) < 4 n, so a walk takes
// fewer than four applications on average.
__host__ __device__ __forceinline__ long long feistel_perm(long long i, long long n, unsigned long long key, int h)
{
    const unsigned long long mask = (1ull << h) - 1ull;
    unsigned long long v = (unsigned long long)i;
    do {
        unsigned long long L = v >> h, R = v & mask;
        for (int r = 0; r < 4; ++r) {
            const unsigned long long f = mix64(key ^ (0x9E3779B97F4A7C15ull * (unsigned long long)(r + 1)) ^ R) & mask;
            const unsigned long long t = L ^ f;
            L = R;
            R = t;
        }
        v = (L << h) | R;
    } while (v >= (unsigned long long)n);
    return (long long)v;
}

__device__ __forceinline__ long long map_row(const RowMap &M, long long pos)
{
    const long long q = M.row0 + pos;
    return M.n_perm > 0 ? feistel_perm(q, M.n_perm, M.key, M.half_bits) : q;
}

// bf16 half i (0 = low) of a packed pair as float
__device__ __forceinline__ float bf16_lo(unsigned v) { return __uint_as_float(v << 16); }
__device__ __forceinline__ float bf16_hi(unsigned v) { return __uint_as_float(v & 0xFFFF0000u); }

// sum over the 16 lanes of a lane group (lanes g*16 .. g*16+15)
__device__ __forceinline__ float group16_sum(float v)
{
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ __launch_bounds__(64) void mlp_train_kernel(const MlpPack *__restrict__ P, const MlpTrainPack *__restrict__ TP,
                                                       const float *__restrict__ par, const float *__restrict__ x,
                                                       const float *__restrict__ tgt, long long n, RowMap rmap,
                                                       float *__restrict__ part, int chunks_per_wave)
{
    __shared__ __attribute__((aligned(16))) unsigned short h1s[kMlpHid * kLd], dh2s[kMlpHid * kLd], dh1s[kMlpHid * kLd],
        xbs[16 * kLd];
    const int l = threadIdx.x, g = l >> 4, j = l & 15;
    const int w = blockIdx.x;
    float *prow = part + (long long)w * kPartStride;
    float xm[kMlpIn], xi[kMlpIn];
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) {
        xm[k] = P->xm[k];
        xi[k] = P->xi[k];
    }
    // bf16-rounded w3 of the 16 units this lane holds (16 mt + 4 g + i)
    float w3r[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) w3r[mt][i] = bf16_val(bf16_rne(par[kOffW3 + 16 * mt + 4 * g + i]));
    const float inv_n2 = 2.0f / (float)n;
    for (int c = 0; c < chunks_per_wave; ++c) {
        const long long pos = ((long long)c * gridDim.x + w) * 64 + l;   // this lane's sample
        if (((long long)c * gridDim.x + w) * 64 >= n) break;             // the same for the whole wave
        const bool act = pos < n;
        const long long r = act ? map_row(rmap, pos) : 0;
        float z[kMlpIn];
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) z[k] = act ? (x[r * kMlpIn + k] - xm[k]) * xi[k] : 0.f;
        const float tv = act ? tgt[r] : 0.f;
        const unsigned p01 = pack_bf16(z[0], z[1]), p23 = pack_bf16(z[2], z[3]), p4 = pack_bf16(z[4], 0.f);
        // xb transposed: row k (feature), column = sample
        xbs[0 * kLd + l] = (unsigned short)(p01 & 0xFFFF);
        xbs[1 * kLd + l] = (unsigned short)(p01 >> 16);
        xbs[2 * kLd + l] = (unsigned short)(p23 & 0xFFFF);
        xbs[3 * kLd + l] = (unsigned short)(p23 >> 16);
        xbs[4 * kLd + l] = (unsigned short)(p4 & 0xFFFF);
#pragma unroll
        for (int k = 5; k < 16; ++k) xbs[k * kLd + l] = 0;
        // ---- forward (as inference, all four column tiles) ----
        unsigned h1[4][8], h2[4][8];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x4_t w1 = P->w1[mt][l];
            const f32x4_t b1 = *reinterpret_cast<const f32x4_t *>(&P->b1[16 * mt + 4 * g]);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const int src = 16 * nt + j;
                const unsigned a01 = __shfl(p01, src, 64), a23 = __shfl(p23, src, 64), a4 = __shfl(p4, src, 64);
                const unsigned lo = g == 0 ? a01 : (g == 1 ? a4 : 0u), hi = g == 0 ? a23 : 0u;
                const bf16x4_t bx = __builtin_bit_cast(bf16x4_t, (u32x2_t){lo, hi});
                const f32x4_t d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1, bx, b1, 0, 0, 0);
                h1[nt][2 * mt] = pack_relu(d[0], d[1]);
                h1[nt][2 * mt + 1] = pack_relu(d[2], d[3]);
            }
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x8_t wa = P->w2[mt][0][l], wb = P->w2[mt][1][l];
            const f32x4_t b2 = *reinterpret_cast<const f32x4_t *>(&P->b2[16 * mt + 4 * g]);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const bf16x8_t k0 = __builtin_bit_cast(bf16x8_t, (u32x4_t){h1[nt][0], h1[nt][1], h1[nt][2], h1[nt][3]});
                const bf16x8_t k1 = __builtin_bit_cast(bf16x8_t, (u32x4_t){h1[nt][4], h1[nt][5], h1[nt][6], h1[nt][7]});
                f32x4_t d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, k0, b2, 0, 0, 0);
                d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb, k1, d, 0, 0, 0);
                h2[nt][2 * mt] = pack_relu(d[0], d[1]);
                h2[nt][2 * mt + 1] = pack_relu(d[2], d[3]);
            }
        }
        float y = 0.f;
        {
            const bf16x8_t w3a = P->w3[0][l], w3b = P->w3[1][l];
            const float b3 = P->b3;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const bf16x8_t q0 = __builtin_bit_cast(bf16x8_t, (u32x4_t){h2[nt][0], h2[nt][1], h2[nt][2], h2[nt][3]});
                const bf16x8_t q1 = __builtin_bit_cast(bf16x8_t, (u32x4_t){h2[nt][4], h2[nt][5], h2[nt][6], h2[nt][7]});
                f32x4_t d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3a, q0, (f32x4_t){b3, b3, b3, b3}, 0, 0, 0);
                d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3b, q1, d, 0, 0, 0);
                if (g == nt) y = d[0];
            }
        }
        const float dlt = act ? y - tv : 0.f;
        const float dy = dlt * inv_n2;
        // ---- backward: dh2 (D tiles), gw3 and gb2 partials, staging ----
        unsigned dh2p[4][8];
        float gw3[4][4], gb2[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) gw3[mt][i] = gb2[mt][i] = 0.f;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const float dyn = __shfl(dy, 16 * nt + j, 64);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                float hv[4], dv[4];
                hv[0] = bf16_lo(h2[nt][2 * mt]);
                hv[1] = bf16_hi(h2[nt][2 * mt]);
                hv[2] = bf16_lo(h2[nt][2 * mt + 1]);
                hv[3] = bf16_hi(h2[nt][2 * mt + 1]);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    dv[i] = hv[i] > 0.f ? dyn * w3r[mt][i] : 0.f;
                    gw3[mt][i] = fmaf(dyn, hv[i], gw3[mt][i]);
                    gb2[mt][i] += dv[i];
                }
                dh2p[nt][2 * mt] = pack_bf16(dv[0], dv[1]);
                dh2p[nt][2 * mt + 1] = pack_bf16(dv[2], dv[3]);
                // transposed staging: row = unit, column = sample 16 nt + j
                const int u = 16 * mt + 4 * g, sc = 16 * nt + j;
                dh2s[(u + 0) * kLd + sc] = (unsigned short)(dh2p[nt][2 * mt] & 0xFFFF);
                dh2s[(u + 1) * kLd + sc] = (unsigned short)(dh2p[nt][2 * mt] >> 16);
                dh2s[(u + 2) * kLd + sc] = (unsigned short)(dh2p[nt][2 * mt + 1] & 0xFFFF);
                dh2s[(u + 3) * kLd + sc] = (unsigned short)(dh2p[nt][2 * mt + 1] >> 16);
                h1s[(u + 0) * kLd + sc] = (unsigned short)(h1[nt][2 * mt] & 0xFFFF);
                h1s[(u + 1) * kLd + sc] = (unsigned short)(h1[nt][2 * mt] >> 16);
                h1s[(u + 2) * kLd + sc] = (unsigned short)(h1[nt][2 * mt + 1] & 0xFFFF);
                h1s[(u + 3) * kLd + sc] = (unsigned short)(h1[nt][2 * mt + 1] >> 16);
            }
        }
        // ---- dh1 = (W2^T dh2) (h1 > 0), gb1 partial, staging ----
        float gb1[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x8_t wa = TP->w2t[mt][0][l], wb = TP->w2t[mt][1][l];
#pragma unroll
            for (int i = 0; i < 4; ++i) gb1[mt][i] = 0.f;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const bf16x8_t k0 = __builtin_bit_cast(bf16x8_t, (u32x4_t){dh2p[nt][0], dh2p[nt][1], dh2p[nt][2], dh2p[nt][3]});
                const bf16x8_t k1 = __builtin_bit_cast(bf16x8_t, (u32x4_t){dh2p[nt][4], dh2p[nt][5], dh2p[nt][6], dh2p[nt][7]});
                f32x4_t d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, k0, (f32x4_t){0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb, k1, d, 0, 0, 0);
                float hv[4];
                hv[0] = bf16_lo(h1[nt][2 * mt]);
                hv[1] = bf16_hi(h1[nt][2 * mt]);
                hv[2] = bf16_lo(h1[nt][2 * mt + 1]);
                hv[3] = bf16_hi(h1[nt][2 * mt + 1]);
                float dv[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    dv[i] = hv[i] > 0.f ? d[i] : 0.f;
                    gb1[mt][i] += dv[i];
                }
                const unsigned q0 = pack_bf16(dv[0], dv[1]), q1 = pack_bf16(dv[2], dv[3]);
                const int u = 16 * mt + 4 * g, sc = 16 * nt + j;
                dh1s[(u + 0) * kLd + sc] = (unsigned short)(q0 & 0xFFFF);
                dh1s[(u + 1) * kLd + sc] = (unsigned short)(q0 >> 16);
                dh1s[(u + 2) * kLd + sc] = (unsigned short)(q1 & 0xFFFF);
                dh1s[(u + 3) * kLd + sc] = (unsigned short)(q1 >> 16);
            }
        }
        __syncthreads();   // one wave: its LDS writes are visible to its reads after this
        // ---- gW2 = dh2 h1^T and gW1 = dh1 xb^T on the matrix cores (K = samples) ----
        const bool first = c == 0;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const bf16x8_t a0 = *reinterpret_cast<const bf16x8_t *>(&dh2s[(16 * mu + j) * kLd + 8 * g]);
            const bf16x8_t a1 = *reinterpret_cast<const bf16x8_t *>(&dh2s[(16 * mu + j) * kLd + 32 + 8 * g]);
#pragma unroll
            for (int mk = 0; mk < 4; ++mk) {
                const bf16x8_t b0 = *reinterpret_cast<const bf16x8_t *>(&h1s[(16 * mk + j) * kLd + 8 * g]);
                const bf16x8_t b1 = *reinterpret_cast<const bf16x8_t *>(&h1s[(16 * mk + j) * kLd + 32 + 8 * g]);
                f32x4_t d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, (f32x4_t){0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, d, 0, 0, 0);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float *dst = prow + kOffW2 + (16 * mu + 4 * g + i) * kMlpHid + 16 * mk + j;
                    *dst = first ? d[i] : *dst + d[i];
                }
            }
            const bf16x8_t e0 = *reinterpret_cast<const bf16x8_t *>(&dh1s[(16 * mu + j) * kLd + 8 * g]);
            const bf16x8_t e1 = *reinterpret_cast<const bf16x8_t *>(&dh1s[(16 * mu + j) * kLd + 32 + 8 * g]);
            const bf16x8_t f0 = *reinterpret_cast<const bf16x8_t *>(&xbs[j * kLd + 8 * g]);
            const bf16x8_t f1 = *reinterpret_cast<const bf16x8_t *>(&xbs[j * kLd + 32 + 8 * g]);
            f32x4_t d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(e0, f0, (f32x4_t){0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(e1, f1, d, 0, 0, 0);
            if (j < kMlpIn) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float *dst = prow + kOffW1 + (16 * mu + 4 * g + i) * kMlpIn + j;
                    *dst = first ? d[i] : *dst + d[i];
                }
            }
        }
        // ---- bias and w3 partials: sums over the 16 lanes of a group ----
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float s1 = group16_sum(gb1[mt][i]), s2 = group16_sum(gb2[mt][i]), s3 = group16_sum(gw3[mt][i]);
                if (j == i) {
                    const int u = 16 * mt + 4 * g + i;
                    float *d1 = prow + kOffB1 + u, *d2 = prow + kOffB2 + u, *d3 = prow + kOffW3 + u;
                    *d1 = first ? s1 : *d1 + s1;
                    *d2 = first ? s2 : *d2 + s2;
                    *d3 = first ? s3 : *d3 + s3;
                }
            }
        float sdy = dy, sl = dlt * dlt;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            sdy += __shfl_xor(sdy, o, 64);
            sl += __shfl_xor(sl, o, 64);
        }
        if (l == 0) {
            prow[kOffB3] = first ? sdy : prow[kOffB3] + sdy;
            prow[kMlpNParam] = first ? sl : prow[kMlpNParam] + sl;
        }
        __syncthreads();   // the staging is rewritten by the next chunk
    }
}

// grad = fixed-order sum of the partial rows; loss = their loss sum / n
// (added to *loss_acc when given); optionally one bias-corrected Adam step
// on the masters.  A work-group takes 64 parameters; its four waves sum the
// rows r = q (mod 4) (q the wave) in four interleaved accumulators each, and
// wave 0 adds the four wave sums in order: the same order for every call
// with the same row count.
constexpr int kRedParams = 64;
__global__ __launch_bounds__(256) void mlp_reduce_adam_kernel(const float *__restrict__ part, int rows, long long n,
                                                              float *__restrict__ grad, float *__restrict__ loss,
                                                              double *__restrict__ loss_acc, float *__restrict__ par,
                                                              float *__restrict__ mo, float *__restrict__ vo, int adam,
                                                              float lr, float b1, float b2, float eps, float bc1,
                                                              float bc2)
{
    __shared__ float red[4][kRedParams];
    const int q = threadIdx.x >> 6, j = threadIdx.x & 63;
    const int pi = blockIdx.x * kRedParams + j;
    float a[4] = {0.f, 0.f, 0.f, 0.f};
    if (pi <= kMlpNParam) {
        int r = q;
        for (; r + 12 < rows; r += 16) {
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] += part[(long long)(r + 4 * u) * kPartStride + pi];
        }
        for (int u = 0; r < rows; r += 4, ++u) a[u & 3] += part[(long long)r * kPartStride + pi];
    }
    red[q][j] = (a[0] + a[1]) + (a[2] + a[3]);
    __syncthreads();
    if (q != 0 || pi > kMlpNParam) return;
    const float gsum = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
    if (pi == kMlpNParam) {
        const float L = gsum / (float)n;
        loss[0] = L;
        if (loss_acc) loss_acc[0] += (double)L;
        return;
    }
    grad[pi] = gsum;
    if (adam) {
        const float m1 = b1 * mo[pi] + (1.f - b1) * gsum;
        const float v1 = b2 * vo[pi] + (1.f - b2) * gsum * gsum;
        mo[pi] = m1;
        vo[pi] = v1;
        par[pi] -= lr * (m1 / bc1) / (sqrtf(v1 / bc2) + eps);
    }
}

// raw features of conserved states cons [5][n] (SoA doubles) -> x [n][5]
__global__ __launch_bounds__(kT) void mlp_features_kernel(const double *__restrict__ cons, float *__restrict__ x,
                                                          long long n)
{
    const long long i = (long long)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const C2pIn in = c2p_setup(cons[i], cons[n + i], cons[2 * n + i], cons[3 * n + i], cons[4 * n + i], 5.0 / 3.0);
    float f[kMlpIn];
    mlp_features(in, f);
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) x[i * kMlpIn + k] = f[k];
}

// training inputs: raw features x [n][5] of cons [5][n] and the target
// y = log(p / E), formed in FP64 and rounded to binary32
__global__ __launch_bounds__(kT) void mlp_prepare_kernel(const double *__restrict__ cons, const double *__restrict__ p,
                                                         float *__restrict__ x, float *__restrict__ y, long long n)
{
    const long long i = (long long)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const C2pIn in = c2p_setup(cons[i], cons[n + i], cons[2 * n + i], cons[3 * n + i], cons[4 * n + i], 5.0 / 3.0);
    float f[kMlpIn];
    mlp_features(in, f);
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) x[i * kMlpIn + k] = f[k];
    y[i] = (float)log(p[i] / in.E);
}

// Normalisation statistics of the training set in FP64, in a fixed order
// (bitwise reproducible): pass 0 sums the six columns (five features, the
// target), pass 1 the squared deviations from the means.  Work-group b
// takes rows b, b + G, b + 2G, ... in a grid-stride walk, reduces its lanes
// by a fixed shuffle tree and its waves in order, and writes one partial per
// column; the finishing kernel adds the G partials in order.
__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__global__ __launch_bounds__(kT) void mlp_stats_kernel(const float *__restrict__ x, const float *__restrict__ y,
                                                       long long n, int pass, const double *__restrict__ mean,
                                                       double *__restrict__ partial)
{
    __shared__ double red[6][kT / kWave];
    double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double mu[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (pass == 1)
        for (int c = 0; c < 6; ++c) mu[c] = mean[c];
    const long long stride = (long long)gridDim.x * kT;
    for (long long i = (long long)blockIdx.x * kT + threadIdx.x; i < n; i += stride) {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const double v = (double)(c < kMlpIn ? x[i * kMlpIn + c] : y[i]) - mu[c];
            a[c] += pass == 0 ? v : v * v;
        }
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const double v = wave_sum(a[c]);
        if (lane == 0) red[c][w] = v;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double v = 0.0;
        for (int i = 0; i < kT / kWave; ++i) v += red[threadIdx.x][i];
        partial[(long long)threadIdx.x * gridDim.x + blockIdx.x] = v;
    }
}

// pass 0: mean[c] = sum / n; pass 1: std[c] = sqrt(sum / (n - 1)) (features
// floored at 1e-6) and the FP32 normalisation block
__global__ void mlp_stats_finish_kernel(const double *__restrict__ partial, int G, long long n, int pass,
                                        double *__restrict__ mean, float *__restrict__ norm)
{
    const int c = threadIdx.x;
    if (c >= 6) return;
    double v = 0.0;
    for (int b = 0; b < G; ++b) v += partial[(long long)c * G + b];
    if (pass == 0) {
        mean[c] = v / (double)n;
        return;
    }
    double sd = n > 1 ? sqrt(v / (double)(n - 1)) : 0.0;
    if (c < kMlpIn) {
        sd = fmax(sd, 1e-6);
        norm[c] = (float)mean[c];
        norm[5 + c] = (float)sd;
    } else {
        norm[10] = (float)mean[c];
        norm[11] = (float)sd;
    }
}

// t = binary32((y - y_mean) / y_std), with the stored binary32 y_mean, y_std
// taken as doubles
__global__ __launch_bounds__(kT) void mlp_standardise_kernel(const float *__restrict__ norm, const float *__restrict__ y,
                                                             float *__restrict__ t, long long n)
{
    const long long i = (long long)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    t[i] = (float)(((double)y[i] - (double)norm[10]) / (double)norm[11]);
}

__global__ __launch_bounds__(kT) void mlp_permutation_kernel(long long n, unsigned long long key, int h,
                                                             long long *__restrict__ idx)
{
    const long long i = (long long)blockIdx.x * kT + threadIdx.x;
    if (i < n) idx[i] = feistel_perm(i, n, key, h);
}

pb_status refresh(pb_mlp *m, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_refresh_kernel, dim3(1), dim3(256), 0, s, m->par, m->norm, m->pack, m->tpack);
    PB_HIP(hipGetLastError());
    return PB_OK;
}

// the permutation key of (seed, epoch) and the Feistel half width for n
unsigned long long perm_key(unsigned long long seed, long long epoch)
{
    return mix64(seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(epoch + 1));
}

int perm_half_bits(long long n)
{
    int m = 2;
    while (m < 62 && (1ll << m) < n) ++m;
    return (m + 1) / 2;
}

// forward + backward over n rows (mapped by rmap) into the partial buffer
// `part`, then the fixed-order reduction (and Adam); shared by the entry
// points that take the library's scratch and the one that takes a caller's
pb_status run_grad_into(pb_mlp *m, float *part, float *grad, float *loss, const float *x, const float *t, long long n,
                        const RowMap &rmap, hipStream_t s, int adam, float lr, float b1, float b2, float eps, int step,
                        double *loss_acc)
{
    const long long nchunks = (n + 63) / 64;
    const int waves = (int)std::min<long long>(kTrainWavesMax, nchunks);
    const int cpw = (int)((nchunks + waves - 1) / waves);
    hipLaunchKernelGGL(mlp_train_kernel, dim3(waves), dim3(64), 0, s, m->pack, m->tpack, m->par, x, t, n, rmap, part,
                       cpw);
    PB_HIP(hipGetLastError());
    const float bc1 = adam ? 1.f - std::pow(b1, (float)step) : 1.f;
    const float bc2 = adam ? 1.f - std::pow(b2, (float)step) : 1.f;
    hipLaunchKernelGGL(mlp_reduce_adam_kernel, dim3((kMlpNParam + 1 + kRedParams - 1) / kRedParams), dim3(256), 0, s,
                       part, waves, n,
                       grad, loss, loss_acc, m->par, m->madam, m->vadam, adam, lr, b1, b2, eps, bc1, bc2);
    PB_HIP(hipGetLastError());
    if (adam) return refresh(m, s);
    return PB_OK;
}

pb_status run_grad(pb_mlp *m, const float *x, const float *t, long long n, const RowMap &rmap, hipStream_t s, int adam,
                   float lr, float b1, float b2, float eps, int step, double *loss_acc)
{
    return run_grad_into(m, m->part, m->grad, m->loss, x, t, n, rmap, s, adam, lr, b1, b2, eps, step, loss_acc);
}

// The partial-gradient scratch of pb_mlp_grad_noalloc: one file-scope
// device array (each GPU the library runs on holds its own copy until the
// process ends).  Host code never passes the array's name to a kernel (on
// the host it is a stand-in, not a device address): it takes the address
// hipGetSymbolAddress reports for the current device, once per device.
constexpr long long kNoAllocMaxRows = 1ll << 30;
__device__ __align__(256) float scratch[kTrainWavesMax * kPartStride];

pb_status scratch_address(float **out)
{
    constexpr int kMaxDev = 64;
    static std::mutex mu;
    static float *addr[kMaxDev] = {};
    int dev = 0;
    PB_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) { set_error("device index out of range"); return PB_EUNSUPPORTED; }
    std::lock_guard<std::mutex> g(mu);
    if (!addr[dev]) {
        void *ptr = nullptr;
        PB_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) { set_error("hipGetSymbolAddress(scratch) returned NULL"); return PB_EHIP; }
        addr[dev] = static_cast<float *>(ptr);
    }
    *out = addr[dev];
    return PB_OK;
}

bool adam_ok(float lr, float beta1, float beta2, float eps)
{
    return lr > 0.f && std::isfinite(lr) && beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f &&
           std::isfinite(eps);
}

}  // namespace

pb_status mlp_device_view(const pb_mlp *m, MlpDev *out)
{
    if (!m || !out) { set_error("MLP is NULL"); return PB_EINVAL; }
    out->pack = m->pack;
    out->par = m->par;
    out->norm = m->norm;
    return PB_OK;
}

}  // namespace pb

using namespace pb;

extern "C" {

pb_status pb_mlp_create(pb_mlp **out)
{
    PB_API_BEGIN
    if (!out) { set_error("out is NULL"); return PB_EINVAL; }
    *out = nullptr;
    pb_mlp *m = new (std::nothrow) pb_mlp();
    if (!m) { set_error("out of host memory"); return PB_ENOMEM; }
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t bytes = al(sizeof(MlpPack)) + al(sizeof(MlpTrainPack)) + 4 * al(kMlpNParam * sizeof(float)) +
                         al(16 * sizeof(float)) + al(sizeof(float)) +
                         al((size_t)kTrainWavesMax * kPartStride * sizeof(float)) +
                         al((size_t)(6 * kStatBlocks + 16) * sizeof(double));
    hipError_t e = hipMalloc(&m->dev, bytes);
    if (e != hipSuccess) { delete m; return hip_fail(e, "hipMalloc(mlp)"); }
    e = hipMemset(m->dev, 0, bytes);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) { (void)hipFree(m->dev); delete m; return hip_fail(e, "hipMemset(mlp)"); }
    char *p = m->dev;
    auto take = [&](size_t b) { char *r = p; p += al(b); return r; };
    m->pack = reinterpret_cast<MlpPack *>(take(sizeof(MlpPack)));
    m->tpack = reinterpret_cast<MlpTrainPack *>(take(sizeof(MlpTrainPack)));
    m->par = reinterpret_cast<float *>(take(kMlpNParam * sizeof(float)));
    m->madam = reinterpret_cast<float *>(take(kMlpNParam * sizeof(float)));
    m->vadam = reinterpret_cast<float *>(take(kMlpNParam * sizeof(float)));
    m->grad = reinterpret_cast<float *>(take(kMlpNParam * sizeof(float)));
    m->norm = reinterpret_cast<float *>(take(16 * sizeof(float)));
    m->loss = reinterpret_cast<float *>(take(sizeof(float)));
    m->part = reinterpret_cast<float *>(take((size_t)kTrainWavesMax * kPartStride * sizeof(float)));
    m->stats = reinterpret_cast<double *>(take((size_t)(6 * kStatBlocks + 16) * sizeof(double)));
    *out = m;
    return PB_OK;
    PB_API_END
}

pb_status pb_mlp_destroy(pb_mlp *m)
{
    PB_API_BEGIN
    if (!m) return PB_OK;
    (void)hipFree(m->dev);
    delete m;
    return PB_OK;
    PB_API_END
}

pb_status pb_mlp_set_params(pb_mlp *m, const float *params, const float *norm)
{
    PB_API_BEGIN
    if (!m || !params || !norm) { set_error("NULL argument"); return PB_EINVAL; }
    for (int i = 0; i < kMlpNParam; ++i)
        if (!std::isfinite(params[i])) { set_error("MLP parameters must be finite"); return PB_EINVAL; }
    for (int i = 0; i < kMlpNNorm; ++i)
        if (!std::isfinite(norm[i])) { set_error("MLP normalisation must be finite"); return PB_EINVAL; }
    for (int i = 5; i < 10; ++i)
        if (!(norm[i] > 0.f)) { set_error("feature std must be > 0"); return PB_EINVAL; }
    if (!(norm[11] > 0.f)) { set_error("target std must be > 0"); return PB_EINVAL; }
    PB_HIP(hipMemcpy(m->par, params, kMlpNParam * sizeof(float), hipMemcpyHostToDevice));
    PB_HIP(hipMemcpy(m->norm, norm, kMlpNNorm * sizeof(float), hipMemcpyHostToDevice));
    PB_HIP(hipMemset(m->madam, 0, kMlpNParam * sizeof(float)));
    PB_HIP(hipMemset(m->vadam, 0, kMlpNParam * sizeof(float)));
    pb_status st = refresh(m, nullptr);
    if (st != PB_OK) return st;
    PB_HIP(hipDeviceSynchronize());
    return PB_OK;
    PB_API_END
}

pb_status pb_mlp_get_params(pb_mlp *m, float *params, float *norm)
{
    PB_API_BEGIN
    if (!m) { set_error("NULL argument"); return PB_EINVAL; }
    PB_HIP(hipDeviceSynchronize());
    if (params) PB_HIP(hipMemcpy(params, m->par, kMlpNParam * sizeof(float), hipMemcpyDeviceToHost));
    if (norm) PB_HIP(hipMemcpy(norm, m->norm, kMlpNNorm * sizeof(float), hipMemcpyDeviceToHost));
    return PB_OK;
    PB_API_END
}

pb_status pb_mlp_forward(const pb_mlp *m, const void *x, void *y, int64_t n, void *stream)
{
    PB_API_BEGIN
    if (!m || !x || !y) { set_error("NULL argument"); return PB_EINVAL; }
    if (n < 0) { set_error("n must be >= 0"); return PB_EINVAL; }
    if (n == 0) return PB_OK;
    MlpDev md;
    mlp_device_view(m, &md);
    const long long nb = (n + kT - 1) / kT;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)nb), dim3(kT), 0, static_cast<hipStream_t>(stream), md,
                       static_cast<const float *>(x), static_cast<float *>(y), (long long)n);
    PB_HIP(hipGetLastError());
    return PB_OK;
    PB_API_END
}

pb_status pb_mlp_features(const void *cons, void *x, int64_t n, void *stream)
{
    PB_API_BEGIN
    if (!cons || !x) { set_error("NULL argument"); return PB_EINVAL; }
    if (n < 0) { set_error("n must be >= 0"); return PB_EINVAL; }
    if (n == 0) return PB_OK;
    const long long nb = (n + kT - 1) / kT;
    hipLaunchKernelGGL(mlp_features_kernel, dim3((unsigned)nb), dim3(kT), 0, static_cast<hipStream_t>(stream),
                       static_cast<const double *>(cons), static_cast<float *>(x), (long long)n);
    PB_HIP(hipGetLastError());
    return PB_OK;
    PB_API_END
}

pb_status pb_mlp_prepare(const void *cons, const void *p, void *x, void *y, int64_t n, void *stream)
{
    PB_API_BEGIN
    if (n < 0) { set_error("n must be >= 0"); return PB_EINVAL; }
    if (n == 0) return PB_OK;
    if (!cons || !p || !x || !y) { set_error("NULL argument"); return PB_EINVAL; }
    const long long nb = (n + kT - 1) / kT;
    hipLaunchKernelGGL(mlp_prepare_kernel, dim3((unsigned)nb), dim3(kT), 0, static_cast<hipStream_t>(stream),
                       static_cast<const double *>(cons), static_cast<const double *>(p), static_cast<float *>(x),
                       static_cast<float *>(y), (long long)n);
    PB_HIP(hipGetLastError());
    return PB_OK;
    PB_API_END
}

pb_status pb_mlp_fit_norm(pb_mlp *m, const void *x, const void *y, int64_t n, void *stream)
{
    PB_API_BEGIN
    if (!m || !x || !y) { set_error("NULL argument"); return PB_EINVAL; }
    if (n < 2) { set_error("n must be >= 2"); return PB_EINVAL; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int G = (int)std::min<long long>(kStatBlocks, (n + kT - 1) / kT);
    double *mean = m->stats, *partial = m->stats + 16;
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(mlp_stats_kernel, dim3(G), dim3(kT), 0, s, static_cast<const float *>(x),
                           static_cast<const float *>(y), (long long)n, pass, mean, partial);
        PB_HIP(hipGetLastError());
        hipLaunchKernelGGL(mlp_stats_finish_kernel, dim3(1), dim3(64), 0, s, partial, G, (long long)n, pass, mean,
                           m->norm);
        PB_HIP(hipGetLastError());
    }
    return refresh(m, s);
    PB_API_END
}

pb_status pb_mlp_standardise_target(const pb_mlp *m, const void *y, void *t, int64_t n, void *stream)
{
    PB_API_BEGIN
    if (!m) { set_error("NULL argument"); return PB_EINVAL; }
    if (n < 0) { set_error("n must be >= 0"); return PB_EINVAL; }
    if (n == 0) return PB_OK;
    if (!y || !t) { set_error("NULL argument"); return PB_EINVAL; }
    const long long nb = (n + kT - 1) / kT;
    hipLaunchKernelGGL(mlp_standardise_kernel, dim3((unsigned)nb), dim3(kT), 0, static_cast<hipStream_t>(stream),
                       m->norm, static_cast<const float *>(y), static_cast<float *>(t), (long long)n);
    PB_HIP(hipGetLastError());
    return PB_OK;
    PB_API_END
}

pb_status pb_mlp_permutation(uint64_t seed, int64_t epoch, int64_t n, void *idx, void *stream)
{
    PB_API_BEGIN
    if (n < 0 || epoch < 0) { set_error("n and epoch must be >= 0"); return PB_EINVAL; }
    if (n == 0) return PB_OK;
    if (!idx) { set_error("NULL argument"); return PB_EINVAL; }
    if (n > (1ll << 60)) { set_error("n too large"); return PB_EINVAL; }
    const long long nb = (n + kT - 1) / kT;
    hipLaunchKernelGGL(mlp_permutation_kernel, dim3((unsigned)nb), dim3(kT), 0, static_cast<hipStream_t>(stream),
                       (long long)n, perm_key(seed, epoch), perm_half_bits(n), static_cast<long long *>(idx));
    PB_HIP(hipGetLastError());
    return PB_OK;
    PB_API_END
}

pb_status pb_mlp_grad(const pb_mlp *m, const void *x, const void *t, int64_t n, void *grad, void *loss, void *stream)
{
    PB_API_BEGIN
    if (!m || !x || !t || !grad || !loss) { set_error("NULL argument"); return PB_EINVAL; }
    if (n < 1) { set_error("n must be >= 1"); return PB_EINVAL; }
    pb_mlp *mm = const_cast<pb_mlp *>(m);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const RowMap ident{0, 0, 0ull, 0};
    pb_status st = run_grad(mm, static_cast<const float *>(x), static_cast<const float *>(t), n, ident, s, 0, 0.f, 0.f,
                            0.f, 0.f, 1, nullptr);
    if (st != PB_OK) return st;
    PB_HIP(hipMemcpyAsync(grad, mm->grad, kMlpNParam * sizeof(float), hipMemcpyDeviceToDevice, s));
    PB_HIP(hipMemcpyAsync(loss, mm->loss, sizeof(float), hipMemcpyDeviceToDevice, s));
    return PB_OK;
    PB_API_END
}

pb_status pb_mlp_grad_noalloc(const pb_mlp *m, const void *x, const void *t, int64_t n, void *grad, void *loss,
                              void *stream)
{
    PB_API_BEGIN
    if (!m || !x || !t || !grad || !loss) { set_error("NULL argument"); return PB_EINVAL; }
    if (n < 1) { set_error("n must be >= 1"); return PB_EINVAL; }
    if (n > kNoAllocMaxRows) {
        set_error("pb_mlp_grad_noalloc: n exceeds the maximum of 2^30 rows");
        return PB_EINVAL;
    }
    float *part = nullptr;
    pb_status st = scratch_address(&part);
    if (st != PB_OK) return st;
    const RowMap ident{0, 0, 0ull, 0};
    return run_grad_into(const_cast<pb_mlp *>(m), part, static_cast<float *>(grad), static_cast<float *>(loss),
                         static_cast<const float *>(x), static_cast<const float *>(t), n, ident,
                         static_cast<hipStream_t>(stream), 0, 0.f, 0.f, 0.f, 0.f, 1, nullptr);
    PB_API_END
}

pb_status pb_mlp_train_step(pb_mlp *m, const void *x, const void *t, int64_t n, float lr, float beta1, float beta2,
                            float eps, int32_t step, void *loss, void *stream)
{
    PB_API_BEGIN
    if (!m || !x || !t) { set_error("NULL argument"); return PB_EINVAL; }
    if (n < 1) { set_error("n must be >= 1"); return PB_EINVAL; }
    if (step < 1) { set_error("step must be >= 1"); return PB_EINVAL; }
    if (!adam_ok(lr, beta1, beta2, eps)) { set_error("bad Adam hyper-parameters"); return PB_EINVAL; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const RowMap ident{0, 0, 0ull, 0};
    pb_status st = run_grad(m, static_cast<const float *>(x), static_cast<const float *>(t), n, ident, s, 1, lr, beta1,
                            beta2, eps, step, nullptr);
    if (st != PB_OK) return st;
    if (loss) PB_HIP(hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToDevice, s));
    return PB_OK;
    PB_API_END
}

pb_status pb_mlp_train_epoch(pb_mlp *m, const void *x, const void *t, int64_t n, int32_t batch, uint64_t seed,
                             int32_t epoch, float lr_max, int64_t step0, int64_t total_steps, float beta1, float beta2,
                             float eps, void *loss_sum, void *stream)
{
    PB_API_BEGIN
    if (!m || !x || !t) { set_error("NULL argument"); return PB_EINVAL; }
    if (batch < 1 || n < batch) { set_error("need 1 <= batch <= n"); return PB_EINVAL; }
    if (epoch < 0 || step0 < 0) { set_error("epoch and step0 must be >= 0"); return PB_EINVAL; }
    const long long spe = n / batch;
    if (total_steps < step0 + spe) { set_error("total_steps must cover this epoch"); return PB_EINVAL; }
    if (!adam_ok(lr_max, beta1, beta2, eps)) { set_error("bad Adam hyper-parameters"); return PB_EINVAL; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const unsigned long long key = perm_key(seed, epoch);
    const int h = perm_half_bits(n);
    for (long long b = 0; b < spe; ++b) {
        const long long step = step0 + b + 1;
        const double ph = 3.14159265358979323846 * (double)(step - 1) / (double)total_steps;
        const float lr = (float)(0.5 * (double)lr_max * (1.0 + std::cos(ph)));
        const RowMap rm{b * batch, (long long)n, key, h};
        pb_status st = run_grad(m, static_cast<const float *>(x), static_cast<const float *>(t), batch, rm, s, 1, lr,
                                beta1, beta2, eps, (int)step, static_cast<double *>(loss_sum));
        if (st != PB_OK) return st;
    }
    return PB_OK;
    PB_API_END
}

}  // extern "C"

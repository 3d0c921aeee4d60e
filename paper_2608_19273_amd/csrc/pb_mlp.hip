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
#include <new>

#include "pb_common.h"
#include "pb_mlp.h"

struct pb_mlp {
    char *dev = nullptr;        // one device allocation holding everything below
    float *par = nullptr;       // FP32 master parameters [kMlpNParam]
    float *madam = nullptr;     // Adam first moments
    float *vadam = nullptr;     // Adam second moments
    float *norm = nullptr;      // [kMlpNNorm]
    pb::MlpPack *pack = nullptr;  // inference operands (bf16, lane-swizzled), see pb_mlp.h
    float *grad = nullptr;      // [kMlpNParam] gradient of the last train step
    float *loss = nullptr;      // [1]
    float *scratch = nullptr;   // training activations, library-owned
    long long scratch_rows = 0;
    float *partial = nullptr;   // [kChunks][kMlpNParam]
    float *lpart = nullptr;     // per-block loss partials
    long long lpart_cap = 0;
};

namespace pb {

namespace {

constexpr int kChunks = 32;
constexpr int kT = 256;

// the inference blob from the FP32 masters and the normalisation block
// (layout of pb_mlp.h)
__global__ __launch_bounds__(256) void mlp_refresh_kernel(const float *__restrict__ par, const float *__restrict__ norm,
                                                          MlpPack *__restrict__ P)
{
    const int t = threadIdx.x;
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

// Training rows: per sample XB[5], H1[64], H2[64], DH1[64], DH2[64], DY[1]
constexpr int kRow = kMlpIn + 4 * kMlpHid + 1;
constexpr int kOXB = 0, kOH1 = kMlpIn, kOH2 = kOH1 + kMlpHid, kODH1 = kOH2 + kMlpHid, kODH2 = kODH1 + kMlpHid,
              kODY = kODH2 + kMlpHid;

// forward + backward per sample (one lane per sample), weights staged in LDS
__global__ __launch_bounds__(kT) void mlp_fwd_bwd_kernel(const float *__restrict__ par, const float *__restrict__ norm,
                                                         const float *__restrict__ x, const float *__restrict__ tgt,
                                                         long long n, float *__restrict__ rows,
                                                         float *__restrict__ lpart)
{
    __shared__ float W1[kMlpHid * kMlpIn], B1[kMlpHid], W2[kMlpHid * kMlpHid], B2[kMlpHid], W3[kMlpHid];
    __shared__ float red[kT / kWave];
    for (int i = threadIdx.x; i < kMlpHid * kMlpHid; i += kT) W2[i] = bf16_val(bf16_rne(par[kOffW2 + i]));
    for (int i = threadIdx.x; i < kMlpHid * kMlpIn; i += kT) W1[i] = bf16_val(bf16_rne(par[kOffW1 + i]));
    for (int i = threadIdx.x; i < kMlpHid; i += kT) {
        B1[i] = par[kOffB1 + i];
        B2[i] = par[kOffB2 + i];
        W3[i] = bf16_val(bf16_rne(par[kOffW3 + i]));
    }
    __syncthreads();
    const long long s = (long long)blockIdx.x * kT + threadIdx.x;
    float lsum = 0.f;
    if (s < n) {
        float* r = rows + s * kRow;
        float xr[kMlpIn];
        unsigned short xb16[kMlpIn];
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) xr[k] = x[s * kMlpIn + k];
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) xb16[k] = bf16_rne((xr[k] - norm[k]) * (1.0f / norm[5 + k]));
        float xb[kMlpIn];
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) {
            xb[k] = bf16_val(xb16[k]);
            r[kOXB + k] = xb[k];
        }
        float h1[kMlpHid];
#pragma unroll
        for (int m = 0; m < kMlpHid; ++m) {
            float a = 0.f;
#pragma unroll
            for (int k = 0; k < kMlpIn; ++k) a = fmaf(W1[m * kMlpIn + k], xb[k], a);
            h1[m] = bf16_val(bf16_rne(fmaxf(a + B1[m], 0.f)));
            r[kOH1 + m] = h1[m];
        }
        float y = 0.f;
        unsigned long long mask2 = 0ull;
        for (int m = 0; m < kMlpHid; ++m) {
            float a = 0.f;
#pragma unroll
            for (int k = 0; k < kMlpHid; ++k) a = fmaf(W2[m * kMlpHid + k], h1[k], a);
            const float h2 = bf16_val(bf16_rne(fmaxf(a + B2[m], 0.f)));
            r[kOH2 + m] = h2;
            if (h2 > 0.f) mask2 |= 1ull << m;
            y = fmaf(W3[m], h2, y);
        }
        y += par[kOffB3];
        const float d = y - tgt[s];
        lsum = d * d;
        const float dy = 2.f * d / (float)n;
        r[kODY] = dy;
        float dh2[kMlpHid];
#pragma unroll
        for (int m = 0; m < kMlpHid; ++m) {
            dh2[m] = ((mask2 >> m) & 1ull) ? dy * W3[m] : 0.f;
            r[kODH2 + m] = dh2[m];
        }
        for (int k = 0; k < kMlpHid; ++k) {
            float a = 0.f;
            if (h1[k] > 0.f) {
#pragma unroll
                for (int m = 0; m < kMlpHid; ++m) a = fmaf(W2[m * kMlpHid + k], dh2[m], a);
            }
            r[kODH1 + k] = a;
        }
    }
    // loss partial of this block (fixed-order reduction)
    for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, kWave);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / kWave] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        float a = 0.f;
        for (int w = 0; w < kT / kWave; ++w) a += red[w];
        lpart[blockIdx.x] = a;
    }
}

// weight gradients: partial[chunk][param] = sum over the chunk's samples
__global__ __launch_bounds__(kT) void mlp_wgrad_kernel(const float *__restrict__ rows, long long n,
                                                       float *__restrict__ partial)
{
    const int pi = blockIdx.x * kT + threadIdx.x;
    if (pi >= kMlpNParam) return;
    const long long per = (n + kChunks - 1) / kChunks;
    const long long s0 = blockIdx.y * per, s1 = std::min(n, s0 + per);
    float a = 0.f;
    if (pi < kOffB1) {  // W1[m][k]
        const int m = pi / kMlpIn, k = pi % kMlpIn;
        for (long long s = s0; s < s1; ++s) a = fmaf(rows[s * kRow + kODH1 + m], rows[s * kRow + kOXB + k], a);
    } else if (pi < kOffW2) {  // b1[m]
        const int m = pi - kOffB1;
        for (long long s = s0; s < s1; ++s) a += rows[s * kRow + kODH1 + m];
    } else if (pi < kOffB2) {  // W2[m][k]
        const int m = (pi - kOffW2) / kMlpHid, k = (pi - kOffW2) % kMlpHid;
        for (long long s = s0; s < s1; ++s) a = fmaf(rows[s * kRow + kODH2 + m], rows[s * kRow + kOH1 + k], a);
    } else if (pi < kOffW3) {  // b2[m]
        const int m = pi - kOffB2;
        for (long long s = s0; s < s1; ++s) a += rows[s * kRow + kODH2 + m];
    } else if (pi < kOffB3) {  // w3[m]
        const int m = pi - kOffW3;
        for (long long s = s0; s < s1; ++s) a = fmaf(rows[s * kRow + kODY], rows[s * kRow + kOH2 + m], a);
    } else {  // b3
        for (long long s = s0; s < s1; ++s) a += rows[s * kRow + kODY];
    }
    partial[(long long)blockIdx.y * kMlpNParam + pi] = a;
}

// grad = fixed-order sum of the chunk partials; loss = sum of block partials / n;
// optionally one Adam step (bias-corrected) on the masters
__global__ __launch_bounds__(kT) void mlp_reduce_adam_kernel(const float *__restrict__ partial,
                                                             const float *__restrict__ lpart, int nlp, long long n,
                                                             float *__restrict__ grad, float *__restrict__ loss,
                                                             float *__restrict__ par, float *__restrict__ mo,
                                                             float *__restrict__ vo, int adam, float lr, float b1,
                                                             float b2, float eps, float bc1, float bc2)
{
    const int pi = blockIdx.x * kT + threadIdx.x;
    if (pi == 0) {
        float a = 0.f;
        for (int i = 0; i < nlp; ++i) a += lpart[i];
        loss[0] = a / (float)n;
    }
    if (pi >= kMlpNParam) return;
    float g = 0.f;
    for (int c = 0; c < kChunks; ++c) g += partial[(long long)c * kMlpNParam + pi];
    grad[pi] = g;
    if (adam) {
        const float m1 = b1 * mo[pi] + (1.f - b1) * g;
        const float v1 = b2 * vo[pi] + (1.f - b2) * g * g;
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

pb_status refresh(pb_mlp *m, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_refresh_kernel, dim3(1), dim3(256), 0, s, m->par, m->norm, m->pack);
    PB_HIP(hipGetLastError());
    return PB_OK;
}

pb_status ensure_scratch(pb_mlp *m, long long n)
{
    if (n > m->scratch_rows) {
        if (m->scratch) PB_HIP(hipFree(m->scratch));
        m->scratch = nullptr;
        m->scratch_rows = 0;
        PB_HIP(hipMalloc(&m->scratch, (size_t)n * kRow * sizeof(float)));
        m->scratch_rows = n;
    }
    const long long nb = (n + kT - 1) / kT;
    if (nb > m->lpart_cap) {
        if (m->lpart) PB_HIP(hipFree(m->lpart));
        m->lpart = nullptr;
        m->lpart_cap = 0;
        PB_HIP(hipMalloc(&m->lpart, (size_t)nb * sizeof(float)));
        m->lpart_cap = nb;
    }
    return PB_OK;
}

pb_status run_grad(pb_mlp *m, const float *x, const float *t, long long n, hipStream_t s, int adam, float lr,
                   float b1, float b2, float eps, int step)
{
    pb_status st = ensure_scratch(m, n);
    if (st != PB_OK) return st;
    const long long nb = (n + kT - 1) / kT;
    hipLaunchKernelGGL(mlp_fwd_bwd_kernel, dim3((unsigned)nb), dim3(kT), 0, s, m->par, m->norm, x, t, n, m->scratch,
                       m->lpart);
    PB_HIP(hipGetLastError());
    hipLaunchKernelGGL(mlp_wgrad_kernel, dim3((kMlpNParam + kT - 1) / kT, kChunks), dim3(kT), 0, s, m->scratch, n,
                       m->partial);
    PB_HIP(hipGetLastError());
    const float bc1 = adam ? 1.f - std::pow(b1, (float)step) : 1.f;
    const float bc2 = adam ? 1.f - std::pow(b2, (float)step) : 1.f;
    hipLaunchKernelGGL(mlp_reduce_adam_kernel, dim3((kMlpNParam + kT - 1) / kT), dim3(kT), 0, s, m->partial, m->lpart,
                       (int)nb, n, m->grad, m->loss, m->par, m->madam, m->vadam, adam, lr, b1, b2, eps, bc1, bc2);
    PB_HIP(hipGetLastError());
    if (adam) return refresh(m, s);
    return PB_OK;
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
    const size_t nf = (size_t)kMlpNParam * 5 + 16 + (size_t)kChunks * kMlpNParam;
    const size_t bytes = nf * sizeof(float) + sizeof(MlpPack) + 4096;
    hipError_t e = hipMalloc(&m->dev, bytes);
    if (e != hipSuccess) { delete m; return hip_fail(e, "hipMalloc(mlp)"); }
    e = hipMemset(m->dev, 0, bytes);
    if (e != hipSuccess) { (void)hipFree(m->dev); delete m; return hip_fail(e, "hipMemset(mlp)"); }
    char *p = m->dev;
    auto take = [&](size_t b) { char *r = p; p += (b + 255) & ~(size_t)255; return r; };
    m->pack = reinterpret_cast<MlpPack *>(take(sizeof(MlpPack)));
    m->par = reinterpret_cast<float *>(take(kMlpNParam * sizeof(float)));
    m->madam = reinterpret_cast<float *>(take(kMlpNParam * sizeof(float)));
    m->vadam = reinterpret_cast<float *>(take(kMlpNParam * sizeof(float)));
    m->grad = reinterpret_cast<float *>(take(kMlpNParam * sizeof(float)));
    m->norm = reinterpret_cast<float *>(take(16 * sizeof(float)));
    m->loss = reinterpret_cast<float *>(take(sizeof(float)));
    m->partial = reinterpret_cast<float *>(take((size_t)kChunks * kMlpNParam * sizeof(float)));
    *out = m;
    return PB_OK;
    PB_API_END
}

pb_status pb_mlp_destroy(pb_mlp *m)
{
    PB_API_BEGIN
    if (!m) return PB_OK;
    if (m->scratch) (void)hipFree(m->scratch);
    if (m->lpart) (void)hipFree(m->lpart);
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

pb_status pb_mlp_grad(const pb_mlp *m, const void *x, const void *t, int64_t n, void *grad, void *loss, void *stream)
{
    PB_API_BEGIN
    if (!m || !x || !t || !grad || !loss) { set_error("NULL argument"); return PB_EINVAL; }
    if (n < 1) { set_error("n must be >= 1"); return PB_EINVAL; }
    pb_mlp *mm = const_cast<pb_mlp *>(m);
    hipStream_t s = static_cast<hipStream_t>(stream);
    pb_status st = run_grad(mm, static_cast<const float *>(x), static_cast<const float *>(t), n, s, 0, 0.f, 0.f, 0.f,
                            0.f, 1);
    if (st != PB_OK) return st;
    PB_HIP(hipMemcpyAsync(grad, mm->grad, kMlpNParam * sizeof(float), hipMemcpyDeviceToDevice, s));
    PB_HIP(hipMemcpyAsync(loss, mm->loss, sizeof(float), hipMemcpyDeviceToDevice, s));
    return PB_OK;
    PB_API_END
}

pb_status pb_mlp_train_step(pb_mlp *m, const void *x, const void *t, int64_t n, float lr, float beta1, float beta2,
                            float eps, int32_t step, void *loss, void *stream)
{
    PB_API_BEGIN
    if (!m || !x || !t) { set_error("NULL argument"); return PB_EINVAL; }
    if (n < 1) { set_error("n must be >= 1"); return PB_EINVAL; }
    if (step < 1) { set_error("step must be >= 1"); return PB_EINVAL; }
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f)) {
        set_error("bad Adam hyper-parameters");
        return PB_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    pb_status st = run_grad(m, static_cast<const float *>(x), static_cast<const float *>(t), n, s, 1, lr, beta1, beta2,
                            eps, step);
    if (st != PB_OK) return st;
    if (loss) PB_HIP(hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToDevice, s));
    return PB_OK;
    PB_API_END
}

}  // extern "C"

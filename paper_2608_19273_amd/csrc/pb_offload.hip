// pb_offload.hip -- offload mode: pure kernel offloading of K patches handed
// over as K separate host chunks (each patch with its halo, per-point order:
// the N unknowns of one point contiguous, points x fastest over the
// (p+2h)^3 box; paper Sec. II-B), returned as K chunks of the updated
// interiors (p^3 points, same order).  The gather prologue and scatter
// epilogue of Sec. III-C, Eq. (4) become the packing of the chunks into
// pinned staging and back; the host-device mapping of Sec. III-D becomes a
// two-slot copy pipeline (Sec. IV: ExaHyPE keeps no cell data on the
// device, so transfers are part of every call).
//
// Pipeline: batches of up to B patches alternate between two slots, each
// with pinned input/output staging, device buffers and its own stream.
// While the GPU copies and computes the batch of one slot, the host unpacks
// the finished batch of the other slot and packs the next one into it; the
// host-to-device and device-to-host copies of the two slots use the two
// copy engines.
//
// Kernel: one work-group per patch, one thread per (x, y) column (p <= 16),
// marching up z over a three-plane LDS ring of the (p+2)^2 inner box (Q and
// the per-point aux).  Each plane of the chunk is loaded point by point (one
// thread per point, its N unknowns contiguous); edges and corners of the box
// are never read.  The cell update is the difference form of the resident
// FV kernels.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "pb_common.h"
#include "pb_physics.h"

namespace pb {

namespace {

template <class Ph>
__global__ __launch_bounds__(kFvThreads) void fv_offload_kernel(const double *__restrict__ in,
                                                                 double *__restrict__ out,
                                                                 const double *__restrict__ dxs, int p, int h,
                                                                 double dt, Ph ph)
{
    constexpr int N = Ph::N, A = Ph::A, W = N + A, AA = A > 0 ? A : 1;
    extern __shared__ double ring[];   // [3][W][(p+2)^2]
    const int k = blockIdx.x, t = threadIdx.x;
    const int pe = p + 2, Pl = pe * pe, pb = p + 2 * h;
    const double *chunk = in + (long long)k * pb * pb * pb * N;
    double *dst = out + (long long)k * p * p * p * N;
    const double hr = 0.5 * dt / dxs[k];

    // inner-box plane zz in [-1, p] into ring slot (zz + 1) % 3
    auto load_plane = [&](int zz) {
        double *r = ring + ((zz + 1) % 3) * W * Pl;
        const bool zin = zz >= 0 && zz < p;
        for (int pt = t; pt < Pl; pt += blockDim.x) {
            const int xx = pt % pe - 1, yy = pt / pe - 1;
            const bool xin = xx >= 0 && xx < p, yin = yy >= 0 && yy < p;
            if ((!xin && !yin) || (!zin && !(xin && yin))) continue;   // edges and corners: never read
            const double *src = chunk + ((long long)((zz + h) * pb + (yy + h)) * pb + (xx + h)) * N;
            double q[N], a[AA], e[1] = {0.0};
#pragma unroll
            for (int v = 0; v < N; ++v) q[v] = src[v];
            ph.aux(q, e, a);
#pragma unroll
            for (int v = 0; v < N; ++v) r[v * Pl + pt] = q[v];
#pragma unroll
            for (int j = 0; j < A; ++j) r[(N + j) * Pl + pt] = a[j];
        }
    };

    const bool active = t < p * p;
    const int x = active ? t % p : 0, y = active ? t / p : 0;
    const int c = (y + 1) * pe + (x + 1);
    load_plane(-1);
    load_plane(0);
    for (int z = 0; z < p; ++z) {
        load_plane(z + 1);   // into the slot of plane z - 2, free since the last barrier
        lds_barrier();       // (no thread reads what another writes to global memory)
        if (active) {
            const double *rm = ring + (z % 3) * W * Pl, *r0 = ring + ((z + 1) % 3) * W * Pl,
                         *rp = ring + ((z + 2) % 3) * W * Pl;
            double qc[N], ac[AA], acc2[N];
#pragma unroll
            for (int v = 0; v < N; ++v) { qc[v] = r0[v * Pl + c]; acc2[v] = 0.0; }
#pragma unroll
            for (int j = 0; j < A; ++j) ac[j] = r0[(N + j) * Pl + c];
            auto dirn = [&](auto D, const double *lo, int cl, const double *hi, int ch) {
                double qL[N], aL[AA], qR[N], aR[AA];
#pragma unroll
                for (int v = 0; v < N; ++v) { qL[v] = lo[v * Pl + cl]; qR[v] = hi[v * Pl + ch]; }
#pragma unroll
                for (int j = 0; j < A; ++j) { aL[j] = lo[(N + j) * Pl + cl]; aR[j] = hi[(N + j) * Pl + ch]; }
                rusanov_pair2<Ph, decltype(D)::value>(ph, qL, aL, qc, ac, qR, aR, acc2);
            };
            dirn(std::integral_constant<int, 0>(), r0, c - 1, r0, c + 1);
            dirn(std::integral_constant<int, 1>(), r0, c - pe, r0, c + pe);
            dirn(std::integral_constant<int, 2>(), rm, c, rp, c);
            double S[N];
            if (Ph::kSrc) {
                ph.source(qc, ac, S);
            } else {
#pragma unroll
                for (int v = 0; v < N; ++v) S[v] = 0.0;
            }
            double *o = dst + ((long long)(z * p + y) * p + x) * N;
#pragma unroll
            for (int v = 0; v < N; ++v) o[v] = qc[v] - hr * acc2[v] + dt * S[v];
        }
        lds_barrier();   // the slot of plane z - 1 is free for the next load
    }
}

double ms_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// run f(i) for i in [0, n) on up to 8 host threads (inline when small; 16
// threads measured slower on a 16-core host share)
template <class F>
void parallel_for(int n, size_t bytes, F &&f)
{
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int T = (int)std::min<unsigned>(8u, hw);
    if (T <= 1 || n < 2 || bytes < (1u << 20)) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    std::vector<std::thread> th;
    try {
        th.reserve(T);
    } catch (...) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    const int per = (n + T - 1) / T;
    for (int w = 0; w < T; ++w) {
        const int a = w * per, b = std::min(n, a + per);
        if (a >= b) break;
        try {
            th.emplace_back([&f, a, b] {
                for (int i = a; i < b; ++i) f(i);
            });
        } catch (...) {
            for (int i = a; i < b; ++i) f(i);   // no thread for this range: run it here
        }
    }
    for (auto &x : th) x.join();
}

}  // namespace
}  // namespace pb

using namespace pb;

struct pb_offload {
    int p = 0, h = 0, pde = 0, N = 0;
    std::vector<double> params;
    int B = 0;                  // patches per batch
    size_t in_pp = 0, out_pp = 0;   // doubles per patch in and out
    struct Slot {
        double *h_in = nullptr, *h_out = nullptr, *h_dx = nullptr;
        double *d_in = nullptr, *d_out = nullptr, *d_dx = nullptr;
        hipStream_t s = nullptr;
        hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
        int k0 = 0, n = 0;
        bool busy = false;
    } slot[2];
};

namespace {

void free_offload(pb_offload *o)
{
    for (auto &S : o->slot) {
        if (S.s) (void)hipStreamSynchronize(S.s);
        if (S.h_in) (void)hipHostFree(S.h_in);
        if (S.h_out) (void)hipHostFree(S.h_out);
        if (S.h_dx) (void)hipHostFree(S.h_dx);
        if (S.d_in) (void)hipFree(S.d_in);
        if (S.d_out) (void)hipFree(S.d_out);
        if (S.d_dx) (void)hipFree(S.d_dx);
        for (auto &e : S.ev)
            if (e) (void)hipEventDestroy(e);
        if (S.s) (void)hipStreamDestroy(S.s);
    }
    delete o;
}

pb_status launch_offload(const pb_offload *o, const pb_offload::Slot &S, double dt)
{
    const int W = o->N + (o->pde == PB_PDE_EULER ? 3 : 0);
    const size_t lds = (size_t)3 * W * (o->p + 2) * (o->p + 2) * sizeof(double);
    const double *pr = o->params.data();
    switch (o->pde) {
    case PB_PDE_ADVECTION_F:
        hipLaunchKernelGGL(fv_offload_kernel<AdvF>, dim3(S.n), dim3(kFvThreads), lds, S.s, S.d_in, S.d_out, S.d_dx,
                           o->p, o->h, dt, AdvF{{pr[0], pr[1], pr[2]}, pr[3]});
        break;
    case PB_PDE_ADVECTION_B:
        hipLaunchKernelGGL(fv_offload_kernel<AdvB>, dim3(S.n), dim3(kFvThreads), lds, S.s, S.d_in, S.d_out, S.d_dx,
                           o->p, o->h, dt, AdvB{{pr[0], pr[1], pr[2]}, pr[3]});
        break;
    default:
        hipLaunchKernelGGL(fv_offload_kernel<Euler<3>>, dim3(S.n), dim3(kFvThreads), lds, S.s, S.d_in, S.d_out,
                           S.d_dx, o->p, o->h, dt, Euler<3>{pr[0]});
        break;
    }
    PB_HIP(hipGetLastError());
    return PB_OK;
}

// wait for a slot's batch, add its copy and kernel times, unpack its output
pb_status finish_slot(pb_offload *o, pb_offload::Slot &S, double *const *out_chunks, pb_offload_timing &tm)
{
    if (!S.busy) return PB_OK;
    S.busy = false;
    PB_HIP(hipEventSynchronize(S.ev[3]));
    float a = 0.f, b = 0.f, c = 0.f;
    PB_HIP(hipEventElapsedTime(&a, S.ev[0], S.ev[1]));
    PB_HIP(hipEventElapsedTime(&b, S.ev[1], S.ev[2]));
    PB_HIP(hipEventElapsedTime(&c, S.ev[2], S.ev[3]));
    tm.h2d_ms += a;
    tm.compute_ms += b;
    tm.d2h_ms += c;
    const auto t0 = std::chrono::steady_clock::now();
    const size_t n = o->out_pp;
    parallel_for(S.n, (size_t)S.n * n * sizeof(double), [&](int i) {
        std::memcpy(out_chunks[S.k0 + i], S.h_out + (size_t)i * n, n * sizeof(double));
    });
    tm.unpack_ms += ms_since(t0);
    return PB_OK;
}

}  // namespace

extern "C" {

pb_status pb_offload_create(const pb_offload_desc *d, pb_offload **out)
{
    PB_API_BEGIN
    if (!d || !out) { set_error("NULL argument"); return PB_EINVAL; }
    *out = nullptr;
    if (d->dim != 3) { set_error("offload mode: dim 3 only"); return PB_EUNSUPPORTED; }
    if (d->p < 1 || d->p > kFvPmax) { set_error("offload mode: 1 <= p <= 16"); return PB_EINVAL; }
    if (d->halo < 1 || d->halo > 8) { set_error("offload mode: 1 <= halo <= 8"); return PB_EINVAL; }
    if (d->batch_patches < 0) { set_error("batch_patches must be >= 0"); return PB_EINVAL; }
    int need_n = 0, need_prm = 0;
    switch (d->pde) {
    case PB_PDE_ADVECTION_F:
    case PB_PDE_ADVECTION_B: need_n = 1; need_prm = 4; break;
    case PB_PDE_EULER: need_n = 5; need_prm = 1; break;
    default: set_error("offload mode: ADVECTION_F, ADVECTION_B or EULER"); return PB_EUNSUPPORTED;
    }
    if (d->n_unknowns != need_n) { set_error("offload mode: n_unknowns does not match the PDE"); return PB_EINVAL; }
    if (!d->pde_params || d->n_pde_params < need_prm) { set_error("pde_params missing"); return PB_EINVAL; }
    for (int i = 0; i < need_prm; ++i)
        if (!std::isfinite(d->pde_params[i])) { set_error("pde_params must be finite"); return PB_EINVAL; }
    if (d->pde == PB_PDE_EULER && !(d->pde_params[0] > 1.0)) { set_error("gamma must be > 1"); return PB_EINVAL; }
    pb_offload *o = new (std::nothrow) pb_offload();
    if (!o) { set_error("out of host memory"); return PB_ENOMEM; }
    o->p = d->p;
    o->h = d->halo;
    o->pde = d->pde;
    o->N = d->n_unknowns;
    o->params.assign(d->pde_params, d->pde_params + need_prm);
    const size_t pb_ = (size_t)(d->p + 2 * d->halo);
    o->in_pp = pb_ * pb_ * pb_ * o->N;
    o->out_pp = (size_t)d->p * d->p * d->p * o->N;
    o->B = d->batch_patches > 0 ? d->batch_patches
                                : (int)std::max<size_t>(1, (32u << 20) / (o->in_pp * sizeof(double)));
    for (auto &S : o->slot) {
        hipError_t e = hipHostMalloc((void **)&S.h_in, (size_t)o->B * o->in_pp * sizeof(double), hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void **)&S.h_out, (size_t)o->B * o->out_pp * sizeof(double), hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void **)&S.h_dx, (size_t)o->B * sizeof(double), hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc((void **)&S.d_in, (size_t)o->B * o->in_pp * sizeof(double));
        if (e == hipSuccess) e = hipMalloc((void **)&S.d_out, (size_t)o->B * o->out_pp * sizeof(double));
        if (e == hipSuccess) e = hipMalloc((void **)&S.d_dx, (size_t)o->B * sizeof(double));
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&S.s, hipStreamNonBlocking);
        for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventCreate(&S.ev[i]);
        if (e != hipSuccess) {
            free_offload(o);
            return hip_fail(e, "pb_offload_create");
        }
    }
    *out = o;
    return PB_OK;
    PB_API_END
}

pb_status pb_offload_destroy(pb_offload *o)
{
    PB_API_BEGIN
    if (!o) { set_error("offload object is NULL"); return PB_EINVAL; }
    free_offload(o);
    return PB_OK;
    PB_API_END
}

pb_status pb_offload_fv_step(pb_offload *o, int32_t K, const double *const *in_chunks, double *const *out_chunks,
                             const double *dx, double dt, pb_offload_timing *timing)
{
    PB_API_BEGIN
    if (!o) { set_error("offload object is NULL"); return PB_EINVAL; }
    if (K < 0) { set_error("K must be >= 0"); return PB_EINVAL; }
    if (!(dt > 0.0) || !std::isfinite(dt)) { set_error("dt must be finite and > 0"); return PB_EINVAL; }
    pb_offload_timing tm{};
    const auto t_start = std::chrono::steady_clock::now();
    if (K > 0) {
        if (!in_chunks || !out_chunks || !dx) { set_error("NULL chunk or dx array"); return PB_EINVAL; }
        for (int k = 0; k < K; ++k) {
            if (!in_chunks[k] || !out_chunks[k]) { set_error("NULL chunk " + std::to_string(k)); return PB_EINVAL; }
            if (!(dx[k] > 0.0) || !std::isfinite(dx[k])) { set_error("dx must be finite and > 0"); return PB_EINVAL; }
        }
    }
    pb_status st = PB_OK;
    const int nb = (K + o->B - 1) / o->B;
    for (int i = 0; i < nb && st == PB_OK; ++i) {
        pb_offload::Slot &S = o->slot[i & 1];
        if ((st = finish_slot(o, S, out_chunks, tm)) != PB_OK) break;
        S.k0 = i * o->B;
        S.n = std::min(o->B, K - S.k0);
        const auto t0 = std::chrono::steady_clock::now();
        const size_t n = o->in_pp;
        parallel_for(S.n, (size_t)S.n * n * sizeof(double), [&](int j) {
            std::memcpy(S.h_in + (size_t)j * n, in_chunks[S.k0 + j], n * sizeof(double));
        });
        for (int j = 0; j < S.n; ++j) S.h_dx[j] = dx[S.k0 + j];
        tm.pack_ms += ms_since(t0);
        hipError_t e = hipEventRecord(S.ev[0], S.s);
        if (e == hipSuccess) e = hipMemcpyAsync(S.d_in, S.h_in, (size_t)S.n * n * sizeof(double), hipMemcpyHostToDevice, S.s);
        if (e == hipSuccess) e = hipMemcpyAsync(S.d_dx, S.h_dx, (size_t)S.n * sizeof(double), hipMemcpyHostToDevice, S.s);
        if (e == hipSuccess) e = hipEventRecord(S.ev[1], S.s);
        if (e != hipSuccess) { st = hip_fail(e, "pb_offload_fv_step (copy in)"); break; }
        if ((st = launch_offload(o, S, dt)) != PB_OK) break;
        e = hipEventRecord(S.ev[2], S.s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(S.h_out, S.d_out, (size_t)S.n * o->out_pp * sizeof(double), hipMemcpyDeviceToHost, S.s);
        if (e == hipSuccess) e = hipEventRecord(S.ev[3], S.s);
        if (e != hipSuccess) { st = hip_fail(e, "pb_offload_fv_step (copy out)"); break; }
        S.busy = true;
        ++tm.batches;
    }
    // drain: the batch started first finishes first
    for (int j = 0; j < 2; ++j) {
        pb_offload::Slot &S = o->slot[(nb + j) & 1];
        if (st == PB_OK) {
            st = finish_slot(o, S, out_chunks, tm);
        } else {
            (void)hipStreamSynchronize(S.s);
            S.busy = false;
        }
    }
    tm.total_ms = ms_since(t_start);
    if (timing) *timing = tm;
    return st;
    PB_API_END
}

}  // extern "C"

// pb_fv.hip -- fused first-order Rusanov finite-volume step on a patch batch
// (the FV composition of paper Sec. II-A, Eq. (3): source term, face fluxes
// from the two adjacent cell values, update), one launch per time step.
//
// Work decomposition (MI355X): a work-group of 256 threads owns one z-slab of
// one patch and marches through it plane by plane.  Thread t owns column
// (x, y) = (t % p, t / p).  For each plane the work-group
//   1. stores its cells' Q and per-cell aux (1/rho, p, c ...) in LDS, and the
//      4p face-halo cells of the plane, read straight from the face
//      neighbours' interiors (this is the halo gather, fused into the tile
//      load: no halo array ever exists in HBM);
//   2. after one barrier, evaluates the x and y face fluxes from LDS and the
//      z face flux from registers (the lower z face is carried over from the
//      previous plane, so every z face is evaluated once);
//   3. updates the cell, stores it, and (CFL mode) folds the largest speed of
//      the new state into a per-thread maximum.
// LDS is double-buffered by plane parity, so one barrier per plane suffices.
// At the end the work-group reduces its maxima (wave shuffle, then LDS) and
// does one atomicMax per direction on the IEEE bits (exact and
// order-independent for non-negative doubles); the last work-group to finish
// turns the maxima into the next step's dt, so dt never leaves the device.
#include <algorithm>
#include <type_traits>

#include "pb_common.h"
#include "pb_physics.h"

namespace pb {

namespace {

template <class Ph, typename T>
__device__ __forceinline__ void load_cell(const T *__restrict__ q, const double *__restrict__ ex,
                                          long long off, long long C, long long c, double *out,
                                          double *e)
{
    constexpr int N = Ph::N;
    const T *base = q + off * N + c;
#pragma unroll
    for (int v = 0; v < N; ++v) out[v] = (double)base[(long long)v * C];
    if (Ph::E) e[0] = ex[off + c];
}

template <class Ph, int DIM>
__device__ __forceinline__ void cell_speeds(const Ph &ph, const double *q, const double *a,
                                            double *lm)
{
    lm[0] = fmax(lm[0], ph.template eig<0>(q, a));
    lm[1] = fmax(lm[1], ph.template eig<1>(q, a));
    if (DIM == 3) lm[2] = fmax(lm[2], ph.template eig<2>(q, a));
}

// work-group max of lm[0..DIM) -> atomicMax into ctrl->lam; the last
// work-group of the launch writes dt = cfl / sum_d(Lambda_d / dx_min) into
// ctrl->dt[slot_out] and clears the accumulators for the next launch.
template <int DIM>
__device__ __forceinline__ void finish_lambda(Ctrl *ctrl, const double *lm, int n_units, int slot_out,
                                              double cfl, double dxmin)
{
    __shared__ double red[3][kFvThreads / kWave];
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const double m = wave_max(lm[d]);
        if (lane == 0) red[d][w] = m;
    }
    __syncthreads();
    if (t == 0) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            double m = red[d][0];
            for (int i = 1; i < (int)(blockDim.x / kWave); ++i) m = fmax(m, red[d][i]);
            atomicMax(&ctrl->lam[d], dbits(m));
        }
        __threadfence();
        const unsigned prev = atomicAdd(&ctrl->done, 1u);
        if (prev == (unsigned)n_units - 1u) {
            __threadfence();
            double den = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                const double L = __longlong_as_double((long long)atomicAdd(&ctrl->lam[d], 0ull));
                den += L / dxmin;
            }
            const double dt = cfl / den;
            ctrl->dt[slot_out] = dt;
            ctrl->last_dt = dt;
#pragma unroll
            for (int d = 0; d < 3; ++d) atomicExch(&ctrl->lam[d], 0ull);
            atomicExch(&ctrl->done, 0u);
        }
    }
}

}  // namespace

template <class Ph, int DIM, typename T, bool kLam>
__global__ __launch_bounds__(kFvThreads) void fv_step_kernel(
    const T *__restrict__ qin, T *__restrict__ qout, const double *__restrict__ ex,
    const PatchDev *__restrict__ patches, int n_units, int n_slabs, int slab, int remap,
    Ctrl *__restrict__ ctrl, int slot_in, double dt_fixed, double cfl, double dxmin, Ph ph)
{
    constexpr int N = Ph::N, A = Ph::A, W = N + A;
    constexpr int PH = kFvPmax + 2;
    __shared__ double lds[2][W][PH * PH];

    const int t = threadIdx.x;
    const int unit = remap ? xcd_remap(blockIdx.x, n_units) : (int)blockIdx.x;
    const int k = unit / n_slabs, sl = unit - k * n_slabs;
    const PatchDev P = patches[k];
    const int p = P.p;
    const long long C = (DIM == 3) ? (long long)p * p * p : (long long)p * p;
    long long onb[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) onb[f] = (f < 2 * DIM) ? patches[P.nbr[f]].off : P.off;

    const int z0 = (DIM == 3) ? sl * slab : 0;
    const int z1 = (DIM == 3) ? min(p, z0 + slab) : 1;
    // a slab can start beyond the last plane of a patch smaller than the
    // batch maximum: such a unit only takes part in the reductions
    const bool active = (z0 < p) && t < p * p;
    const int x = active ? t % p : 0, y = active ? t / p : 0;
    const double dt = dt_fixed > 0.0 ? dt_fixed : ctrl->dt[slot_in];
    const double r = dt * P.inv_dx;
    const int li = (y + 1) * PH + (x + 1);

    double qc[N], ac[A > 0 ? A : 1], qn[N], an[A > 0 ? A : 1], fzl[N], dzl[N], e[1];
    double lm[3] = {0.0, 0.0, 0.0};
    bool bad = false;

    if (active) {
        load_cell<Ph>(qin, ex, P.off, C, ((long long)z0 * p + y) * p + x, qc, e);
        ph.aux(qc, e, ac);
        if (DIM == 3) {
            double qm[N], am[A > 0 ? A : 1];
            const long long om = (z0 == 0) ? onb[4] : P.off;
            const int zm = (z0 == 0) ? p - 1 : z0 - 1;
            load_cell<Ph>(qin, ex, om, C, ((long long)zm * p + y) * p + x, qm, e);
            ph.aux(qm, e, am);
            rusanov_face<Ph, (DIM == 3 ? 2 : 1)>(ph, qm, am, qc, ac, fzl, dzl);
        }
    }

    for (int z = z0; z < z1; ++z) {
        double(*buf)[PH * PH] = lds[z & 1];
        if (DIM == 3 && active) {
            const long long on = (z + 1 == p) ? onb[5] : P.off;
            const int zn = (z + 1 == p) ? 0 : z + 1;
            load_cell<Ph>(qin, ex, on, C, ((long long)zn * p + y) * p + x, qn, e);
            ph.aux(qn, e, an);
        }
        if (active) {
#pragma unroll
            for (int v = 0; v < N; ++v) buf[v][li] = qc[v];
#pragma unroll
            for (int a = 0; a < A; ++a) buf[N + a][li] = ac[a];
        }
        if (t < 4 * p) {
            // face-halo cell of this plane, gathered from the face neighbour
            const int side = t / p, j = t - side * p;
            int hx, hy, sx, sy;
            long long o;
            if (side == 0)      { hx = -1; hy = j;  sx = p - 1; sy = j;     o = onb[0]; }
            else if (side == 1) { hx = p;  hy = j;  sx = 0;     sy = j;     o = onb[1]; }
            else if (side == 2) { hx = j;  hy = -1; sx = j;     sy = p - 1; o = onb[2]; }
            else                { hx = j;  hy = p;  sx = j;     sy = 0;     o = onb[3]; }
            double hq[N], ha[A > 0 ? A : 1];
            load_cell<Ph>(qin, ex, o, C, ((long long)z * p + sy) * p + sx, hq, e);
            ph.aux(hq, e, ha);
            const int hi = (hy + 1) * PH + (hx + 1);
#pragma unroll
            for (int v = 0; v < N; ++v) buf[v][hi] = hq[v];
#pragma unroll
            for (int a = 0; a < A; ++a) buf[N + a][hi] = ha[a];
        }
        __syncthreads();
        if (active) {
            double acc[N];
#pragma unroll
            for (int v = 0; v < N; ++v) acc[v] = 0.0;
            double qs[N], as[A > 0 ? A : 1], F0[N], D0[N], F1[N], D1[N];
            // x faces
#pragma unroll
            for (int v = 0; v < N; ++v) qs[v] = buf[v][li - 1];
#pragma unroll
            for (int a = 0; a < A; ++a) as[a] = buf[N + a][li - 1];
            rusanov_face<Ph, 0>(ph, qs, as, qc, ac, F0, D0);
#pragma unroll
            for (int v = 0; v < N; ++v) qs[v] = buf[v][li + 1];
#pragma unroll
            for (int a = 0; a < A; ++a) as[a] = buf[N + a][li + 1];
            rusanov_face<Ph, 0>(ph, qc, ac, qs, as, F1, D1);
#pragma unroll
            for (int v = 0; v < N; ++v) acc[v] += (F1[v] - F0[v]) + (D1[v] + D0[v]);
            // y faces
#pragma unroll
            for (int v = 0; v < N; ++v) qs[v] = buf[v][li - PH];
#pragma unroll
            for (int a = 0; a < A; ++a) as[a] = buf[N + a][li - PH];
            rusanov_face<Ph, 1>(ph, qs, as, qc, ac, F0, D0);
#pragma unroll
            for (int v = 0; v < N; ++v) qs[v] = buf[v][li + PH];
#pragma unroll
            for (int a = 0; a < A; ++a) as[a] = buf[N + a][li + PH];
            rusanov_face<Ph, 1>(ph, qc, ac, qs, as, F1, D1);
#pragma unroll
            for (int v = 0; v < N; ++v) acc[v] += (F1[v] - F0[v]) + (D1[v] + D0[v]);
            // z faces: lower one carried from the previous plane
            if (DIM == 3) {
                rusanov_face<Ph, (DIM == 3 ? 2 : 1)>(ph, qc, ac, qn, an, F1, D1);
#pragma unroll
                for (int v = 0; v < N; ++v) {
                    acc[v] += (F1[v] - fzl[v]) + (D1[v] + dzl[v]);
                    fzl[v] = F1[v];
                    dzl[v] = D1[v];
                }
            }
            double S[N];
            if (Ph::kSrc) {
                ph.source(qc, ac, S);
            } else {
#pragma unroll
                for (int v = 0; v < N; ++v) S[v] = 0.0;
            }
            double qw[N];
            T *dst = qout + P.off * N + ((long long)z * p + y) * p + x;
#pragma unroll
            for (int v = 0; v < N; ++v) {
                const double nv = qc[v] - r * acc[v] + dt * S[v];
                const T st = (T)nv;
                dst[(long long)v * C] = st;
                qw[v] = (double)st;
                bad |= !isfinite(qw[v]);
            }
            if (kLam) {
                double aw[A > 0 ? A : 1];
                ph.aux(qw, e, aw);
                cell_speeds<Ph, DIM>(ph, qw, aw, lm);
            }
        }
        if (DIM == 3) {
#pragma unroll
            for (int v = 0; v < N; ++v) qc[v] = qn[v];
#pragma unroll
            for (int a = 0; a < A; ++a) ac[a] = an[a];
        }
    }
    if (__syncthreads_or(bad) && t == 0) atomicAdd(&ctrl->nonfinite, 1ull);
    if (kLam) finish_lambda<DIM>(ctrl, lm, n_units, slot_in ^ 1, cfl, dxmin);
}

// Largest speeds of the current state (first step of a call in CFL mode):
// one work-group per patch, dt written into ctrl->dt[0].
template <class Ph, int DIM, typename T>
__global__ __launch_bounds__(kFvThreads) void fv_lambda_kernel(const T *__restrict__ q,
                                                               const PatchDev *__restrict__ patches,
                                                               int n_units, Ctrl *__restrict__ ctrl,
                                                               double cfl, double dxmin, Ph ph)
{
    constexpr int N = Ph::N, A = Ph::A;
    const PatchDev P = patches[blockIdx.x];
    const int p = P.p;
    const long long C = (DIM == 3) ? (long long)p * p * p : (long long)p * p;
    double lm[3] = {0.0, 0.0, 0.0};
    double e[1] = {0.0};
    for (long long c = threadIdx.x; c < C; c += blockDim.x) {
        double qc[N], ac[A > 0 ? A : 1];
        load_cell<Ph>(q, (const double *)nullptr, P.off, C, c, qc, e);
        ph.aux(qc, e, ac);
        cell_speeds<Ph, DIM>(ph, qc, ac, lm);
    }
    finish_lambda<DIM>(ctrl, lm, n_units, 0, cfl, dxmin);
}

__global__ void ctrl_init_kernel(Ctrl *ctrl)
{
    // zero the whole control block with vector stores (no memset node, so
    // this is safe inside captured graphs)
    unsigned long long *w = reinterpret_cast<unsigned long long *>(ctrl);
    for (int i = threadIdx.x; i < (int)(sizeof(Ctrl) / 8); i += blockDim.x) w[i] = 0ull;
}

// ------------------------------------------------------------------ host --

namespace {

template <class Ph, int DIM, typename T>
pb_status launch_typed(pb_batch *b, const Ph &ph, const void *qin, void *qout, int slot_in,
                       double dt_fixed, double cfl, hipStream_t s)
{
    const int slab = (DIM == 3) ? (b->fv_slab > 0 ? std::min(b->fv_slab, b->pmax) : b->pmax) : 1;
    const int n_slabs = (DIM == 3) ? (b->pmax + slab - 1) / slab : 1;
    const int n_units = b->K * n_slabs;
    Ctrl *ctrl = reinterpret_cast<Ctrl *>(b->ws);
    const T *qi = static_cast<const T *>(qin);
    T *qo = static_cast<T *>(qout);
    const double *ex = Ph::E ? reinterpret_cast<const double *>(b->ws + ws_layout(b->pde, b->total_cells, b->N, b->storage).pres)
                             : nullptr;
    if constexpr (Ph::E > 0) {  // SRHD: dt comes from the con2prim pass
        hipLaunchKernelGGL((fv_step_kernel<Ph, DIM, T, false>), dim3(n_units), dim3(kFvThreads), 0, s, qi, qo,
                           ex, b->d_patches, n_units, n_slabs, slab, b->fv_xcd_remap, ctrl, slot_in,
                           dt_fixed, cfl, b->dxmin, ph);
    } else {
        if (dt_fixed > 0.0)
            hipLaunchKernelGGL((fv_step_kernel<Ph, DIM, T, false>), dim3(n_units), dim3(kFvThreads), 0, s, qi,
                               qo, ex, b->d_patches, n_units, n_slabs, slab, b->fv_xcd_remap, ctrl, slot_in,
                               dt_fixed, cfl, b->dxmin, ph);
        else
            hipLaunchKernelGGL((fv_step_kernel<Ph, DIM, T, true>), dim3(n_units), dim3(kFvThreads), 0, s, qi,
                               qo, ex, b->d_patches, n_units, n_slabs, slab, b->fv_xcd_remap, ctrl, slot_in,
                               dt_fixed, cfl, b->dxmin, ph);
    }
    PB_HIP(hipGetLastError());
    return PB_OK;
}

template <class Ph, int DIM, typename T>
pb_status launch_lambda_typed(pb_batch *b, const Ph &ph, const void *q, double cfl, hipStream_t s)
{
    Ctrl *ctrl = reinterpret_cast<Ctrl *>(b->ws);
    hipLaunchKernelGGL((fv_lambda_kernel<Ph, DIM, T>), dim3(b->K), dim3(kFvThreads), 0, s,
                       static_cast<const T *>(q), b->d_patches, b->K, ctrl, cfl, b->dxmin, ph);
    PB_HIP(hipGetLastError());
    return PB_OK;
}

// dispatch on (pde, dim, storage); F is a generic lambda taking (phys, dim tag, T tag)
template <class F>
pb_status dispatch(pb_batch *b, F &&f)
{
    const bool f32 = b->storage == PB_STORE_FP32;
    const double *pr = b->params.data();
    switch (b->pde) {
    case PB_PDE_ADVECTION_F: {
        AdvF ph{{pr[0], pr[1], pr[2]}, pr[3]};
        if (b->dim == 2) return f32 ? f(ph, std::integral_constant<int, 2>(), float()) : f(ph, std::integral_constant<int, 2>(), double());
        return f32 ? f(ph, std::integral_constant<int, 3>(), float()) : f(ph, std::integral_constant<int, 3>(), double());
    }
    case PB_PDE_ADVECTION_B: {
        AdvB ph{{pr[0], pr[1], pr[2]}, pr[3]};
        if (b->dim == 2) return f32 ? f(ph, std::integral_constant<int, 2>(), float()) : f(ph, std::integral_constant<int, 2>(), double());
        return f32 ? f(ph, std::integral_constant<int, 3>(), float()) : f(ph, std::integral_constant<int, 3>(), double());
    }
    case PB_PDE_EULER:
        if (b->dim == 2) {
            Euler<2> ph{pr[0]};
            return f32 ? f(ph, std::integral_constant<int, 2>(), float()) : f(ph, std::integral_constant<int, 2>(), double());
        } else {
            Euler<3> ph{pr[0]};
            return f32 ? f(ph, std::integral_constant<int, 3>(), float()) : f(ph, std::integral_constant<int, 3>(), double());
        }
    case PB_PDE_SRHD: {
        Srhd ph{pr[0]};
        if (f32) return f(ph, std::integral_constant<int, 3>(), float());
        return f(ph, std::integral_constant<int, 3>(), double());
    }
    default:
        set_error("fv_rusanov_step: PDE not supported by the finite-volume kernel");
        return PB_EUNSUPPORTED;
    }
}

}  // namespace

pb_status launch_fv_step(pb_batch *b, const void *qin, void *qout, int slot_in, double dt_fixed,
                         double cfl, hipStream_t s)
{
    return dispatch(b, [&](const auto &ph, auto dimc, auto tt) -> pb_status {
        using Ph = std::decay_t<decltype(ph)>;
        using T = decltype(tt);
        constexpr int DIM = decltype(dimc)::value;
        return launch_typed<Ph, DIM, T>(b, ph, qin, qout, slot_in, dt_fixed, cfl, s);
    });
}

pb_status launch_fv_lambda(pb_batch *b, const void *q, double cfl, hipStream_t s)
{
    return dispatch(b, [&](const auto &ph, auto dimc, auto tt) -> pb_status {
        using Ph = std::decay_t<decltype(ph)>;
        using T = decltype(tt);
        constexpr int DIM = decltype(dimc)::value;
        if constexpr (Ph::E > 0) {
            set_error("internal: SRHD speeds come from the con2prim pass");
            return PB_EINVAL;
        } else {
            return launch_lambda_typed<Ph, DIM, T>(b, ph, q, cfl, s);
        }
    });
}

pb_status launch_ctrl_init(pb_batch *b, hipStream_t s)
{
    hipLaunchKernelGGL(ctrl_init_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<Ctrl *>(b->ws));
    PB_HIP(hipGetLastError());
    return PB_OK;
}

}  // namespace pb

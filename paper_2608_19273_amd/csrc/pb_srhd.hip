// pb_srhd.hip -- the per-cell conservative-to-primitive pass of the SRHD
// finite-volume step, and the standalone con2prim entry point.
//
// The SRHD step is two launches (plus the one-work-group dt reduction):
//   1. this pass: one lane per cell recovers the pressure by the bracketed
//      FP64 Newton iteration (pb_c2p.h), seeded by the plain guess, the
//      previous step's pressure (warm) or the MLP (learned); writes p to the
//      workspace and per-work-group partials: largest speeds of Q^n (for dt),
//      Newton iterations, failures, fallbacks;
//   2. the fused Rusanov kernel (pb_fv.hip) with the SRHD functor, which
//      reads p of each cell and its face neighbours.
// Failures never stop the step; they are counted and reported by
// pb_batch_stats (a failed cell carries the last Newton iterate).
#include <algorithm>

#include "pb_c2p.h"
#include "pb_common.h"
#include "pb_mlp.h"
#include "pb_physics.h"

namespace pb {

namespace {

constexpr int kC2pThreads = 256;

// sums (and maxima) over the work-group of the per-lane statistics; lane 0 of
// wave 0 ends up with the totals
struct C2pStats {
    double lam[3];
    double iters, fails, maxit, fallbacks, cells;
};

__device__ __forceinline__ void reduce_stats(C2pStats &s)
{
    __shared__ double red[8][kC2pThreads / kWave];
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    double v[8] = {s.lam[0], s.lam[1], s.lam[2], s.iters, s.fails, s.maxit, s.fallbacks, s.cells};
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const bool mx = (r < 3 || r == 5);
        for (int o = 32; o > 0; o >>= 1) {
            const double u = __shfl_xor(v[r], o, kWave);
            v[r] = mx ? fmax(v[r], u) : v[r] + u;
        }
        if (lane == 0) red[r][w] = v[r];
    }
    __syncthreads();
    if (t == 0) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const bool mx = (r < 3 || r == 5);
            double a = red[r][0];
            for (int i = 1; i < kC2pThreads / kWave; ++i) a = mx ? fmax(a, red[r][i]) : a + red[r][i];
            v[r] = a;
        }
        s.lam[0] = v[0]; s.lam[1] = v[1]; s.lam[2] = v[2];
        s.iters = v[3]; s.fails = v[4]; s.maxit = v[5]; s.fallbacks = v[6]; s.cells = v[7];
    }
}

// guess: 0 plain, 1 learned (mlp), 2 warm (pres holds the previous pressure)
template <int GUESS>
__global__ __launch_bounds__(kC2pThreads) void srhd_c2p_kernel(
    const double *__restrict__ q, double *__restrict__ pres, const PatchDev *__restrict__ patches,
    int chunks, int n_units, double *__restrict__ part, double gam, double tol, int maxit, MlpDev mlp)
{
    const int unit = blockIdx.x;
    const int k = unit / chunks, ch = unit - k * chunks;
    const PatchDev P = patches[k];
    const long long C = (long long)P.p * P.p * P.p;
    const long long c = (long long)ch * kC2pThreads + threadIdx.x;
    const bool active = c < C;
    C2pStats s = {{0.0, 0.0, 0.0}, 0.0, 0.0, 0.0, 0.0, 0.0};
    double qv[5] = {1.0, 0.0, 0.0, 0.0, 1.0};
    if (active) {
        const double *base = q + P.off * 5 + c;
#pragma unroll
        for (int v = 0; v < 5; ++v) qv[v] = base[(long long)v * C];
    }
    const C2pIn in = c2p_setup(qv[0], qv[1], qv[2], qv[3], qv[4], gam);
    double p0 = in.hi;
    // warm: previous pressure; learned: the guess the network pass stored
    if (GUESS != 0 && active) p0 = pres[P.off + c];
    if (active) {
        C2pOut o = c2p_solve(in, gam, tol, maxit, p0);
        if (GUESS != 0 && o.status == C2P_NOTCONV) {
            const C2pOut o2 = c2p_solve(in, gam, tol, maxit, in.hi);
            s.fallbacks = 1.0;
            o.p = o2.p;
            o.status = o2.status;
            o.it += o2.it;
        }
        pres[P.off + c] = o.p;
        const Srhd ph{gam};
        double a[Srhd::A], e[1] = {o.p};
        ph.aux(qv, e, a);
        s.lam[0] = a[4];
        s.lam[1] = a[5];
        s.lam[2] = a[6];
        s.iters = o.it;
        s.fails = o.status != C2P_OK ? 1.0 : 0.0;
        s.maxit = o.it;
        s.cells = 1.0;
    }
    reduce_stats(s);
    if (threadIdx.x == 0) {
        const double v[8] = {s.lam[0], s.lam[1], s.lam[2], s.iters, s.fails, s.maxit, s.fallbacks, s.cells};
#pragma unroll
        for (int r = 0; r < 8; ++r) part[(long long)r * n_units + unit] = v[r];
    }
}

// Learned guesses: each wave loads the network once and pushes
// kGuessGroups groups of 64 cells through it (a work-group covers
// 256 * kGuessGroups cells).
constexpr int kGuessGroups = 4;

__device__ __forceinline__ double guess_of(const MlpRegs &r, const float *norm, const double *qv, bool active,
                                           double gam)
{
    const double d0[5] = {1.0, 0.0, 0.0, 0.0, 1.0};
    const double *u = active ? qv : d0;
    const C2pIn in = c2p_setup(u[0], u[1], u[2], u[3], u[4], gam);
    return mlp_guess(r, norm, in);
}

// p0 of every cell of the SRHD pass into `pres`
__global__ __launch_bounds__(kC2pThreads) void srhd_guess_kernel(const double *__restrict__ q,
                                                                 double *__restrict__ pres,
                                                                 const PatchDev *__restrict__ patches, int gchunks,
                                                                 double gam, MlpDev mlp)
{
    const int unit = blockIdx.x;
    const int k = unit / gchunks, ch = unit - k * gchunks;
    const PatchDev P = patches[k];
    const long long C = (long long)P.p * P.p * P.p;
    MlpRegs r;
    mlp_load(mlp, r);
#pragma unroll 1
    for (int gi = 0; gi < kGuessGroups; ++gi) {
        const long long c = ((long long)ch * kGuessGroups + gi) * kC2pThreads + threadIdx.x;
        const bool active = c < C;
        double qv[5];
        if (active) {
            const double *base = q + P.off * 5 + c;
#pragma unroll
            for (int v = 0; v < 5; ++v) qv[v] = base[(long long)v * C];
        }
        const double g = guess_of(r, mlp.norm, qv, active, gam);
        if (active) pres[P.off + c] = g;
    }
}

// learned guesses for the standalone entry point, into p0[n]
__global__ __launch_bounds__(kC2pThreads) void flat_guess_kernel(const double *__restrict__ cons,
                                                                 double *__restrict__ p0, long long n, double gam,
                                                                 MlpDev mlp)
{
    MlpRegs r;
    mlp_load(mlp, r);
#pragma unroll 1
    for (int gi = 0; gi < kGuessGroups; ++gi) {
        const long long i = ((long long)blockIdx.x * kGuessGroups + gi) * kC2pThreads + threadIdx.x;
        const bool active = i < n;
        double qv[5];
        if (active) {
#pragma unroll
            for (int v = 0; v < 5; ++v) qv[v] = cons[(long long)v * n + i];
        }
        const double g = guess_of(r, mlp.norm, qv, active, gam);
        if (active) p0[i] = g;
    }
}

// standalone con2prim over n cells of SoA arrays
template <int GUESS>
__global__ __launch_bounds__(kC2pThreads) void con2prim_kernel(
    const double *__restrict__ cons, double *prim, long long n, double gam, double tol, int maxit,
    const double *p_prev, int *__restrict__ iters, int *__restrict__ status,
    unsigned long long *__restrict__ counters, MlpDev mlp)
{
    const long long i = (long long)blockIdx.x * kC2pThreads + threadIdx.x;
    const bool active = i < n;
    double qv[5] = {1.0, 0.0, 0.0, 0.0, 1.0};
    if (active) {
#pragma unroll
        for (int v = 0; v < 5; ++v) qv[v] = cons[(long long)v * n + i];
    }
    const C2pIn in = c2p_setup(qv[0], qv[1], qv[2], qv[3], qv[4], gam);
    double p0 = in.hi;
    // warm: caller's previous pressures; learned: the guesses the network
    // pass stored in prim[4]
    if (GUESS != 0 && active) p0 = p_prev[i];
    C2pStats s = {{0.0, 0.0, 0.0}, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (active) {
        C2pOut o = c2p_solve(in, gam, tol, maxit, p0);
        if (GUESS != 0 && o.status == C2P_NOTCONV) {
            const C2pOut o2 = c2p_solve(in, gam, tol, maxit, in.hi);
            s.fallbacks = 1.0;
            o.p = o2.p;
            o.status = o2.status;
            o.it += o2.it;
        }
        const double iEp = 1.0 / (in.E + o.p);
        const double vx = qv[1] * iEp, vy = qv[2] * iEp, vz = qv[3] * iEp;
        const double v2 = vx * vx + vy * vy + vz * vz;
        prim[i] = qv[0] * sqrt(1.0 - v2);
        prim[n + i] = vx;
        prim[2 * n + i] = vy;
        prim[3 * n + i] = vz;
        prim[4 * n + i] = o.p;
        if (iters) iters[i] = o.it;
        if (status) status[i] = o.status;
        s.iters = o.it;
        s.fails = o.status != C2P_OK ? 1.0 : 0.0;
        s.maxit = o.it;
    }
    if (counters) {
        reduce_stats(s);
        if (threadIdx.x == 0) {
            if (s.fails > 0.0) atomicAdd(&counters[0], (unsigned long long)s.fails);
            atomicAdd(&counters[1], (unsigned long long)s.iters);
            if (s.fallbacks > 0.0) atomicAdd(&counters[2], (unsigned long long)s.fallbacks);
            atomicMax(&counters[3], (unsigned long long)s.maxit);
        }
    }
}

}  // namespace

pb_status launch_srhd_c2p(pb_batch *b, const void *q, int slot_out, bool want_dt, double cfl, hipStream_t s)
{
    const WsLayout L = ws_layout(b->pde, b->total_cells, b->N, b->storage, b->K);
    double *pres = reinterpret_cast<double *>(b->ws + L.pres);
    double *part = reinterpret_cast<double *>(b->ws + L.part);
    const long long cmax = (long long)b->pmax * b->pmax * b->pmax;
    const int chunks = (int)((cmax + kC2pThreads - 1) / kC2pThreads);
    const int n_units = b->K * chunks;
    const double gam = b->params[0], tol = b->params[1];
    const int maxit = (int)b->params[2];
    int guess = b->guess;
    if (guess == PB_GUESS_WARM && !b->pres_valid) guess = PB_GUESS_PLAIN;
    MlpDev md{};
    if (guess == PB_GUESS_LEARNED) {
        pb_status st = mlp_device_view(b->mlp, &md);
        if (st != PB_OK) return st;
    }
    const double *qd = static_cast<const double *>(q);
    switch (guess) {
    case PB_GUESS_PLAIN:
        hipLaunchKernelGGL(srhd_c2p_kernel<0>, dim3(n_units), dim3(kC2pThreads), 0, s, qd, pres, b->d_patches, chunks,
                           n_units, part, gam, tol, maxit, md);
        break;
    case PB_GUESS_LEARNED:
        hipLaunchKernelGGL(srhd_guess_kernel, dim3(b->K * ((chunks + kGuessGroups - 1) / kGuessGroups)),
                           dim3(kC2pThreads), 0, s, qd, pres, b->d_patches, (chunks + kGuessGroups - 1) / kGuessGroups,
                           gam, md);
        PB_HIP(hipGetLastError());
        hipLaunchKernelGGL(srhd_c2p_kernel<1>, dim3(n_units), dim3(kC2pThreads), 0, s, qd, pres, b->d_patches, chunks,
                           n_units, part, gam, tol, maxit, md);
        break;
    default:
        hipLaunchKernelGGL(srhd_c2p_kernel<2>, dim3(n_units), dim3(kC2pThreads), 0, s, qd, pres, b->d_patches, chunks,
                           n_units, part, gam, tol, maxit, md);
    }
    PB_HIP(hipGetLastError());
    b->pres_valid = true;
    return launch_dt_reduce(b, part, n_units, 3, slot_out, cfl, want_dt, true, s);
}

}  // namespace pb

using namespace pb;

extern "C" pb_status con2prim(const void *cons, void *prim, int64_t n, double gamma, double tol, int32_t max_iter,
                              int32_t guess, const pb_mlp *mlp, const void *p_prev, void *iters, void *status,
                              void *counters, void *stream)
{
    if (!cons || !prim) { set_error("con2prim: cons and prim are required"); return PB_EINVAL; }
    if (n < 0) { set_error("con2prim: n must be >= 0"); return PB_EINVAL; }
    if (!(gamma > 1.0 && gamma <= 2.0)) { set_error("con2prim: Gamma must be in (1, 2]"); return PB_EINVAL; }
    if (!(tol > 0.0)) { set_error("con2prim: tol must be > 0"); return PB_EINVAL; }
    if (max_iter < 0 || max_iter > 1000) { set_error("con2prim: max_iter must be in [0, 1000]"); return PB_EINVAL; }
    if (guess < PB_GUESS_PLAIN || guess > PB_GUESS_WARM) { set_error("con2prim: unknown guess"); return PB_EINVAL; }
    if (guess == PB_GUESS_LEARNED && !mlp) { set_error("con2prim: learned guess needs an MLP"); return PB_EINVAL; }
    if (guess == PB_GUESS_WARM && !p_prev) { set_error("con2prim: warm guess needs p_prev"); return PB_EINVAL; }
    if (n == 0) return PB_OK;
    MlpDev md{};
    if (guess == PB_GUESS_LEARNED) {
        pb_status st = mlp_device_view(mlp, &md);
        if (st != PB_OK) return st;
    }
    const long long blocks = (n + kC2pThreads - 1) / kC2pThreads;
    if (blocks > 0x7fffffffll) { set_error("con2prim: n too large"); return PB_EINVAL; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double *cd = static_cast<const double *>(cons);
    double *pd = static_cast<double *>(prim);
    const double *pp = static_cast<const double *>(p_prev);
    int *it = static_cast<int *>(iters);
    int *stp = static_cast<int *>(status);
    unsigned long long *cnt = static_cast<unsigned long long *>(counters);
    switch (guess) {
    case PB_GUESS_PLAIN:
        hipLaunchKernelGGL(con2prim_kernel<0>, dim3((unsigned)blocks), dim3(kC2pThreads), 0, s, cd, pd, (long long)n,
                           gamma, tol, max_iter, pp, it, stp, cnt, md);
        break;
    case PB_GUESS_LEARNED:
        // guesses go to prim[4] (the pressure row), which the solve overwrites
        hipLaunchKernelGGL(flat_guess_kernel, dim3((unsigned)((blocks + kGuessGroups - 1) / kGuessGroups)),
                           dim3(kC2pThreads), 0, s, cd, pd + 4 * n, (long long)n, gamma, md);
        PB_HIP(hipGetLastError());
        hipLaunchKernelGGL(con2prim_kernel<1>, dim3((unsigned)blocks), dim3(kC2pThreads), 0, s, cd, pd, (long long)n,
                           gamma, tol, max_iter, pd + 4 * n, it, stp, cnt, md);
        break;
    default:
        hipLaunchKernelGGL(con2prim_kernel<2>, dim3((unsigned)blocks), dim3(kC2pThreads), 0, s, cd, pd, (long long)n,
                           gamma, tol, max_iter, pp, it, stp, cnt, md);
    }
    PB_HIP(hipGetLastError());
    return PB_OK;
}

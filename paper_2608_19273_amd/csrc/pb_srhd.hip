// pb_srhd.hip -- the per-cell conservative-to-primitive pass of the SRHD
// finite-volume step, and the standalone con2prim entry point.
//
// The SRHD step is two launches (plus the small dt reduction):
//   1. this pass: one lane per cell recovers the pressure by the bracketed
//      FP64 Newton iteration (pb_c2p.h), seeded by the plain guess, the
//      previous step's pressure (warm) or the MLP (learned, evaluated in the
//      same pass on the matrix cores: see pb_mlp.h); writes p to the
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

// Newton from p0; a learned guess that does not converge is retried from the
// plain guess (counted as a fallback)
__device__ __forceinline__ C2pOut solve_cell(const C2pIn &in, double gam, double tol, int maxit, double p0,
                                             bool retry, double &fallbacks)
{
    C2pOut o = c2p_solve(in, gam, tol, maxit, p0);
    if (retry && o.status == C2P_NOTCONV) {
        const C2pOut o2 = c2p_solve(in, gam, tol, maxit, in.hi);
        fallbacks += 1.0;
        o.p = o2.p;
        o.status = o2.status;
        o.it += o2.it;
    }
    return o;
}

__device__ __forceinline__ void add_cell(C2pStats &s, const C2pOut &o)
{
    s.iters += o.it;
    s.fails += o.status != C2P_OK ? 1.0 : 0.0;
    s.maxit = fmax(s.maxit, (double)o.it);
    s.cells += 1.0;
}

// per-lane totals over the cells a lane visits (integers where they count)
struct CellAcc {
    double lam[3] = {0.0, 0.0, 0.0};
    int iters = 0, fails = 0, maxit = 0, fallbacks = 0, cells = 0;
    __device__ __forceinline__ void add(const C2pOut &o)
    {
        iters += o.it;
        fails += o.status != C2P_OK;
        maxit = max(maxit, o.it);
        ++cells;
    }
    __device__ __forceinline__ C2pStats stats() const
    {
        return {{lam[0], lam[1], lam[2]}, (double)iters, (double)fails, (double)maxit, (double)fallbacks,
                (double)cells};
    }
};

__device__ __forceinline__ C2pOut solve_cell_i(const C2pIn &in, double gam, double tol, int maxit, double p0,
                                               int &fallbacks)
{
    C2pOut o = c2p_solve(in, gam, tol, maxit, p0);
    if (o.status == C2P_NOTCONV) {
        const C2pOut o2 = c2p_solve(in, gam, tol, maxit, in.hi);
        ++fallbacks;
        o.p = o2.p;
        o.status = o2.status;
        o.it += o2.it;
    }
    return o;
}

// Chunks of 256 cells a work-group of the con2prim passes walks: the
// learned pass copies the network to LDS once per work-group, and every
// pass reduces its statistics once per work-group.
constexpr int kLearnChunks = 8;

// the same LDS object behind an offset the compiler cannot see through: keeps
// it from hoisting the (loop-invariant) weight reads out of the cell loop,
// which would hold every weight tile in registers for the whole launch
__device__ __forceinline__ const MlpPack &lds_fresh(const MlpPack &sp)
{
    unsigned off = 0;
    __asm__ volatile("" : "+v"(off));
    return *reinterpret_cast<const MlpPack *>(reinterpret_cast<const char *>(&sp) + off);
}

struct MlpLane {
    float xm[kMlpIn], xi[kMlpIn], ym, ys;
};

// copies the blob to the work-group's LDS (returned) and the standardisation
// constants to L
__device__ __forceinline__ const MlpPack &mlp_lane_setup(const MlpPack *__restrict__ pack, MlpLane &L)
{
    __shared__ MlpPack sp;
    const u32x4_t *src = reinterpret_cast<const u32x4_t *>(pack);
    u32x4_t *dst = reinterpret_cast<u32x4_t *>(&sp);
    for (int i = threadIdx.x; i < (int)(sizeof(MlpPack) / 16); i += kC2pThreads) dst[i] = src[i];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) {
        L.xm[k] = pack->xm[k];
        L.xi[k] = pack->xi[k];
    }
    L.ym = pack->ym;
    L.ys = pack->ys;
    return sp;
}

// The con2prim pass of one work-group: kLearnChunks chunks of 256 cells of
// its patch, the next chunk's state (and, for the warm start, the previous
// pressure) loaded while the current one is solved, one statistics
// reduction for all of them.  GUESS: PB_GUESS_PLAIN (Newton from p_hi),
// PB_GUESS_WARM (from the previous pressure in pres), PB_GUESS_LEARNED (from
// the network, evaluated here on the matrix cores; `pack` is the inference
// blob, copied to LDS once).  A guessed start that does not converge is
// redone from p_hi.  The speeds of the recovered state feed the next dt.
template <int GUESS>
__device__ __forceinline__ void c2p_pass(const double *__restrict__ q, double *__restrict__ pres,
                                         const PatchDev *__restrict__ patches, int gchunks, int n_units,
                                         double *__restrict__ part, double gam, double tol, int maxit,
                                         const MlpPack *__restrict__ pack)
{
    constexpr bool kLearned = GUESS == PB_GUESS_LEARNED, kWarm = GUESS == PB_GUESS_WARM;
    MlpLane L;
    const MlpPack *sp = nullptr;
    if constexpr (kLearned) sp = &mlp_lane_setup(pack, L);
    const int unit = blockIdx.x;
    const int k = unit / gchunks, gc = unit - k * gchunks;
    const PatchDev P = patches[k];
    const long long C = (long long)P.p * P.p * P.p;
    const double *base = q + P.off * 5;
    double *pb = pres + P.off;
    CellAcc acc;
    const long long c0 = (long long)gc * kLearnChunks * kC2pThreads + threadIdx.x;
    double nx[5] = {1.0, 0.0, 0.0, 0.0, 1.0}, npv = 0.0;
    if (c0 < C) {
#pragma unroll
        for (int v = 0; v < 5; ++v) nx[v] = base[(long long)v * C + c0];
        if (kWarm) npv = pb[c0];
    }
#pragma unroll 1
    for (int gi = 0; gi < kLearnChunks; ++gi) {
        const long long c = c0 + (long long)gi * kC2pThreads;
        if (c - threadIdx.x >= C) break;   // the same for the whole work-group
        const bool active = c < C;
        double qv[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) qv[v] = nx[v];
        const double pprev = npv;
        const long long cn = c + kC2pThreads;
        if (gi + 1 < kLearnChunks && cn < C) {
#pragma unroll
            for (int v = 0; v < 5; ++v) nx[v] = base[(long long)v * C + cn];
            if (kWarm) npv = pb[cn];
        }
        const C2pIn in = c2p_setup(qv[0], qv[1], qv[2], qv[3], qv[4], gam);
        double p0 = in.hi;
        if constexpr (kLearned) p0 = mlp_guess(lds_fresh(*sp), L.xm, L.xi, L.ym, L.ys, in);   // whole wave
        if constexpr (kWarm) p0 = pprev;
        if (active) {
            C2pOut o;
            if constexpr (GUESS == PB_GUESS_PLAIN) o = c2p_solve(in, gam, tol, maxit, p0);
            else o = solve_cell_i(in, gam, tol, maxit, p0, acc.fallbacks);
            pb[c] = o.p;
            const Srhd ph{gam};
            double a[Srhd::A], e[1] = {o.p};
            ph.aux_fast(qv, e, a);
#pragma unroll
            for (int d = 0; d < 3; ++d) acc.lam[d] = fmax(acc.lam[d], a[4 + d]);
            acc.add(o);
        }
    }
    C2pStats s = acc.stats();
    reduce_stats(s);
    if (threadIdx.x == 0) {
        const double v[8] = {s.lam[0], s.lam[1], s.lam[2], s.iters, s.fails, s.maxit, s.fallbacks, s.cells};
#pragma unroll
        for (int r = 0; r < 8; ++r) part[(long long)r * n_units + unit] = v[r];
    }
}

// plain (GUESS 0) or warm (GUESS 2) start
template <int GUESS>
__global__ __launch_bounds__(kC2pThreads) void srhd_c2p_kernel(
    const double *__restrict__ q, double *__restrict__ pres, const PatchDev *__restrict__ patches, int gchunks,
    int n_units, double *__restrict__ part, double gam, double tol, int maxit)
{
    c2p_pass<GUESS>(q, pres, patches, gchunks, n_units, part, gam, tol, maxit, nullptr);
}

__global__ __launch_bounds__(kC2pThreads, 4) void srhd_c2p_learned_kernel(
    const double *__restrict__ q, double *__restrict__ pres, const PatchDev *__restrict__ patches, int gchunks,
    int n_units, double *__restrict__ part, double gam, double tol, int maxit, const MlpPack *__restrict__ pack)
{
    c2p_pass<PB_GUESS_LEARNED>(q, pres, patches, gchunks, n_units, part, gam, tol, maxit, pack);
}

// standalone con2prim, one cell of SoA arrays: primitives out
__device__ __forceinline__ void prim_out(const double *qv, const C2pIn &in, const C2pOut &o, double *prim,
                                         long long n, long long i, int *iters, int *status)
{
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
}

__device__ __forceinline__ void counters_out(C2pStats &s, unsigned long long *counters)
{
    reduce_stats(s);
    if (threadIdx.x == 0) {
        if (s.fails > 0.0) atomicAdd(&counters[0], (unsigned long long)s.fails);
        atomicAdd(&counters[1], (unsigned long long)s.iters);
        if (s.fallbacks > 0.0) atomicAdd(&counters[2], (unsigned long long)s.fallbacks);
        atomicMax(&counters[3], (unsigned long long)s.maxit);
    }
}

// standalone con2prim over n cells, plain (0) or warm (2) guess
template <int GUESS>
__global__ __launch_bounds__(kC2pThreads) void con2prim_kernel(
    const double *__restrict__ cons, double *__restrict__ prim, long long n, double gam, double tol, int maxit,
    const double *__restrict__ p_prev, int *__restrict__ iters, int *__restrict__ status,
    unsigned long long *__restrict__ counters)
{
    const long long i = (long long)blockIdx.x * kC2pThreads + threadIdx.x;
    const bool active = i < n;
    double qv[5] = {1.0, 0.0, 0.0, 0.0, 1.0};
    if (active) {
#pragma unroll
        for (int v = 0; v < 5; ++v) qv[v] = cons[(long long)v * n + i];
    }
    const C2pIn in = c2p_setup(qv[0], qv[1], qv[2], qv[3], qv[4], gam);
    C2pStats s = {{0.0, 0.0, 0.0}, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (active) {
        const double p0 = GUESS == 2 ? p_prev[i] : in.hi;
        const C2pOut o = solve_cell(in, gam, tol, maxit, p0, GUESS != 0, s.fallbacks);
        prim_out(qv, in, o, prim, n, i, iters, status);
        add_cell(s, o);
    }
    if (counters) counters_out(s, counters);
}

// standalone con2prim with the learned guess: kLearnChunks x 256 cells per
// work-group, the network evaluated in the same pass
__global__ __launch_bounds__(kC2pThreads, 4) void con2prim_learned_kernel(
    const double *__restrict__ cons, double *__restrict__ prim, long long n, double gam, double tol, int maxit,
    int *__restrict__ iters, int *__restrict__ status, unsigned long long *__restrict__ counters,
    const MlpPack *__restrict__ pack)
{
    MlpLane L;
    const MlpPack &sp = mlp_lane_setup(pack, L);
    CellAcc acc;
    const long long i0 = (long long)blockIdx.x * kLearnChunks * kC2pThreads + threadIdx.x;
#pragma unroll 1
    for (int gi = 0; gi < kLearnChunks; ++gi) {
        const long long i = i0 + (long long)gi * kC2pThreads;
        if (i - threadIdx.x >= n) break;   // the same for the whole work-group
        const bool active = i < n;
        double qv[5] = {1.0, 0.0, 0.0, 0.0, 1.0};
        if (active) {
#pragma unroll
            for (int v = 0; v < 5; ++v) qv[v] = cons[(long long)v * n + i];
        }
        const C2pIn in = c2p_setup(qv[0], qv[1], qv[2], qv[3], qv[4], gam);
        const double p0 = mlp_guess(lds_fresh(sp), L.xm, L.xi, L.ym, L.ys, in);   // whole wave
        if (active) {
            const C2pOut o = solve_cell_i(in, gam, tol, maxit, p0, acc.fallbacks);
            prim_out(qv, in, o, prim, n, i, iters, status);
            acc.add(o);
        }
    }
    if (counters) {
        C2pStats s = acc.stats();
        counters_out(s, counters);
    }
}

}  // namespace

pb_status launch_srhd_c2p(pb_batch *b, const void *q, int slot_out, bool want_dt, double cfl, hipStream_t s)
{
    const WsLayout L = ws_layout(b->pde, b->dim, b->h, b->total_cells, b->N, b->storage, b->K);
    double *pres = reinterpret_cast<double *>(b->ws + L.pres);
    double *part = reinterpret_cast<double *>(b->ws + L.part);
    const long long cmax = (long long)b->pmax * b->pmax * b->pmax;
    const int chunks = (int)((cmax + kC2pThreads - 1) / kC2pThreads);
    const double gam = b->params[0], tol = b->params[1];
    const int maxit = (int)b->params[2];
    int guess = b->guess;
    if (guess == PB_GUESS_WARM && !b->pres_valid) guess = PB_GUESS_PLAIN;
    const double *qd = static_cast<const double *>(q);
    const int gchunks = (chunks + kLearnChunks - 1) / kLearnChunks;
    const int n_units = b->K * gchunks;
    switch (guess) {
    case PB_GUESS_PLAIN:
        hipLaunchKernelGGL(srhd_c2p_kernel<PB_GUESS_PLAIN>, dim3(n_units), dim3(kC2pThreads), 0, s, qd, pres,
                           b->d_patches, gchunks, n_units, part, gam, tol, maxit);
        break;
    case PB_GUESS_LEARNED: {
        MlpDev md{};
        pb_status st = mlp_device_view(b->mlp, &md);
        if (st != PB_OK) return st;
        hipLaunchKernelGGL(srhd_c2p_learned_kernel, dim3(n_units), dim3(kC2pThreads), 0, s, qd, pres, b->d_patches,
                           gchunks, n_units, part, gam, tol, maxit, md.pack);
        break;
    }
    default:
        hipLaunchKernelGGL(srhd_c2p_kernel<PB_GUESS_WARM>, dim3(n_units), dim3(kC2pThreads), 0, s, qd, pres,
                           b->d_patches, gchunks, n_units, part, gam, tol, maxit);
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
    PB_API_BEGIN
    if (n < 0) { set_error("con2prim: n must be >= 0"); return PB_EINVAL; }
    if (n > 0 && (!cons || !prim)) { set_error("con2prim: cons and prim are required"); return PB_EINVAL; }
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
                           gamma, tol, max_iter, pp, it, stp, cnt);
        break;
    case PB_GUESS_LEARNED:
        hipLaunchKernelGGL(con2prim_learned_kernel, dim3((unsigned)((blocks + kLearnChunks - 1) / kLearnChunks)),
                           dim3(kC2pThreads), 0, s, cd, pd, (long long)n, gamma, tol, max_iter, it, stp, cnt, md.pack);
        break;
    default:
        hipLaunchKernelGGL(con2prim_kernel<2>, dim3((unsigned)blocks), dim3(kC2pThreads), 0, s, cd, pd, (long long)n,
                           gamma, tol, max_iter, pp, it, stp, cnt);
    }
    PB_HIP(hipGetLastError());
    return PB_OK;
    PB_API_END
}

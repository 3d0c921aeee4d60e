// pb_api.hip -- host runtime behind the C ABI of include/patchhip.h:
// argument validation (always before any HIP call), the patch table upload,
// workspace layout, step sequencing with the device-resident dt, HIP-graph
// capture and replay of step sequences, statistics.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "pb_common.h"

namespace pb {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

pb_status hip_fail(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return PB_EHIP;
}

pb_status api_fail(const char *what, pb_status st) noexcept
{
    try {
        set_error(what);
    } catch (...) {
    }
    return st;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

WsLayout ws_layout(int pde, int dim, int h, long long total_cells, int N, int storage, int K)
{
    WsLayout L;
    size_t o = 0;
    L.ctrl = o;
    o += sizeof(Ctrl);
    o = align256(o);
    L.part = o;
    // [8][units] partials, then [8][units / 256 + 1] for the second reduction stage
    o = align256(o + (size_t)8 * ((size_t)max_units(K) + (size_t)max_units(K) / 256 + 1) * sizeof(double));
    if (pde == PB_PDE_SRHD) {
        L.pres = o;
        o = align256(o + (size_t)total_cells * sizeof(double));
    }
    if (fd_buffers(pde, dim, h)) {
        const size_t es = storage == PB_STORE_FP32 ? 4 : 8;
        L.yA = o;
        o = align256(o + (size_t)total_cells * N * es);
        L.yB = o;
        o = align256(o + (size_t)total_cells * N * es);
    }
    L.total = o;
    return L;
}

static int n_params_needed(int pde, int N)
{
    switch (pde) {
    case PB_PDE_ADVECTION_F:
    case PB_PDE_ADVECTION_B: return 4;
    case PB_PDE_EULER: return 1;
    case PB_PDE_LINSYM: return 3 + 3 * N * N;
    case PB_PDE_SRHD: return 3;
    case PB_PDE_ADVECTION_VAR: return 1;
    }
    return -1;
}

// host-only validation of a descriptor; returns PB_OK or PB_EINVAL with text
static pb_status validate(const pb_batch_desc *d, bool need_buffers, long long *cells_out,
                          double *dxmin_out, int *pmax_out)
{
    if (!d) { set_error("descriptor is NULL"); return PB_EINVAL; }
    if (d->dim != 2 && d->dim != 3) { set_error("dim must be 2 or 3"); return PB_EINVAL; }
    if (d->n_patches < 1) { set_error("n_patches must be >= 1"); return PB_EINVAL; }
    if (!d->p || !d->dx || !d->neighbor) { set_error("p, dx and neighbor tables are required"); return PB_EINVAL; }
    if (d->halo < 1) { set_error("halo must be >= 1"); return PB_EINVAL; }
    if (d->pde < PB_PDE_ADVECTION_F || d->pde > PB_PDE_ADVECTION_VAR) { set_error("unknown pde"); return PB_EINVAL; }
    if (d->storage != PB_STORE_FP64 && d->storage != PB_STORE_FP32) { set_error("unknown storage"); return PB_EINVAL; }
    if (d->n_unknowns < 1 || d->n_aux < 0 || d->n_aux > 64) { set_error("need n_unknowns >= 1 and 0 <= n_aux <= 64"); return PB_EINVAL; }
    if (d->pde == PB_PDE_ADVECTION_VAR) {
        if (d->n_unknowns != 1 || d->n_aux != d->dim) {
            set_error("variable advection needs n_unknowns = 1 and n_aux = dim");
            return PB_EINVAL;
        }
    } else if (d->n_aux != 0) {
        set_error("n_aux > 0 (material parameters) is implemented for ADVECTION_VAR only");
        return PB_EUNSUPPORTED;
    }
    const int N = d->n_unknowns + d->n_aux;   // values per point
    switch (d->pde) {
    case PB_PDE_ADVECTION_F:
    case PB_PDE_ADVECTION_B:
        if (N != 1) { set_error("advection needs n_unknowns = 1"); return PB_EINVAL; }
        break;
    case PB_PDE_EULER:
        if (N != d->dim + 2) { set_error("Euler needs n_unknowns = dim + 2"); return PB_EINVAL; }
        break;
    case PB_PDE_LINSYM:
        if (N < 1 || N > 64) { set_error("linear system needs 1 <= n_unknowns <= 64"); return PB_EINVAL; }
        break;
    case PB_PDE_SRHD:
        if (N != 5 || d->dim != 3) { set_error("SRHD needs dim = 3 and n_unknowns = 5"); return PB_EINVAL; }
        break;
    case PB_PDE_ADVECTION_VAR:
        break;
    }
    const int np = n_params_needed(d->pde, N);
    if (d->n_pde_params < np || (np > 0 && !d->pde_params)) {
        set_error("pde_params: expected " + std::to_string(np) + " values");
        return PB_EINVAL;
    }
    for (int i = 0; i < np; ++i)
        if (!std::isfinite(d->pde_params[i])) { set_error("pde_params must be finite"); return PB_EINVAL; }
    if (d->pde == PB_PDE_EULER && !(d->pde_params[0] > 1.0)) { set_error("gamma must be > 1"); return PB_EINVAL; }
    if (d->pde == PB_PDE_SRHD) {
        if (!(d->pde_params[0] > 1.0 && d->pde_params[0] <= 2.0)) { set_error("SRHD Gamma must be in (1, 2]"); return PB_EINVAL; }
        if (!(d->pde_params[1] > 0.0)) { set_error("con2prim tol must be > 0"); return PB_EINVAL; }
        if (!(d->pde_params[2] >= 0.0 && d->pde_params[2] <= 1000.0)) { set_error("con2prim max_iter must be in [0, 1000]"); return PB_EINVAL; }
    }
    long long cells = 0;
    double dxmin = INFINITY;
    int pmax = 0;
    for (int k = 0; k < d->n_patches; ++k) {
        const int p = d->p[k];
        if (p < 1 || p > 1024) { set_error("patch " + std::to_string(k) + ": p out of range"); return PB_EINVAL; }
        if (p < d->halo) { set_error("patch " + std::to_string(k) + ": p must be >= halo"); return PB_EINVAL; }
        if (!(d->dx[k] > 0.0) || !std::isfinite(d->dx[k])) { set_error("patch " + std::to_string(k) + ": dx must be > 0"); return PB_EINVAL; }
        for (int f = 0; f < 2 * d->dim; ++f) {
            const int nb = d->neighbor[(size_t)k * 2 * d->dim + f];
            if (nb < 0 || nb >= d->n_patches) { set_error("patch " + std::to_string(k) + ": neighbour index out of range"); return PB_EINVAL; }
            if (d->p[nb] != p) { set_error("patch " + std::to_string(k) + ": neighbour has a different p"); return PB_EINVAL; }
        }
        long long c = p;
        for (int e = 1; e < d->dim; ++e) c *= p;
        cells += c;
        dxmin = std::min(dxmin, d->dx[k]);
        pmax = std::max(pmax, p);
    }
    if (cells > (1ll << 40)) { set_error("batch too large"); return PB_EINVAL; }
    if (need_buffers) {
        if (!d->state || !d->state_alt) { set_error("state and state_alt are required"); return PB_EINVAL; }
        if (d->state == d->state_alt) { set_error("state and state_alt must differ"); return PB_EINVAL; }
        const WsLayout L = ws_layout(d->pde, d->dim, d->halo, cells, N, d->storage, d->n_patches);
        if (!d->workspace) { set_error("workspace is required"); return PB_EINVAL; }
        if (((uintptr_t)d->workspace & 255) != 0) { set_error("workspace must be 256-byte aligned"); return PB_EINVAL; }
        if (d->workspace_bytes < L.total) {
            set_error("workspace too small: need " + std::to_string(L.total) + " bytes");
            return PB_EINVAL;
        }
    }
    if (cells_out) *cells_out = cells;
    if (dxmin_out) *dxmin_out = dxmin;
    if (pmax_out) *pmax_out = pmax;
    return PB_OK;
}

// profiling: hand the next pair's start event (first launch of the pair)
// and end event (last launch) to the next main-kernel launch (launch_main),
// then count the launch once it has been enqueued and the pair once its end
// is on the stream
static void arm_events(pb_batch *b, bool first = true, bool last = true)
{
    if (!b->profiling) return;
    b->kev[0] = first ? b->prof_ev[0][b->prof_n] : nullptr;
    b->kev[1] = last ? b->prof_ev[1][b->prof_n] : nullptr;
}

static pb_status disarm_events(pb_batch *b, pb_status st)
{
    if (b->profiling) {
        if (st != PB_OK) {
            b->prof_pending = 0;   // an unfinished pair is dropped
        } else {
            if (b->kev[0]) b->prof_pending = 0;
            ++b->prof_pending;
            if (b->kev[1]) {
                ++b->prof_n;
                b->prof_launches += b->prof_pending;
                b->prof_pending = 0;
            }
        }
    }
    b->kev[0] = b->kev[1] = nullptr;
    return st;
}

// enqueue n FV steps on stream s starting from buffer `cur`; returns the new cur
static pb_status enqueue_fv(pb_batch *b, double cfl, double dt_fixed, int n, hipStream_t s, int *cur_io)
{
    int cur = *cur_io;
    pb_status st;
    const bool cfl_mode = !(dt_fixed > 0.0);
    if (cfl_mode && b->pde != PB_PDE_SRHD)
        if ((st = launch_fv_lambda(b, b->state[cur], cfl, s)) != PB_OK) return st;
    // span mode: without the con2prim pass the n step launches follow each
    // other with nothing in between, so one pair brackets all of them
    const bool span = b->prof_span && b->pde != PB_PDE_SRHD;
    for (int i = 0; i < n; ++i) {
        const int slot = i & 1;
        if (b->pde == PB_PDE_SRHD)
            if ((st = launch_srhd_c2p(b, b->state[cur], slot, cfl_mode, cfl, s)) != PB_OK) return st;
        if (span)
            arm_events(b, i == 0, i == n - 1);
        else
            arm_events(b);
        st = disarm_events(b, launch_fv_step(b, b->state[cur], b->state[cur ^ 1], slot, i, dt_fixed, cfl, s));
        if (st != PB_OK) return st;
        cur ^= 1;
    }
    *cur_io = cur;
    return PB_OK;
}

// dt of the linear system: its largest speeds are the spectral radii rho_d
// of B_d (part of the PDE parameters), so dt = cfl / sum_d (rho_d / dx_min)
double fd_dt(const pb_batch *b, double cfl, double dt_fixed)
{
    if (dt_fixed > 0.0) return dt_fixed;
    double den = 0.0;
    for (int d = 0; d < b->dim; ++d) den += b->params[d] / b->dxmin;
    return cfl / den;
}

static pb_status enqueue_fd(pb_batch *b, double cfl, double dt_fixed, double sigma, int rk, int n,
                            hipStream_t s, int *cur_io)
{
    int cur = *cur_io;
    pb_status st;
    const WsLayout L = ws_layout(b->pde, b->dim, b->h, b->total_cells, b->N, b->storage, b->K);
    void *yA = b->ws + L.yA, *yB = b->ws + L.yB;
    if (b->pde == PB_PDE_EULER) {
        // dt on the device: from Q^n for the first step, then from the last
        // stage of each step (ping-pong slots as in the FV path)
        if (!(dt_fixed > 0.0))
            if ((st = launch_fv_lambda(b, b->state[cur], cfl, s)) != PB_OK) return st;
        for (int i = 0; i < n; ++i) {
            void *q0 = b->state[cur], *acc = b->state[cur ^ 1];
            const int slot = i & 1;
            void *ys[4] = {q0, yA, yB, yA};
            void *yn[4] = {yA, yB, yA, nullptr};
            for (int sg = 0; sg < (rk == 1 ? 1 : 4); ++sg) {
                arm_events(b);
                st = disarm_events(b, launch_fd_euler_stage(b, sg, rk, q0, ys[sg], rk == 1 ? nullptr : yn[sg], acc,
                                                            slot, dt_fixed, cfl, sigma, s));
                if (st != PB_OK) return st;
            }
            cur ^= 1;
        }
        *cur_io = cur;
        return PB_OK;
    }
    const double dt = fd_dt(b, cfl, dt_fixed);
    for (int i = 0; i < n; ++i) {
        void *q0 = b->state[cur], *acc = b->state[cur ^ 1];
        if (rk == 1) {
            arm_events(b);
            st = disarm_events(b, launch_fd_stage(b, 0, 1, q0, q0, nullptr, acc, dt, sigma, s));
            if (st != PB_OK) return st;
        } else {
            // stage 1 reads Q^n, stages 2-4 read the previous stage value
            void *ys[4] = {q0, yA, yB, yA};
            void *yn[4] = {yA, yB, yA, nullptr};
            for (int sg = 0; sg < 4; ++sg) {
                arm_events(b);
                st = disarm_events(b, launch_fd_stage(b, sg, 4, q0, ys[sg], yn[sg], acc, dt, sigma, s));
                if (st != PB_OK) return st;
            }
        }
        cur ^= 1;
    }
    *cur_io = cur;
    return PB_OK;
}

}  // namespace pb

using namespace pb;

extern "C" {

const char *pb_last_error(void) { return g_err.c_str(); }

pb_status pb_workspace_size(const pb_batch_desc *desc, size_t *bytes)
{
    PB_API_BEGIN
    if (!bytes) { set_error("bytes is NULL"); return PB_EINVAL; }
    long long cells = 0;
    pb_status st = validate(desc, false, &cells, nullptr, nullptr);
    if (st != PB_OK) return st;
    *bytes = ws_layout(desc->pde, desc->dim, desc->halo, cells, desc->n_unknowns + desc->n_aux, desc->storage,
                       desc->n_patches).total;
    return PB_OK;
    PB_API_END
}

pb_status pb_column_runs(const pb_batch_desc *desc, int32_t kind, int32_t w, int32_t cus, int32_t *runs,
                         int32_t max_runs, int32_t *n_runs)
{
    PB_API_BEGIN
    if (!n_runs || (max_runs > 0 && !runs)) { set_error("NULL argument"); return PB_EINVAL; }
    *n_runs = 0;
    long long cells = 0;
    pb_status st = validate(desc, false, &cells, nullptr, nullptr);
    if (st != PB_OK) return st;
    if (desc->dim != 3) { set_error("column runs apply to 3D batches"); return PB_EINVAL; }
    if (kind != 0 && kind != 1) { set_error("kind must be 0 (FV) or 1 (Euler FD)"); return PB_EINVAL; }
    if (w < 1 || w > 8 || cus < 1) { set_error("need w in [1, 8] and cus >= 1"); return PB_EINVAL; }
    const std::vector<int4> r = column_runs(kind, desc->n_patches, desc->p, desc->neighbor, w, cus);
    *n_runs = (int32_t)r.size();
    if ((int32_t)r.size() > max_runs) { set_error("runs buffer too small"); return PB_EINVAL; }
    for (size_t i = 0; i < r.size(); ++i) {
        runs[4 * i + 0] = r[i].x;
        runs[4 * i + 1] = r[i].y;
        runs[4 * i + 2] = r[i].z;
        runs[4 * i + 3] = r[i].w;
    }
    return PB_OK;
    PB_API_END
}

pb_status patch_batch_create(const pb_batch_desc *d, pb_batch **out)
{
    PB_API_BEGIN
    if (!out) { set_error("out is NULL"); return PB_EINVAL; }
    *out = nullptr;
    long long cells = 0;
    double dxmin = 0.0;
    int pmax = 0;
    pb_status st = validate(d, true, &cells, &dxmin, &pmax);
    if (st != PB_OK) return st;
    pb_batch *b = new (std::nothrow) pb_batch();
    if (!b) { set_error("out of host memory"); return PB_ENOMEM; }
    b->dim = d->dim;
    b->K = d->n_patches;
    b->N = d->n_unknowns + d->n_aux;   // values per point: the kernels carry the last n_aux unchanged
    b->h = d->halo;
    b->pde = d->pde;
    b->storage = d->storage;
    b->p.assign(d->p, d->p + d->n_patches);
    b->dx.assign(d->dx, d->dx + d->n_patches);
    b->nbr.assign(d->neighbor, d->neighbor + (size_t)d->n_patches * 2 * d->dim);
    b->params.assign(d->pde_params, d->pde_params + n_params_needed(d->pde, b->N));
    b->state[0] = d->state;
    b->state[1] = d->state_alt;
    b->ws = static_cast<char *>(d->workspace);
    b->ws_bytes = d->workspace_bytes;
    b->stream = static_cast<hipStream_t>(d->stream);
    b->total_cells = cells;
    b->dxmin = dxmin;
    b->pmax = pmax;
    b->uniform_p = std::all_of(b->p.begin(), b->p.end(), [&](int v) { return v == b->p[0]; });

    std::vector<PatchDev> tab((size_t)b->K);
    long long off = 0;
    for (int k = 0; k < b->K; ++k) {
        PatchDev &P = tab[k];
        std::memset(&P, 0, sizeof P);
        P.off = off;
        P.p = b->p[k];
        for (int f = 0; f < 6; ++f) P.nbr[f] = f < 2 * b->dim ? b->nbr[(size_t)k * 2 * b->dim + f] : k;
        P.inv_dx = 1.0 / b->dx[k];
        long long c = P.p;
        for (int e = 1; e < b->dim; ++e) c *= P.p;
        off += c;
    }
    hipError_t e = hipMalloc(&b->d_patches, tab.size() * sizeof(PatchDev));
    if (e != hipSuccess) { delete b; return hip_fail(e, "hipMalloc(patch table)"); }
    e = hipMemcpy(b->d_patches, tab.data(), tab.size() * sizeof(PatchDev), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipFree(b->d_patches);
        delete b;
        return hip_fail(e, "patch_batch_create");
    }
    st = launch_ctrl_init(b, b->stream);
    if (st == PB_OK) st = runs_prepare(b);   // the default tunings' run tables
    if (st != PB_OK) { patch_batch_destroy(b); return st; }
    *out = b;
    return PB_OK;
    PB_API_END
}

pb_status patch_batch_destroy(pb_batch *b)
{
    PB_API_BEGIN
    if (!b) return PB_OK;
    for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    for (int w = 0; w < 2; ++w)
        for (auto ev : b->prof_ev[w]) (void)hipEventDestroy(ev);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    (void)hipFree(b->d_patches);
    if (b->d_fd_items) (void)hipFree(b->d_fd_items);
    if (b->d_fd_ws_items) (void)hipFree(b->d_fd_ws_items);
    if (b->d_fd_B) (void)hipFree(b->d_fd_B);
    if (b->d_fd_A) (void)hipFree(b->d_fd_A);
    if (b->fv_runs.d) (void)hipFree(b->fv_runs.d);
    if (b->fd_runs.d) (void)hipFree(b->fd_runs.d);
    delete b;
    return PB_OK;
    PB_API_END
}

pb_status pb_batch_reset(pb_batch *b, int32_t which)
{
    PB_API_BEGIN
    if (!b) { set_error("batch is NULL"); return PB_EINVAL; }
    if (which != 0 && which != 1) { set_error("which must be 0 or 1"); return PB_EINVAL; }
    b->cur = which;
    b->steps = 0;
    b->pres_valid = false;
    return launch_ctrl_init(b, b->stream);
    PB_API_END
}

pb_status pb_batch_set_tuning(pb_batch *b, const pb_tuning *t)
{
    PB_API_BEGIN
    if (!b || !t) { set_error("NULL argument"); return PB_EINVAL; }
    if (t->fv_slab < 0 || t->fv_slab > kFvPmax) { set_error("fv_slab must be in [0, 16]"); return PB_EINVAL; }
    if (t->fd_wg_per_cu < 0 || t->fd_wg_per_cu > 2) { set_error("fd_wg_per_cu must be 0, 1 or 2"); return PB_EINVAL; }
    if (t->fv_persist < 0 || t->fv_persist > 8) { set_error("fv_persist must be in [0, 8]"); return PB_EINVAL; }
    if (t->fv_column < 0 || t->fv_column > 8) { set_error("fv_column must be in [0, 8]"); return PB_EINVAL; }
    if (t->fd_column < 0 || t->fd_column > 8) { set_error("fd_column must be in [0, 8]"); return PB_EINVAL; }
    if (t->fd_ws < 0 || t->fd_ws > 2) { set_error("fd_ws must be 0, 1 or 2"); return PB_EINVAL; }
    b->fv_slab = t->fv_slab;
    b->fv_xcd_remap = t->fv_xcd_remap ? 1 : 0;
    b->fd_xcd_remap = t->fd_xcd_remap ? 1 : 0;
    b->fd_wg_per_cu = t->fd_wg_per_cu == 0 ? 2 : t->fd_wg_per_cu;
    b->fv_dma = t->fv_dma ? 1 : 0;
    b->fd_ws = t->fd_ws;
    b->fv_persist = t->fv_persist;
    b->fv_column = t->fv_column;
    b->fd_column = t->fd_column;
    for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    b->graphs.clear();
    return runs_prepare(b);
    PB_API_END
}

pb_status pb_batch_get_tuning(const pb_batch *b, pb_tuning *out)
{
    PB_API_BEGIN
    if (!b || !out) { set_error("NULL argument"); return PB_EINVAL; }
    out->fv_slab = b->fv_slab;
    out->fv_xcd_remap = b->fv_xcd_remap;
    out->fd_xcd_remap = b->fd_xcd_remap;
    out->fd_wg_per_cu = b->fd_wg_per_cu;
    out->fv_dma = b->fv_dma;
    out->fd_ws = b->fd_ws;
    out->fv_persist = b->fv_persist;
    out->fv_column = b->fv_column;
    out->fd_column = b->fd_column;
    return PB_OK;
    PB_API_END
}

pb_status pb_batch_set_c2p_guess(pb_batch *b, int32_t guess, const pb_mlp *mlp)
{
    PB_API_BEGIN
    if (!b) { set_error("batch is NULL"); return PB_EINVAL; }
    if (b->pde != PB_PDE_SRHD) { set_error("con2prim guess applies to SRHD batches"); return PB_EINVAL; }
    if (guess < PB_GUESS_PLAIN || guess > PB_GUESS_WARM) { set_error("unknown guess mode"); return PB_EINVAL; }
    if (guess == PB_GUESS_LEARNED && !mlp) { set_error("learned guess needs an MLP"); return PB_EINVAL; }
    b->guess = guess;
    b->mlp = mlp;
    for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    b->graphs.clear();
    return PB_OK;
    PB_API_END
}

pb_status pb_batch_stats(pb_batch *b, pb_stats *out)
{
    PB_API_BEGIN
    if (!b || !out) { set_error("NULL argument"); return PB_EINVAL; }
    Ctrl c;
    PB_HIP(hipMemcpyAsync(&c, b->ws, sizeof c, hipMemcpyDeviceToHost, b->stream));
    PB_HIP(hipStreamSynchronize(b->stream));
    std::memset(out, 0, sizeof *out);
    out->steps = b->steps;
    out->nonfinite_units = (int64_t)c.nonfinite;
    out->c2p_cells = (int64_t)c.c2p_cells;
    out->c2p_failures = (int64_t)c.c2p_fail;
    out->c2p_iterations = (int64_t)c.c2p_iters;
    out->c2p_fallbacks = (int64_t)c.c2p_fallback;
    out->c2p_max_iterations = (int32_t)c.c2p_maxit;
    out->current = b->cur;
    out->last_dt = b->last_dt_host > 0.0 ? b->last_dt_host : c.dt[b->last_slot];
    return PB_OK;
    PB_API_END
}

// run or replay a step sequence; `kind` 0 = FV, 1 = FD
static pb_status run_steps(pb_batch *b, int kind, double cfl, double dt_fixed, double sigma, int rk,
                           int n, int use_graph)
{
    pb_status st;
    if (b->profiling && use_graph) { set_error("profiling records events between launches; use eager mode"); return PB_EINVAL; }
    if (b->profiling) {
        const size_t need = (size_t)b->prof_n + (size_t)n * 4 + 4;
        for (int w = 0; w < 2; ++w)
            while (b->prof_ev[w].size() < need) {
                hipEvent_t ev;
                PB_HIP(hipEventCreate(&ev));
                b->prof_ev[w].push_back(ev);
            }
    }
    if (!use_graph) {
        int cur = b->cur;
        st = kind == 0 ? enqueue_fv(b, cfl, dt_fixed, n, b->stream, &cur)
                       : enqueue_fd(b, cfl, dt_fixed, sigma, rk, n, b->stream, &cur);
        if (st != PB_OK) return st;
        b->cur = cur;
        return PB_OK;
    }
    for (auto &g : b->graphs) {
        if (g.kind == kind && g.n_steps == n && g.parity_cur == b->cur && g.key0 == cfl &&
            g.key1 == dt_fixed && g.key2 == sigma && g.key3 == rk) {
            PB_HIP(hipGraphLaunch(g.exec, b->stream));
            b->cur ^= (n & 1);
            return PB_OK;
        }
    }
    // capture on the library's own stream, replay on the caller's
    PB_HIP(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
    int cur = b->cur;
    st = kind == 0 ? enqueue_fv(b, cfl, dt_fixed, n, b->capture_stream, &cur)
                   : enqueue_fd(b, cfl, dt_fixed, sigma, rk, n, b->capture_stream, &cur);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(b->capture_stream, &graph);
    if (st != PB_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    b->graphs.push_back({kind, n, b->cur, cfl, dt_fixed, sigma, rk, exec});
    PB_HIP(hipGraphLaunch(exec, b->stream));
    b->cur = cur;
    return PB_OK;
}

static pb_status finish_call(pb_batch *b, int n, double dt_fixed, double *dt_last_host)
{
    b->steps += n;
    b->last_dt_host = dt_fixed > 0.0 ? dt_fixed : 0.0;
    if (n > 0) b->last_slot = (n - 1) & 1;
    if (dt_last_host) {
        if (dt_fixed > 0.0) {
            *dt_last_host = dt_fixed;
        } else {
            double v = 0.0;
            const size_t o = offsetof(Ctrl, dt) + sizeof(double) * (size_t)b->last_slot;
            PB_HIP(hipMemcpyAsync(&v, b->ws + o, sizeof v, hipMemcpyDeviceToHost, b->stream));
            PB_HIP(hipStreamSynchronize(b->stream));
            *dt_last_host = v;
        }
    }
    return PB_OK;
}

static constexpr int kProfPool = 1024;   // launches recorded without growing the event pool

pb_status pb_batch_profile(pb_batch *b, int32_t on)
{
    PB_API_BEGIN
    if (!b) { set_error("batch is NULL"); return PB_EINVAL; }
    if (on < 0 || on > 2) { set_error("profile mode must be 0, 1 or 2"); return PB_EINVAL; }
    if (on) {
        // create the event pool now, so that a profiled call spends no time
        // creating events (the pool still grows for a call of more launches)
        for (int w = 0; w < 2; ++w)
            while (b->prof_ev[w].size() < (size_t)kProfPool) {
                hipEvent_t ev;
                PB_HIP(hipEventCreate(&ev));
                b->prof_ev[w].push_back(ev);
            }
    }
    b->profiling = on != 0;
    b->prof_span = on == 2;
    b->prof_n = 0;
    b->prof_launches = b->prof_pending = 0;
    return PB_OK;
    PB_API_END
}

pb_status pb_batch_profile_read(pb_batch *b, double *total_ms, int64_t *launches)
{
    PB_API_BEGIN
    if (!b || !total_ms || !launches) { set_error("NULL argument"); return PB_EINVAL; }
    PB_HIP(hipStreamSynchronize(b->stream));
    double sum = 0.0;
    for (int i = 0; i < b->prof_n; ++i) {
        float ms = 0.f;
        PB_HIP(hipEventElapsedTime(&ms, b->prof_ev[0][i], b->prof_ev[1][i]));
        sum += ms;
    }
    *total_ms = sum;
    *launches = b->prof_launches;
    b->prof_n = 0;
    b->prof_launches = b->prof_pending = 0;
    return PB_OK;
    PB_API_END
}

pb_status fv_rusanov_step(pb_batch *b, double cfl, double dt_fixed, int32_t n_steps, int32_t use_graph,
                          double *dt_last_host)
{
    PB_API_BEGIN
    if (!b) { set_error("batch is NULL"); return PB_EINVAL; }
    if (n_steps < 0) { set_error("n_steps must be >= 0"); return PB_EINVAL; }
    if (!std::isfinite(dt_fixed) || (!(dt_fixed > 0.0) && !(cfl > 0.0 && std::isfinite(cfl)))) {
        set_error("need dt_fixed > 0 or a finite cfl > 0");
        return PB_EINVAL;
    }
    if (b->pde == PB_PDE_LINSYM) { set_error("fv_rusanov_step: the linear system runs through fd_ko_step"); return PB_EUNSUPPORTED; }
    if (b->pmax > kFvPmax) { set_error("fv_rusanov_step: p > 16 is not supported"); return PB_EUNSUPPORTED; }
    if (b->pde == PB_PDE_SRHD && b->storage != PB_STORE_FP64) { set_error("SRHD runs in FP64 storage"); return PB_EUNSUPPORTED; }
    if (n_steps == 0) return finish_call(b, 0, dt_fixed, dt_last_host);
    pb_status st = run_steps(b, 0, cfl, dt_fixed, 0.0, 0, n_steps, use_graph);
    if (st != PB_OK) return st;
    return finish_call(b, n_steps, dt_fixed, dt_last_host);
    PB_API_END
}

pb_status fd_ko_step(pb_batch *b, double cfl, double dt_fixed, double sigma_ko, int32_t rk_stages,
                     int32_t n_steps, int32_t use_graph, double *dt_last_host)
{
    PB_API_BEGIN
    if (!b) { set_error("batch is NULL"); return PB_EINVAL; }
    if (n_steps < 0) { set_error("n_steps must be >= 0"); return PB_EINVAL; }
    if (rk_stages != 1 && rk_stages != 4) { set_error("rk_stages must be 1 or 4"); return PB_EINVAL; }
    if (!std::isfinite(sigma_ko) || sigma_ko < 0.0) { set_error("sigma_ko must be finite and >= 0"); return PB_EINVAL; }
    if (!std::isfinite(dt_fixed) || (!(dt_fixed > 0.0) && !(cfl > 0.0 && std::isfinite(cfl)))) {
        set_error("need dt_fixed > 0 or a finite cfl > 0");
        return PB_EINVAL;
    }
    if (b->pde != PB_PDE_LINSYM && b->pde != PB_PDE_EULER) {
        set_error("fd_ko_step: implemented for LINSYM and EULER");
        return PB_EUNSUPPORTED;
    }
    if (b->h < 3) { set_error("fd_ko_step needs halo >= 3"); return PB_EINVAL; }
    if (b->dim != 3 || b->storage != PB_STORE_FP64) { set_error("fd_ko_step: dim 3, FP64 storage"); return PB_EUNSUPPORTED; }
    if (b->pde == PB_PDE_EULER) {
        if (b->pmax > kFvPmax) { set_error("fd_ko_step: p > 16 is not supported for EULER"); return PB_EUNSUPPORTED; }
        if (n_steps == 0) return finish_call(b, 0, dt_fixed, dt_last_host);
        pb_status st = run_steps(b, 1, cfl, dt_fixed, sigma_ko, rk_stages, n_steps, use_graph);
        if (st != PB_OK) return st;
        return finish_call(b, n_steps, dt_fixed, dt_last_host);
    }
    if (b->N > 60) { set_error("fd_ko_step: at most 60 unknowns"); return PB_EUNSUPPORTED; }
    for (int k = 0; k < b->K; ++k) {
        if (b->p[k] != 4 && b->p[k] != 8 && b->p[k] != 16) { set_error("fd_ko_step: p must be 4, 8 or 16"); return PB_EUNSUPPORTED; }
        for (int f = 0; f < 6; ++f)
            if (b->nbr[(size_t)k * 6 + f] != k) { set_error("fd_ko_step: patches must be periodic on themselves"); return PB_EUNSUPPORTED; }
    }
    const double dt = fd_dt(b, cfl, dt_fixed);
    if (n_steps == 0) return finish_call(b, 0, dt, dt_last_host);
    pb_status st = fd_prepare(b);
    if (st != PB_OK) return st;
    st = run_steps(b, 1, cfl, dt_fixed, sigma_ko, rk_stages, n_steps, use_graph);
    if (st != PB_OK) return st;
    return finish_call(b, n_steps, dt, dt_last_host);
    PB_API_END
}

}  // extern "C"

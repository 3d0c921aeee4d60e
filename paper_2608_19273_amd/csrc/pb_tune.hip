// pb_tune.hip -- measured launch-shape search for the step kernels of a
// batch, and the process-wide cache of its results (text-file persistence).
//
// The search times real launches on the batch's own input: the trial
// launches read the current state and write only the other state buffer and
// the workspace, and the control block is restored afterwards, so tuning
// never advances or perturbs the simulation.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "pb_common.h"

namespace pb {
namespace {

std::mutex g_mu;
std::map<std::string, pb_tuning> g_cache;

std::string tune_key(const pb_batch *b, int kind)
{
    std::map<int, int> hist;
    for (int p : b->p) ++hist[p];
    std::ostringstream k;
    k << (kind == 0 ? "fv" : "fd") << "/pde" << b->pde << "/d" << b->dim << "/N" << b->N << "/s" << b->storage
      << "/h" << b->h << "/";
    bool first = true;
    for (auto &e : hist) {
        k << (first ? "" : ",") << e.first << "x" << e.second;
        first = false;
    }
    return k.str();
}

pb_tuning current(const pb_batch *b)
{
    pb_tuning t;
    t.fv_slab = b->fv_slab;
    t.fv_xcd_remap = b->fv_xcd_remap;
    t.fd_xcd_remap = b->fd_xcd_remap;
    t.fd_wg_per_cu = b->fd_wg_per_cu;
    t.fv_dma = b->fv_dma;
    t.fd_ws = b->fd_ws;
    t.fv_persist = b->fv_persist;
    t.fv_column = b->fv_column;
    t.fd_column = b->fd_column;
    return t;
}

pb_status apply(pb_batch *b, const pb_tuning &t)
{
    b->fv_slab = t.fv_slab;
    b->fv_xcd_remap = t.fv_xcd_remap;
    b->fd_xcd_remap = t.fd_xcd_remap;
    b->fd_wg_per_cu = t.fd_wg_per_cu == 0 ? 2 : t.fd_wg_per_cu;
    b->fv_dma = t.fv_dma;
    b->fd_ws = t.fd_ws;
    b->fv_persist = t.fv_persist;
    b->fv_column = t.fv_column;
    b->fd_column = t.fd_column;
    return runs_prepare(b);
}

std::vector<pb_tuning> candidates(const pb_batch *b, int kind)
{
    std::vector<pb_tuning> c;
    const pb_tuning base = current(b);
    if (kind == 0 && fv_small_eligible(b)) {
        c.push_back(base);   // the small-patch kernel has no launch-shape choices
    } else if (kind == 0) {
        std::vector<int> slabs;
        if (b->dim == 3) {
            for (int s = b->pmax; s >= 2 && slabs.size() < 3; s /= 2) slabs.push_back(s);
            if (slabs.empty()) slabs.push_back(b->pmax);
        } else {
            slabs.push_back(0);
        }
        auto plain = [&](int remap) {
            pb_tuning t = base;
            t.fv_persist = 0;
            t.fv_column = 0;
            t.fv_dma = 0;
            t.fv_slab = 0;
            t.fv_xcd_remap = remap;
            return t;
        };
        if (b->dim == 3)
            for (int w = 3; w >= 2; --w)
                for (int remap = 1; remap >= 0; --remap) {
                    pb_tuning t = plain(remap);
                    t.fv_column = w;
                    c.push_back(t);
                }
        if (b->dim == 3 && b->uniform_p)
            for (int remap = 1; remap >= 0; --remap) {
                pb_tuning t = plain(remap);
                t.fv_persist = 3;
                c.push_back(t);
            }
        for (int remap = 1; remap >= 0; --remap)
            for (int s : slabs) {
                pb_tuning t = plain(remap);
                t.fv_slab = s;
                c.push_back(t);
            }
        if (fv_dma_eligible(b))
            for (int remap = 1; remap >= 0; --remap)
                for (int i = 0; i < 2 && i < (int)slabs.size(); ++i) {
                    pb_tuning t = plain(remap);
                    t.fv_slab = slabs[i];
                    t.fv_dma = 1;
                    c.push_back(t);
                }
    } else if (b->pde == PB_PDE_EULER) {
        if (b->uniform_p && b->p[0] * b->p[0] * b->p[0] <= 256) {
            c.push_back(base);   // the small-patch kernel has no launch-shape choices
        } else {
            for (int w : {2, 4, 0})
                for (int remap = 1; remap >= 0; --remap) {
                    pb_tuning t = base;
                    t.fd_column = w;
                    t.fd_xcd_remap = remap;
                    c.push_back(t);
                }
        }
    } else {
        for (int ws = 2; ws >= 1; --ws)
            for (int remap = 1; remap >= 0; --remap) {
                pb_tuning t = base;
                t.fd_ws = ws;
                t.fd_xcd_remap = remap;
                c.push_back(t);
            }
        for (int wg = 2; wg >= 1; --wg)
            for (int remap = 1; remap >= 0; --remap) {
                pb_tuning t = base;
                t.fd_ws = 0;
                t.fd_xcd_remap = remap;
                t.fd_wg_per_cu = wg;
                c.push_back(t);
            }
    }
    if ((int)c.size() > PB_TUNE_MAX) c.resize(PB_TUNE_MAX);
    return c;
}

// one trial launch of the tuned kernel (see the header of this file)
pb_status trial(pb_batch *b, int kind, double cfl, double dt_fixed, double sigma, hipStream_t s)
{
    void *qin = b->state[b->cur], *qout = b->state[b->cur ^ 1];
    if (kind == 0) return launch_fv_step(b, qin, qout, 0, 0, dt_fixed, cfl, s);
    const WsLayout L = ws_layout(b->pde, b->dim, b->h, b->total_cells, b->N, b->storage, b->K);
    if (b->pde == PB_PDE_EULER)   // RK stage 1: reads Q^n, writes the stage value and the other state buffer
        return launch_fd_euler_stage(b, 0, 4, qin, qin, b->ws + L.yA, qout, 0, dt_fixed, cfl, sigma, s);
    return launch_fd_stage(b, 0, 4, qin, qin, b->ws + L.yA, qout, fd_dt(b, cfl, dt_fixed), sigma, s);
}

}  // namespace
}  // namespace pb

using namespace pb;

extern "C" {

pb_status pb_autotune(pb_batch *b, int32_t kind, double cfl, double dt_fixed, double sigma_ko, int32_t trials,
                      int32_t use_cache, pb_autotune_result *out)
{
    PB_API_BEGIN
    if (!b || !out) { set_error("NULL argument"); return PB_EINVAL; }
    if (kind != 0 && kind != 1) { set_error("pb_autotune: kind must be 0 (FV) or 1 (FD)"); return PB_EINVAL; }
    if (trials < 1 || trials > 1000) { set_error("pb_autotune: trials must be in [1, 1000]"); return PB_EINVAL; }
    if (kind == 0 && b->pde == PB_PDE_LINSYM) { set_error("pb_autotune: the linear system has no FV step"); return PB_EINVAL; }
    if (kind == 1 && b->pde != PB_PDE_LINSYM && b->pde != PB_PDE_EULER) {
        set_error("pb_autotune: FD tuning applies to the linear system and to Euler");
        return PB_EINVAL;
    }
    if (kind == 1 && b->pde == PB_PDE_EULER &&
        (b->dim != 3 || b->storage != PB_STORE_FP64 || b->pmax > kFvPmax || b->h < 3)) {
        set_error("pb_autotune: the Euler FD step needs dim 3, FP64 storage, p <= 16 and a halo of 3");
        return PB_EUNSUPPORTED;
    }
    if (kind == 0 && b->pde == PB_PDE_SRHD && b->storage != PB_STORE_FP64) { set_error("SRHD runs in FP64 storage"); return PB_EUNSUPPORTED; }
    if (kind == 0 && b->pmax > kFvPmax) { set_error("fv_rusanov_step: p > 16 is not supported"); return PB_EUNSUPPORTED; }
    if (!std::isfinite(dt_fixed) || (!(dt_fixed > 0.0) && !(cfl > 0.0 && std::isfinite(cfl)))) {
        set_error("need dt_fixed > 0 or a finite cfl > 0");
        return PB_EINVAL;
    }
    if (kind == 1 && (!std::isfinite(sigma_ko) || sigma_ko < 0.0)) { set_error("sigma_ko must be finite and >= 0"); return PB_EINVAL; }
    *out = pb_autotune_result{};
    const std::string key = tune_key(b, kind);
    const std::vector<pb_tuning> cand = candidates(b, kind);
    out->n_candidates = (int32_t)cand.size();
    for (size_t i = 0; i < cand.size(); ++i) out->cand[i] = cand[i];
    if (use_cache) {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            out->from_cache = 1;
            out->n_candidates = 1;
            out->cand[0] = it->second;
            out->cand_us[0] = 0.0;
            return pb_batch_set_tuning(b, &it->second);
        }
    }
    if (kind == 1 && b->pde == PB_PDE_LINSYM) {
        pb_status st = fd_prepare(b);
        if (st != PB_OK) return st;
    }
    hipStream_t s = b->stream;
    const pb_tuning before = current(b);
    // save the control block; prepare the dt / pressure inputs of the trials
    Ctrl saved;
    PB_HIP(hipMemcpyAsync(&saved, b->ws, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    PB_HIP(hipStreamSynchronize(s));
    const bool cfl_mode = !(dt_fixed > 0.0);
    pb_status st = PB_OK;
    if (kind == 0) {
        if (b->pde == PB_PDE_SRHD)
            st = launch_srhd_c2p(b, b->state[b->cur], 0, cfl_mode, cfl, s);
        else if (cfl_mode)
            st = launch_fv_lambda(b, b->state[b->cur], cfl, s);
    } else if (b->pde == PB_PDE_EULER && cfl_mode) {
        st = launch_fv_lambda(b, b->state[b->cur], cfl, s);   // dt of Q^n into slot 0, as a step's start
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st == PB_OK && hipEventCreate(&e0) != hipSuccess) st = hip_fail(hipErrorUnknown, "hipEventCreate");
    if (st == PB_OK && hipEventCreate(&e1) != hipSuccess) st = hip_fail(hipErrorUnknown, "hipEventCreate");
    std::vector<double> best_avg(cand.size(), 1e300);
    for (int pass = 0; pass < 2 && st == PB_OK; ++pass) {
        for (size_t ci = 0; ci < cand.size() && st == PB_OK; ++ci) {
            // second pass in reverse order, so drift does not favour one end
            const size_t i = pass == 0 ? ci : cand.size() - 1 - ci;
            if ((st = apply(b, cand[i])) != PB_OK) break;
            if ((st = trial(b, kind, cfl, dt_fixed, sigma_ko, s)) != PB_OK) break;
            hipError_t e = hipEventRecord(e0, s);
            for (int r = 0; r < trials && e == hipSuccess && st == PB_OK; ++r)
                st = trial(b, kind, cfl, dt_fixed, sigma_ko, s);
            if (st != PB_OK) break;
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) { st = hip_fail(e, "pb_autotune timing"); break; }
            best_avg[i] = std::min(best_avg[i], 1e3 * (double)ms / trials);
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    // restore the control block whatever happened
    hipError_t er = hipMemcpyAsync(b->ws, &saved, sizeof(Ctrl), hipMemcpyHostToDevice, s);
    if (er == hipSuccess) er = hipStreamSynchronize(s);
    if (st != PB_OK) {
        (void)pb_batch_set_tuning(b, &before);   // (also drops graphs that hold an older run table)
        return st;
    }
    if (er != hipSuccess) return hip_fail(er, "pb_autotune: restoring the control block");
    size_t bi = 0;
    for (size_t i = 0; i < cand.size(); ++i) {
        out->cand_us[i] = best_avg[i];
        if (best_avg[i] < best_avg[bi]) bi = i;
    }
    out->best = (int32_t)bi;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[key] = cand[bi];
    }
    return pb_batch_set_tuning(b, &cand[bi]);
    PB_API_END
}

pb_status pb_autotune_cache_save(const char *path)
{
    PB_API_BEGIN
    if (!path) { set_error("NULL path"); return PB_EINVAL; }
    std::ofstream f(path, std::ios::trunc);
    if (!f) { set_error(std::string("cannot open ") + path + " for writing"); return PB_EINVAL; }
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &e : g_cache)
        f << e.first << ' ' << e.second.fv_slab << ' ' << e.second.fv_xcd_remap << ' ' << e.second.fd_xcd_remap << ' '
          << e.second.fd_wg_per_cu << ' ' << e.second.fv_dma << ' ' << e.second.fd_ws << ' ' << e.second.fv_persist
          << ' ' << e.second.fv_column << ' ' << e.second.fd_column << '\n';
    if (!f) { set_error(std::string("write failed: ") + path); return PB_EINVAL; }
    return PB_OK;
    PB_API_END
}

pb_status pb_autotune_cache_load(const char *path, int32_t *n_loaded)
{
    PB_API_BEGIN
    if (!path) { set_error("NULL path"); return PB_EINVAL; }
    if (n_loaded) *n_loaded = 0;
    std::ifstream f(path);
    if (!f) { set_error(std::string("cannot open ") + path); return PB_EINVAL; }
    std::string line;
    int n = 0, lineno = 0;
    while (std::getline(f, line)) {
        ++lineno;
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        std::istringstream in(line);
        std::string key, extra;
        pb_tuning t{};
        bool ok = (bool)(in >> key >> t.fv_slab >> t.fv_xcd_remap >> t.fd_xcd_remap >> t.fd_wg_per_cu >> t.fv_dma >>
                         t.fd_ws);
        // shorter lines (written before the later fields existed) load those
        // fields at their defaults: fv_persist 0, fv_column 0, fd_column 2
        t.fd_column = 2;
        if (ok && !(in >> t.fv_persist)) {
            t.fv_persist = 0;
            in.clear();
        } else if (ok && !(in >> t.fv_column)) {
            t.fv_column = 0;
            in.clear();
        } else if (ok && !(in >> t.fd_column)) {
            t.fd_column = 2;
            in.clear();
        }
        if (!ok || (in >> extra) || t.fv_persist < 0 || t.fv_persist > 8 || t.fv_column < 0 || t.fv_column > 8 ||
            t.fd_column < 0 || t.fd_column > 8 ||
            t.fv_slab < 0 || t.fv_slab > kFvPmax || t.fv_xcd_remap < 0 || t.fv_xcd_remap > 1 ||
            t.fd_xcd_remap < 0 || t.fd_xcd_remap > 1 || t.fd_wg_per_cu < 0 || t.fd_wg_per_cu > 2 || t.fv_dma < 0 ||
            t.fv_dma > 1 || t.fd_ws < 0 || t.fd_ws > 2) {
            set_error(std::string(path) + ":" + std::to_string(lineno) + ": malformed tuning entry");
            if (n_loaded) *n_loaded = n;
            return PB_EINVAL;
        }
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[key] = t;
        ++n;
    }
    if (n_loaded) *n_loaded = n;
    return PB_OK;
    PB_API_END
}

pb_status pb_autotune_cache_clear(void)
{
    PB_API_BEGIN
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache.clear();
    return PB_OK;
    PB_API_END
}

}  // extern "C"

// pb_common.h -- internal declarations shared by the library's translation
// units (host runtime and HIP kernels).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <exception>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/patchhip.h"

namespace pb {

constexpr int kWave = 64;
constexpr int kFvThreads = 256;   // one 16x16 plane per work-group
constexpr int kFvPmax = 16;

// One patch as the kernels see it (48 bytes, 16-aligned).
struct alignas(16) PatchDev {
    long long off;   // first cell of the patch (cells, not elements)
    int p;           // cells per direction
    int nbr[6];      // face neighbours -x,+x,-y,+y,-z,+z
    int pad;
    double inv_dx;   // 1 / dx
};
static_assert(sizeof(PatchDev) == 48, "PatchDev layout");

// Control block at the start of the workspace (256 bytes).
struct Ctrl {
    double dt[2];                       // step sizes, ping-ponged by step parity
    unsigned long long reserved[4];
    unsigned long long nonfinite;       // units that produced NaN/Inf
    unsigned long long c2p_cells;
    unsigned long long c2p_fail;
    unsigned long long c2p_iters;
    unsigned long long c2p_fallback;
    unsigned int c2p_maxit;
    unsigned int pad0;
    double last_dt;
    unsigned long long lmax[3][3];      // FV steps of a call: largest speeds (IEEE bits) by step % 3
    unsigned long long pad[10];
};
static_assert(sizeof(Ctrl) == 256, "Ctrl layout");

// thread-local error text
void set_error(const std::string &msg);
pb_status hip_fail(hipError_t e, const char *what);

// Every C-ABI entry point runs its body between PB_API_BEGIN and PB_API_END,
// so no C++ exception (a failed host allocation, a thread that could not
// start) crosses the C boundary: it becomes PB_ENOMEM or PB_EINVAL with a
// message.
pb_status api_fail(const char *what, pb_status st) noexcept;
#define PB_API_BEGIN try {
#define PB_API_END                                                                                    \
    }                                                                                                 \
    catch (const std::bad_alloc &) { return ::pb::api_fail("out of host memory", PB_ENOMEM); }        \
    catch (const std::exception &e_) { return ::pb::api_fail(e_.what(), PB_EINVAL); }               \
    catch (...) { return ::pb::api_fail("unexpected host error", PB_EINVAL); }

#define PB_HIP(call)                                          \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return ::pb::hip_fail(e_, #call); \
    } while (0)

// ------------------------------------------------------------ device utils

__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ unsigned long long dbits(double v)
{
    return (unsigned long long)__double_as_longlong(v);
}

// Work-group order -> unit order such that the units one XCD runs (the
// hardware deals work-groups round-robin over the 8 XCDs) are consecutive:
// neighbouring patches then share that XCD's L2 for their halo reads.
// Global -> LDS DMA (gfx950 global_load_lds_dword / _dwordx4): every active
// lane copies 4 / 16 bytes from its global address to lds + 4 / 16 * lane.
// The destination is wave-uniform (M0).  They are issued from inline
// assembly on purpose: the compiler then does not add conservative waits for
// them before unrelated LDS reads (its alias tracking of such copies gives up
// when a kernel has many of them), and the callers wait explicitly
// (s_waitcnt vmcnt) before they read the copied data.  The instructions have
// no register results; the memory clobber keeps LDS accesses in order.
__device__ __forceinline__ unsigned lds_address(const void *p)
{
    return (unsigned)(size_t)((__attribute__((address_space(3))) const void *)p);
}

__device__ __forceinline__ void dma_to_lds16(const void *g, const void *lds)
{
    const unsigned a = __builtin_amdgcn_readfirstlane(lds_address(lds));
    __asm__ volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off" : : "s"(a), "v"(g) : "memory", "m0");
}

__device__ __forceinline__ void dma_to_lds4(const void *g, const void *lds)
{
    const unsigned a = __builtin_amdgcn_readfirstlane(lds_address(lds));
    __asm__ volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dword %1, off" : : "s"(a), "v"(g) : "memory", "m0");
}

// Work-group max of lm[0..DIM) stored as this unit's partial (plain stores,
// no atomics and no fence: the kernel boundary makes them visible to the
// reduction kernel that follows).  Layout: part[d * n_units + unit].
template <int DIM>
__device__ __forceinline__ void store_partial(double *__restrict__ part, const double *lm, int unit,
                                              int n_units)
{
    __shared__ double red[3][kFvThreads / kWave];
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const double m = wave_max(lm[d]);
        if (lane == 0) red[d][w] = m;
    }
    __syncthreads();
    if (t < DIM) {
        double m = red[t][0];
        for (int i = 1; i < (int)(blockDim.x / kWave); ++i) m = fmax(m, red[t][i]);
        part[(long long)t * n_units + unit] = m;
    }
}

// Hand-over of the CFL maxima between the FV steps of one call, with no
// reduction kernel between them.  Step i of a call (step >= 0) folds the
// largest speeds of its new state into lmax[i % 3] by atomicMax on the
// IEEE-754 bit patterns: exact and independent of the order, since the
// maxima are >= 0 and never NaN (fmax from 0 drops NaN speeds) and such
// doubles order as their bit patterns.  Step i > 0 takes dt from
// lmax[(i - 1) % 3] with the reduction kernel's arithmetic
// (dt = cfl / sum_d Lambda_d / dx_min); its work-group 0 records that dt in
// ctrl->dt[slot] for the host and clears lmax[(i + 1) % 3] for step i + 1
// (last written two steps before and last read one step before, by kernels
// that have finished).  Step 0 reads ctrl->dt[slot], which the reduction at
// the start of the call writes; that reduction also clears lmax[0].
// step < 0: the step stores its partials for a reduction kernel instead.
struct FvChain {
    int step;
    double cfl, dxmin;
};

template <int DIM>
__device__ __forceinline__ double chain_dt(const Ctrl *ctrl, const FvChain &c)
{
    const int r = (c.step + 2) % 3;
    double den = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) den += __longlong_as_double((long long)ctrl->lmax[r][d]) / c.dxmin;
    return c.cfl / den;
}

// the step's dt: fixed, handed over from the previous step of the call, or
// from the reduction kernel (see FvChain)
template <int DIM, bool kLam>
__device__ __forceinline__ double step_dt(Ctrl *ctrl, int slot_in, double dt_fixed, const FvChain &c)
{
    if (dt_fixed > 0.0) return dt_fixed;
    if (kLam && c.step > 0) {
        const double dt = chain_dt<DIM>(ctrl, c);
        if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->dt[slot_in] = dt;
        return dt;
    }
    return ctrl->dt[slot_in];
}

// the largest speeds of a work-group's cells: to the partials (c.step < 0)
// or folded into the control block (see FvChain)
template <int DIM>
__device__ __forceinline__ void fold_speeds(Ctrl *ctrl, double *__restrict__ part, const double *lm, int unit,
                                            int n_units, const FvChain &c)
{
    if (c.step < 0) {
        store_partial<DIM>(part, lm, unit, n_units);
        return;
    }
    __shared__ double red[3][kFvThreads / kWave];
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const double m = wave_max(lm[d]);
        if (lane == 0) red[d][w] = m;
    }
    __syncthreads();
    if (t < DIM) {
        double m = red[t][0];
        for (int i = 1; i < (int)(blockDim.x / kWave); ++i) m = fmax(m, red[t][i]);
        atomicMax(&ctrl->lmax[c.step % 3][t], (unsigned long long)__double_as_longlong(m));
    }
    if (blockIdx.x == 0 && t >= kWave && t < kWave + 3) ctrl->lmax[(c.step + 1) % 3][t - kWave] = 0ull;
}

// Work-group barrier for the LDS exchange only: wait for this wave's LDS
// writes, then the bare barrier instruction (the compiler memory clobber
// keeps LDS accesses on their side of it).  __syncthreads() would also wait
// for every global load and store the wave has in flight (its fence covers
// global memory), draining the prefetch of the next planes and the stores of
// the last one at every barrier.  Only for kernels in which no thread reads
// global data another thread of the launch writes.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0), vmcnt and expcnt unconstrained
    __asm__ volatile("s_barrier" ::: "memory");
}

__device__ __forceinline__ int xcd_remap(int bid, int n)
{
    const int q = n >> 3, r = n & 7;
    const int x = bid & 7, j = bid >> 3;
    return x * q + (x < r ? x : r) + j;
}

}  // namespace pb

// ------------------------------------------------------------------------
// Host runtime object (defined here so that every translation unit of the
// library can read it).
struct pb_batch {
    int dim = 0, K = 0, N = 0, h = 0, pde = 0, storage = 0;
    std::vector<int> p;
    std::vector<double> dx;
    std::vector<int> nbr;
    std::vector<double> params;
    void *state[2] = {nullptr, nullptr};
    int cur = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    long long total_cells = 0;
    double dxmin = 0.0;
    int pmax = 0;
    bool uniform_p = true;
    pb::PatchDev *d_patches = nullptr;
    long long steps = 0;
    double last_dt_host = 0.0;
    // tuning
    int fv_slab = 0;
    int fv_xcd_remap = 1;
    int fd_xcd_remap = 1;
    int fd_wg_per_cu = 2;
    int fd_ws = 1;   // linear-system FD: wave-specialised kernel
    int fv_dma = 0;
    int fv_persist = 0;   // FV 3D, one p: > 0 = balanced plane schedule over this many work-groups per CU
    int fv_column = 0;    // FV 3D: > 0 = column runs along +z chains, about this many work-groups per CU
    int fd_column = 2;    // Euler FD: likewise (runs of whole patches at least); 0 = one work-group per patch
    // column-run tables (int4: patch, first plane, planes, 0; one per unit)
    // of the FV and the Euler FD plane kernels, and the w each was built for
    struct RunTable {
        void *d = nullptr;
        int n = 0, w = 0;
    };
    RunTable fv_runs, fd_runs;
    // SRHD guess mode
    int guess = PB_GUESS_PLAIN;
    const pb_mlp *mlp = nullptr;
    bool pres_valid = false;         // SRHD: the workspace holds a previous pressure
    // FD: tile work list (largest patches first) and the B_d matrices
    bool fd_ready = false;
    void *d_fd_items = nullptr;
    void *d_fd_ws_items = nullptr;   // per-tile geometry of the wave-specialised kernel
    int fd_n_items = 0;
    double *d_fd_B = nullptr;
    double *d_fd_A = nullptr;        // A operands of the one-wave-per-tile FD kernel
    // graph cache
    struct GraphEntry {
        int kind, n_steps, parity_cur;
        double key0, key1, key2;
        int key3;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    hipStream_t capture_stream = nullptr;
    int last_slot = 0;
    // event timing of the step kernels (eager mode only): one event pair per
    // launch, or in span mode one pair per run of back-to-back launches of
    // the FV step kernel (the first launch's start, the last launch's end)
    bool profiling = false, prof_span = false;
    int prof_n = 0;                 // completed event pairs
    long long prof_launches = 0;    // launches those pairs cover
    long long prof_pending = 0;     // launches of the pair still open
    std::vector<hipEvent_t> prof_ev[2];
    // events the next main-kernel launch sets from its own start and end
    // (null: that end is not recorded)
    hipEvent_t kev[2] = {nullptr, nullptr};
};

namespace pb {
// workspace sub-ranges (byte offsets), from the batch description
struct WsLayout {
    size_t ctrl = 0;       // Ctrl
    size_t part = 0;       // per-unit partials [8][units]: speeds (3), con2prim stats (5)
    size_t pres = 0;       // SRHD: pressure per cell (double)
    size_t yA = 0, yB = 0; // FD: stage buffers
    size_t total = 0;
};
// the FD step's two stage buffers exist for the linear system and for 3D
// Euler batches whose halo reaches the FD stencil (h >= 3)
inline bool fd_buffers(int pde, int dim, int h)
{
    return pde == PB_PDE_LINSYM || (pde == PB_PDE_EULER && dim == 3 && h >= 3);
}
WsLayout ws_layout(int pde, int dim, int h, long long total_cells, int N, int storage, int K);
// largest number of work units any launch uses (partials are sized for it)
inline long long max_units(int K) { return (long long)K * kFvPmax; }

// launches a step's main kernel (the FV step, an FD stage) with its arguments
// converted to the kernel's parameter types; when the batch is profiling, the
// dispatch itself sets the events it is given to its start and end
// (hipExtLaunchKernel), so a pair on one launch times the kernel alone,
// without the launch gap or the dt reduction that may follow it on the stream
template <typename... P, typename... Args>
inline void launch_main(const pb_batch *b, void (*kern)(P...), dim3 grid, dim3 block, size_t lds, hipStream_t s,
                        Args... args)
{
    static_assert(sizeof...(P) == sizeof...(Args), "kernel argument count");
    std::tuple<P...> a{static_cast<P>(args)...};
    void *ptrs[sizeof...(P)];
    std::apply([&ptrs](auto &...x) { int i = 0; ((ptrs[i++] = static_cast<void *>(&x)), ...); }, a);
    if (b->kev[0] || b->kev[1])
        (void)hipExtLaunchKernel(reinterpret_cast<const void *>(kern), grid, block, ptrs, lds, s, b->kev[0],
                                 b->kev[1], 0);
    else
        (void)hipLaunchKernel(reinterpret_cast<const void *>(kern), grid, block, ptrs, lds, s);
}

// launchers (implemented in the kernel translation units)
pb_status launch_fv_lambda(pb_batch *b, const void *q, double cfl, hipStream_t s);
pb_status launch_fv_step(pb_batch *b, const void *qin, void *qout, int slot_in, int step, double dt_fixed,
                         double cfl, hipStream_t s);
pb_status launch_srhd_c2p(pb_batch *b, const void *q, int slot_out, bool want_dt, double cfl,
                          hipStream_t s);
pb_status launch_fd_stage(pb_batch *b, int stage, int rk_stages, const void *q0, const void *y,
                          void *ynext, void *acc, double dt, double sigma, hipStream_t s);
// one stage of the Euler FD4 + KO6 step (dt from ctrl->dt[slot] unless
// dt_fixed > 0; the last stage writes the next step's dt to slot ^ 1)
pb_status launch_fd_euler_stage(pb_batch *b, int stage, int rk_stages, const void *q0, const void *y, void *ynext,
                                void *acc, int slot, double dt_fixed, double cfl, double sigma, hipStream_t s);
// the DMA-fed FV kernel applies to this batch (3D, no extra per-cell input,
// every p a multiple of 4, 16-byte aligned state buffers)
bool fv_dma_eligible(const pb_batch *b);
// the small-patch FV kernel applies (3D, one p, p^3 <= 256 threads); its
// work-groups take as many patches as fit 256 threads and an LDS box of
// (p+2)^3 slots of N + A doubles per patch within kFvSmallLds bytes
constexpr size_t kFvSmallLds = 64 * 1024;
bool fv_small_eligible(const pb_batch *b);
// the column runs (patch, first plane, planes, 0) of a 3D batch with
// neighbour table nbr [K][6], about w work-groups per CU on `cus` CUs.
// kind 0 (FV): links between patches of one p >= 2, runs of any length;
// kind 1 (Euler FD, halo 3): links between patches of one p >= 4, runs of
// whole patches at least.
std::vector<int4> column_runs(int kind, int K, const int *p, const int *nbr, int w, int cus);
// (re)builds the column-run tables for b->fv_column and b->fd_column (a
// table is freed when its w is 0 or does not apply); host call, done when
// the batch is created and when its tuning is set, never inside a capture
pb_status runs_prepare(pb_batch *b);
// dt of an FD step: dt_fixed if > 0, else cfl / sum_d (rho(B_d) / dx_min)
double fd_dt(const pb_batch *b, double cfl, double dt_fixed);
// uploads the FD work list and B_d (library-owned; done once, before any capture)
pb_status fd_prepare(pb_batch *b);
pb_status launch_ctrl_init(pb_batch *b, hipStream_t s);
pb_status launch_dt_reduce(pb_batch *b, const double *part, int n_units, int dim, int slot, double cfl, bool want_dt,
                           bool want_stats, hipStream_t s);
}  // namespace pb

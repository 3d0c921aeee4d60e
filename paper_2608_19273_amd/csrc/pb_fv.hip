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
#include <mutex>
#include <type_traits>
#include <vector>

#include "pb_common.h"
#include "pb_physics.h"

namespace pb {

constexpr int kReduceSpan = 256;    // units per work-group of the first reduction stage
constexpr int kReduceOne = 8192;    // up to this many units the single-work-group reduction runs alone

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

// Largest speeds of a freshly written cell, for the next step's dt only: the
// aux evaluation uses the reciprocal / rsqrt estimates refined by Newton
// steps (a max over cells needs no correctly rounded quotient).
template <class Ph, int DIM>
__device__ __forceinline__ void cell_speeds_fast(const Ph &ph, const double *q, double *lm)
{
    constexpr int AA = Ph::A > 0 ? Ph::A : 1;
    double a[AA], e[1] = {0.0};
    ph.aux_fast(q, e, a);
    cell_speeds<Ph, DIM>(ph, q, a, lm);
}

}  // namespace

// raw (storage-type) values of one cell: N unknowns plus the extra input
template <class Ph, typename T>
struct RawCell {
    T q[Ph::N];
    double e;
};

template <class Ph, typename T>
__device__ __forceinline__ void issue_load(const T *__restrict__ q, const double *__restrict__ ex,
                                           long long off, long long C, long long c, RawCell<Ph, T> &r)
{
    const T *base = q + off * Ph::N + c;
#pragma unroll
    for (int v = 0; v < Ph::N; ++v) r.q[v] = base[(long long)v * C];
    if (Ph::E) r.e = ex[off + c];
}

template <class Ph, typename T>
__device__ __forceinline__ void unpack(const RawCell<Ph, T> &r, double *q, double *e)
{
#pragma unroll
    for (int v = 0; v < Ph::N; ++v) q[v] = (double)r.q[v];
    e[0] = Ph::E ? r.e : 0.0;
}

template <class Ph, int D>
__device__ __forceinline__ void phys_flux_or_zero(const Ph &ph, const double *q, const double *a, double *F)
{
    if (Ph::kFlux) {
        ph.template flux<D>(q, a, F);
    } else {
#pragma unroll
        for (int v = 0; v < Ph::N; ++v) F[v] = 0.0;
    }
}

// The aux values an x or y neighbour's flux and speed read, which the plane
// kernel passes through LDS: all of them, except for SRHD, whose direction d
// reads p, v_d and lambda_d only, so v_z and lambda_z stay in the z carry
// (10 instead of 12 values per cell: three work-groups fit a CU's LDS).
template <class Ph> struct PlaneAux {
    static constexpr int n = Ph::A;
    static __device__ __forceinline__ constexpr int idx(int j) { return j; }
};
template <> struct PlaneAux<Srhd> {
    static constexpr int n = 5;
    static __device__ __forceinline__ constexpr int idx(int j) { return j < 3 ? j : j + 1; }   // p, v_x, v_y, l_x, l_y
};

// Work schedule of the plane-march kernel.  Slab mode (plan.planes == 0):
// work-group (unit) u marches slab u % n_slabs of patch u / n_slabs (a slab
// can start beyond the last plane of a patch smaller than the batch maximum:
// such a unit only takes part in the reductions).  Balanced mode (uniform
// patch size p, plan.planes = K p planes in patch order): the grid is a
// chosen number of work-groups per CU (those that fit at once: no second
// round) and work-group r marches the planes
// [r T / G, (r + 1) T / G) of that sequence, one segment per patch it
// crosses, so every work-group moves the same number of planes and the last
// round of a grid of whole patches, partly filled, disappears.  Column mode
// (plan.runs): unit u marches runs[u].z planes starting at plane runs[u].y of
// patch runs[u].x and continuing, without a restart, into the +z neighbour
// (the z halo between consecutive patches of a run is the plane the march
// has just processed: it is never read twice).
struct FvPlan {
    int n_units, n_slabs, slab, remap;
    long long planes;   // balanced mode: total planes (0: slab mode)
    const int4 *runs;   // column mode (non-null): unit u marches runs[u] = (patch, first plane, planes)
};

template <class Ph, int DIM, typename T, bool kLam>
__global__ __launch_bounds__(kFvThreads) __attribute__((amdgpu_waves_per_eu(3))) void fv_step_kernel(
    const T *__restrict__ qin, T *__restrict__ qout, const double *__restrict__ ex,
    const PatchDev *__restrict__ patches, FvPlan plan, Ctrl *__restrict__ ctrl, double *__restrict__ part,
    int slot_in, double dt_fixed, FvChain chain, Ph ph)
{
    constexpr int N = Ph::N, A = Ph::A, AP = PlaneAux<Ph>::n, W = N + AP, AA = A > 0 ? A : 1;
    constexpr int PH = kFvPmax + 2;
    constexpr int DZ = DIM == 3 ? 2 : 1;   // z direction index (unused in 2D)
    __shared__ double lds[2][W][PH * PH];

    const int t = threadIdx.x;
    const int unit = plan.remap ? xcd_remap(blockIdx.x, plan.n_units) : (int)blockIdx.x;
    const double dt = step_dt<DIM, kLam>(ctrl, slot_in, dt_fixed, chain);
    double lm[3] = {0.0, 0.0, 0.0};
    bool bad = false;
    int parity = 0;   // LDS buffer of the next plane (alternates over every plane the work-group marches)

    // one segment: n planes starting at plane z0 of patch k, continuing into
    // the +z neighbour at the patch's top (the patches of a run share p)
    auto segment = [&](int k, int z0, int n) {
    const int p = patches[k].p;
    const long long C = (DIM == 3) ? (long long)p * p * p : (long long)p * p;

    const bool work = n > 0;
    const bool active = work && t < p * p;
    const int x = active ? t % p : 0, y = active ? t / p : 0;
    const int li = (y + 1) * PH + (x + 1);

    // face-halo cell of each plane: wave w serves side w (-x, +x, -y, +y),
    // so the extra loads and aux evaluations spread over all four waves
    const int side = __builtin_amdgcn_readfirstlane(t >> 6), j = t & 63;
    const bool halo = work && j < p;
    int hsrc = 0, hdst = 0;
    if (halo) {
        int hx, hy, sx, sy;
        if (side == 0)      { hx = -1; hy = j;  sx = p - 1; sy = j;     }
        else if (side == 1) { hx = p;  hy = j;  sx = 0;     sy = j;     }
        else if (side == 2) { hx = j;  hy = -1; sx = j;     sy = p - 1; }
        else                { hx = j;  hy = p;  sx = j;     sy = 0;     }
        hsrc = sy * p + sx;
        hdst = (hy + 1) * PH + (hx + 1);
    }
    const long long cxy = (long long)y * p + x;
    const long long pp = (long long)p * p;
    // the current patch and its +z neighbour (the run's next patch): cell
    // offsets of the patch and of the wave's halo-side neighbour (lanes
    // without a halo cell load cell 0 of that neighbour and drop it)
    long long offc = patches[k].off, hoffc = patches[patches[k].nbr[side]].off;
    double hr_ = 0.5 * dt * patches[k].inv_dx;   // the face sums below are doubled
    int kn = (DIM == 3) ? patches[k].nbr[5] : k;
    long long offn = patches[kn].off, hoffn = patches[patches[kn].nbr[side]].off;
    int zl = z0;   // the current plane's z inside the current patch

    // per thread, two sets that swap roles from plane to plane (the loop runs
    // two planes per trip, so nothing is copied between them): a plane's
    // values (q, a), its z flux and speed (fz, lz), and the doubled flux and
    // fluctuation of its lower z face (fs, dn)
    struct Carry {
        double q[N], a[AA], fz[N], fs[N], dn[N];
        double lz;
    };
    Carry cA, cB;
    double e[1];
    double *qc = cA.q, *ac = cA.a, *fzc = cA.fz, *fs2l = cA.fs, *dn2l = cA.dn;
    double &lzc = cA.lz;
    lzc = 0.0;
    // one-plane prefetch (raw storage-type values): the own column for plane
    // z+1 and the halo cell for plane z.  One plane ahead is as fast as two or
    // three, and with the next plane's flux evaluated after the x and y
    // directions the kernel fits in 3 waves per SIMD without spilling.
    RawCell<Ph, T> rnA, hrA;

    // plane zl + d (d = 0, 1, 2; p >= 2) of the run: the current patch or the next
    auto own_plane_off = [&](int zz) -> long long { return zz >= p ? offn : offc; };
    auto own_plane_c = [&](int zz) -> long long { return (zz >= p ? zz - p : zz) * pp + cxy; };

    // Every lane issues every load (idle lanes at a valid address they do not
    // use), and the prefetch at the slab's top reloads a plane in reach
    // instead of skipping: a load under a divergent or conditional branch
    // makes the compiler copy its target registers at the join, which waits
    // for the load right there and empties the prefetch ring.
    if (work) {
        RawCell<Ph, T> rc;
        issue_load<Ph>(qin, ex, offc, C, z0 * pp + cxy, rc);
        if (DIM == 3) {
            RawCell<Ph, T> rm;
            const long long om = (z0 == 0) ? patches[patches[k].nbr[4]].off : offc;
            const int zm = (z0 == 0) ? p - 1 : z0 - 1;
            issue_load<Ph>(qin, ex, om, C, zm * pp + cxy, rm);
            issue_load<Ph>(qin, ex, own_plane_off(z0 + 1), C, own_plane_c(z0 + 1), rnA);
            double qm[N], am[AA], fzm[N];
            unpack<Ph>(rm, qm, e);
            ph.aux(qm, e, am);
            phys_flux_or_zero<Ph, DZ>(ph, qm, am, fzm);
            unpack<Ph>(rc, qc, e);
            ph.aux(qc, e, ac);
            phys_flux_or_zero<Ph, DZ>(ph, qc, ac, fzc);
            lzc = ph.template eig<DZ>(qc, ac);
            rusanov_face2<Ph, DZ>(ph, qm, fzm, ph.template eig<DZ>(qm, am), qc, fzc, lzc, fs2l, dn2l);
        } else {
            unpack<Ph>(rc, qc, e);
            ph.aux(qc, e, ac);
        }
    }
    if (work) {
        issue_load<Ph>(qin, ex, hoffc, C, z0 * pp + hsrc, hrA);
    }

    // run plane i (at zl of the current patch): consumes rn (own plane i+1)
    // and hr (halo of plane i), then refills them with planes i+2 and i+1,
    // clamped to the plane after the run and to the run's last plane
    auto plane = [&](int i, RawCell<Ph, T> &rn, RawCell<Ph, T> &hr, Carry &cur, Carry &nxt) {
        const double *qc = cur.q, *ac = cur.a, *fzc = cur.fz, *fs2l = cur.fs, *dn2l = cur.dn;
        const double lzc = cur.lz;
        double(*buf)[PH * PH] = lds[parity];
        parity ^= 1;
        double hq[N], he[1];
        unpack<Ph>(hr, hq, he);
        {
            const int zh = zl + min(1, n - 1 - i);
            issue_load<Ph>(qin, ex, zh >= p ? hoffn : hoffc, C, (zh >= p ? zh - p : zh) * pp + hsrc, hr);
        }
        if (halo) {
            double ha[AA];
            ph.aux(hq, he, ha);
#pragma unroll
            for (int v = 0; v < N; ++v) buf[v][hdst] = hq[v];
#pragma unroll
            for (int j = 0; j < AP; ++j) buf[N + j][hdst] = ha[PlaneAux<Ph>::idx(j)];
        }
        if (active) {
#pragma unroll
            for (int v = 0; v < N; ++v) buf[v][li] = qc[v];
#pragma unroll
            for (int j = 0; j < AP; ++j) buf[N + j][li] = ac[PlaneAux<Ph>::idx(j)];
        }
        lds_barrier();   // (no thread reads what another writes to global memory)
        double acc2[N];
#pragma unroll
        for (int v = 0; v < N; ++v) acc2[v] = 0.0;
        if (active) {
            {
                double qL[N], aL[AA], qR[N], aR[AA];
#pragma unroll
                for (int v = 0; v < N; ++v) { qL[v] = buf[v][li - 1]; qR[v] = buf[v][li + 1]; }
#pragma unroll
                for (int a = 0; a < AA; ++a) { aL[a] = 0.0; aR[a] = 0.0; }
#pragma unroll
                for (int j = 0; j < AP; ++j) {
                    aL[PlaneAux<Ph>::idx(j)] = buf[N + j][li - 1];
                    aR[PlaneAux<Ph>::idx(j)] = buf[N + j][li + 1];
                }
                rusanov_pair2<Ph, 0>(ph, qL, aL, qc, ac, qR, aR, acc2);
            }
            {
                double qL[N], aL[AA], qR[N], aR[AA];
#pragma unroll
                for (int v = 0; v < N; ++v) { qL[v] = buf[v][li - PH]; qR[v] = buf[v][li + PH]; }
#pragma unroll
                for (int a = 0; a < AA; ++a) { aL[a] = 0.0; aR[a] = 0.0; }
#pragma unroll
                for (int j = 0; j < AP; ++j) {
                    aL[PlaneAux<Ph>::idx(j)] = buf[N + j][li - PH];
                    aR[PlaneAux<Ph>::idx(j)] = buf[N + j][li + PH];
                }
                rusanov_pair2<Ph, 1>(ph, qL, aL, qc, ac, qR, aR, acc2);
            }
        }
        // the next plane's primitives, flux and speed, after the x and y
        // directions: fewer values are live at once (3 waves per SIMD)
        double *qn = nxt.q, *an = nxt.a, *fzn = nxt.fz;
        double &lzn = nxt.lz;
        lzn = 0.0;
        if (DIM == 3) {
            unpack<Ph>(rn, qn, e);
            const int z2 = zl + min(2, n - i);
            issue_load<Ph>(qin, ex, own_plane_off(z2), C, own_plane_c(z2), rn);
            ph.aux(qn, e, an);
            phys_flux_or_zero<Ph, DZ>(ph, qn, an, fzn);
            lzn = ph.template eig<DZ>(qn, an);
        }
        if (active) {
            if (DIM == 3) {
                double *fs2u = nxt.fs, *dn2u = nxt.dn;
                rusanov_face2<Ph, DZ>(ph, qc, fzc, lzc, qn, fzn, lzn, fs2u, dn2u);
#pragma unroll
                for (int v = 0; v < N; ++v) acc2[v] += (fs2u[v] - fs2l[v]) + (dn2u[v] + dn2l[v]);
            }
            double S[N];
            if (Ph::kSrc) {
                ph.source(qc, ac, S);
            } else {
#pragma unroll
                for (int v = 0; v < N; ++v) S[v] = 0.0;
            }
            double qw[N];
            T *dst = qout + offc * N + zl * pp + cxy;
#pragma unroll
            for (int v = 0; v < N; ++v) {
                const double nv = v < N - Ph::M ? qc[v] - hr_ * acc2[v] + dt * S[v] : qc[v];   // material: carried
                const T st = (T)nv;
                __builtin_nontemporal_store(st, dst + (long long)v * C);
                qw[v] = (double)st;
                bad |= !isfinite(qw[v]);
            }
            if (kLam) cell_speeds_fast<Ph, DIM>(ph, qw, lm);
        }
    };
    // after plane i: the run continues in the +z neighbour at the patch's top
    // (already the source of the loads issued for its first planes)
    auto advance = [&](int i) {
        if (DIM == 3 && ++zl == p && i + 1 < n) {
            zl = 0;
            offc = offn;
            hoffc = hoffn;
            hr_ = 0.5 * dt * patches[kn].inv_dx;
            kn = patches[kn].nbr[5];
            offn = patches[kn].off;
            hoffn = patches[patches[kn].nbr[side]].off;
        }
    };

    int i = 0;
    for (; i + 1 < n; i += 2) {
        plane(i, rnA, hrA, cA, cB);
        advance(i);
        plane(i + 1, rnA, hrA, cB, cA);
        advance(i + 1);
    }
    if (i < n) plane(i, rnA, hrA, cA, cB);
    };

    if (DIM == 3 && plan.runs) {
        const int4 r = plan.runs[unit];
        segment(r.x, r.y, r.z);
    } else if (DIM == 3 && plan.planes > 0) {
        // balanced mode: a contiguous run of planes (every patch has p planes)
        const int p = patches[0].p;
        const long long G = plan.n_units;
        long long s = plan.planes * unit / G;
        const long long s1 = plan.planes * (unit + 1) / G;
        while (s < s1) {
            const int k = (int)(s / p);
            const int za = (int)(s - (long long)k * p);
            const int zb = (int)min((long long)p, za + (s1 - s));
            segment(k, za, zb - za);
            s += zb - za;
        }
    } else {
        const int k = unit / plan.n_slabs, sl = unit - k * plan.n_slabs;
        const int p = patches[k].p;
        const int z0 = (DIM == 3) ? sl * plan.slab : 0;
        const int z1 = (DIM == 3) ? min(p, z0 + plan.slab) : 1;
        segment(k, min(z0, z1), max(0, z1 - z0));
    }
    if (__syncthreads_or(bad) && t == 0) atomicAdd(&ctrl->nonfinite, 1ull);
    if (kLam) fold_speeds<DIM>(ctrl, part, lm, unit, plan.n_units, chain);
}

// ---------------------------------------------------------------------------
// DMA-fed variant of the same step (3D, no extra per-cell input, p a
// multiple of 4): the state planes do not pass through registers.  Each
// plane of the slab (interior p x p cells and the four face-halo strips read
// from the neighbours) is copied HBM/L2 -> LDS by the gfx950 global->LDS DMA
// loads three planes ahead into a ring of four plane buffers, so about three
// planes of loads per work-group are always in flight and the waves only
// compute.  Interior and +-y strips move in 16-byte pieces, the strided
// +-x strips as 4-byte words.  Per plane z the work-group
//   1. writes the aux of its cells (computed one plane earlier) and of the
//      halo cells (computed now from the halo strips in LDS) to LDS;
//   2. waits for the DMA of plane z+1 (exact vmcnt: only the DMA and stores
//      issued after it may still be in flight) and meets at a bare barrier;
//   3. issues the DMA of plane z+3 into the buffer plane z-1 used;
//   4. evaluates the faces and updates the cell exactly as fv_step_kernel.
// The plane loop is dispatched on z % 4 to four copies of the body, each
// naming its buffers statically, so the compiler can tell the ring's buffers
// apart and does not wait for DMA into a buffer it is not reading.
namespace {

constexpr int kDmaNP = kFvPmax * kFvPmax + 4 * kFvPmax;   // slots per unknown and plane

// the wave index, as a value the compiler knows is the same in every lane
__device__ __forceinline__ int wave_index() { return __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6); }

// wait until at most n of this wave's vector-memory operations are in flight
__device__ __forceinline__ void wait_vm(int n)
{
    switch (n) {
    case 0: __builtin_amdgcn_s_waitcnt(0x0070); break;
    case 1: __builtin_amdgcn_s_waitcnt(0x0071); break;
    case 2: __builtin_amdgcn_s_waitcnt(0x0072); break;
    case 3: __builtin_amdgcn_s_waitcnt(0x0073); break;
    case 4: __builtin_amdgcn_s_waitcnt(0x0074); break;
    case 5: __builtin_amdgcn_s_waitcnt(0x0075); break;
    case 6: __builtin_amdgcn_s_waitcnt(0x0076); break;
    case 7: __builtin_amdgcn_s_waitcnt(0x0077); break;
    case 8: __builtin_amdgcn_s_waitcnt(0x0078); break;
    case 9: __builtin_amdgcn_s_waitcnt(0x0079); break;
    case 10: __builtin_amdgcn_s_waitcnt(0x007a); break;
    case 11: __builtin_amdgcn_s_waitcnt(0x007b); break;
    case 12: __builtin_amdgcn_s_waitcnt(0x007c); break;
    case 13: __builtin_amdgcn_s_waitcnt(0x007d); break;
    case 14: __builtin_amdgcn_s_waitcnt(0x007e); break;
    default: __builtin_amdgcn_s_waitcnt(0x007f); break;   // 15 (larger counts are clamped down: still safe)
    }
}

// the bare work-group barrier (no memory fence: callers wait for what they need)
__device__ __forceinline__ void bare_barrier() { __asm__ volatile("s_barrier" ::: "memory"); }

// DMA of one plane (plane index zl inside the source patch `own` for the
// interior; the halo strips from the face neighbours) into buf[N][kDmaNP].
// Jobs: per unknown `ji` interior pieces of 1 KB, one +-x job, one +-y job;
// job k runs on wave k % 4.  Every wave issues the same number of DMA
// instructions in every plane (lanes without data are masked).
__device__ __forceinline__ void dma_plane(void *buf_v, const void *q_v, int esz, int N, long long C, int p,
                                          long long own, const long long *onb, int zl, int ji, int w)
{
    char *buf = static_cast<char *>(buf_v);
    const char *q = static_cast<const char *>(q_v);
    const int epp = 16 / esz;   // elements per 16-byte piece
    const int dpe = esz / 4;    // 4-byte words per element
    const int L = threadIdx.x & 63;
    const long long pp = (long long)p * p;
    const int J = N * (ji + 2);
    for (int k = w; k < J; k += 4) {
        const int v = k / (ji + 2), r = k - v * (ji + 2);
        char *dst = buf + (long long)v * kDmaNP * esz;
        const long long row = (long long)v * C + zl * pp;   // element offset of the plane row in a patch block
        if (r < ji) {
            const int piece = 64 * r + L;
            if (piece * epp < pp)
                dma_to_lds16(q + (own * N + row + (long long)piece * epp) * esz, dst + 1024 * r);
        } else if (r == ji) {
            const int j = L / dpe, word = L - j * dpe;
            if (j < 2 * p) {
                const int side = j / p, yy = j - side * p;
                const long long e = onb[side] * N + row + (long long)yy * p + (side == 0 ? p - 1 : 0);
                dma_to_lds4(q + e * esz + 4 * word, dst + pp * esz);
            }
        } else {
            const int pps = p / epp;   // pieces per strip
            if (L < 2 * pps) {
                const int side = L / pps, kk = L - side * pps;
                const long long e = onb[2 + side] * N + row + (long long)(side == 0 ? p - 1 : 0) * p + kk * epp;
                dma_to_lds16(q + e * esz, dst + (pp + 2 * p) * esz);
            }
        }
    }
}

}  // namespace

template <class Ph, typename T, bool kLam>
__global__ __launch_bounds__(kFvThreads, 2) void fv_step_dma_kernel(
    const T *__restrict__ qin, T *__restrict__ qout, const PatchDev *__restrict__ patches, int n_units,
    int n_slabs, int slab, int remap, Ctrl *__restrict__ ctrl, double *__restrict__ part, int slot_in,
    double dt_fixed, FvChain chain, Ph ph)
{
    constexpr int N = Ph::N, A = Ph::A, AA = A > 0 ? A : 1;
    static_assert(Ph::E == 0, "the DMA variant has no extra per-cell input");
    __shared__ T sq0[N * kDmaNP], sq1[N * kDmaNP], sq2[N * kDmaNP], sq3[N * kDmaNP];
    __shared__ double sa[2][AA][kDmaNP];

    const int t = threadIdx.x, w = wave_index();
    const int unit = remap ? xcd_remap(blockIdx.x, n_units) : (int)blockIdx.x;
    const int k = unit / n_slabs, sl = unit - k * n_slabs;
    const PatchDev P = patches[k];
    const int p = P.p;
    const long long C = (long long)p * p * p, pp = (long long)p * p;
    long long onb[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) onb[f] = patches[P.nbr[f]].off;
    const int z0 = sl * slab, z1 = min(p, z0 + slab);
    const bool work = z0 < p;
    const bool active = work && t < pp;
    const int x = active ? t % p : 0, y = active ? t / p : 0;
    const double dt = step_dt<3, kLam>(ctrl, slot_in, dt_fixed, chain);
    const double hr_ = 0.5 * dt * P.inv_dx;
    // LDS slots of the cell and its four in-plane neighbours (halo strips
    // follow the p x p interior: -x, +x, -y, +y, p cells each)
    const int li = y * p + x;
    const int lxm = x == 0 ? (int)pp + y : li - 1, lxp = x == p - 1 ? (int)pp + p + y : li + 1;
    const int lym = y == 0 ? (int)pp + 2 * p + x : li - p, lyp = y == p - 1 ? (int)pp + 3 * p + x : li + p;
    // halo cells whose aux this thread evaluates: wave w serves strip w
    const int j = t & 63;
    const bool halo = work && j < p;
    const int hslot = (int)pp + w * p + j;
    // DMA instructions per wave and plane, and stores per wave and plane
    const int ji = (int)((pp * (long long)sizeof(T) + 1023) / 1024);
    const int J = N * (ji + 2);
    const int dw = (J - w + 3) / 4;
    const int sw = (64 * w < pp) ? N : 0;

    double lm[3] = {0.0, 0.0, 0.0};
    bool bad = false;
    if (work) {
        double qc[N], ac[AA], fzc[N], fs2l[N], dn2l[N], e[1] = {0.0};
        double lzc = 0.0;
        auto src_of = [&](int zz) __device__ -> long long { return zz >= p ? onb[5] : P.off; };
        auto dma = [&](int zz) __device__ {   // plane zz into ring buffer zz % 4
            T *b = (zz & 3) == 0 ? sq0 : (zz & 3) == 1 ? sq1 : (zz & 3) == 2 ? sq2 : sq3;
            dma_plane(b, qin, (int)sizeof(T), N, C, p, src_of(zz), onb, zz >= p ? zz - p : zz, ji, w);
        };
        auto d_of = [&](int zz) __device__ { return zz <= z1 ? dw : 0; };
        // the plane below the slab (for the first z face): a register load,
        // issued before the DMA so that waiting for it leaves the DMA in flight
        double qm[N];
        if (active) {
            const long long om = (z0 == 0) ? onb[4] : P.off;
            const int zm = (z0 == 0) ? p - 1 : z0 - 1;
            const T *b = qin + om * N + (long long)zm * pp + li;
#pragma unroll
            for (int v = 0; v < N; ++v) qm[v] = (double)b[(long long)v * C];
        }
        dma(z0);
        if (z0 + 1 <= z1) dma(z0 + 1);
        if (z0 + 2 <= z1) dma(z0 + 2);
        wait_vm(d_of(z0 + 1) + d_of(z0 + 2));
        bare_barrier();
        if (active) {
            const T *cb = (z0 & 3) == 0 ? sq0 : (z0 & 3) == 1 ? sq1 : (z0 & 3) == 2 ? sq2 : sq3;
#pragma unroll
            for (int v = 0; v < N; ++v) qc[v] = (double)cb[v * kDmaNP + li];
            double am[AA], fzm[N];
            ph.aux(qm, e, am);
            phys_flux_or_zero<Ph, 2>(ph, qm, am, fzm);
            ph.aux(qc, e, ac);
            phys_flux_or_zero<Ph, 2>(ph, qc, ac, fzc);
            lzc = ph.template eig<2>(qc, ac);
            rusanov_face2<Ph, 2>(ph, qm, fzm, ph.template eig<2>(qm, am), qc, fzc, lzc, fs2l, dn2l);
        }

        auto plane = [&](auto bufc, int z) __device__ {
            constexpr int B = decltype(bufc)::value;
            T *cur = B == 0 ? sq0 : B == 1 ? sq1 : B == 2 ? sq2 : sq3;
            T *nxt = B == 3 ? sq0 : B == 0 ? sq1 : B == 1 ? sq2 : sq3;
            T *prv = B == 1 ? sq0 : B == 2 ? sq1 : B == 3 ? sq2 : sq3;   // buffer of plane z-1 (= z+3)
            double(*sab)[kDmaNP] = sa[z & 1];
            // 1. aux of this plane's cells and halo cells to LDS
            if (active) {
#pragma unroll
                for (int a = 0; a < A; ++a) sab[a][li] = ac[a];
            }
            if (halo) {
                double hq[N], ha[AA];
#pragma unroll
                for (int v = 0; v < N; ++v) hq[v] = (double)cur[v * kDmaNP + hslot];
                ph.aux(hq, e, ha);
#pragma unroll
                for (int a = 0; a < A; ++a) sab[a][hslot] = ha[a];
            }
            // 2. plane z+1 landed (all but the DMA and stores issued after it)
            wait_vm(d_of(z + 2) + sw * min(2, z - z0));
            __builtin_amdgcn_s_waitcnt(0xc07f);   // this wave's LDS writes done
            bare_barrier();
            // 3. prefetch plane z+3 into the buffer plane z-1 used
            if (z + 3 <= z1)
                dma_plane(prv, qin, (int)sizeof(T), N, C, p, src_of(z + 3), onb, z + 3 >= p ? z + 3 - p : z + 3, ji, w);
            // 4. faces and update
            if (active) {
                double qn[N], an[AA], fzn[N];
#pragma unroll
                for (int v = 0; v < N; ++v) qn[v] = (double)nxt[v * kDmaNP + li];
                ph.aux(qn, e, an);
                phys_flux_or_zero<Ph, 2>(ph, qn, an, fzn);
                const double lzn = ph.template eig<2>(qn, an);
                double acc2[N];
#pragma unroll
                for (int v = 0; v < N; ++v) acc2[v] = 0.0;
                {
                    double qL[N], aL[AA], qR[N], aR[AA];
#pragma unroll
                    for (int v = 0; v < N; ++v) { qL[v] = (double)cur[v * kDmaNP + lxm]; qR[v] = (double)cur[v * kDmaNP + lxp]; }
#pragma unroll
                    for (int a = 0; a < A; ++a) { aL[a] = sab[a][lxm]; aR[a] = sab[a][lxp]; }
                    rusanov_pair2<Ph, 0>(ph, qL, aL, qc, ac, qR, aR, acc2);
                }
                {
                    double qL[N], aL[AA], qR[N], aR[AA];
#pragma unroll
                    for (int v = 0; v < N; ++v) { qL[v] = (double)cur[v * kDmaNP + lym]; qR[v] = (double)cur[v * kDmaNP + lyp]; }
#pragma unroll
                    for (int a = 0; a < A; ++a) { aL[a] = sab[a][lym]; aR[a] = sab[a][lyp]; }
                    rusanov_pair2<Ph, 1>(ph, qL, aL, qc, ac, qR, aR, acc2);
                }
                {
                    double fs2u[N], dn2u[N];
                    rusanov_face2<Ph, 2>(ph, qc, fzc, lzc, qn, fzn, lzn, fs2u, dn2u);
#pragma unroll
                    for (int v = 0; v < N; ++v) {
                        acc2[v] += (fs2u[v] - fs2l[v]) + (dn2u[v] + dn2l[v]);
                        fs2l[v] = fs2u[v];
                        dn2l[v] = dn2u[v];
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
                T *dst = qout + P.off * N + (long long)z * pp + li;
#pragma unroll
                for (int v = 0; v < N; ++v) {
                    const double nv = v < N - Ph::M ? qc[v] - hr_ * acc2[v] + dt * S[v] : qc[v];   // material: carried
                    const T st = (T)nv;
                    __builtin_nontemporal_store(st, dst + (long long)v * C);
                    qw[v] = (double)st;
                    bad |= !isfinite(qw[v]);
                }
                if (kLam) cell_speeds_fast<Ph, 3>(ph, qw, lm);
#pragma unroll
                for (int v = 0; v < N; ++v) { qc[v] = qn[v]; fzc[v] = fzn[v]; }
#pragma unroll
                for (int a = 0; a < A; ++a) ac[a] = an[a];
                lzc = lzn;
            }
        };
        for (int z = z0; z < z1; ++z) {
            switch (z & 3) {
            case 0: plane(std::integral_constant<int, 0>(), z); break;
            case 1: plane(std::integral_constant<int, 1>(), z); break;
            case 2: plane(std::integral_constant<int, 2>(), z); break;
            default: plane(std::integral_constant<int, 3>(), z); break;
            }
        }
        // no DMA may still write LDS when the work-group ends
        wait_vm(0);
    }
    if (__syncthreads_or(bad) && t == 0) atomicAdd(&ctrl->nonfinite, 1ull);
    if (kLam) fold_speeds<3>(ctrl, part, lm, unit, n_units, chain);
}

// ---------------------------------------------------------------------------
// Small patches (3D, one p for the whole batch, p^3 <= 256).  The plane march
// leaves most of a work-group idle when p^2 is small (9 of 256 threads for
// p = 3).  Here a work-group takes G whole patches, one thread per cell:
//   1. every thread stages its cell's Q and aux in an LDS box of (p+2)^3
//      slots per patch (edges and corners unused), and the work-group stages
//      the G * 6p^2 face-halo cells read from the neighbours (the halo
//      gather, again fused into the load);
//   2. after one barrier every thread evaluates the three directions in the
//      difference form of the plane kernel from its six face neighbours,
//      updates, stores and folds the speeds of the new state.
// G = min(256 / p^3, 64 KB / box) is chosen by the launcher.
template <class Ph, typename T, bool kLam>
__global__ __launch_bounds__(kFvThreads) void fv_small_kernel(
    const T *__restrict__ qin, T *__restrict__ qout, const double *__restrict__ ex,
    const PatchDev *__restrict__ patches, int K, int p, int G, Ctrl *__restrict__ ctrl,
    double *__restrict__ part, int slot_in, double dt_fixed, FvChain chain, Ph ph)
{
    constexpr int N = Ph::N, A = Ph::A, AA = A > 0 ? A : 1;
    extern __shared__ double box[];   // [N + A][G * B]
    const int t = threadIdx.x;
    const int P3 = p * p * p, pb = p + 2, B = pb * pb * pb, SL = G * B;
    const int k0 = blockIdx.x * G;
    const int g = t / P3, l = t - g * P3;
    const bool active = g < G && k0 + g < K;
    const int x = l % p, y = (l / p) % p, z = l / (p * p);
    const double dt = step_dt<3, kLam>(ctrl, slot_in, dt_fixed, chain);
    auto slot = [&](int gg, int xx, int yy, int zz) { return gg * B + ((zz + 1) * pb + (yy + 1)) * pb + (xx + 1); };

    double qc[N], ac[AA], e[1] = {0.0};
    double inv_dx = 0.0;
    const int s = slot(active ? g : 0, x, y, z);
    if (active) {
        const PatchDev P = patches[k0 + g];
        inv_dx = P.inv_dx;
        load_cell<Ph>(qin, ex, P.off, P3, l, qc, e);
        ph.aux(qc, e, ac);
#pragma unroll
        for (int v = 0; v < N; ++v) box[v * SL + s] = qc[v];
#pragma unroll
        for (int a = 0; a < A; ++a) box[(N + a) * SL + s] = ac[a];
    }
    // face halos: face f = 2 dir + side of patch gg, position (i, j) on it
    const int HF = p * p, HP = 6 * HF;
    for (int h = t; h < G * HP; h += blockDim.x) {
        const int gg = h / HP, r = h - gg * HP, f = r / HF, ij = r - f * HF, i = ij % p, j = ij / p;
        if (k0 + gg >= K) break;   // h only grows, and so does gg
        const int dir = f >> 1, side = f & 1;
        const int nb = patches[k0 + gg].nbr[f];
        const int at = side ? p : -1, from = side ? 0 : p - 1;
        int dx_, dy_, dz_, sx, sy, sz;
        if (dir == 0)      { dx_ = at; sx = from; dy_ = sy = i; dz_ = sz = j; }
        else if (dir == 1) { dy_ = at; sy = from; dx_ = sx = i; dz_ = sz = j; }
        else               { dz_ = at; sz = from; dx_ = sx = i; dy_ = sy = j; }
        double hq[N], ha[AA], he[1] = {0.0};
        load_cell<Ph>(qin, ex, patches[nb].off, P3, (sz * p + sy) * p + sx, hq, he);
        ph.aux(hq, he, ha);
        const int d = slot(gg, dx_, dy_, dz_);
#pragma unroll
        for (int v = 0; v < N; ++v) box[v * SL + d] = hq[v];
#pragma unroll
        for (int a = 0; a < A; ++a) box[(N + a) * SL + d] = ha[a];
    }
    lds_barrier();   // (no thread reads what another writes to global memory)

    double lm[3] = {0.0, 0.0, 0.0};
    bool bad = false;
    if (active) {
        double acc2[N];
#pragma unroll
        for (int v = 0; v < N; ++v) acc2[v] = 0.0;
        auto dirn = [&](auto D, int st) {
            double qL[N], aL[AA], qR[N], aR[AA];
#pragma unroll
            for (int v = 0; v < N; ++v) { qL[v] = box[v * SL + s - st]; qR[v] = box[v * SL + s + st]; }
#pragma unroll
            for (int a = 0; a < A; ++a) { aL[a] = box[(N + a) * SL + s - st]; aR[a] = box[(N + a) * SL + s + st]; }
            rusanov_pair2<Ph, decltype(D)::value>(ph, qL, aL, qc, ac, qR, aR, acc2);
        };
        dirn(std::integral_constant<int, 0>(), 1);
        dirn(std::integral_constant<int, 1>(), pb);
        dirn(std::integral_constant<int, 2>(), pb * pb);
        double S[N];
        if (Ph::kSrc) {
            ph.source(qc, ac, S);
        } else {
#pragma unroll
            for (int v = 0; v < N; ++v) S[v] = 0.0;
        }
        const double hr_ = 0.5 * dt * inv_dx;
        const PatchDev P = patches[k0 + g];
        T *dst = qout + P.off * N + l;
        double qw[N];
#pragma unroll
        for (int v = 0; v < N; ++v) {
            const T st = (T)(v < N - Ph::M ? qc[v] - hr_ * acc2[v] + dt * S[v] : qc[v]);
            __builtin_nontemporal_store(st, dst + (long long)v * P3);
            qw[v] = (double)st;
            bad |= !isfinite(qw[v]);
        }
        if (kLam) cell_speeds_fast<Ph, 3>(ph, qw, lm);
    }
    if (__syncthreads_or(bad) && t == 0) atomicAdd(&ctrl->nonfinite, 1ull);
    if (kLam) fold_speeds<3>(ctrl, part, lm, blockIdx.x, gridDim.x, chain);
}

// Largest speeds of the current state (first step of a call in CFL mode):
// one work-group per patch, partial maxima per patch.
template <class Ph, int DIM, typename T>
__global__ __launch_bounds__(kFvThreads) void fv_lambda_kernel(const T *__restrict__ q,
                                                               const PatchDev *__restrict__ patches,
                                                               double *__restrict__ part, Ph ph)
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
    store_partial<DIM>(part, lm, blockIdx.x, gridDim.x);
}

// dt from the partial maxima: Lambda_d = max over units, then
// dt = cfl / sum_d (Lambda_d / dx_min), written to ctrl->dt[slot].  With
// stats, rows 3..7 of the partials (con2prim iterations, failures, largest
// iteration count, fallbacks, cells) are folded into the control block.
// One work-group; every thread issues the loads of all rows of a unit
// together (one memory round trip per unit, not one per row).  Maxima are
// exact and the sums are of integers held exactly in doubles, so the result
// does not depend on the order.
__global__ __launch_bounds__(1024) void dt_reduce_kernel(const double *__restrict__ part, int n_units, int dim,
                                                         Ctrl *__restrict__ ctrl, int slot, double cfl,
                                                         double dxmin, int want_dt, int want_stats)
{
    __shared__ double red[8][1024 / kWave];
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    const int rows = want_stats ? 8 : dim;
    // row r is used when r < dim, or r >= 3 with stats; max for rows 0-2 and 5
    double m[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) m[r] = 0.0;
    for (int i = t; i < n_units; i += blockDim.x) {
        double v[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = (r < rows && !(r >= dim && r < 3)) ? part[(long long)r * n_units + i] : 0.0;
#pragma unroll
        for (int r = 0; r < 8; ++r) m[r] = (r < 3 || r == 5) ? fmax(m[r], v[r]) : m[r] + v[r];
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const bool mx = r < 3 || r == 5;
        double a = m[r];
        for (int o = 32; o > 0; o >>= 1) {
            const double u = __shfl_xor(a, o, kWave);
            a = mx ? fmax(a, u) : a + u;
        }
        if (lane == 0) red[r][w] = a;
    }
    __syncthreads();
    if (t == 0) {
        double tot[8];
        for (int r = 0; r < rows; ++r) {
            if (r >= dim && r < 3) continue;
            const bool mx = r < 3 || r == 5;
            double a = red[r][0];
            for (int i = 1; i < (int)(blockDim.x / kWave); ++i) a = mx ? fmax(a, red[r][i]) : a + red[r][i];
            tot[r] = a;
        }
        if (want_dt) {
            double den = 0.0;
            for (int d = 0; d < dim; ++d) den += tot[d] / dxmin;
            const double dt = cfl / den;
            ctrl->dt[slot] = dt;
            ctrl->last_dt = dt;
            // the first FV step of a call folds its speeds into lmax[0]
            for (int d = 0; d < 3; ++d) ctrl->lmax[0][d] = 0ull;
        }
        if (want_stats) {
            ctrl->c2p_iters += (unsigned long long)tot[3];
            ctrl->c2p_fail += (unsigned long long)tot[4];
            if ((unsigned)tot[5] > ctrl->c2p_maxit) ctrl->c2p_maxit = (unsigned)tot[5];
            ctrl->c2p_fallback += (unsigned long long)tot[6];
            ctrl->c2p_cells += (unsigned long long)tot[7];
        }
    }
}

// first stage of the partial reduction: work-group g folds units
// [g*kReduceSpan, (g+1)*kReduceSpan) of every row (max for rows 0-2 and 5,
// sum otherwise) into out[r * n_out + g]
__global__ __launch_bounds__(256) void partial_reduce_kernel(const double *__restrict__ part, int n_units, int rows,
                                                             int dim, double *__restrict__ out, int n_out)
{
    __shared__ double red[256 / kWave];
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    const int u0 = blockIdx.x * kReduceSpan, u1 = min(n_units, u0 + kReduceSpan);
    for (int r = 0; r < rows; ++r) {
        if (r >= dim && r < 3) continue;
        const bool mx = r < 3 || r == 5;
        double m = 0.0;
        for (int i = u0 + t; i < u1; i += 256) {
            const double v = part[(long long)r * n_units + i];
            m = mx ? fmax(m, v) : m + v;
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double u = __shfl_xor(m, o, kWave);
            m = mx ? fmax(m, u) : m + u;
        }
        if (lane == 0) red[w] = m;
        __syncthreads();
        if (t == 0) {
            double a = red[0];
            for (int i = 1; i < 256 / kWave; ++i) a = mx ? fmax(a, red[i]) : a + red[i];
            out[(long long)r * n_out + blockIdx.x] = a;
        }
        __syncthreads();
    }
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

// compute units of the current device (cached per device)
pb_status device_cus(int *out)
{
    static std::mutex mu;
    static std::vector<std::pair<int, int>> cache;
    int dev = 0;
    PB_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(mu);
    for (const auto &e : cache)
        if (e.first == dev) { *out = e.second; return PB_OK; }
    int cus = 0;
    PB_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    cache.push_back({dev, std::max(1, cus)});
    *out = std::max(1, cus);
    return PB_OK;
}

template <class Ph, int DIM, typename T>
pb_status launch_typed(pb_batch *b, const Ph &ph, const void *qin, void *qout, int slot_in, int step,
                       double dt_fixed, double cfl, hipStream_t s)
{
    // in CFL mode the steps of a call hand the speed maxima to each other
    // through the control block (FvChain); step < 0 stores partials and
    // runs the reduction kernel after the step
    const FvChain chain{step, cfl, b->dxmin};
    const int slab = (DIM == 3) ? (b->fv_slab > 0 ? std::min(b->fv_slab, b->pmax) : b->pmax) : 1;
    const int n_slabs = (DIM == 3) ? (b->pmax + slab - 1) / slab : 1;
    int n_units = b->K * n_slabs;
    Ctrl *ctrl = reinterpret_cast<Ctrl *>(b->ws);
    const WsLayout L = ws_layout(b->pde, b->dim, b->h, b->total_cells, b->N, b->storage, b->K);
    double *part = reinterpret_cast<double *>(b->ws + L.part);
    const T *qi = static_cast<const T *>(qin);
    T *qo = static_cast<T *>(qout);
    const double *ex = Ph::E ? reinterpret_cast<const double *>(b->ws + L.pres)
                             : nullptr;
    if constexpr (DIM == 3) {
      if (fv_small_eligible(b)) {
        const int p = b->p[0], box = (p + 2) * (p + 2) * (p + 2);
        const int G = std::max(1, std::min(kFvThreads / (p * p * p),
                                           (int)(kFvSmallLds / ((Ph::N + Ph::A) * box * sizeof(double)))));
        const int nwg = (b->K + G - 1) / G;
        const size_t lds = (size_t)(Ph::N + Ph::A) * G * (p + 2) * (p + 2) * (p + 2) * sizeof(double);
        const bool lam = !(dt_fixed > 0.0) && Ph::E == 0;
        if (lam)
            launch_main(b, fv_small_kernel<Ph, T, true>, dim3(nwg), dim3(kFvThreads), lds, s, qi, qo, ex,
                               b->d_patches, b->K, p, G, ctrl, part, slot_in, dt_fixed, chain, ph);
        else
            launch_main(b, fv_small_kernel<Ph, T, false>, dim3(nwg), dim3(kFvThreads), lds, s, qi, qo, ex,
                               b->d_patches, b->K, p, G, ctrl, part, slot_in, dt_fixed, chain, ph);
        PB_HIP(hipGetLastError());
        if (lam && step < 0) return launch_dt_reduce(b, part, nwg, DIM, slot_in ^ 1, cfl, true, false, s);
        return PB_OK;
      }
    }
    // the plane-march kernel: slab units, column runs along +z chains, or
    // the balanced plane schedule over the work-groups that are resident at
    // once (uniform p)
    FvPlan plan{n_units, n_slabs, slab, b->fv_xcd_remap, 0, nullptr};
    auto plane_kernel = [&](auto kern) -> pb_status {
        if (DIM == 3 && b->fv_column > 0 && b->fv_runs.d) {
            plan.runs = static_cast<const int4 *>(b->fv_runs.d);
            plan.n_units = b->fv_runs.n;
        } else if (DIM == 3 && b->fv_persist > 0 && b->uniform_p) {
            int cus = 0;
            pb_status st = device_cus(&cus);
            if (st != PB_OK) return st;
            const long long slots = (long long)b->fv_persist * cus;
            const long long planes = (long long)b->K * b->p[0];
            plan.planes = planes;
            plan.n_units = (int)std::min<long long>(slots, planes);
        }
        n_units = plan.n_units;
        launch_main(b, kern, dim3(plan.n_units), dim3(kFvThreads), 0, s, qi, qo, ex, b->d_patches, plan, ctrl, part,
                    slot_in, dt_fixed, chain, ph);
        return PB_OK;
    };
    pb_status lst = PB_OK;
    if constexpr (Ph::E > 0) {  // SRHD: dt comes from the con2prim pass
        lst = plane_kernel(fv_step_kernel<Ph, DIM, T, false>);
    } else if (DIM == 3 && b->fv_dma && fv_dma_eligible(b)) {
        if (dt_fixed > 0.0)
            launch_main(b, fv_step_dma_kernel<Ph, T, false>, dim3(n_units), dim3(kFvThreads), 0, s, qi, qo,
                               b->d_patches, n_units, n_slabs, slab, b->fv_xcd_remap, ctrl, part, slot_in, dt_fixed,
                               chain, ph);
        else
            launch_main(b, fv_step_dma_kernel<Ph, T, true>, dim3(n_units), dim3(kFvThreads), 0, s, qi, qo,
                               b->d_patches, n_units, n_slabs, slab, b->fv_xcd_remap, ctrl, part, slot_in, dt_fixed,
                               chain, ph);
    } else {
        if (dt_fixed > 0.0)
            lst = plane_kernel(fv_step_kernel<Ph, DIM, T, false>);
        else
            lst = plane_kernel(fv_step_kernel<Ph, DIM, T, true>);
    }
    if (lst != PB_OK) return lst;
    PB_HIP(hipGetLastError());
    if (!(dt_fixed > 0.0) && Ph::E == 0 && step < 0) {
        pb_status st = launch_dt_reduce(b, part, n_units, DIM, slot_in ^ 1, cfl, true, false, s);
        if (st != PB_OK) return st;
    }
    return PB_OK;
}

template <class Ph, int DIM, typename T>
pb_status launch_lambda_typed(pb_batch *b, const Ph &ph, const void *q, double cfl, hipStream_t s)
{
    Ctrl *ctrl = reinterpret_cast<Ctrl *>(b->ws);
    const WsLayout L = ws_layout(b->pde, b->dim, b->h, b->total_cells, b->N, b->storage, b->K);
    double *part = reinterpret_cast<double *>(b->ws + L.part);
    hipLaunchKernelGGL((fv_lambda_kernel<Ph, DIM, T>), dim3(b->K), dim3(kFvThreads), 0, s,
                       static_cast<const T *>(q), b->d_patches, part, ph);
    PB_HIP(hipGetLastError());
    (void)ctrl;
    return launch_dt_reduce(b, part, b->K, DIM, 0, cfl, true, false, s);
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
    case PB_PDE_ADVECTION_VAR:
        if (b->dim == 2) {
            AdvVar<2> ph{pr[0]};
            return f32 ? f(ph, std::integral_constant<int, 2>(), float()) : f(ph, std::integral_constant<int, 2>(), double());
        } else {
            AdvVar<3> ph{pr[0]};
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

// Column runs: the +z link k -> s = nbr[k][+z] holds where s's -z neighbour
// is k and both patches have the same p (>= 2 for the FV march, >= 4 for the
// FD march, whose window reaches 4 planes ahead), so the march reads s's
// first planes as the continuation of k's column.  Links form chains and
// cycles; each gets a number of runs proportional to its planes (at least
// one; at most one per plane for FV, per patch for FD), about w work-groups
// per CU in total, and runs of one chain split its planes as evenly as
// integers allow.  Units are ordered layer-major: the lowest run of every
// chain (chains by their smallest patch index), then every chain's second
// run, and so on.  With the XCD remap an XCD then holds the runs of one
// height layer over a block of neighbouring chains of a grid in patch order
// (several whole rows of them), which start at equal heights, march in step
// and find their x and y neighbours' planes in the same L2.  (Chain after
// chain gave each XCD every layer of fewer chains, two rows on the headline
// grid, so half the y-halo strips came from other XCDs: HBM reads 1.48x
// the algorithmic reads instead of 1.16x.)
std::vector<int4> column_runs(int kind, int K, const int *p, const int *nbr, int w, int cus)
{
    const int pmin = kind == 0 ? 2 : 4;
    std::vector<int> succ(K, -1), pred(K, -1);
    for (int k = 0; k < K; ++k) {
        const int s = nbr[6 * k + 5];
        if (p[k] >= pmin && p[s] == p[k] && nbr[6 * s + 4] == k) {
            succ[k] = s;
            pred[s] = k;
        }
    }
    std::vector<std::vector<int>> chains;
    std::vector<char> seen(K, 0);
    for (int k = 0; k < K; ++k) {   // open chains, from their first patch
        if (pred[k] >= 0) continue;
        chains.emplace_back();
        for (int j = k; j >= 0; j = succ[j]) {
            seen[j] = 1;
            chains.back().push_back(j);
        }
    }
    for (int k = 0; k < K; ++k) {   // cycles, from their smallest patch
        if (seen[k]) continue;
        chains.emplace_back();
        int j = k;
        do {
            seen[j] = 1;
            chains.back().push_back(j);
            j = succ[j];
        } while (j != k);
    }
    std::vector<std::pair<int, int>> order;   // (smallest patch, chain)
    for (int c = 0; c < (int)chains.size(); ++c)
        order.push_back({*std::min_element(chains[c].begin(), chains[c].end()), c});
    std::sort(order.begin(), order.end());
    long long total = 0;
    for (const auto &c : chains) total += (long long)c.size() * p[c[0]];
    const double slots = (double)w * cus;
    std::vector<std::vector<int4>> per;   // the runs of each chain, bottom to top
    size_t rm = 0;
    for (const auto &o : order) {
        const std::vector<int> &c = chains[o.second];
        const int pc = p[c[0]];
        const long long planes = (long long)c.size() * pc;
        const long long rmax = kind == 0 ? planes : (long long)c.size();
        const long long r = std::max(1LL, std::min(rmax, std::llround(slots * (double)planes / (double)total)));
        per.emplace_back();
        for (long long j = 0; j < r; ++j) {
            const long long s0 = j * planes / r, s1 = (j + 1) * planes / r;
            per.back().push_back(make_int4(c[s0 / pc], (int)(s0 % pc), (int)(s1 - s0), 0));
        }
        rm = std::max(rm, per.back().size());
    }
    // layer-major: the first run of every chain, then every second run, ...
    std::vector<int4> runs;
    for (size_t j = 0; j < rm; ++j)
        for (const auto &v : per)
            if (j < v.size()) runs.push_back(v[j]);
    return runs;
}

namespace {

pb_status build_table(pb_batch *b, pb_batch::RunTable &tab, int kind, int w, bool applies)
{
    if (tab.w == w && (tab.d || w <= 0 || !applies)) return PB_OK;
    tab.w = 0;
    if (tab.d) {
        PB_HIP(hipFree(tab.d));
        tab.d = nullptr;
        tab.n = 0;
    }
    if (w <= 0 || !applies) {
        tab.w = w;
        return PB_OK;
    }
    int cus = 0;
    pb_status st = device_cus(&cus);
    if (st != PB_OK) return st;
    const std::vector<int4> runs = column_runs(kind, b->K, b->p.data(), b->nbr.data(), w, cus);
    if ((long long)runs.size() > max_units(b->K)) { set_error("column runs exceed the partial buffers"); return PB_EINVAL; }
    void *d = nullptr;
    PB_HIP(hipMalloc(&d, runs.size() * sizeof(int4)));
    if (hipMemcpy(d, runs.data(), runs.size() * sizeof(int4), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        set_error("hipMemcpy of the column runs failed");
        return PB_EHIP;
    }
    tab.d = d;
    tab.n = (int)runs.size();
    tab.w = w;
    return PB_OK;
}

}  // namespace

pb_status runs_prepare(pb_batch *b)
{
    pb_status st = build_table(b, b->fv_runs, 0, b->fv_column, b->dim == 3);
    if (st != PB_OK) return st;
    return build_table(b, b->fd_runs, 1, b->fd_column, b->dim == 3 && b->pde == PB_PDE_EULER);
}

bool fv_small_eligible(const pb_batch *b)
{
    return b->dim == 3 && b->uniform_p && b->p[0] * b->p[0] * b->p[0] <= kFvThreads;
}

bool fv_dma_eligible(const pb_batch *b)
{
    if (b->dim != 3 || b->pde == PB_PDE_SRHD || b->pde == PB_PDE_LINSYM) return false;
    for (int pk : b->p)
        if (pk % 4 != 0 || pk > kFvPmax) return false;
    for (int i = 0; i < 2; ++i)
        if (reinterpret_cast<uintptr_t>(b->state[i]) % 16 != 0) return false;
    return true;
}

pb_status launch_fv_step(pb_batch *b, const void *qin, void *qout, int slot_in, int step, double dt_fixed,
                         double cfl, hipStream_t s)
{
    return dispatch(b, [&](const auto &ph, auto dimc, auto tt) -> pb_status {
        using Ph = std::decay_t<decltype(ph)>;
        using T = decltype(tt);
        constexpr int DIM = decltype(dimc)::value;
        return launch_typed<Ph, DIM, T>(b, ph, qin, qout, slot_in, step, dt_fixed, cfl, s);
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

pb_status launch_dt_reduce(pb_batch *b, const double *part, int n_units, int dim, int slot, double cfl, bool want_dt,
                           bool want_stats, hipStream_t s)
{
    if (!want_dt && !want_stats) return PB_OK;
    const int rows = want_stats ? 8 : dim;
    if (n_units > kReduceOne) {
        // first stage: one work-group per kReduceSpan units, partials of the
        // partials into the tail of the partial buffer
        const int g = (n_units + kReduceSpan - 1) / kReduceSpan;
        double *part2 = const_cast<double *>(part) + (size_t)8 * max_units(b->K);
        hipLaunchKernelGGL(partial_reduce_kernel, dim3(g), dim3(256), 0, s, part, n_units, rows, dim, part2, g);
        PB_HIP(hipGetLastError());
        part = part2;
        n_units = g;
    }
    hipLaunchKernelGGL(dt_reduce_kernel, dim3(1), dim3(1024), 0, s, part, n_units, dim, reinterpret_cast<Ctrl *>(b->ws),
                       slot, cfl, b->dxmin, want_dt ? 1 : 0, want_stats ? 1 : 0);
    PB_HIP(hipGetLastError());
    return PB_OK;
}

pb_status launch_ctrl_init(pb_batch *b, hipStream_t s)
{
    hipLaunchKernelGGL(ctrl_init_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<Ctrl *>(b->ws));
    PB_HIP(hipGetLastError());
    return PB_OK;
}

}  // namespace pb

// pb_fdeuler.hip -- one Runge-Kutta stage of the fourth-order finite-difference
// scheme with sixth-order Kreiss-Oliger dissipation for the 3D Euler equations
// in flux form (the paper's fourth scheme, Sec. IV, with the flux-divergence
// term of Eq. (1)), on a batch of patches joined through their face
// neighbours:
//   R(Q) = sum_d ( -D4_d F_d(Q) + KO6_d Q ),
//   D4 f  = [(f_-2 - f_+2) + 8 (f_+1 - f_-1)] / (12 dx),
//   KO6 u = sigma/(64 dx) [(u_-3 + u_+3) - 6 (u_-2 + u_+2) + 15 (u_-1 + u_+1) - 20 u_0].
// The stencil reaches 3 cells along each axis and never diagonally, so the
// halo is the three face layers of each side (no edges or corners).
//
// Work decomposition (MI355X): as the FV step, one work-group of 256 threads
// per z-slab of one patch; thread t owns column (x, y) = (t % p, t / p) and
// the work-group marches up the slab plane by plane.  Per output plane z:
//   1. each thread holds its column's Q on planes z-3..z+3 and 1/rho, p on
//      planes z-2..z+2 in registers (plane z+3 arrives from a load issued one
//      plane earlier; its division happens once, as it enters the flux
//      window), so the z derivatives need no LDS; F_z is re-formed from the
//      window per unknown (a multiplication or two each, cheaper in
//      registers than a window of fluxes).  The window's seven register sets
//      rotate with the plane (the loop body is instantiated for the seven
//      phases), so no value moves from set to set;
//   2. the work-group writes Q, F_x and F_y of plane z to LDS, together with
//      the 12p face-halo cells of the plane (three layers per side, read
//      straight from the face neighbours' interiors: the halo gather of
//      Sec. II, Eq. (2), fused into the stage) and, for the two inner
//      layers, their F_x or F_y, so every x and y flux is evaluated once.
//      The halo cells are loaded four planes ahead, when the neighbour's
//      own work-group loads that plane (so they are still in L2), and wait
//      in a small LDS ring until their plane comes;
//   3. after a barrier each thread forms R of its cell, meets the others at
//      a second barrier (the plane LDS is single-buffered: 45 KB, 68 KB with
//      the halo ring, two work-groups per CU), applies the RK stage update
//      and stores.
// The last stage of a step also folds the largest characteristic speeds of
// the new state into per-unit partials for the next step's dt, and counts
// non-finite results.
#include <algorithm>

#include "pb_common.h"
#include "pb_physics.h"

namespace pb {

namespace {

constexpr int kEN = 5;                      // unknowns of 3D Euler
constexpr int kQS = kFvPmax + 6;            // row stride of the Q plane: x in [-3, p + 3)
constexpr int kFxS = kFvPmax + 4;           // row stride of F_x: x in [-2, p + 2)
constexpr int kPlaneQ = kQS * kQS;          // Q plane slots (corners unused)
constexpr int kPlaneF = kFvPmax * kFxS;     // F_x and F_y plane slots
constexpr int kHaloRing = 3;                 // halo ring slots: halo loads run kHaloRing + 1 planes ahead

__device__ __forceinline__ int q_slot(int x, int y) { return (y + 3) * kQS + x + 3; }
__device__ __forceinline__ int fx_slot(int x, int y) { return y * kFxS + x + 2; }
__device__ __forceinline__ int fy_slot(int x, int y) { return (y + 2) * kFvPmax + x; }

// 1/rho and the pressure (all the fluxes need; no sound speed), in the
// aux layout the Euler functor's flux reads
__device__ __forceinline__ void euler_ip(const double *q, double gm1, double *a)
{
    const double ir = recip(q[0]);
    const double m2 = q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    a[0] = ir;
    a[1] = gm1 * (q[4] - 0.5 * m2 * ir);
}

__device__ __forceinline__ double d4(double m2, double m1, double p1, double p2)
{
    return (m2 - p2) + 8.0 * (p1 - m1);
}

__device__ __forceinline__ double ko6(double m3, double m2, double m1, double c, double p1, double p2, double p3)
{
    return (((m3 + p3) - 6.0 * (m2 + p2)) + 15.0 * (m1 + p1)) - 20.0 * c;
}

// the 5 unknowns of one cell: base points at unknown 0 of the patch block,
// o is the cell's offset in it, C the unknown stride (all offsets fit 32
// bits: p <= 16)
__device__ __forceinline__ void load5(const double *__restrict__ base, unsigned o, unsigned C, double *out)
{
#pragma unroll
    for (int v = 0; v < kEN; ++v) out[v] = base[o + v * C];
}

// The plane kernel's own-column accesses: base is the same for the whole
// wave (unknown 0 of a plane of a patch block) and ob the lane's byte offset
// in the plane, below 2 KB.  The per-unknown base then stays in scalar
// registers and every access takes the scalar-base + 32-bit vector-offset
// form, with no per-lane 64-bit address arithmetic.
// The empty asm hands the offset over as a fresh 32-bit value at each access
// (one 32-bit register copy): otherwise the compiler hoists its widening to
// 64 bits out of the plane loop and forms 64-bit vector addresses again.
__device__ __forceinline__ const double *at(const double *base, unsigned ob)
{
    __asm__ volatile("" : "+v"(ob));
    return reinterpret_cast<const double *>(reinterpret_cast<const char *>(base) + ob);
}
__device__ __forceinline__ double *at(double *base, unsigned ob)
{
    __asm__ volatile("" : "+v"(ob));
    return reinterpret_cast<double *>(reinterpret_cast<char *>(base) + ob);
}

__device__ __forceinline__ void load5u(const double *__restrict__ base, unsigned ob, unsigned C, double *out)
{
#pragma unroll
    for (int v = 0; v < kEN; ++v) out[v] = *at(base + (size_t)v * C, ob);
}

// the same, as streaming loads (read once, no halo reuse: they should not
// displace the stage input's lines from L2)
__device__ __forceinline__ void load5u_nt(const double *__restrict__ base, unsigned ob, unsigned C, double *out)
{
#pragma unroll
    for (int v = 0; v < kEN; ++v) out[v] = __builtin_nontemporal_load(at(base + (size_t)v * C, ob));
}

}  // namespace

// S: RK4 stage 0..3, or 4 for the single forward-Euler stage.
//   S = 0: ynext = y + dt/2 R, acc = y + dt/6 R      (y = Q^n)
//   S = 1: ynext = q0 + dt/2 R, acc += dt/3 R
//   S = 2: ynext = q0 + dt R,   acc += dt/3 R
//   S = 3: acc += dt/6 R                              (acc = Q^{n+1})
//   S = 4: acc = y + dt R                             (y = Q^n)
// kLam: fold the speeds of the new state (last stage, CFL mode).
// runs (non-null): unit u marches runs[u] = (patch, first plane, planes, 0)
// up the patch's +z chain, crossing patch tops without a restart (the
// column-run table of the FV kernel); else unit u is slab u % n_slabs of
// patch u / n_slabs.
template <int S, bool kLam>
__global__ __launch_bounds__(kFvThreads, 2) void fd_euler_stage_kernel(
    const double *__restrict__ y, const double *__restrict__ q0, double *__restrict__ ynext,
    double *__restrict__ acc, const PatchDev *__restrict__ patches, int n_units, int n_slabs, int slab, int remap,
    const int4 *__restrict__ runs, Ctrl *__restrict__ ctrl, double *__restrict__ part, int slot, double dt_fixed,
    double gamma, double sigma)
{
    constexpr int N = kEN;
    constexpr bool kReadQ0 = S == 1 || S == 2;
    constexpr bool kReadAcc = S == 1 || S == 2 || S == 3;
    constexpr bool kFinal = S == 3 || S == 4;
    __shared__ double sQ[N][kPlaneQ];
    __shared__ double sFx[N][kPlaneF];
    __shared__ double sFy[N][kPlaneF];
    __shared__ double sH[kHaloRing][N][12 * kFvPmax];   // halo ring: the halo cells of run planes i .. i+kHaloRing-1

    const int t = threadIdx.x;
    const int unit = remap ? xcd_remap(blockIdx.x, n_units) : (int)blockIdx.x;
    int kc, z0, n;   // the unit's first patch and plane, and its planes
    if (runs) {
        const int4 r = runs[unit];
        kc = r.x;
        z0 = r.y;
        n = r.z;
    } else {
        kc = unit / n_slabs;
        const int sl = unit - kc * n_slabs;
        z0 = sl * slab;
        n = max(0, min(patches[kc].p, z0 + slab) - z0);
    }
    const int p = patches[kc].p;
    const unsigned C = (unsigned)(p * p * p), pp = (unsigned)(p * p);
    // patch blocks of the current patch in every buffer and its z neighbours
    // in y (they move up one patch when the march crosses a patch top)
    const double *yo = y + patches[kc].off * N, *ylo = y + patches[patches[kc].nbr[4]].off * N;
    int kn = patches[kc].nbr[5];
    const double *yhi = y + patches[kn].off * N;
    const double *q0o = q0 + patches[kc].off * N, *acco = acc + patches[kc].off * N;
    double *yno = ynext + patches[kc].off * N, *accw = acc + patches[kc].off * N;
    double inv_dx = patches[kc].inv_dx;
    // a slab can start beyond the last plane of a patch smaller than the
    // batch maximum: such a unit only takes part in the reductions
    const bool work = n > 0;
    const bool active = work && t < p * p;
    const int x = active ? t % p : 0, yy = active ? t / p : 0;
    const unsigned cxy = (unsigned)(yy * p + x), cxy8 = 8u * cxy;
    const double dt = dt_fixed > 0.0 ? dt_fixed : ctrl->dt[slot];
    const double gm1 = gamma - 1.0;
    double c4 = inv_dx / 12.0, cko = sigma * inv_dx / 64.0;
    const Euler<3> ph{gamma};
    const int qs = q_slot(x, yy), fxs = fx_slot(x, yy), fys = fy_slot(x, yy);

    // this thread's face-halo cell (threads 0 .. 12p-1): side (-x, +x, -y, +y),
    // layer 0..2 outwards, position j along the face.  Every lane loads (the
    // others a valid cell they do not use), so no load sits in a divergent
    // branch: a load under one makes the compiler copy its target registers
    // at the join, which waits for the load there and then.
    const bool halo = work && t < 12 * p;
    int hq, hf, hside, hcell;
    bool hflux, hx;
    {
        const int th = halo ? t : 0;
        const int side = th / (3 * p), r = th - side * 3 * p, layer = r / p, j = r - layer * p;
        int dx_, dy_, sx, sy;
        if (side == 0)      { dx_ = -1 - layer; dy_ = j; sx = p - 1 - layer; sy = j; }
        else if (side == 1) { dx_ = p + layer;  dy_ = j; sx = layer;         sy = j; }
        else if (side == 2) { dx_ = j; dy_ = -1 - layer; sx = j; sy = p - 1 - layer; }
        else                { dx_ = j; dy_ = p + layer;  sx = j; sy = layer; }
        hside = side;
        hcell = sy * p + sx;
        hq = q_slot(dx_, dy_);
        hflux = layer < 2;
        hx = side < 2;
        hf = hx ? fx_slot(dx_, dy_) : fy_slot(dx_, dy_);
    }
    // unknown 0 of the halo cell's source column, plane 0, for patch kk (a
    // select over the record's entries, not nbr[side]: a lane-varying index
    // would send the patch record to scratch memory)
    auto halo_src = [&](int kk) -> const double * {
        const PatchDev &Q = patches[kk];
        const int nb = hside == 0 ? Q.nbr[0] : hside == 1 ? Q.nbr[1] : hside == 2 ? Q.nbr[2] : Q.nbr[3];
        return y + patches[nb].off * N + hcell;
    };
    const double *hsrc = halo_src(kc);   // the current patch
    const double *hsrcn = halo_src(kn);  // its +z neighbour (the run's next patch)
    // this thread's column on plane zz (zz in [-3, p + 3): the planes outside
    // the patch come from the z neighbours; the choice is uniform)
    auto col = [&](int zz, unsigned o8, double *out) {
        const double *b = zz < 0 ? ylo : (zz >= p ? yhi : yo);
        const int zl = zz < 0 ? zz + p : (zz >= p ? zz - p : zz);
        load5u(b + (size_t)zl * pp, o8, C, out);
    };

    // The window of planes z-3 .. z+3 (slots w = 0..6) lives in seven
    // register sets that rotate instead of sliding: the plane loop is
    // unrolled over the seven phases, and at phase PH slot w is set
    // (w + PH) % 7, so the plane entering at slot 6 takes the set of the
    // plane leaving slot 0 and no value is copied (a slide moved 38 doubles
    // per plane).  ar holds 1/rho and p of the same sets (slots 1..5 live).
    double qr[7][N];
    double ar[7][2];
    double rl[N], hr[N];   // loads in flight: own plane z+3, halo cell of plane z+3
    double lm[3] = {0.0, 0.0, 0.0};
    bool bad = false;

    if (work) {
#pragma unroll
        for (int i = 0; i < 6; ++i) col(z0 - 3 + i, cxy8, qr[i]);
        col(z0 + 3, cxy8, rl);
#pragma unroll
        for (int i = 0; i < 4; ++i) euler_ip(qr[1 + i], gm1, ar[1 + i]);
        // the halo cells of run planes 0..2 go to the ring, plane 3 stays in
        // flight (clamped to the run's last plane, a plane past the patch top
        // comes from the +z neighbour: p >= 4 keeps it inside that one)
#pragma unroll 1
        for (int k = 0; k < kHaloRing; ++k) {
            const int zh = z0 + min(k, n - 1);
            double hv[N];
            load5(zh >= p ? hsrcn : hsrc, (unsigned)(zh >= p ? zh - p : zh) * pp, C, hv);
            if (halo) {
#pragma unroll
                for (int v = 0; v < N; ++v) sH[k][v][t] = hv[v];
            }
        }
        const int zh = z0 + min(kHaloRing, n - 1);
        load5(zh >= p ? hsrcn : hsrc, (unsigned)(zh >= p ? zh - p : zh) * pp, C, hr);
    }
    int hs = 0;   // ring slot of the current run plane (i % kHaloRing)

    int z = z0;   // the current plane, inside the current patch
    int i = 0;    // the current run plane
    auto plane = [&](auto phase) __attribute__((always_inline)) {
        constexpr int PH = decltype(phase)::value;
        auto Q = [&](int w) -> double * { return qr[(w + PH) % 7]; };
        auto A = [&](int w) -> double * { return ar[(w + PH) % 7]; };
        const size_t zo = (size_t)z * pp;   // the plane's first cell in the patch block
        const unsigned ob = cxy8;
        double q0v[N], accv[N];
        {
            // plane z+3 enters the window; the load of plane z+4 replaces it
            // (near the run's top a plane inside the window's reach is
            // loaded again instead, unused; p >= 4 keeps every plane read
            // inside the current patch or the next)
#pragma unroll
            for (int v = 0; v < N; ++v) Q(6)[v] = rl[v];
            col(z + min(4, n + 2 - i), ob, rl);
            if (kReadQ0) load5u_nt(q0o + zo, ob, C, q0v);
            if (kReadAcc) load5u_nt(acco + zo, ob, C, accv);
            euler_ip(Q(5), gm1, A(5));
        }
        if (active) {
            double fx[N], fy[N];
            ph.flux<0>(Q(3), A(3), fx);
            ph.flux<1>(Q(3), A(3), fy);
#pragma unroll
            for (int v = 0; v < N; ++v) {
                sQ[v][qs] = Q(3)[v];
                sFx[v][fxs] = fx[v];
                sFy[v][fys] = fy[v];
            }
        }
        // The halo cells of this plane come from the ring; the cells of run
        // plane i + 3 (loaded one plane ago) take their slot, and the load of
        // plane i + 4 is issued: halo strips are read four planes ahead, at
        // the time the neighbour's own work-group loads that plane into its
        // window, so the strips are still in L2 (read one plane ahead, three
        // planes after the neighbour, they had mostly left it).  Each thread
        // reads back only what it wrote: no barrier.
        double hv[N];
        if (halo) {
#pragma unroll
            for (int v = 0; v < N; ++v) hv[v] = sH[hs][v][t];
#pragma unroll
            for (int v = 0; v < N; ++v) sH[hs][v][t] = hr[v];
        }
        hs = hs == kHaloRing - 1 ? 0 : hs + 1;
        {
            const int zh = z + min(kHaloRing + 1, n - 1 - i);   // run plane i + kHaloRing + 1, or the run's last plane near its top
            load5(zh >= p ? hsrcn : hsrc, (unsigned)(zh >= p ? zh - p : zh) * pp, C, hr);
        }
        if (halo) {
#pragma unroll
            for (int v = 0; v < N; ++v) sQ[v][hq] = hv[v];
            if (hflux) {
                double a[2], F[N];
                euler_ip(hv, gm1, a);
                if (hx) {
                    ph.flux<0>(hv, a, F);
#pragma unroll
                    for (int v = 0; v < N; ++v) sFx[v][hf] = F[v];
                } else {
                    ph.flux<1>(hv, a, F);
#pragma unroll
                    for (int v = 0; v < N; ++v) sFy[v][hf] = F[v];
                }
            }
        }
        lds_barrier();
        double R[N];
        if (active) {
            // u_z of planes z-2, z-1, z+1, z+2 (window slots 1, 2, 4, 5); the
            // components of F_z are formed per unknown below
            double uz[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int w = k < 2 ? k + 1 : k + 2;
                uz[k] = Q(w)[3] * A(w)[0];
            }
            auto fzv = [&](int k, int v) -> double {
                const int w = k < 2 ? k + 1 : k + 2;
                const double pr = A(w)[1];
                if (v == 0) return Q(w)[3];
                if (v == 3) return Q(w)[3] * uz[k] + pr;
                if (v == 4) return (Q(w)[4] + pr) * uz[k];
                return Q(w)[v] * uz[k];
            };
#pragma unroll
            for (int v = 0; v < N; ++v) {
                const double *u = sQ[v], *fxv = sFx[v], *fyv = sFy[v];
                const double dfx = d4(fxv[fxs - 2], fxv[fxs - 1], fxv[fxs + 1], fxv[fxs + 2]);
                const double dfy = d4(fyv[fys - 2 * kFvPmax], fyv[fys - kFvPmax], fyv[fys + kFvPmax],
                                      fyv[fys + 2 * kFvPmax]);
                const double dfz = d4(fzv(0, v), fzv(1, v), fzv(2, v), fzv(3, v));
                const double c = Q(3)[v];
                const double kx = ko6(u[qs - 3], u[qs - 2], u[qs - 1], c, u[qs + 1], u[qs + 2], u[qs + 3]);
                const double ky = ko6(u[qs - 3 * kQS], u[qs - 2 * kQS], u[qs - kQS], c, u[qs + kQS],
                                      u[qs + 2 * kQS], u[qs + 3 * kQS]);
                const double kz = ko6(Q(0)[v], Q(1)[v], Q(2)[v], c, Q(4)[v], Q(5)[v], Q(6)[v]);
                R[v] = cko * ((kx + ky) + kz) - c4 * ((dfx + dfy) + dfz);
                // one unknown's 20 LDS reads at a time: hoisting all of them
                // would not fit the register budget
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        lds_barrier();   // the plane's LDS is free for the next one
        if (active) {
            double nv[N];
#pragma unroll
            for (int v = 0; v < N; ++v) {
                double *const yg = at(yno + zo + (size_t)v * C, ob), *const ag = at(accw + zo + (size_t)v * C, ob);
                if (S == 0) {
                    __builtin_nontemporal_store(Q(3)[v] + (0.5 * dt) * R[v], yg);
                    nv[v] = Q(3)[v] + (dt / 6.0) * R[v];
                } else if (S == 1) {
                    __builtin_nontemporal_store(q0v[v] + (0.5 * dt) * R[v], yg);
                    nv[v] = accv[v] + (dt / 3.0) * R[v];
                } else if (S == 2) {
                    __builtin_nontemporal_store(q0v[v] + dt * R[v], yg);
                    nv[v] = accv[v] + (dt / 3.0) * R[v];
                } else if (S == 3) {
                    nv[v] = accv[v] + (dt / 6.0) * R[v];
                } else {
                    nv[v] = Q(3)[v] + dt * R[v];
                }
                __builtin_nontemporal_store(nv[v], ag);
            }
            if (kFinal) {
#pragma unroll
                for (int v = 0; v < N; ++v) bad |= !isfinite(nv[v]);
                if (kLam) {
                    double a[3];
                    ph.aux_fast(nv, nullptr, a);
                    lm[0] = fmax(lm[0], ph.eig<0>(nv, a));
                    lm[1] = fmax(lm[1], ph.eig<1>(nv, a));
                    lm[2] = fmax(lm[2], ph.eig<2>(nv, a));
                }
            }
        }
        if (++z == p && i + 1 < n) {
            // the run continues in the +z neighbour: every buffer's patch
            // block moves up one patch (the window and the loads in flight
            // already come from it)
            z = 0;
            const long long off = patches[kn].off;
            ylo = yo;
            yo = yhi;
            q0o = q0 + off * N;
            acco = acc + off * N;
            yno = ynext + off * N;
            accw = acc + off * N;
            inv_dx = patches[kn].inv_dx;
            c4 = inv_dx / 12.0;
            cko = sigma * inv_dx / 64.0;
            hsrc = hsrcn;
            kn = patches[kn].nbr[5];
            yhi = y + patches[kn].off * N;
            hsrcn = halo_src(kn);
        }
    };
    // the plane of phase PH is run plane i with i % 7 == PH
    while (i < n) {
        plane(std::integral_constant<int, 0>());
        if (++i == n) break;
        plane(std::integral_constant<int, 1>());
        if (++i == n) break;
        plane(std::integral_constant<int, 2>());
        if (++i == n) break;
        plane(std::integral_constant<int, 3>());
        if (++i == n) break;
        plane(std::integral_constant<int, 4>());
        if (++i == n) break;
        plane(std::integral_constant<int, 5>());
        if (++i == n) break;
        plane(std::integral_constant<int, 6>());
        ++i;
    }
    if (kFinal) {
        if (__syncthreads_or(bad) && t == 0) atomicAdd(&ctrl->nonfinite, 1ull);
        if (kLam) store_partial<3>(part, lm, unit, n_units);
    }
}

// ---------------------------------------------------------------------------
// Small patches (one p for the batch, p^3 <= 256, so 3 <= p <= 6 with the
// halo of 3).  The plane march would leave all but p^2 threads of a
// work-group idle; here a work-group takes G whole patches, one thread per
// cell, and stages each patch with its face halos in LDS in a cross layout:
// the p^3 interior slots, then for faces -x, +x, -y, +y, -z, +z three
// layers of p^2 slots each (layer 0 touching the patch), 7 doubles per slot
// (Q, 1/rho, p).  Every thread then reads its 18 stencil slots, evaluates
// the 12 fluxes its D4 terms need (F_d at +-1, +-2 along d) from the staged
// Q and aux, and updates as the plane kernel does.
namespace {

struct SmallGeom {
    int p, p2, p3, slots;   // slots per patch: p^3 + 18 p^2
};

// slot of tile-local (x, y, z), at most one coordinate outside [0, p)
__device__ __forceinline__ int cross_slot(const SmallGeom &g, int x, int y, int z)
{
    const int lay = 3 * g.p2;
    if (x < 0) return g.p3 + 0 * lay + (-x - 1) * g.p2 + z * g.p + y;
    if (x >= g.p) return g.p3 + 1 * lay + (x - g.p) * g.p2 + z * g.p + y;
    if (y < 0) return g.p3 + 2 * lay + (-y - 1) * g.p2 + z * g.p + x;
    if (y >= g.p) return g.p3 + 3 * lay + (y - g.p) * g.p2 + z * g.p + x;
    if (z < 0) return g.p3 + 4 * lay + (-z - 1) * g.p2 + y * g.p + x;
    if (z >= g.p) return g.p3 + 5 * lay + (z - g.p) * g.p2 + y * g.p + x;
    return (z * g.p + y) * g.p + x;
}

constexpr int kSmallW = 7;   // Q (5), 1/rho, p per slot

}  // namespace

template <int S, bool kLam>
__global__ __launch_bounds__(kFvThreads) void fd_euler_small_kernel(
    const double *__restrict__ y, const double *__restrict__ q0, double *__restrict__ ynext,
    double *__restrict__ acc, const PatchDev *__restrict__ patches, int K, int p, int G, Ctrl *__restrict__ ctrl,
    double *__restrict__ part, int slot, double dt_fixed, double gamma, double sigma)
{
    constexpr int N = kEN;
    constexpr bool kReadQ0 = S == 1 || S == 2;
    constexpr bool kReadAcc = S == 1 || S == 2 || S == 3;
    constexpr bool kFinal = S == 3 || S == 4;
    extern __shared__ double sm[];   // [kSmallW][G * slots]
    const SmallGeom geo{p, p * p, p * p * p, p * p * p + 18 * p * p};
    const int SL = G * geo.slots;
    const int t = threadIdx.x;
    const int k0 = blockIdx.x * G;
    const int g = t / geo.p3, l = t - g * geo.p3;
    const bool active = g < G && k0 + g < K;
    const int x = l % p, yy = (l / p) % p, z = l / geo.p2;
    const double dt = dt_fixed > 0.0 ? dt_fixed : ctrl->dt[slot];
    const double gm1 = gamma - 1.0;
    const Euler<3> ph{gamma};
    const unsigned C = (unsigned)geo.p3;

    // 1. stage the interior cells and the face halos
    double qc[N];
    long long off = 0;
    double inv_dx = 0.0;
    if (active) {
        const PatchDev P = patches[k0 + g];
        off = P.off;
        inv_dx = P.inv_dx;
        load5(y + off * N, (unsigned)l, C, qc);
        double a[2];
        euler_ip(qc, gm1, a);
        const int s0 = g * geo.slots + l;
#pragma unroll
        for (int v = 0; v < N; ++v) sm[v * SL + s0] = qc[v];
        sm[5 * SL + s0] = a[0];
        sm[6 * SL + s0] = a[1];
    }
    const int HP = 18 * geo.p2;   // halo cells per patch
    for (int h = t; h < G * HP; h += blockDim.x) {
        const int gg = h / HP, r = h - gg * HP;
        if (k0 + gg >= K) break;   // h only grows, and so does gg
        const int f = r / (3 * geo.p2), rr = r - f * 3 * geo.p2, L = rr / geo.p2, ab = rr - L * geo.p2;
        const int a_ = ab / p, b_ = ab - a_ * p;
        const int in = L, out = p - 1 - L;   // source layer for the + and - faces
        int sx, sy, sz;
        switch (f) {
        case 0: sx = out; sy = b_; sz = a_; break;
        case 1: sx = in;  sy = b_; sz = a_; break;
        case 2: sx = b_; sy = out; sz = a_; break;
        case 3: sx = b_; sy = in;  sz = a_; break;
        case 4: sx = b_; sy = a_; sz = out; break;
        default: sx = b_; sy = a_; sz = in; break;
        }
        const int nb = patches[k0 + gg].nbr[f];
        double hq[N], a[2];
        load5(y + patches[nb].off * N, (unsigned)((sz * p + sy) * p + sx), C, hq);
        euler_ip(hq, gm1, a);
        const int d = gg * geo.slots + geo.p3 + r;
#pragma unroll
        for (int v = 0; v < N; ++v) sm[v * SL + d] = hq[v];
        sm[5 * SL + d] = a[0];
        sm[6 * SL + d] = a[1];
    }
    lds_barrier();

    double lm[3] = {0.0, 0.0, 0.0};
    bool bad = false;
    if (active) {
        const int base = g * geo.slots;
        // stencil slots along each direction: offsets -3, -2, -1, +1, +2, +3
        int st[3][6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int o = k < 3 ? k - 3 : k - 2;
            st[0][k] = base + cross_slot(geo, x + o, yy, z);
            st[1][k] = base + cross_slot(geo, x, yy + o, z);
            st[2][k] = base + cross_slot(geo, x, yy, z + o);
        }
        const double c4 = inv_dx / 12.0, cko = sigma * inv_dx / 64.0;
        double R[N], kox[N];
#pragma unroll
        for (int v = 0; v < N; ++v) { R[v] = 0.0; kox[v] = 0.0; }
        auto dir = [&](auto D) {
            constexpr int d = decltype(D)::value;
            // D4 of F_d from the fluxes at -2, -1, +1, +2 (slots 1, 2, 3, 4)
            double F[4][N];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int sl = st[d][i + 1];
                double q[N], a[2];
#pragma unroll
                for (int v = 0; v < N; ++v) q[v] = sm[v * SL + sl];
                a[0] = sm[5 * SL + sl];
                a[1] = sm[6 * SL + sl];
                ph.flux<d>(q, a, F[i]);
            }
#pragma unroll
            for (int v = 0; v < N; ++v) {
                R[v] += d4(F[0][v], F[1][v], F[2][v], F[3][v]);
                kox[v] += ko6(sm[v * SL + st[d][0]], sm[v * SL + st[d][1]], sm[v * SL + st[d][2]], qc[v],
                              sm[v * SL + st[d][3]], sm[v * SL + st[d][4]], sm[v * SL + st[d][5]]);
            }
        };
        dir(std::integral_constant<int, 0>());
        dir(std::integral_constant<int, 1>());
        dir(std::integral_constant<int, 2>());
        const unsigned own = (unsigned)l;
        double q0v[N], accv[N], nv[N];
        if (kReadQ0) load5(q0 + off * N, own, C, q0v);
        if (kReadAcc) load5(acc + off * N, own, C, accv);
        double *yno = ynext + off * N, *accw = acc + off * N;
#pragma unroll
        for (int v = 0; v < N; ++v) {
            const double Rv = cko * kox[v] - c4 * R[v];
            const unsigned gi = own + v * C;
            if (S == 0) {
                yno[gi] = qc[v] + (0.5 * dt) * Rv;
                nv[v] = qc[v] + (dt / 6.0) * Rv;
            } else if (S == 1) {
                yno[gi] = q0v[v] + (0.5 * dt) * Rv;
                nv[v] = accv[v] + (dt / 3.0) * Rv;
            } else if (S == 2) {
                yno[gi] = q0v[v] + dt * Rv;
                nv[v] = accv[v] + (dt / 3.0) * Rv;
            } else if (S == 3) {
                nv[v] = accv[v] + (dt / 6.0) * Rv;
            } else {
                nv[v] = qc[v] + dt * Rv;
            }
            accw[gi] = nv[v];
        }
        if (kFinal) {
#pragma unroll
            for (int v = 0; v < N; ++v) bad |= !isfinite(nv[v]);
            if (kLam) {
                double a[3];
                ph.aux_fast(nv, nullptr, a);
                lm[0] = fmax(lm[0], ph.eig<0>(nv, a));
                lm[1] = fmax(lm[1], ph.eig<1>(nv, a));
                lm[2] = fmax(lm[2], ph.eig<2>(nv, a));
            }
        }
    }
    if (kFinal) {
        if (__syncthreads_or(bad) && t == 0) atomicAdd(&ctrl->nonfinite, 1ull);
        if (kLam) store_partial<3>(part, lm, blockIdx.x, gridDim.x);
    }
}

// ------------------------------------------------------------------ host --

namespace {

// G > 0: the small-patch kernel with G patches per work-group (n_units = work-groups)
template <int S, bool kLam>
void launch_s(dim3 g, hipStream_t s, const double *y, const double *q0, double *yn, double *acc, const pb_batch *b,
              int n_units, int n_slabs, int slab, const int4 *runs, int G, Ctrl *ctrl, double *part, int slot,
              double dt_fixed, double sigma)
{
    if (G > 0) {
        const int p = b->p[0];
        const size_t lds = (size_t)kSmallW * G * (p * p * p + 18 * p * p) * sizeof(double);
        launch_main(b, fd_euler_small_kernel<S, kLam>, g, dim3(kFvThreads), lds, s, y, q0, yn, acc,
                           b->d_patches, b->K, p, G, ctrl, part, slot, dt_fixed, b->params[0], sigma);
    } else {
        launch_main(b, fd_euler_stage_kernel<S, kLam>, g, dim3(kFvThreads), 0, s, y, q0, yn, acc, b->d_patches,
                           n_units, n_slabs, slab, b->fd_xcd_remap, runs, ctrl, part, slot, dt_fixed, b->params[0],
                           sigma);
    }
}

}  // namespace

pb_status launch_fd_euler_stage(pb_batch *b, int stage, int rk_stages, const void *q0, const void *y, void *ynext,
                                void *acc, int slot, double dt_fixed, double cfl, double sigma, hipStream_t s)
{
    if (b->pmax > kFvPmax) { set_error("fd_ko_step: p > 16 is not supported for EULER"); return PB_EUNSUPPORTED; }
    const int slab = b->pmax, n_slabs = 1;
    // one p with p^3 <= 256: whole patches per work-group (LDS cross layout
    // of 7 doubles per slot, at most 64 KB per work-group)
    int G = 0;
    if (b->uniform_p && b->p[0] * b->p[0] * b->p[0] <= kFvThreads) {
        const int p = b->p[0];
        const size_t per = (size_t)kSmallW * (p * p * p + 18 * p * p) * sizeof(double);
        G = std::max(1, std::min(kFvThreads / (p * p * p), (int)(kFvSmallLds / per)));
    }
    // column runs along +z chains when the tuning asks for them (the table is
    // built when the batch is created or its tuning set)
    const int4 *runs = (G == 0 && b->fd_column > 0 && b->fd_runs.d) ? static_cast<const int4 *>(b->fd_runs.d) : nullptr;
    const int n_units = G > 0 ? (b->K + G - 1) / G : runs ? b->fd_runs.n : b->K * n_slabs;
    Ctrl *ctrl = reinterpret_cast<Ctrl *>(b->ws);
    const WsLayout L = ws_layout(b->pde, b->dim, b->h, b->total_cells, b->N, b->storage, b->K);
    double *part = reinterpret_cast<double *>(b->ws + L.part);
    const int S = rk_stages == 1 ? 4 : stage;
    const bool final_stage = S == 3 || S == 4;
    const bool lam = final_stage && !(dt_fixed > 0.0);
    const double *yi = static_cast<const double *>(y), *q0i = static_cast<const double *>(q0);
    double *yn = static_cast<double *>(ynext), *ac = static_cast<double *>(acc);
    const dim3 g(n_units);
#define PB_FDE_ARGS g, s, yi, q0i, yn, ac, b, n_units, n_slabs, slab, runs, G, ctrl, part, slot, dt_fixed, sigma
    switch (S) {
    case 0: launch_s<0, false>(PB_FDE_ARGS); break;
    case 1: launch_s<1, false>(PB_FDE_ARGS); break;
    case 2: launch_s<2, false>(PB_FDE_ARGS); break;
    case 3: lam ? launch_s<3, true>(PB_FDE_ARGS) : launch_s<3, false>(PB_FDE_ARGS); break;
    default: lam ? launch_s<4, true>(PB_FDE_ARGS) : launch_s<4, false>(PB_FDE_ARGS); break;
    }
#undef PB_FDE_ARGS
    PB_HIP(hipGetLastError());
    if (lam) return launch_dt_reduce(b, part, n_units, 3, slot ^ 1, cfl, true, false, s);
    return PB_OK;
}

}  // namespace pb

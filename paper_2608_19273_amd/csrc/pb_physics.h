// pb_physics.h -- the PDE terms of dQ/dt + div F(Q) + B(Q).grad Q = S(Q)
// (paper Sec. I, Eq. (1)) as device functors that the kernels inline, which
// is how the physics gets fused into the numerical kernel (paper Sec. III-B
// does this with an MLIR pass; here C++ templates do it).
//
// Every functor splits its work into a per-cell part, `aux`, holding the
// expensive operations (divisions, square roots, the SRHD primitive state),
// and cheap per-face parts (flux along d, largest speed along d,
// non-conservative product) that read the cached aux values.  The kernels
// evaluate aux once per cell and keep it in LDS next to Q.
//
// Functor interface:
//   N, A, E            unknowns, aux values, extra per-cell inputs (SRHD: p)
//   M                  material parameters: the last M of the N values per
//                      point, read by the physics and carried through every
//                      update unchanged (fixed in time)
//   kFlux, kNcp, kSrc  which terms exist
//   aux(q, e, a)       a[0..A) from Q and the extra inputs
//   eig<D>(q, a)       largest |characteristic speed| along D
//   flux<D>(q, a, F)   F_D(Q)
//   ncp<D>(qL, qR, o)  B_D((qL+qR)/2) (qR - qL)
//   source(q, a, S)    S(Q)
#pragma once

#include <hip/hip_runtime.h>

namespace pb {

// 1/x from the hardware reciprocal estimate refined by two Newton steps
// (error within an ulp or two of the correctly rounded quotient; x finite, nonzero).
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// sqrt(a) from the hardware reciprocal-square-root estimate refined by
// Goldschmidt/Newton steps; a <= 0, inf and NaN take the library path.
__device__ __forceinline__ double root(double a)
{
    if (!(a > 0.0 && a < 1e300)) return sqrt(a);
    const double y = __builtin_amdgcn_rsq(a);
    double g = a * y, h = 0.5 * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, a);
    return fma(d, h, g);
}

// Linear advection, conservative form: F_d = a_d q, S = -kappa q.
struct AdvF {
    static constexpr int N = 1, A = 0, E = 0, M = 0, DIMS = 3;
    static constexpr bool kFlux = true, kNcp = false, kSrc = true;
    double a[3];
    double kappa;
    __device__ __forceinline__ void aux(const double *, const double *, double *) const {}
    __device__ __forceinline__ void aux_fast(const double *, const double *, double *) const {}
    template <int D> __device__ __forceinline__ double eig(const double *, const double *) const
    {
        return fabs(a[D]);
    }
    template <int D> __device__ __forceinline__ void flux(const double *q, const double *, double *F) const
    {
        F[0] = a[D] * q[0];
    }
    template <int D> __device__ __forceinline__ void ncp(const double *, const double *, double *) const {}
    __device__ __forceinline__ void source(const double *q, const double *, double *S) const
    {
        S[0] = -kappa * q[0];
    }
};

// Linear advection, non-conservative form: B_d = a_d, F = 0.
struct AdvB {
    static constexpr int N = 1, A = 0, E = 0, M = 0, DIMS = 3;
    static constexpr bool kFlux = false, kNcp = true, kSrc = true;
    double a[3];
    double kappa;
    __device__ __forceinline__ void aux(const double *, const double *, double *) const {}
    __device__ __forceinline__ void aux_fast(const double *, const double *, double *) const {}
    template <int D> __device__ __forceinline__ double eig(const double *, const double *) const
    {
        return fabs(a[D]);
    }
    template <int D> __device__ __forceinline__ void flux(const double *, const double *, double *F) const
    {
        F[0] = 0.0;
    }
    template <int D> __device__ __forceinline__ void ncp(const double *qL, const double *qR, double *o) const
    {
        o[0] = a[D] * (qR[0] - qL[0]);
    }
    __device__ __forceinline__ void source(const double *q, const double *, double *S) const
    {
        S[0] = -kappa * q[0];
    }
};

// Linear advection by a velocity field carried as material parameters (the
// N + M values per point of paper Sec. II, here N = 1 evolving, M = DIM):
// Q = (q, a_1..a_DIM), F_d = a_d(x) q, speed |a_d(x)|, S = -kappa q.  The
// Rusanov face uses the speeds and fluxes of the two adjacent cells, so a
// field that varies in space gives the usual variable-coefficient flux.
template <int DIM>
struct AdvVar {
    static constexpr int N = 1 + DIM, A = 0, E = 0, M = DIM, DIMS = DIM;
    static constexpr bool kFlux = true, kNcp = false, kSrc = true;
    double kappa;
    __device__ __forceinline__ void aux(const double *, const double *, double *) const {}
    __device__ __forceinline__ void aux_fast(const double *, const double *, double *) const {}
    template <int D> __device__ __forceinline__ double eig(const double *q, const double *) const
    {
        return fabs(q[1 + D]);
    }
    template <int D> __device__ __forceinline__ void flux(const double *q, const double *, double *F) const
    {
        F[0] = q[1 + D] * q[0];
#pragma unroll
        for (int v = 1; v < N; ++v) F[v] = 0.0;
    }
    template <int D> __device__ __forceinline__ void ncp(const double *, const double *, double *) const {}
    __device__ __forceinline__ void source(const double *q, const double *, double *S) const
    {
        S[0] = -kappa * q[0];
#pragma unroll
        for (int v = 1; v < N; ++v) S[v] = 0.0;
    }
};

// Compressible Euler, ideal gas: Q = (rho, m, E), p = (gamma-1)(E - |m|^2/(2 rho)),
// F_d = (m_d, m_d m/rho + p e_d, (E + p) m_d/rho), speed |m_d/rho| + sqrt(gamma p/rho).
// aux = (1/rho, p, c).
template <int DIM>
struct Euler {
    static constexpr int N = DIM + 2, A = 3, E = 0, M = 0, DIMS = DIM;
    static constexpr bool kFlux = true, kNcp = false, kSrc = false;
    double gamma;
    __device__ __forceinline__ void aux(const double *q, const double *, double *a) const
    {
        const double ir = 1.0 / q[0];
        double m2 = q[1] * q[1] + q[2] * q[2];
        if (DIM == 3) m2 += q[3] * q[3];
        const double p = (gamma - 1.0) * (q[DIM + 1] - 0.5 * m2 * ir);
        a[0] = ir;
        a[1] = p;
        a[2] = sqrt(gamma * p * ir);
    }
    __device__ __forceinline__ void aux_fast(const double *q, const double *, double *a) const
    {
        const double ir = recip(q[0]);
        double m2 = q[1] * q[1] + q[2] * q[2];
        if (DIM == 3) m2 += q[3] * q[3];
        const double p = (gamma - 1.0) * (q[DIM + 1] - 0.5 * m2 * ir);
        a[0] = ir;
        a[1] = p;
        a[2] = root(gamma * p * ir);
    }
    template <int D> __device__ __forceinline__ double eig(const double *q, const double *a) const
    {
        return fabs(q[1 + D] * a[0]) + a[2];
    }
    template <int D> __device__ __forceinline__ void flux(const double *q, const double *a, double *F) const
    {
        const double ud = q[1 + D] * a[0];
        F[0] = q[1 + D];
#pragma unroll
        for (int e = 0; e < DIM; ++e) F[1 + e] = q[1 + e] * ud + (e == D ? a[1] : 0.0);
        F[DIM + 1] = (q[DIM + 1] + a[1]) * ud;
    }
    template <int D> __device__ __forceinline__ void ncp(const double *, const double *, double *) const {}
    __device__ __forceinline__ void source(const double *, const double *, double *) const {}
};

// Special-relativistic hydrodynamics, ideal gas, Q = (D, S, tau); the
// pressure comes from the con2prim pass (extra input).  With E = tau + D:
//   v = S/(E + p), W = (1 - v^2)^(-1/2), rho = D/W, rho h = rho + Gamma p/(Gamma-1),
//   c_s^2 = Gamma p/(rho h),
//   lambda_pm = [v_d (1 - c_s^2) +- c_s sqrt((1 - v^2)(1 - v^2 c_s^2 - v_d^2 (1 - c_s^2)))]
//               / (1 - v^2 c_s^2),
//   F_d = (D v_d, S v_d + p e_d, S_d - D v_d).
// aux = (p, v_x, v_y, v_z, lambda_x, lambda_y, lambda_z).
struct Srhd {
    static constexpr int N = 5, A = 7, E = 1, M = 0, DIMS = 3;
    static constexpr bool kFlux = true, kNcp = false, kSrc = false;
    double gam;
    // The reciprocals and roots come from the refined hardware estimates
    // (recip, root: within an ulp or two of the correctly rounded values);
    // the primitives feed the fluxes of the step and the speeds its dt.
    __device__ __forceinline__ void aux(const double *q, const double *e, double *a) const
    {
        const double p = e[0];
        const double iEp = recip(q[4] + q[0] + p);
        const double v[3] = {q[1] * iEp, q[2] * iEp, q[3] * iEp};
        const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        const double rho = q[0] * root(1.0 - v2);
        const double rhoh = rho + gam / (gam - 1.0) * p;
        const double cs2 = gam * p * recip(rhoh);
        const double cs = root(cs2);
        const double iden = recip(1.0 - v2 * cs2);
        a[0] = p;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            a[1 + d] = v[d];
            const double rt = root((1.0 - v2) * (1.0 - v2 * cs2 - v[d] * v[d] * (1.0 - cs2)));
            const double lp = (v[d] * (1.0 - cs2) + cs * rt) * iden;
            const double lm = (v[d] * (1.0 - cs2) - cs * rt) * iden;
            a[4 + d] = fmax(fabs(lp), fabs(lm));
        }
    }
    __device__ __forceinline__ void aux_fast(const double *q, const double *e, double *a) const { aux(q, e, a); }
    template <int D> __device__ __forceinline__ double eig(const double *, const double *a) const
    {
        return a[4 + D];
    }
    template <int D> __device__ __forceinline__ void flux(const double *q, const double *a, double *F) const
    {
        const double vd = a[1 + D];
        F[0] = q[0] * vd;
#pragma unroll
        for (int e = 0; e < 3; ++e) F[1 + e] = q[1 + e] * vd + (e == D ? a[0] : 0.0);
        F[4] = q[1 + D] - q[0] * vd;
    }
    template <int D> __device__ __forceinline__ void ncp(const double *, const double *, double *) const {}
    __device__ __forceinline__ void source(const double *, const double *, double *) const {}
};

// Rusanov face flux along D between cells L and R, plus half the midpoint
// non-conservative fluctuation:
//   F* = (F(L) + F(R))/2 - max(lambda_L, lambda_R) (Q_R - Q_L)/2,
//   Dn = B((Q_L + Q_R)/2) (Q_R - Q_L)/2.
template <class Ph, int D>
__device__ __forceinline__ void rusanov_face(const Ph &ph, const double *qL, const double *aL,
                                             const double *qR, const double *aR, double *Fs,
                                             double *Dn)
{
    constexpr int N = Ph::N;
    const double s = fmax(ph.template eig<D>(qL, aL), ph.template eig<D>(qR, aR));
    double FL[N], FR[N];
    if (Ph::kFlux) {
        ph.template flux<D>(qL, aL, FL);
        ph.template flux<D>(qR, aR, FR);
    } else {
#pragma unroll
        for (int v = 0; v < N; ++v) FL[v] = FR[v] = 0.0;
    }
#pragma unroll
    for (int v = 0; v < N; ++v) Fs[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * s * (qR[v] - qL[v]);
    if (Ph::kNcp) {
        double o[N];
        ph.template ncp<D>(qL, qR, o);
#pragma unroll
        for (int v = 0; v < N; ++v) Dn[v] = 0.5 * o[v];
    } else {
#pragma unroll
        for (int v = 0; v < N; ++v) Dn[v] = 0.0;
    }
}

// Both faces of a cell along D at once, times two:
//   2 [(F*_{+} - F*_{-}) + (Dn_{+} + Dn_{-})]
//   = (F(R) - F(L)) - s_{+} (Q_R - Q) + s_{-} (Q - Q_L)
//     + B(mid_{+}) (Q_R - Q) + B(mid_{-}) (Q - Q_L),
// with s_{+-} the Rusanov speeds of the two faces.  F(Q) of the cell itself
// cancels, so only the two neighbours' fluxes are evaluated.
template <class Ph, int D>
__device__ __forceinline__ void rusanov_pair2(const Ph &ph, const double *qL, const double *aL,
                                              const double *q, const double *a, const double *qR,
                                              const double *aR, double *acc2)
{
    constexpr int N = Ph::N;
    const double l0 = ph.template eig<D>(q, a);
    const double sp = fmax(l0, ph.template eig<D>(qR, aR));
    const double sm = fmax(l0, ph.template eig<D>(qL, aL));
    if (Ph::kFlux) {
        double FL[N], FR[N];
        ph.template flux<D>(qL, aL, FL);
        ph.template flux<D>(qR, aR, FR);
#pragma unroll
        for (int v = 0; v < N; ++v) acc2[v] += (FR[v] - FL[v]) - sp * (qR[v] - q[v]) + sm * (q[v] - qL[v]);
    } else {
#pragma unroll
        for (int v = 0; v < N; ++v) acc2[v] += sm * (q[v] - qL[v]) - sp * (qR[v] - q[v]);
    }
    if (Ph::kNcp) {
        double o0[N], o1[N];
        ph.template ncp<D>(qL, q, o0);
        ph.template ncp<D>(q, qR, o1);
#pragma unroll
        for (int v = 0; v < N; ++v) acc2[v] += o1[v] + o0[v];
    }
}

// Twice the Rusanov face flux between L and R along D, given the two
// physical fluxes and speeds (used for the z faces, whose fluxes are carried
// from plane to plane), and twice the midpoint fluctuation, kept apart because
// the flux enters the two cells with opposite signs and the fluctuation with
// the same sign:  2 F* = F_L + F_R - s (Q_R - Q_L),  2 Dn = B(mid)(Q_R - Q_L).
template <class Ph, int D>
__device__ __forceinline__ void rusanov_face2(const Ph &ph, const double *qL, const double *FL,
                                              double lL, const double *qR, const double *FR,
                                              double lR, double *Fs2, double *Dn2)
{
    constexpr int N = Ph::N;
    const double s = fmax(lL, lR);
#pragma unroll
    for (int v = 0; v < N; ++v) Fs2[v] = (FL[v] + FR[v]) - s * (qR[v] - qL[v]);
    if (Ph::kNcp) {
        ph.template ncp<D>(qL, qR, Dn2);
    } else {
#pragma unroll
        for (int v = 0; v < N; ++v) Dn2[v] = 0.0;
    }
}

}  // namespace pb

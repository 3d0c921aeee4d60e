// pb_c2p.h -- conservative-to-primitive recovery of special-relativistic
// hydrodynamics as a device function (one cell per lane), shared by the
// standalone con2prim entry point and the SRHD finite-volume pass.
//
// Ideal gas p = (Gamma-1) rho eps.  With E = tau + D, s = |S| and a trial
// pressure p: v = S/(E+p), W = (1 - v^2)^(-1/2), rho = D/W and
//   f(p)  = (Gamma-1) [E - s^2/(E+p) - D sqrt(1 - s^2/(E+p)^2)] - p,
//   f'(p) = (Gamma-1) v^2 (1 - D W/(E+p)) - 1  (< 0, so the root is unique),
// with the root bracketed by (max(s - E, 0), (Gamma-1) tau].  Newton steps
// that leave the bracket are replaced by bisection; every evaluated point
// narrows the bracket by the sign of f.  Converged when
// |f| <= tol (Gamma-1)(E+p) (the size of the terms that cancel in f); one
// more Newton step polishes the root if it stays in the bracket.  The
// iteration count is the number of updates before convergence.
#pragma once

#include <hip/hip_runtime.h>

namespace pb {

enum { C2P_OK = 0, C2P_NOTCONV = 1, C2P_BAD = 2 };

struct C2pOut {
    double p;
    int it;
    int status;
};

struct C2pIn {
    double D, s2, s, tau, E;   // s = |S|
    double lo, hi;   // bracket
    bool ok;         // admissible input
};

__device__ __forceinline__ C2pIn c2p_setup(double D, double Sx, double Sy, double Sz, double tau, double gam)
{
    C2pIn in;
    in.D = D;
    in.tau = tau;
    in.s2 = Sx * Sx + Sy * Sy + Sz * Sz;
    in.E = tau + D;
    const double s = sqrt(in.s2);
    in.s = s;
    in.ok = isfinite(D) && isfinite(in.s2) && isfinite(tau) && D > 0.0 && tau > 0.0;
    double lo = s - in.E;
    in.lo = lo > 0.0 ? lo : 0.0;
    in.hi = (gam - 1.0) * tau;
    in.ok = in.ok && (in.hi > in.lo);
    return in;
}

// 1/x from the hardware reciprocal estimate refined by two Newton steps
// (within an ulp or two of the correctly rounded quotient; x finite, nonzero)
__device__ __forceinline__ double c2p_recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// sqrt(a) and 1/sqrt(a) together, for 0 < a <= 1: Goldschmidt's coupled
// iteration g -> sqrt(a), h -> 1/(2 sqrt(a)) from the hardware reciprocal-
// square-root estimate, two steps, then one correction of the root
// (g + (a - g^2) h)
__device__ __forceinline__ double c2p_sqrt_rsqrt(double a, double &rs)
{
    const double y = __builtin_amdgcn_rsq(a);
    double g = a * y, h = 0.5 * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    rs = h + h;
    return fma(fma(-g, g, a), h, g);
}

// Newton from p0 (p0 outside (lo, hi] or NaN -> the plain guess hi).  Per
// step one reciprocal of E + p, one coupled root (sqrt(1 - v^2) and the
// Lorentz factor W = 1/sqrt(1 - v^2)) and one reciprocal of f'; the
// divisions of the closed forms become products with these.
__device__ __forceinline__ C2pOut c2p_solve(const C2pIn &in, double gam, double tol, int maxit, double p0)
{
    C2pOut o;
    if (!in.ok) {
        o.p = __builtin_nan("");
        o.it = 0;
        o.status = C2P_BAD;
        return o;
    }
    const double g1 = gam - 1.0;
    double lo = in.lo, hi = in.hi;
    double p = (p0 > lo && p0 <= hi) ? p0 : hi;
    for (int it = 0;; ++it) {
        const double Ep = in.E + p;
        const double iEp = c2p_recip(Ep);
        const double v2 = in.s2 * iEp * iEp;
        double W;
        const double sq = c2p_sqrt_rsqrt(1.0 - v2, W);
        const double f = g1 * (in.E - in.s2 * iEp - in.D * sq) - p;
        const double df = g1 * v2 * (1.0 - in.D * iEp * W) - 1.0;
        const double step = f * c2p_recip(df);
        if (fabs(f) <= tol * g1 * Ep) {
            const double pp = p - step;
            if (pp > lo && pp <= hi) p = pp;
            o.p = p;
            o.it = it;
            o.status = C2P_OK;
            return o;
        }
        if (it >= maxit) {
            o.p = p;
            o.it = it;
            o.status = C2P_NOTCONV;
            return o;
        }
        if (f > 0.0) lo = p; else hi = p;
        double pn = p - step;
        if (!(pn > lo && pn <= hi)) pn = 0.5 * (lo + hi);
        p = pn;
    }
}

}  // namespace pb

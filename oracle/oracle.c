/*
 * oracle.c -- plain CPU reference ("oracle") for the batched explicit update
 * of Cartesian patches with halos, for systems of the form
 *
 *     dQ/dt + div F(Q) + B(Q) . grad Q = S(Q)          (paper Sec. I, Eq. (1))
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition that the HIP library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never calls it, and it shares no code, header, table or
 * helper with the HIP library.
 *
 * Conventions
 *   - single-threaded, IEEE double, built with -O2 -ffp-contract=off
 *     -fno-fast-math so that every expression is evaluated as written;
 *   - each patch is expanded into its own array-of-structs block *with* halo,
 *     (p+2h)^d cells x N unknowns, the "natural" per-cell layout of the
 *     paper (Sec. II-B): one contiguous run of unknowns per cell;
 *   - halo edges and corners are filled with NaN so that a stencil that
 *     strays off the axis shows up as NaN in the result;
 *   - the state exchanged with the caller is patch-blocked SoA:
 *     element (k, v, cell) sits at  off_k*N + v*p_k^d + cell,  cell index
 *     (z*p + y)*p + x, x fastest, off_k = sum_{j<k} p_j^d.
 *
 * What each function follows is cited in its comment.  Formulas the paper
 * names but does not spell out (Rusanov flux, Kreiss-Oliger dissipation,
 * classical RK4, special-relativistic hydrodynamics and its
 * conservative-to-primitive recovery) are the textbook definitions cited at
 * the function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- types -- */

enum { ORC_ADV_F = 0, ORC_ADV_B = 1, ORC_EULER = 2, ORC_LINSYM = 3, ORC_SRHD = 4, ORC_ADV_VAR = 5 };

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2 };

/* con2prim per-cell status */
enum { C2P_OK = 0, C2P_NOTCONV = 1, C2P_BADINPUT = 2 };

typedef struct {
    int dim;              /* 2 or 3 */
    int K;                /* number of patches */
    int N;                /* evolved unknowns per cell */
    int h;                /* halo width */
    const int *p;         /* [K] cells per direction */
    const double *dx;     /* [K] cell width */
    const int *nbr;       /* [K][2*dim] face neighbours (-x,+x,-y,+y,-z,+z) */
    int pde;              /* ORC_* */
    const double *prm;    /* PDE parameters, see pde_* below */
    /* SRHD con2prim settings used inside the FV step */
    double c2p_tol;
    int c2p_maxit;
    /* material parameters (Sec. II: N evolving unknowns plus M parameters
     * per point that are fixed in time): the last M of the N values per cell
     * are read by the physics and copied through every update unchanged */
    int M;
} orc_desc;

typedef struct {
    long c2p_fail;        /* cells whose con2prim did not converge / bad input */
    long c2p_iters;       /* total Newton updates */
    int c2p_maxiter_seen;
} orc_stats;

/* --------------------------------------------------------- patch access -- */

static long cells_of(const orc_desc *b, int k)
{
    long c = 1;
    for (int d = 0; d < b->dim; d++) c *= b->p[k];
    return c;
}

static long hcells_of(const orc_desc *b, int k)
{
    long c = 1;
    for (int d = 0; d < b->dim; d++) c *= (b->p[k] + 2 * b->h);
    return c;
}

/* index of cell (i[0],i[1],i[2]) (halo-relative, interior starts at 0) in the
 * with-halo block of patch k */
static long hidx(const orc_desc *b, int k, const int *i)
{
    long ph = b->p[k] + 2 * b->h;
    long r = 0;
    for (int d = b->dim - 1; d >= 0; d--) r = r * ph + (i[d] + b->h);
    return r;
}

static long iidx(const orc_desc *b, int k, const int *i)
{
    long p = b->p[k];
    long r = 0;
    for (int d = b->dim - 1; d >= 0; d--) r = r * p + i[d];
    return r;
}

/* iterate i over [lo,hi)^dim, returns 0 when done */
static int next_index(int dim, int *i, const int *lo, const int *hi)
{
    for (int d = 0; d < dim; d++) {
        if (++i[d] < hi[d]) return 1;
        i[d] = lo[d];
    }
    return 0;
}

typedef struct {
    double **U;           /* [K] -> with-halo AoS blocks, hcells*N doubles */
    long *off;            /* [K] cell offsets in the exchange layout */
} hblocks;

static void free_blocks(const orc_desc *b, hblocks *hb)
{
    if (hb->U) {
        for (int k = 0; k < b->K; k++) free(hb->U[k]);
        free(hb->U);
    }
    free(hb->off);
    hb->U = NULL;
    hb->off = NULL;
}

static int alloc_blocks(const orc_desc *b, hblocks *hb, int width)
{
    hb->U = (double **)calloc((size_t)b->K, sizeof(double *));
    hb->off = (long *)calloc((size_t)b->K + 1, sizeof(long));
    if (!hb->U || !hb->off) { free_blocks(b, hb); return ORC_ENOMEM; }
    for (int k = 0; k < b->K; k++) {
        hb->off[k + 1] = hb->off[k] + cells_of(b, k);
        size_t n = (size_t)hcells_of(b, k) * (size_t)width;
        hb->U[k] = (double *)malloc(n * sizeof(double));
        if (!hb->U[k]) { free_blocks(b, hb); return ORC_ENOMEM; }
        for (size_t j = 0; j < n; j++) hb->U[k][j] = NAN;
    }
    return ORC_OK;
}

/* exchange layout -> interior of the AoS blocks (halo left untouched) */
static void load_interior(const orc_desc *b, const double *Q, hblocks *hb, int W)
{
    int lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, i[3];
    for (int k = 0; k < b->K; k++) {
        long C = cells_of(b, k);
        for (int d = 0; d < b->dim; d++) hi[d] = b->p[k];
        memcpy(i, lo, sizeof i);
        do {
            long hc = hidx(b, k, i), ic = iidx(b, k, i);
            for (int v = 0; v < W; v++)
                hb->U[k][hc * W + v] = Q[hb->off[k] * W + (long)v * C + ic];
        } while (next_index(b->dim, i, lo, hi));
    }
}

static void store_interior(const orc_desc *b, const hblocks *hb, double *Q, int W)
{
    int lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, i[3];
    for (int k = 0; k < b->K; k++) {
        long C = cells_of(b, k);
        for (int d = 0; d < b->dim; d++) hi[d] = b->p[k];
        memcpy(i, lo, sizeof i);
        do {
            long hc = hidx(b, k, i), ic = iidx(b, k, i);
            for (int v = 0; v < W; v++)
                Q[hb->off[k] * W + (long)v * C + ic] = hb->U[k][hc * W + v];
        } while (next_index(b->dim, i, lo, hi));
    }
}

/*
 * Halo fill (paper Sec. II, cell kernel Eq. (2): every patch is read with a
 * halo of width h, p^ = p + 2h; the halo holds the face-adjacent cells'
 * values).  For the face in direction d on side s the h layers are copied
 * from the interior of the face neighbour at the wrapped index; all other
 * indices stay interior, so edges and corners are never written (they keep
 * the NaN they were allocated with).  Requires p_nb == p_k and p >= h.
 */
static void fill_halo(const orc_desc *b, hblocks *hb, int W)
{
    int i[3], j[3], lo[3], hi[3];
    for (int k = 0; k < b->K; k++) {
        int p = b->p[k];
        for (int d = 0; d < b->dim; d++) {
            for (int s = 0; s < 2; s++) {
                int nb = b->nbr[k * 2 * b->dim + 2 * d + s];
                for (int l = 0; l < b->h; l++) {
                    int id = (s == 0) ? -1 - l : p + l;     /* halo index */
                    int jd = (s == 0) ? p - 1 - l : l;      /* source index */
                    for (int e = 0; e < 3; e++) { lo[e] = 0; hi[e] = (e < b->dim) ? p : 1; }
                    lo[d] = id; hi[d] = id + 1;
                    memcpy(i, lo, sizeof i);
                    do {
                        memcpy(j, i, sizeof j);
                        j[d] = jd;
                        long dst = hidx(b, k, i), src = hidx(b, nb, j);
                        for (int v = 0; v < W; v++)
                            hb->U[k][dst * W + v] = hb->U[nb][src * W + v];
                    } while (next_index(b->dim, i, lo, hi));
                }
            }
        }
    }
}

/* ------------------------------------------------------------- physics -- */
/*
 * Parameters (prm):
 *   ORC_ADV_F / ORC_ADV_B : a_x, a_y, a_z, kappa      (N >= 1, every unknown
 *                           advected with velocity a; source S = -kappa Q)
 *   ORC_EULER             : gamma                     (N = dim + 2)
 *   ORC_LINSYM            : rho_x, rho_y, rho_z, B_x[N][N], B_y[N][N],
 *                           B_z[N][N] (row-major)     (rho_d = spectral radius)
 *   ORC_SRHD              : Gamma                     (N = 5, dim = 3)
 *   ORC_ADV_VAR           : kappa                     (N = 1 + dim, M = dim:
 *                           q and the velocity field a(x) as material
 *                           parameters; F_d = a_d(x) q, S = -kappa q)
 */

/*
 * Special-relativistic hydrodynamics, ideal gas p = (Gamma-1) rho eps
 * (Marti & Mueller, Living Rev. Relativity, "Numerical hydrodynamics in
 * special relativity"):
 *   W = (1 - v^2)^(-1/2),  h = 1 + eps + p/rho,
 *   D = rho W,  S = rho h W^2 v,  tau = rho h W^2 - p - D,
 *   F_d = (D v_d, S v_d + p e_d, S_d - D v_d),
 *   c_s^2 = Gamma p / (rho h),
 *   lambda_pm = [v_d (1 - c_s^2) +- c_s sqrt((1 - v^2)(1 - v^2 c_s^2
 *               - v_d^2 (1 - c_s^2)))] / (1 - v^2 c_s^2).
 */
void orc_srhd_prim2cons(long n, const double *prim, double *cons, double Gam)
{
    /* prim SoA [5][n] = (rho, vx, vy, vz, p) -> cons SoA [5][n] = (D,Sx,Sy,Sz,tau) */
    for (long c = 0; c < n; c++) {
        double rho = prim[c], vx = prim[n + c], vy = prim[2 * n + c], vz = prim[3 * n + c];
        double p = prim[4 * n + c];
        double v2 = vx * vx + vy * vy + vz * vz;
        double W = 1.0 / sqrt(1.0 - v2);
        double eps = p / ((Gam - 1.0) * rho);
        double h = 1.0 + eps + p / rho;
        double rhW2 = rho * h * W * W;
        cons[c] = rho * W;
        cons[n + c] = rhW2 * vx;
        cons[2 * n + c] = rhW2 * vy;
        cons[3 * n + c] = rhW2 * vz;
        cons[4 * n + c] = rhW2 - p - rho * W;
    }
}

/*
 * Conservative-to-primitive recovery for SRHD by a bracketed Newton iteration
 * on the pressure.  With E = tau + D and s = |S|, a trial pressure p gives
 *   v = S / (E + p),  W = (1 - v^2)^(-1/2),  rho = D / W,
 *   rho eps = (E + p)(1 - v^2) - p - D sqrt(1 - v^2),
 * and the root of
 *   f(p) = (Gamma-1) [E - s^2/(E+p) - D sqrt(1 - s^2/(E+p)^2)] - p
 * is the pressure.  Its derivative is
 *   f'(p) = (Gamma-1) v^2 (1 - D W / (E+p)) - 1  (< 0),
 * so f decreases and the root lies in (p_lo, p_hi] with
 *   p_lo = max(s - E, 0),   p_hi = (Gamma-1) tau
 * (tau >= rho eps follows from tau = rho W (W-1) + rho eps W^2 + p (W^2-1)).
 * Newton steps that leave the bracket are replaced by bisection; the bracket
 * is narrowed with the sign of f at every evaluated point.  Convergence:
 * |f(p)| <= tol (Gamma-1)(E+p), i.e. relative to the size of the terms that
 * cancel in f; then one more Newton step ("polish") is taken if it stays in
 * the bracket.  The iteration count is the number of Newton/bisection updates
 * before convergence (the polish is not counted).
 *
 * Returns C2P_* and writes p, iterations.
 */
static int c2p_newton(double D, double Sx, double Sy, double Sz, double tau,
                      double Gam, double tol, int maxit, double p0,
                      double *p_out, int *it_out)
{
    double E = tau + D;
    double s2 = Sx * Sx + Sy * Sy + Sz * Sz;
    double s = sqrt(s2);
    if (!(isfinite(D) && isfinite(s2) && isfinite(tau)) || !(D > 0.0) || !(tau > 0.0)) {
        *p_out = NAN; *it_out = 0; return C2P_BADINPUT;
    }
    double lo = s - E; if (lo < 0.0) lo = 0.0;
    double hi = (Gam - 1.0) * tau;
    if (!(hi > lo)) { *p_out = NAN; *it_out = 0; return C2P_BADINPUT; }
    double p = p0;
    if (!(p > lo) || !(p <= hi)) p = hi;  /* NaN or outside the bracket */
    for (int it = 0; ; it++) {
        double Ep = E + p;
        double v2 = s2 / (Ep * Ep);
        double sq = sqrt(1.0 - v2);
        double f = (Gam - 1.0) * (E - s2 / Ep - D * sq) - p;
        double W = 1.0 / sq;
        double df = (Gam - 1.0) * v2 * (1.0 - D * W / Ep) - 1.0;
        if (fabs(f) <= tol * (Gam - 1.0) * Ep) {
            double pp = p - f / df;
            if (pp > lo && pp <= hi) p = pp;
            *p_out = p; *it_out = it;
            return C2P_OK;
        }
        if (it >= maxit) { *p_out = p; *it_out = it; return C2P_NOTCONV; }
        if (f > 0.0) lo = p; else hi = p;
        double pn = p - f / df;
        if (!(pn > lo && pn <= hi)) pn = 0.5 * (lo + hi);
        p = pn;
    }
}

/*
 * con2prim over n cells.  cons SoA [5][n]; prim SoA [5][n] = (rho,vx,vy,vz,p).
 * p_guess (nullable): initial pressure per cell; a guess that is NaN or
 * outside (p_lo, p_hi] is replaced by p_hi.  If a guessed start does not
 * converge, the cell is redone from the plain guess p_hi ("fallback") and the
 * iterations of both attempts are counted.
 * iters, status (nullable): per-cell outputs.  Returns the number of cells
 * with status != C2P_OK.
 */
long orc_con2prim(long n, const double *cons, double *prim, double Gam, double tol,
                  int maxit, const double *p_guess, int *iters, int *status,
                  long *n_fallback)
{
    long nfail = 0, nfb = 0;
    for (long c = 0; c < n; c++) {
        double D = cons[c], Sx = cons[n + c], Sy = cons[2 * n + c], Sz = cons[3 * n + c];
        double tau = cons[4 * n + c];
        double p; int it = 0, it2 = 0;
        double g = p_guess ? p_guess[c] : INFINITY;
        int st = c2p_newton(D, Sx, Sy, Sz, tau, Gam, tol, maxit, g, &p, &it);
        if (st == C2P_NOTCONV && p_guess) {
            nfb++;
            st = c2p_newton(D, Sx, Sy, Sz, tau, Gam, tol, maxit, INFINITY, &p, &it2);
            it += it2;
        }
        if (st != C2P_OK) nfail++;
        if (prim) {
            double Ep = tau + D + p;
            double vx = Sx / Ep, vy = Sy / Ep, vz = Sz / Ep;
            double v2 = vx * vx + vy * vy + vz * vz;
            double W = 1.0 / sqrt(1.0 - v2);
            prim[c] = D / W;
            prim[n + c] = vx;
            prim[2 * n + c] = vy;
            prim[3 * n + c] = vz;
            prim[4 * n + c] = p;
        }
        if (iters) iters[c] = it;
        if (status) status[c] = st;
    }
    if (n_fallback) *n_fallback = nfb;
    return nfail;
}

/* f(p) and f'(p) of the con2prim root problem, exported for the tests */
void orc_c2p_residual(double D, double Sx, double Sy, double Sz, double tau,
                      double Gam, double p, double *f, double *df)
{
    double E = tau + D;
    double s2 = Sx * Sx + Sy * Sy + Sz * Sz;
    double Ep = E + p;
    double v2 = s2 / (Ep * Ep);
    double sq = sqrt(1.0 - v2);
    *f = (Gam - 1.0) * (E - s2 / Ep - D * sq) - p;
    *df = (Gam - 1.0) * v2 * (1.0 - D * (1.0 / sq) / Ep) - 1.0;
}

/* per-cell "primitive" data each PDE needs besides Q (only SRHD has any:
 * the pressure, from con2prim) */
static int aux_width(const orc_desc *b) { return b->pde == ORC_SRHD ? 1 : 0; }

/* physical flux F_d(Q) */
static void phys_flux(const orc_desc *b, int d, const double *Q, const double *aux, double *F)
{
    int N = b->N;
    switch (b->pde) {
    case ORC_ADV_F:
        for (int v = 0; v < N; v++) F[v] = b->prm[d] * Q[v];
        break;
    case ORC_ADV_VAR:
        F[0] = Q[1 + d] * Q[0];
        for (int v = 1; v < N; v++) F[v] = 0.0;
        break;
    case ORC_EULER: {
        /* Q = (rho, m, E); F_d = (m_d, m_d m / rho + p e_d, (E + p) m_d / rho) */
        double gam = b->prm[0];
        double rho = Q[0];
        double m2 = 0.0;
        for (int e = 0; e < b->dim; e++) m2 += Q[1 + e] * Q[1 + e];
        double E = Q[1 + b->dim];
        double p = (gam - 1.0) * (E - 0.5 * m2 / rho);
        F[0] = Q[1 + d];
        for (int e = 0; e < b->dim; e++) F[1 + e] = Q[1 + d] * Q[1 + e] / rho + (e == d ? p : 0.0);
        F[1 + b->dim] = (E + p) * Q[1 + d] / rho;
        break;
    }
    case ORC_SRHD: {
        double p = aux[0];
        double Ep = Q[4] + Q[0] + p;
        double vd = Q[1 + d] / Ep;
        F[0] = Q[0] * vd;
        for (int e = 0; e < 3; e++) F[1 + e] = Q[1 + e] * vd + (e == d ? p : 0.0);
        F[4] = Q[1 + d] - Q[0] * vd;
        break;
    }
    default:
        for (int v = 0; v < N; v++) F[v] = 0.0;
    }
}

static int has_flux(const orc_desc *b)
{
    return b->pde == ORC_ADV_F || b->pde == ORC_EULER || b->pde == ORC_SRHD || b->pde == ORC_ADV_VAR;
}

static int has_ncp(const orc_desc *b) { return b->pde == ORC_ADV_B || b->pde == ORC_LINSYM; }

/* B_d(Q) dQ  (the non-conservative product along d) */
static void phys_ncp(const orc_desc *b, int d, const double *Qbar, const double *dQ, double *out)
{
    int N = b->N;
    (void)Qbar;
    switch (b->pde) {
    case ORC_ADV_B:
        for (int v = 0; v < N; v++) out[v] = b->prm[d] * dQ[v];
        break;
    case ORC_LINSYM: {
        const double *B = b->prm + 3 + (long)d * N * N;
        for (int r = 0; r < N; r++) {
            double acc = 0.0;
            for (int c = 0; c < N; c++) acc += B[(long)r * N + c] * dQ[c];
            out[r] = acc;
        }
        break;
    }
    default:
        for (int v = 0; v < N; v++) out[v] = 0.0;
    }
}

/* maximal absolute characteristic speed along d */
static double phys_eig(const orc_desc *b, int d, const double *Q, const double *aux)
{
    switch (b->pde) {
    case ORC_ADV_F:
    case ORC_ADV_B:
        return fabs(b->prm[d]);
    case ORC_ADV_VAR:
        return fabs(Q[1 + d]);
    case ORC_EULER: {
        double gam = b->prm[0];
        double rho = Q[0];
        double m2 = 0.0;
        for (int e = 0; e < b->dim; e++) m2 += Q[1 + e] * Q[1 + e];
        double p = (gam - 1.0) * (Q[1 + b->dim] - 0.5 * m2 / rho);
        return fabs(Q[1 + d] / rho) + sqrt(gam * p / rho);
    }
    case ORC_LINSYM:
        return b->prm[d];
    case ORC_SRHD: {
        double Gam = b->prm[0];
        double p = aux[0];
        double Ep = Q[4] + Q[0] + p;
        double v[3] = {Q[1] / Ep, Q[2] / Ep, Q[3] / Ep};
        double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        double W = 1.0 / sqrt(1.0 - v2);
        double rho = Q[0] / W;
        double rhoh = rho + Gam / (Gam - 1.0) * p;
        double cs2 = Gam * p / rhoh;
        double cs = sqrt(cs2);
        double vd = v[d];
        double den = 1.0 - v2 * cs2;
        double root = sqrt((1.0 - v2) * (1.0 - v2 * cs2 - vd * vd * (1.0 - cs2)));
        double lp = (vd * (1.0 - cs2) + cs * root) / den;
        double lm = (vd * (1.0 - cs2) - cs * root) / den;
        return fmax(fabs(lp), fabs(lm));
    }
    }
    return 0.0;
}

static void phys_source(const orc_desc *b, const double *Q, double *S)
{
    for (int v = 0; v < b->N; v++) S[v] = 0.0;
    if (b->pde == ORC_ADV_F || b->pde == ORC_ADV_B) {
        double kappa = b->prm[3];
        for (int v = 0; v < b->N; v++) S[v] = -kappa * Q[v];
    }
    if (b->pde == ORC_ADV_VAR) S[0] = -b->prm[0] * Q[0];
}

/* ------------------------------------------------------- time step size -- */
/*
 * CFL time step: Lambda_d = max over all interior cells of all patches of the
 * maximal speed along d; dt = cfl / sum_d (Lambda_d / dx_min) with dx_min the
 * smallest cell width in the batch.  (The paper only says that the
 * eigenvalue function returns a scalar, Sec. II-B; the combination over
 * directions is the unsplit CFL rule, which is the exact shift at cfl = 1 for
 * axis-aligned advection.)
 */
static double cfl_dt(const orc_desc *b, const hblocks *hb, const hblocks *ax, double cfl,
                     double *lam_out)
{
    int N = b->N, A = aux_width(b);
    double lam[3] = {0.0, 0.0, 0.0};
    double dxmin = INFINITY;
    int lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, i[3];
    for (int k = 0; k < b->K; k++) {
        if (b->dx[k] < dxmin) dxmin = b->dx[k];
        for (int d = 0; d < b->dim; d++) hi[d] = b->p[k];
        memcpy(i, lo, sizeof i);
        do {
            long hc = hidx(b, k, i);
            const double *Q = hb->U[k] + hc * N;
            const double *a = A ? ax->U[k] + hc * A : NULL;
            for (int d = 0; d < b->dim; d++) {
                double l = phys_eig(b, d, Q, a);
                if (l > lam[d]) lam[d] = l;
            }
        } while (next_index(b->dim, i, lo, hi));
    }
    double den = 0.0;
    for (int d = 0; d < b->dim; d++) den += lam[d] / dxmin;
    if (lam_out) for (int d = 0; d < 3; d++) lam_out[d] = lam[d];
    return cfl / den;
}

/* ------------------------------------------------- validation, helpers -- */

static int check_desc(const orc_desc *b, int stencil_radius)
{
    if (!b || (b->dim != 2 && b->dim != 3) || b->K < 1 || b->N < 1 || !b->p || !b->dx || !b->nbr)
        return ORC_EINVAL;
    if (b->h < stencil_radius) return ORC_EINVAL;
    if (b->pde == ORC_EULER && b->N != b->dim + 2) return ORC_EINVAL;
    if (b->pde == ORC_SRHD && (b->N != 5 || b->dim != 3)) return ORC_EINVAL;
    if (b->pde == ORC_ADV_VAR ? (b->N != 1 + b->dim || b->M != b->dim) : b->M != 0) return ORC_EINVAL;
    for (int k = 0; k < b->K; k++) {
        if (b->p[k] < b->h || !(b->dx[k] > 0.0)) return ORC_EINVAL;
        for (int f = 0; f < 2 * b->dim; f++) {
            int nb = b->nbr[k * 2 * b->dim + f];
            if (nb < 0 || nb >= b->K || b->p[nb] != b->p[k]) return ORC_EINVAL;
        }
    }
    return ORC_OK;
}

/* SRHD: pressure of every cell of every with-halo block (halo included; the
 * halo is a copy of neighbour interiors, so this equals the neighbour's own
 * result).  Corner/edge NaN cells are skipped. */
static void srhd_pressure(const orc_desc *b, const hblocks *hb, hblocks *ax, orc_stats *st)
{
    double Gam = b->prm[0];
    int lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, i[3];
    for (int k = 0; k < b->K; k++) {
        int p = b->p[k];
        for (int d = 0; d < b->dim; d++) { lo[d] = -b->h; hi[d] = p + b->h; }
        memcpy(i, lo, sizeof i);
        do {
            long c = hidx(b, k, i);
            const double *Q = hb->U[k] + c * 5;
            if (isnan(Q[0])) { ax->U[k][c] = NAN; continue; }
            double pr; int it;
            int s = c2p_newton(Q[0], Q[1], Q[2], Q[3], Q[4], Gam, b->c2p_tol, b->c2p_maxit,
                               INFINITY, &pr, &it);
            ax->U[k][c] = pr;
            int interior = 1;
            for (int d = 0; d < b->dim; d++) if (i[d] < 0 || i[d] >= p) interior = 0;
            if (st && interior) {
                if (s != C2P_OK) st->c2p_fail++;
                st->c2p_iters += it;
                if (it > st->c2p_maxiter_seen) st->c2p_maxiter_seen = it;
            }
        } while (next_index(b->dim, i, lo, hi));
    }
}

/* ------------------------------------------------- Rusanov FV step ----- */
/*
 * First-order finite-volume step with a Rusanov (local Lax-Friedrichs) flux
 * (Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 10)
 * on the patch batch, composed as in the paper's kernel-composition example
 * (Sec. II-A, Eq. (3)): source term, face fluxes from the two adjacent cell
 * values (piecewise-constant reconstruction), update.
 *
 * For the face between L and R along d:
 *   s  = max(lambda_d(Q_L), lambda_d(Q_R))
 *   F* = 1/2 (F_d(Q_L) + F_d(Q_R)) - 1/2 s (Q_R - Q_L)
 *   D  = 1/2 B_d((Q_L + Q_R)/2) (Q_R - Q_L)       (non-conservative product,
 *        midpoint path; added to both adjacent cells)
 * and each interior cell i is advanced by explicit Euler with every term
 * taken at Q^n:
 *   Q_i <- Q_i - (dt/dx) sum_d [ (F*_{i+1/2} - F*_{i-1/2}) + (D_{i+1/2} + D_{i-1/2}) ]
 *              + dt S(Q_i).
 * round_fp32 != 0 rounds every stored value to binary32 (round to nearest
 * even) after each step, emulating FP32 state storage.
 *
 * Q: exchange layout, updated in place.  dt_fixed > 0 fixes the step size.
 * dt_used (nullable): dt of every step [n_steps].
 */
int orc_fv_step(const orc_desc *b, double *Q, double cfl, double dt_fixed, int n_steps,
                int round_fp32, double *dt_used, orc_stats *st)
{
    int rc = check_desc(b, 1);
    if (rc) return rc;
    if (b->pde == ORC_SRHD && !(b->c2p_maxit >= 0)) return ORC_EINVAL;
    int N = b->N, A = aux_width(b);
    hblocks hb = {0}, ax = {0}, out = {0};
    if ((rc = alloc_blocks(b, &hb, N))) return rc;
    if ((rc = alloc_blocks(b, &out, N))) { free_blocks(b, &hb); return rc; }
    if (A && (rc = alloc_blocks(b, &ax, A))) { free_blocks(b, &hb); free_blocks(b, &out); return rc; }

    double FL[64], FR[64], Fs[64], QLR[64], dQ[64], Dn[64], acc[64], S[64], Qb[64];
    if (N > 64) { free_blocks(b, &hb); free_blocks(b, &out); free_blocks(b, &ax); return ORC_EINVAL; }

    load_interior(b, Q, &hb, N);
    for (int n = 0; n < n_steps; n++) {
        fill_halo(b, &hb, N);
        if (A) srhd_pressure(b, &hb, &ax, st);
        double dt = dt_fixed > 0.0 ? dt_fixed : cfl_dt(b, &hb, &ax, cfl, NULL);
        if (dt_used) dt_used[n] = dt;
        int lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, i[3], j[3];
        for (int k = 0; k < b->K; k++) {
            double r = dt / b->dx[k];
            for (int d = 0; d < b->dim; d++) hi[d] = b->p[k];
            memcpy(i, lo, sizeof i);
            do {
                long c0 = hidx(b, k, i);
                const double *Qi = hb.U[k] + c0 * N;
                const double *ai = A ? ax.U[k] + c0 * A : NULL;
                for (int v = 0; v < N; v++) acc[v] = 0.0;
                for (int d = 0; d < b->dim; d++) {
                    double Fface[2][64], Dface[2][64];
                    for (int side = 0; side < 2; side++) {
                        /* face i-1/2 (side 0) or i+1/2 (side 1): L, R cells */
                        memcpy(j, i, sizeof j);
                        j[d] += (side == 0) ? -1 : 1;
                        long cj = hidx(b, k, j);
                        const double *QL = side == 0 ? hb.U[k] + cj * N : Qi;
                        const double *QR = side == 0 ? Qi : hb.U[k] + cj * N;
                        const double *aL = A ? (side == 0 ? ax.U[k] + cj * A : ai) : NULL;
                        const double *aR = A ? (side == 0 ? ai : ax.U[k] + cj * A) : NULL;
                        double sL = phys_eig(b, d, QL, aL), sR = phys_eig(b, d, QR, aR);
                        double smax = sL > sR ? sL : sR;
                        phys_flux(b, d, QL, aL, FL);
                        phys_flux(b, d, QR, aR, FR);
                        for (int v = 0; v < N; v++)
                            Fs[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * smax * (QR[v] - QL[v]);
                        if (has_ncp(b)) {
                            for (int v = 0; v < N; v++) {
                                Qb[v] = 0.5 * (QL[v] + QR[v]);
                                dQ[v] = QR[v] - QL[v];
                            }
                            phys_ncp(b, d, Qb, dQ, QLR);
                            for (int v = 0; v < N; v++) Dn[v] = 0.5 * QLR[v];
                        } else {
                            for (int v = 0; v < N; v++) Dn[v] = 0.0;
                        }
                        memcpy(Fface[side], Fs, sizeof(double) * N);
                        memcpy(Dface[side], Dn, sizeof(double) * N);
                    }
                    for (int v = 0; v < N; v++)
                        acc[v] += (Fface[1][v] - Fface[0][v]) + (Dface[1][v] + Dface[0][v]);
                }
                phys_source(b, Qi, S);
                double *Qo = out.U[k] + c0 * N;
                for (int v = 0; v < N; v++) {
                    double q = Qi[v] - r * acc[v] + dt * S[v];
                    if (round_fp32) q = (double)(float)q;
                    Qo[v] = v < N - b->M ? q : Qi[v];   /* material parameters: copied */
                }
            } while (next_index(b->dim, i, lo, hi));
        }
        /* swap */
        double **t = hb.U; hb.U = out.U; out.U = t;
    }
    store_interior(b, &hb, Q, N);
    free_blocks(b, &hb);
    free_blocks(b, &out);
    if (A) free_blocks(b, &ax);
    return ORC_OK;
}

/* ---------------------------------------------- FD4 + KO6 + RK4 step ---- */
/*
 * Fourth-order central finite differences with Kreiss-Oliger dissipation
 * (Kreiss & Oliger 1973, the dissipation the paper names in Sec. I) and
 * classical Runge-Kutta stages (Sec. II: RK schemes call the cell update
 * several times with the Butcher-tableau step sizes and refresh the halo
 * between stages).
 *
 *   D4 u   = [(u_{-2} - u_{+2}) + 8 (u_{+1} - u_{-1})] / (12 dx)
 *   KO6 u  = sigma/(64 dx) [(u_{-3} + u_{+3}) - 6 (u_{-2} + u_{+2})
 *                           + 15 (u_{-1} + u_{+1}) - 20 u_0]
 *   R(Q)_i = sum_d ( -D4_d F_d(Q) - B_d(Q_i) D4_d Q + KO6_d Q ) + S(Q_i)
 *
 * The sixth difference is the dissipation of order 2r = 6 that matches a
 * fourth-order interior scheme (Gustafsson, Kreiss & Oliger, "Time-dependent
 * problems and difference methods"); it needs a halo of 3.  sigma = 0 turns
 * it off (then a halo of 2 suffices).
 *
 * rk_stages = 4: k1 = R(Q), k2 = R(Q + dt/2 k1), k3 = R(Q + dt/2 k2),
 *                k4 = R(Q + dt k3), Q <- Q + dt/6 (k1 + 2 k2 + 2 k3 + k4);
 * rk_stages = 1: Q <- Q + dt R(Q).
 * dt is computed once per step from Q^n by the CFL rule of cfl_dt.
 */
static void fd_rhs(const orc_desc *b, hblocks *hb, hblocks *rhs, double sigma)
{
    int N = b->N;
    double G[64], BG[64], Fm2[64], Fm1[64], Fp1[64], Fp2[64], S[64];
    int lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, i[3], j[3];
    fill_halo(b, hb, N);
    for (int k = 0; k < b->K; k++) {
        double dx = b->dx[k];
        for (int d = 0; d < b->dim; d++) hi[d] = b->p[k];
        memcpy(i, lo, sizeof i);
        do {
            long c0 = hidx(b, k, i);
            const double *Qi = hb->U[k] + c0 * N;
            double *r = rhs->U[k] + c0 * N;
            for (int v = 0; v < N; v++) r[v] = 0.0;
            for (int d = 0; d < b->dim; d++) {
                const double *u[7];
                for (int o = -3; o <= 3; o++) {
                    int oo = (o < -b->h || o > b->h) ? 0 : o;  /* unused when sigma = 0 */
                    memcpy(j, i, sizeof j);
                    j[d] += oo;
                    u[o + 3] = hb->U[k] + hidx(b, k, j) * N;
                }
                for (int v = 0; v < N; v++)
                    G[v] = ((u[1][v] - u[5][v]) + 8.0 * (u[4][v] - u[2][v])) / (12.0 * dx);
                if (has_flux(b)) {
                    phys_flux(b, d, u[1], NULL, Fm2);
                    phys_flux(b, d, u[2], NULL, Fm1);
                    phys_flux(b, d, u[4], NULL, Fp1);
                    phys_flux(b, d, u[5], NULL, Fp2);
                    for (int v = 0; v < N; v++)
                        r[v] -= ((Fm2[v] - Fp2[v]) + 8.0 * (Fp1[v] - Fm1[v])) / (12.0 * dx);
                }
                if (has_ncp(b)) {
                    phys_ncp(b, d, Qi, G, BG);
                    for (int v = 0; v < N; v++) r[v] -= BG[v];
                }
                if (sigma != 0.0) {
                    for (int v = 0; v < N; v++)
                        r[v] += sigma / (64.0 * dx) *
                                ((((u[0][v] + u[6][v]) - 6.0 * (u[1][v] + u[5][v])) +
                                  15.0 * (u[2][v] + u[4][v])) - 20.0 * u[3][v]);
                }
            }
            phys_source(b, Qi, S);
            for (int v = 0; v < N; v++) r[v] += S[v];
            for (int v = N - b->M; v < N; v++) r[v] = 0.0;   /* material parameters do not evolve */
        } while (next_index(b->dim, i, lo, hi));
    }
}

/* y = x0 + a * k over the interiors (halo of y is refilled by fd_rhs) */
static void axpy_blocks(const orc_desc *b, hblocks *y, const hblocks *x0, double a, const hblocks *kk)
{
    int N = b->N;
    int lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, i[3];
    for (int k = 0; k < b->K; k++) {
        for (int d = 0; d < b->dim; d++) hi[d] = b->p[k];
        memcpy(i, lo, sizeof i);
        do {
            long c = hidx(b, k, i) * N;
            for (int v = 0; v < N; v++) y->U[k][c + v] = x0->U[k][c + v] + a * kk->U[k][c + v];
        } while (next_index(b->dim, i, lo, hi));
    }
}

int orc_fd_step(const orc_desc *b, double *Q, double cfl, double dt_fixed, double sigma,
                int rk_stages, int n_steps, double *dt_used)
{
    int rc = check_desc(b, sigma != 0.0 ? 3 : 2);
    if (rc) return rc;
    if (rk_stages != 1 && rk_stages != 4) return ORC_EINVAL;
    if (b->pde == ORC_SRHD) return ORC_EINVAL;
    if (b->N > 64) return ORC_EINVAL;
    hblocks q0 = {0}, y = {0}, k1 = {0}, k2 = {0}, k3 = {0}, k4 = {0};
    hblocks *all[6] = {&q0, &y, &k1, &k2, &k3, &k4};
    int na = rk_stages == 4 ? 6 : 3;
    for (int a = 0; a < na; a++)
        if ((rc = alloc_blocks(b, all[a], b->N))) {
            for (int c = 0; c < a; c++) free_blocks(b, all[c]);
            return rc;
        }
    int N = b->N;
    load_interior(b, Q, &q0, N);
    for (int n = 0; n < n_steps; n++) {
        double dt = dt_fixed > 0.0 ? dt_fixed : cfl_dt(b, &q0, NULL, cfl, NULL);
        if (dt_used) dt_used[n] = dt;
        if (rk_stages == 1) {
            fd_rhs(b, &q0, &k1, sigma);
            axpy_blocks(b, &y, &q0, dt, &k1);
        } else {
            fd_rhs(b, &q0, &k1, sigma);
            axpy_blocks(b, &y, &q0, 0.5 * dt, &k1);
            fd_rhs(b, &y, &k2, sigma);
            axpy_blocks(b, &y, &q0, 0.5 * dt, &k2);
            fd_rhs(b, &y, &k3, sigma);
            axpy_blocks(b, &y, &q0, dt, &k3);
            fd_rhs(b, &y, &k4, sigma);
            int lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, i[3];
            for (int k = 0; k < b->K; k++) {
                for (int d = 0; d < b->dim; d++) hi[d] = b->p[k];
                memcpy(i, lo, sizeof i);
                do {
                    long c = hidx(b, k, i) * N;
                    for (int v = 0; v < N; v++) {
                        double s = ((k1.U[k][c + v] + 2.0 * k2.U[k][c + v]) + 2.0 * k3.U[k][c + v]) +
                                   k4.U[k][c + v];
                        y.U[k][c + v] = q0.U[k][c + v] + dt / 6.0 * s;
                    }
                } while (next_index(b->dim, i, lo, hi));
            }
        }
        double **t = q0.U; q0.U = y.U; y.U = t;
    }
    store_interior(b, &q0, Q, N);
    for (int a = 0; a < na; a++) free_blocks(b, all[a]);
    return ORC_OK;
}

/* the CFL step of the state Q (exchange layout), for the tests; lam[3] out */
double orc_cfl_dt(const orc_desc *b, const double *Q, double cfl, double *lam)
{
    if (check_desc(b, 0)) return NAN;
    hblocks hb = {0}, ax = {0};
    int A = aux_width(b);
    if (alloc_blocks(b, &hb, b->N)) return NAN;
    if (A && alloc_blocks(b, &ax, A)) { free_blocks(b, &hb); return NAN; }
    load_interior(b, Q, &hb, b->N);
    if (A) srhd_pressure(b, &hb, &ax, NULL);
    double dt = cfl_dt(b, &hb, &ax, cfl, lam);
    free_blocks(b, &hb);
    if (A) free_blocks(b, &ax);
    return dt;
}

/* halo fill exported for the tests: state (exchange layout) -> with-halo AoS
 * blocks concatenated patch after patch (NaN in edges and corners) */
int orc_halo_blocks(const orc_desc *b, const double *Q, double *outblocks)
{
    int rc = check_desc(b, 0);
    if (rc) return rc;
    hblocks hb = {0};
    if ((rc = alloc_blocks(b, &hb, b->N))) return rc;
    load_interior(b, Q, &hb, b->N);
    fill_halo(b, &hb, b->N);
    long o = 0;
    for (int k = 0; k < b->K; k++) {
        long n = hcells_of(b, k) * b->N;
        memcpy(outblocks + o, hb.U[k], sizeof(double) * n);
        o += n;
    }
    free_blocks(b, &hb);
    return ORC_OK;
}

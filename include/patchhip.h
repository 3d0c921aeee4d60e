/*
 * patchhip.h -- C ABI of the MI355X (gfx950) patch-batch library.
 *
 * The library advances K Cartesian patches ("cells" of an adaptive mesh, each
 * carrying a p^d sub-grid read with a halo of width h) of a first-order
 * hyperbolic system
 *
 *     dQ/dt + div F(Q) + B(Q) . grad Q = S(Q)            (paper Sec. I, Eq. (1))
 *
 * concurrently by one explicit time step: the batched cell kernel
 * K~_{dt,K} of paper Sec. II (Eq. (2) and the batching paragraph after it).
 * Two schemes are provided: a first-order Rusanov finite-volume step (the
 * composition example of Sec. II-A, Eq. (3)) and a fourth-order central
 * finite-difference step with Kreiss-Oliger dissipation and classical RK4
 * (the FD4 scheme of Sec. IV).  Special-relativistic hydrodynamics adds a
 * per-cell conservative-to-primitive Newton solve (a term that solves a
 * nonlinear problem internally, Sec. II-A last paragraph), optionally seeded
 * by a small bfloat16 MLP trained with the library's own kernels.
 *
 * Conventions (all entry points)
 *   - Every function returns pb_status.  No C++ exception and no abort ever
 *     crosses this boundary.  Argument checks run on the host before any HIP
 *     call, so PB_EINVAL is reported without touching the GPU.
 *   - pb_last_error() returns a thread-local text for the last failure.
 *   - Device buffers (state, workspace, con2prim arrays, MLP data) are owned
 *     by the caller and must stay allocated while a batch uses them.  The
 *     library owns the pb_batch / pb_mlp objects and their small device
 *     tables, released by the matching destroy call.
 *   - Work is enqueued asynchronously on the caller's stream (hipStream_t
 *     passed as void*; NULL = the null stream).  Host synchronisation happens
 *     only where a host output is requested (dt_last_host, stats, weights),
 *     and in offload mode, whose inputs and outputs are host memory.
 *
 * State layout in HBM ("patch-blocked structure of arrays")
 *   patch k with p_k cells per direction owns cells [off_k, off_k + p_k^d),
 *   off_k = sum_{j<k} p_j^d; value v (0 <= v < N + M: the N unknowns, then
 *   the M material parameters) of local cell c sits at element
 *       off_k * (N + M) + v * p_k^d + c,  c = (z * p_k + y) * p_k + x,
 *   x fastest.  Elements are double (PB_STORE_FP64) or float (PB_STORE_FP32:
 *   arithmetic stays double, every stored value is rounded to nearest even).
 */
#ifndef PATCHHIP_H
#define PATCHHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PB_OK = 0,
    PB_EINVAL = -1,        /* bad argument; nothing was enqueued */
    PB_ENOMEM = -2,        /* a library-owned allocation failed */
    PB_EHIP = -3,          /* a HIP runtime call failed (text in pb_last_error) */
    PB_EUNSUPPORTED = -4,  /* valid request the library does not implement */
} pb_status;

typedef enum {
    PB_PDE_ADVECTION_F = 0, /* N = 1, F_d = a_d q, S = -kappa q.
                               params: a_x, a_y, a_z, kappa */
    PB_PDE_ADVECTION_B = 1, /* N = 1, B_d = a_d (non-conservative form), S = -kappa q.
                               params: a_x, a_y, a_z, kappa */
    PB_PDE_EULER = 2,       /* compressible Euler, ideal gas, N = dim + 2,
                               Q = (rho, m, E).  params: gamma */
    PB_PDE_LINSYM = 3,      /* linear symmetric system, F = S = 0, constant B_d,
                               N = 58.  params: rho_x, rho_y, rho_z (spectral
                               radii), B_x, B_y, B_z (each N*N, row-major) */
    PB_PDE_SRHD = 4,        /* special-relativistic hydrodynamics, dim = 3,
                               N = 5, Q = (D, S_x, S_y, S_z, tau).
                               params: Gamma, con2prim tol, con2prim max_iter */
    PB_PDE_ADVECTION_VAR = 5, /* linear advection by a velocity field held as
                               material parameters (paper Sec. II: N evolving
                               plus M fixed values per point): n_unknowns =
                               1, n_aux = dim, per point (q, a_x, a_y(, a_z));
                               F_d = a_d(x) q,
                               S = -kappa q.  The dim field values of every
                               cell are read by the fluxes and speeds and
                               carried through every step unchanged (bitwise).
                               FV only.  params: kappa */
} pb_pde;

typedef enum { PB_STORE_FP64 = 0, PB_STORE_FP32 = 1 } pb_storage;

typedef struct {
    int32_t dim;              /* 2 or 3 */
    int32_t n_patches;        /* K >= 1 */
    const int32_t *p;         /* host [K]: cells per direction of each patch */
    const double *dx;         /* host [K]: cell width of each patch (> 0) */
    const int32_t *neighbor;  /* host [K][2*dim]: face neighbours in the order
                                 -x,+x,-y,+y(,-z,+z); a patch may name itself
                                 (periodic on itself).  p of a neighbour must
                                 equal p of the patch. */
    int32_t halo;             /* h: >= 1 for the FV step, >= 3 for FD4 + KO6 */
    int32_t pde;              /* pb_pde */
    const double *pde_params; /* host, copied at create */
    int64_t n_pde_params;
    int32_t n_unknowns;       /* N: evolving values per point */
    int32_t n_aux;            /* M: material parameters per point (paper Sec.
                                 II: the state holds N + M values per point,
                                 the last M read by the physics and copied
                                 unchanged through every update).  M = dim for
                                 ADVECTION_VAR (the velocity field); every
                                 other PDE takes M = 0 (M > 0 there:
                                 PB_EUNSUPPORTED, checked on the host) */
    int32_t storage;          /* pb_storage */
    void *state;              /* device: the state, in the layout above */
    void *state_alt;          /* device: second buffer of the same size (the
                                 steps ping-pong between the two) */
    void *workspace;          /* device: pb_workspace_size() bytes, 256-aligned */
    size_t workspace_bytes;
    void *stream;             /* hipStream_t; not owned */
} pb_batch_desc;

typedef struct pb_batch pb_batch;

typedef struct {
    int64_t steps;               /* steps taken since create / reset */
    int64_t nonfinite_units;     /* work units that produced a NaN/Inf value */
    int64_t c2p_cells;           /* con2prim cell solves (SRHD) */
    int64_t c2p_failures;        /* cells that did not converge / bad input */
    int64_t c2p_iterations;      /* total Newton updates */
    int64_t c2p_fallbacks;       /* learned guesses redone from the plain guess */
    int32_t c2p_max_iterations;  /* largest per-cell count seen */
    int32_t current;             /* 0: result in state, 1: in state_alt */
    double last_dt;              /* step size of the most recent step */
} pb_stats;

/* Workspace bytes the batch described by `desc` needs (host-only). */
pb_status pb_workspace_size(const pb_batch_desc *desc, size_t *bytes);

/*
 * Validate `desc`, copy its host tables and upload the patch table (the
 * patch sizes, cell offsets, cell widths and face neighbours of paper
 * Sec. II: K patches of p^d cells with a halo of h, p^ = p + 2h).  The
 * descriptor's device pointers are stored, not copied.  Initialises the
 * workspace on `stream`.
 */
pb_status patch_batch_create(const pb_batch_desc *desc, pb_batch **out);
pb_status patch_batch_destroy(pb_batch *b);

/* Declare `state` (which = 0) or `state_alt` (1) to hold the current state,
 * e.g. after the caller uploaded new data; clears the counters. */
pb_status pb_batch_reset(pb_batch *b, int32_t which);

/* Statistics; synchronises the batch stream. */
pb_status pb_batch_stats(pb_batch *b, pb_stats *out);

/*
 * n_steps Rusanov finite-volume steps (paper Sec. II-A, Eq. (3): source,
 * face fluxes from the two adjacent cell values, update).  Per face along d:
 *   s = max(lambda_d(Q_L), lambda_d(Q_R)),
 *   F* = (F_d(Q_L) + F_d(Q_R))/2 - s (Q_R - Q_L)/2,
 *   D  = B_d((Q_L + Q_R)/2) (Q_R - Q_L)/2 added to both cells,
 * Q_i <- Q_i - dt/dx sum_d [(F*_{+} - F*_{-}) + (D_{+} + D_{-})] + dt S(Q_i).
 * dt_fixed > 0 fixes dt; otherwise dt = cfl / sum_d (Lambda_d / dx_min),
 * Lambda_d the maximal |speed| along d over all cells of the current state,
 * computed on the device (no host round trip between steps).
 * use_graph != 0 captures the n_steps launches once into a HIP graph and
 * replays it on later calls with the same n_steps.
 * dt_last_host (nullable): receives the last step's dt (synchronises).
 * 3D batches whose patches all have one p with p^3 <= 256 run a kernel that
 * packs several whole patches into a work-group (one thread per cell); the
 * others march z-slabs of a patch plane by plane.  Both give the same
 * results to roundoff.
 * Supported: ADVECTION_F/B (N = 1), ADVECTION_VAR (N = 1 + dim), EULER, SRHD;
 * 1 <= p <= 16; halo >= 1.
 */
pb_status fv_rusanov_step(pb_batch *b, double cfl, double dt_fixed, int32_t n_steps,
                          int32_t use_graph, double *dt_last_host);

/*
 * n_steps of fourth-order central differences with sixth-order
 * Kreiss-Oliger dissipation (Kreiss & Oliger 1973, named in paper Sec. I)
 * and rk_stages = 4 (classical RK4) or 1 (forward Euler) stages with a halo
 * refresh before each stage (paper Sec. II: RK schemes call the cell update
 * several times with Butcher-tableau step sizes plus neighbour
 * synchronisation):
 *   R(Q) = sum_d ( -D4_d F_d - B_d D4_d Q + KO6_d Q ) + S(Q),
 *   D4 u = [(u_-2 - u_+2) + 8 (u_+1 - u_-1)] / (12 dx),
 *   KO6 u = sigma/(64 dx) [(u_-3 + u_+3) - 6 (u_-2 + u_+2) + 15 (u_-1 + u_+1) - 20 u_0].
 * Two PDEs (other PDEs return PB_EUNSUPPORTED):
 *  - LINSYM (the B_d term): patches must be periodic on themselves
 *    (neighbor = self), so one persistent launch per stage sweeps all
 *    patches from a cost-ordered work list; dt as in fv_rusanov_step with
 *    Lambda_d = spectral radius of B_d (computed on the host).  N <= 60
 *    (the workloads use N = 58), p in {4, 8, 16}.
 *  - EULER (the F_d term, flux differencing; the paper's fourth scheme,
 *    Sec. IV): patches are joined through their face neighbours (the halo
 *    of width 3 is read from the neighbours' interiors inside each stage);
 *    3 <= p <= 16; dt as in fv_rusanov_step, reduced on the device from the
 *    state at the start of each step.
 * Both: dim 3, halo >= 3, FP64 storage; the workspace carries two extra
 * state-sized stage buffers (pb_workspace_size adds them for LINSYM and for
 * 3D EULER with halo >= 3).  The result lands in the state buffer opposite
 * to the current one after every step (the stage sum accumulates there).
 */
pb_status fd_ko_step(pb_batch *b, double cfl, double dt_fixed, double sigma_ko,
                     int32_t rk_stages, int32_t n_steps, int32_t use_graph,
                     double *dt_last_host);

/* ----------------------------------------------------------------- SRHD -- */

typedef struct pb_mlp pb_mlp;

/* con2prim guess modes */
typedef enum { PB_GUESS_PLAIN = 0, PB_GUESS_LEARNED = 1, PB_GUESS_WARM = 2 } pb_guess;

/*
 * Conservative-to-primitive recovery of special-relativistic hydrodynamics
 * (ideal gas, p = (Gamma-1) rho eps) by a bracketed FP64 Newton iteration on
 * the pressure.  With E = tau + D, s = |S|:
 *   f(p)  = (Gamma-1)[E - s^2/(E+p) - D sqrt(1 - s^2/(E+p)^2)] - p,
 *   f'(p) = (Gamma-1) v^2 (1 - D W/(E+p)) - 1,    root in (max(s-E,0), (Gamma-1) tau].
 * Converged when |f| <= tol (Gamma-1)(E+p); one polishing Newton step follows.
 * cons:   device, SoA [5][n] doubles (D, S_x, S_y, S_z, tau).
 * prim:   device, SoA [5][n] doubles (rho, v_x, v_y, v_z, p), written.
 * guess:  PB_GUESS_PLAIN: p0 = (Gamma-1) tau.  PB_GUESS_LEARNED: p0 from
 *         `mlp` (must be non-NULL).  PB_GUESS_WARM: p0 = p_prev[i].
 *         A learned/warm start that fails is redone from the plain guess.
 * p_prev: device [n] doubles (WARM only, else NULL).
 * iters:  device [n] int32 Newton updates per cell (nullable).
 * status: device [n] int32: 0 ok, 1 not converged, 2 bad input (nullable).
 * counters: device, 8 int64 accumulated (nullable):
 *         [0] failures, [1] total iterations, [2] fallbacks, [3] max iterations.
 * stream: hipStream_t (NULL = default stream); asynchronous.
 * Errors (checked on the host before any launch): PB_EINVAL for n < 0, a NULL
 * cons/prim with n > 0, Gamma outside (1, 2], tol <= 0, max_iter outside
 * [0, 1000], an unknown guess, LEARNED without mlp, WARM without p_prev.
 * n = 0 does nothing and returns PB_OK (the pointers are not looked at).
 * Non-convergence and bad inputs are not errors: see status / counters.
 */
pb_status con2prim(const void *cons, void *prim, int64_t n, double gamma, double tol,
                   int32_t max_iter, int32_t guess, const pb_mlp *mlp, const void *p_prev,
                   void *iters, void *status, void *counters, void *stream);

/* How fv_rusanov_step seeds the SRHD con2prim (default PB_GUESS_PLAIN). */
pb_status pb_batch_set_c2p_guess(pb_batch *b, int32_t guess, const pb_mlp *mlp);

/* ------------------------------------------------------------------ MLP -- */
/*
 * The learned con2prim guess: an MLP 5 -> 64 -> 64 -> 1 with ReLU.  Weights
 * and activations are bfloat16 (round to nearest even), products accumulate
 * in FP32 on the matrix cores, biases are FP32, the output stays FP32.
 * Features of a conserved state (all scale-free, since p/E depends only on
 * D/E and |S|/E):
 *   x = [log(D/E), |S|/E, log(1 - |S|/E), log(tau/E), log((tau (tau + 2D) - |S|^2)/E^2)]
 * (the last is log((E^2 - D^2 - |S|^2)/E^2), which measures the internal energy),
 * standardised with the stored mean/std; the target is y = log(p/E),
 * standardised with mu_y, sigma_y: p0 = E exp(mu_y + sigma_y yhat).
 * Training (FP32 master weights, Adam) runs on the device with the library's
 * own forward, backward and update kernels.
 */
#define PB_MLP_IN 5
#define PB_MLP_HID 64
#define PB_MLP_NPARAM (PB_MLP_HID * PB_MLP_IN + PB_MLP_HID + PB_MLP_HID * PB_MLP_HID + PB_MLP_HID + PB_MLP_HID + 1)

/* Parameter vector order (FP32, PB_MLP_NPARAM values):
 * W1[64][5], b1[64], W2[64][64], b2[64], W3[64], b3 -- then normalisation
 * (not trained): x_mean[5], x_std[5], y_mean, y_std  (12 values) */
#define PB_MLP_NNORM 12

pb_status pb_mlp_create(pb_mlp **out);
pb_status pb_mlp_destroy(pb_mlp *m);
/* host <-> library copies of the FP32 master parameters and normalisation */
pb_status pb_mlp_set_params(pb_mlp *m, const float *params, const float *norm);
pb_status pb_mlp_get_params(pb_mlp *m, float *params, float *norm);
/* raw features (the five values listed above, unstandardised) of n conserved
 * states: cons device SoA [5][n] doubles, x device [n][5] FP32 */
pb_status pb_mlp_features(const void *cons, void *x, int64_t n, void *stream);
/* yhat for n feature rows: x device [n][5] FP32 (raw, unstandardised features),
 * y device [n] FP32 */
pb_status pb_mlp_forward(const pb_mlp *m, const void *x, void *y, int64_t n, void *stream);
/* gradient of the mean squared error (1/n) sum (yhat - t)^2 over n rows
 * w.r.t. the parameters: t device [n] FP32 (standardised target),
 * grad device [PB_MLP_NPARAM] FP32 (overwritten), loss device [1] FP32 */
pb_status pb_mlp_grad(const pb_mlp *m, const void *x, const void *t, int64_t n, void *grad,
                      void *loss, void *stream);
/* pb_mlp_grad without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops): the same
 * kernels and results as pb_mlp_grad, with the partial-gradient scratch in a
 * fixed device array of the library (256 rows of 4672 floats, 4.8 MB, held
 * by each GPU the library runs on until the process ends) instead of the
 * MLP's own buffer, and grad / loss written directly by the reduction.
 * n must be in [1, 2^30] (larger n: PB_EINVAL, nothing enqueued).  Calls no
 * hipMalloc / hipFree.  Every call on one GPU shares that GPU's array (each
 * call rewrites the rows it reads, so no clearing is needed): calls that
 * overlap on one GPU (other streams, other threads) race. */
pb_status pb_mlp_grad_noalloc(const pb_mlp *m, const void *x, const void *t, int64_t n, void *grad,
                              void *loss, void *stream);

/* one Adam step on a batch: grad + update of the FP32 master weights and their
 * bfloat16 copies.  step is the 1-based Adam step counter.
 * Forward and backward run on the matrix cores (bf16 operands, FP32
 * accumulation; dh1 and dh2 are rounded to bf16 for the products), the
 * reduction over rows in a fixed order (bitwise reproducible).  Uses the
 * MLP's own partial-gradient buffer (allocated by pb_mlp_create), so calls on
 * one MLP must not overlap. */
pb_status pb_mlp_train_step(pb_mlp *m, const void *x, const void *t, int64_t n, float lr,
                            float beta1, float beta2, float eps, int32_t step, void *loss,
                            void *stream);

/* Training-set preparation on the device (the trainer then only allocates).
 * pb_mlp_prepare: cons device SoA [5][n] doubles and their pressures p device
 *   [n] doubles -> raw features x device [n][5] FP32 (as pb_mlp_features) and
 *   targets y device [n] FP32 = binary32(log(p / E)) with E = tau + D, formed
 *   in FP64.  n = 0 does nothing. */
pb_status pb_mlp_prepare(const void *cons, const void *p, void *x, void *y, int64_t n, void *stream);
/* pb_mlp_fit_norm: means and standard deviations (divisor n - 1) of the five
 * feature columns of x [n][5] and of y [n], accumulated in FP64 in a fixed
 * order, stored (rounded to binary32) as the MLP's normalisation block
 * x_mean, x_std (floored at 1e-6), y_mean, y_std; the inference operands are
 * refreshed.  n >= 2.  Asynchronous on stream. */
pb_status pb_mlp_fit_norm(pb_mlp *m, const void *x, const void *y, int64_t n, void *stream);
/* pb_mlp_standardise_target: t[i] = binary32((y[i] - y_mean) / y_std) in FP64
 * with the MLP's binary32 y_mean, y_std (device [n] FP32 in and out). */
pb_status pb_mlp_standardise_target(const pb_mlp *m, const void *y, void *t, int64_t n, void *stream);
/* pb_mlp_permutation: idx device [n] int64 = the seeded permutation of
 * [0, n) that pb_mlp_train_epoch walks for (seed, epoch): a balanced
 * four-round Feistel network on 2h bits with cycle walking into [0, n)
 * (Black & Rogaway, "Ciphers with arbitrary finite domains", 2002), h the
 * smallest value with 2^(2h) >= n (and 2h >= 2), key = mix(seed + (epoch + 1)
 * 0x9E3779B97F4A7C15), round function mix(key ^ (r + 1) 0x9E3779B97F4A7C15 ^ R)
 * masked to h bits (r = 0..3, L, R <- R, L ^ F), mix = the SplitMix64
 * finaliser (Steele, Lea & Flood, OOPSLA 2014); the value is L 2^h + R. */
pb_status pb_mlp_permutation(uint64_t seed, int64_t epoch, int64_t n, void *idx, void *stream);
/* pb_mlp_train_epoch: floor(n / batch) Adam steps (as pb_mlp_train_step) on
 * the rows x[idx[b batch + j]], t[idx[b batch + j]] (j < batch) of the
 * permutation idx of (seed, epoch), gathered inside the training kernel.
 * Step s = step0 + b + 1 uses lr = binary32(lr_max (1 + cos(pi (s - 1) /
 * total_steps)) / 2).  loss_sum (device double [1], nullable) accumulates
 * the batch losses.  Errors: batch < 1 or > n, total_steps < step0 + the
 * epoch's steps, bad Adam hyper-parameters. */
pb_status pb_mlp_train_epoch(pb_mlp *m, const void *x, const void *t, int64_t n, int32_t batch,
                             uint64_t seed, int32_t epoch, float lr_max, int64_t step0,
                             int64_t total_steps, float beta1, float beta2, float eps,
                             void *loss_sum, void *stream);

/* ---------------------------------------------------------- measurement -- */

/* on == 1: time every step kernel launch (FV step kernel; FD stage kernel)
 * of later eager calls by a HIP event pair that the kernel's own dispatch sets
 * to its start and end (the dt reduction and launch gaps are not included).
 * on == 2 (span): the same, except that the step launches of one FV call on a
 * PDE other than SRHD, which follow each other on the stream with nothing in
 * between, share one pair: the first launch sets its start, the last its end.
 * The elapsed time over the launch count is then their average period (the
 * duration plus whatever gap separates them), recorded with two events per
 * call instead of two per launch, which costs the stream a few microseconds
 * each.  Step calls with use_graph != 0 fail with PB_EINVAL while it is on;
 * on == 0 stops it and drops what was recorded; any other value is PB_EINVAL.
 * Turning it on creates the event pairs of 1,024 launches here (a call with
 * more launches than the pool holds grows it first), so that recording
 * allocates nothing in the calls being timed.  PB_EHIP if an event cannot be
 * created. */
pb_status pb_batch_profile(pb_batch *b, int32_t on);
/* Sum of the recorded pairs' elapsed times (ms) and the number of launches
 * they cover, since the last read; synchronises the batch stream and clears
 * the record. */
pb_status pb_batch_profile_read(pb_batch *b, double *total_ms, int64_t *launches);

/* Plain streaming copy of `bytes` (multiple of 32, 32-byte aligned device
 * pointers) on `stream`: the attainable-bandwidth reference for the kernels'
 * roofline (reads `bytes`, writes `bytes`). */
pb_status pb_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

/* --------------------------------------------------------------- tuning -- */

/* Launch-shape choices of the step kernels.  None of them changes what is
 * computed; the FV slab changes the order of a few additions at slab seams
 * (last-bit differences), the others change nothing in the results. */
typedef struct {
    int32_t fv_slab;          /* FV: z-planes per work-group (0 = whole patch) */
    int32_t fv_xcd_remap;     /* FV: 1 = group consecutive patches per XCD */
    int32_t fd_xcd_remap;     /* FD: 1 = each XCD takes a contiguous run of tiles
                                 (the tiles of one patch share its L2) */
    int32_t fd_wg_per_cu;     /* FD: resident work-groups per CU, 1 or 2 (0 = 2) */
    int32_t fv_dma;           /* FV 3D: 1 = the DMA-fed kernel (state planes copied
                                 HBM -> LDS three planes ahead) where the batch
                                 allows it (no SRHD, every p a multiple of 4,
                                 16-byte aligned state), 0 = the register-prefetch
                                 kernel (the default) */
    int32_t fd_ws;            /* FD: 2 = one wave per 4x4x4 tile, no
                                 work-group barrier (footprints and matrix
                                 operands DMA'd into the wave's own LDS one
                                 chunk of four unknowns ahead; results equal
                                 the other two to roundoff);
                                 1 = the wave-specialised stage kernel (one
                                 work-group of 12 waves per CU: 8 waves stage
                                 data and compute gradients while 4 run the
                                 matrix product and the update; the default),
                                 0 = the kernel in which every wave does every
                                 phase (fd_wg_per_cu applies to it); both give
                                 bitwise equal results */
    int32_t fv_persist;       /* FV 3D, batches of one p (register kernel):
                                 w in 1..8 = a grid of w work-groups per CU,
                                 each marching an equal run of the batch's K*p
                                 planes (patch after patch): with w no larger
                                 than the work-groups a CU holds at once there
                                 is no partly filled last round; fv_slab is
                                 then unused.  0 = one work-group per slab
                                 (fv_slab), the default.  Results differ from
                                 slab mode only where a slab seam changes the
                                 order of additions. */
    int32_t fv_column;        /* FV 3D (register kernel): w in 1..8 = column
                                 runs: the patches are linked along +z (k to
                                 its +z neighbour s where s's -z neighbour is
                                 k and both have the same p >= 2) into chains
                                 and cycles, each split into runs of nearly
                                 equal plane counts, about w work-groups per
                                 CU in total; a work-group marches its run
                                 across patch tops without a restart, so the
                                 plane below and above every patch top inside
                                 a run is read once.  Takes precedence over
                                 fv_persist and fv_slab; builds a small device
                                 table here (host call, PB_EHIP if that
                                 fails).  0 = off, the default.  Results
                                 differ from slab mode only where a run
                                 starts inside a patch, as at a slab seam. */
    int32_t fd_column;        /* Euler FD (plane kernel): w in 1..8 = column
                                 runs as for fv_column (links between patches
                                 of one p >= 4; every run at least one whole
                                 patch long), about w work-groups per CU;
                                 0 = one work-group per patch.  Default 2
                                 (the kernel holds two work-groups per CU).
                                 Results are bitwise those of fd_column = 0.
                                 Builds a small device table here (host call,
                                 PB_EHIP if that fails). */
} pb_tuning;

pb_status pb_batch_set_tuning(pb_batch *b, const pb_tuning *t);
pb_status pb_batch_get_tuning(const pb_batch *b, pb_tuning *out);

/* The column runs that fv_column = w (kind 0) or fd_column = w (kind 1)
 * sets up for the 3D batch `desc` (its host tables only; device pointers
 * are not used) on a device of `cus` compute units, in unit order (the
 * order the XCD remap groups).  Host-only.
 * runs: host [max_runs][4] receiving (patch, first plane, planes, 0): the
 * unit marches `planes` planes from `first plane` of `patch` on up its +z
 * chain.  *n_runs receives the number of runs even when it exceeds max_runs
 * (then PB_EINVAL and nothing is written; runs may be NULL with max_runs 0
 * to ask for the count).  PB_EINVAL also for an invalid desc, a 2D batch,
 * kind other than 0 or 1, w outside [1, 8] or cus < 1. */
pb_status pb_column_runs(const pb_batch_desc *desc, int32_t kind, int32_t w, int32_t cus, int32_t *runs,
                         int32_t max_runs, int32_t *n_runs);

/* ------------------------------------------------------------ autotuner -- */

/* Measured search over the launch shapes of one step kernel for this batch
 * (the tuning frameworks and exhaustive search that Sec. V names as the way
 * to choose kernel variants per architecture).
 *
 * kind 0 = the finite-volume step (fv_rusanov_step with the given cfl /
 * dt_fixed), kind 1 = one FD4+KO6 stage (fd_ko_step with sigma_ko; cfl /
 * dt_fixed as there; the linear system or 3D Euler).  Candidates:
 *   FV 3D: fv_column {3, 2} x fv_xcd_remap {1, 0}, then fv_persist 3 x
 *          fv_xcd_remap {1, 0} (batches of one p), then fv_slab in
 *          {p_max, p_max/2, p_max/4} (>= 2) x fv_xcd_remap {1, 0}, then the
 *          DMA-fed kernel with fv_slab in {p_max, p_max/2} x fv_xcd_remap
 *          {1, 0} where it applies;
 *          a batch of one p with p^3 <= 256 runs the small-patch kernel,
 *          which has no launch-shape choice: one candidate, the current one;
 *   FV 2D: fv_xcd_remap {1, 0};
 *   FD:    fd_ws {2, 1} x fd_xcd_remap {1, 0}, then fd_ws 0 x fd_xcd_remap {1, 0}
 *          x fd_wg_per_cu {2, 1};
 *   Euler FD: fd_column {2, 4, 0} x fd_xcd_remap {1, 0}; a batch of one p
 *          with p^3 <= 256 runs the small-patch kernel: one candidate.
 * Each candidate runs one untimed launch and then `trials` timed launches
 * (HIP events on the batch's stream), over two interleaved passes; its time
 * is the smaller of the two pass averages.  The trial launches read the
 * current state and write only the other state buffer and the workspace, so
 * the current state is unchanged; the control block (dt slots, counters) is
 * saved before and restored after.  SRHD: the con2prim pass runs once first
 * (so afterwards the warm-start guess is the pressure of the current state).
 * The fastest candidate is applied to the batch (captured graphs are
 * dropped) and cached in this process under a key of (kind, PDE, dim, N,
 * storage, halo, patch-size histogram); with use_cache = 1 a cached entry is
 * applied without timing anything (out->from_cache = 1).
 * Synchronises the stream.  Errors: PB_EINVAL for bad arguments or a kind
 * that does not match the PDE, PB_EHIP for HIP failures. */
#define PB_TUNE_MAX 16
typedef struct {
    int32_t n_candidates;
    int32_t from_cache;
    int32_t best;                    /* index into cand / cand_us */
    int32_t pad_;
    pb_tuning cand[PB_TUNE_MAX];
    double cand_us[PB_TUNE_MAX];     /* average launch duration (microseconds) */
} pb_autotune_result;

pb_status pb_autotune(pb_batch *b, int32_t kind, double cfl, double dt_fixed, double sigma_ko, int32_t trials,
                      int32_t use_cache, pb_autotune_result *out);

/* The process-wide tuning cache as a text file, one entry per line:
 * "<key> <fv_slab> <fv_xcd_remap> <fd_xcd_remap> <fd_wg_per_cu> <fv_dma> <fd_ws> <fv_persist> <fv_column>
 *  <fd_column>"
 * (the last three fields may be missing, from the end: they then load at
 * their defaults fv_persist 0, fv_column 0, fd_column 2).
 * save writes every entry (replacing the file); load adds the file's entries
 * (a later entry of the same key wins) and stores their number in *n_loaded
 * (nullable).  Host-only; PB_EINVAL on a file that cannot be opened or a
 * malformed line (entries before it stay loaded). */
pb_status pb_autotune_cache_save(const char *path);
pb_status pb_autotune_cache_load(const char *path, int32_t *n_loaded);
pb_status pb_autotune_cache_clear(void);

/* ---------------------------------------------------------- offload mode -- */

/*
 * Pure kernel offloading, as ExaHyPE ships a bundle of K cells to the
 * accelerator (paper Sec. IV): no cell data stays on the device between
 * calls.  The caller hands K separate host chunks (the AoAoS of Sec. II-B):
 * chunk k is patch k with its halo, the (p+2h)^3 points of the halo box in
 * per-point order (the N unknowns of one point contiguous, points x fastest,
 * then y, then z), and receives K host chunks of the p^3 updated interior
 * points in the same per-point order.  The gather prologue and scatter
 * epilogue of Sec. III-C, Eq. (4) are the packing of the chunks into pinned
 * staging buffers and back; the host-device mapping of Sec. III-D is a copy
 * pipeline: batches of patches go through two slots (pinned staging, device
 * buffers, a stream each), so the packing of one batch, the copies and the
 * kernel of another overlap.  Edges and corners of the halo box are never
 * read (the Rusanov stencil is axis-aligned); only the innermost halo layer
 * is read.
 */
typedef struct pb_offload pb_offload;

typedef struct {
    int32_t dim;              /* 3 */
    int32_t p;                /* cells per direction, 1..16 */
    int32_t halo;             /* 1 <= h <= 8: width of the halo in each chunk */
    int32_t pde;              /* ADVECTION_F, ADVECTION_B or EULER */
    const double *pde_params; /* host, copied at create */
    int64_t n_pde_params;
    int32_t n_unknowns;       /* N (as in pb_batch_desc) */
    int32_t batch_patches;    /* patches per pipeline batch, 0 = the library's
                                 choice (about 32 MiB of input per batch) */
} pb_offload_desc;

/* Allocates the two pipeline slots (pinned host staging, device buffers,
 * streams).  Errors: PB_EINVAL for a bad description, PB_EUNSUPPORTED for
 * another PDE or dim, PB_ENOMEM / PB_EHIP for failed allocations. */
pb_status pb_offload_create(const pb_offload_desc *desc, pb_offload **out);
pb_status pb_offload_destroy(pb_offload *o);

typedef struct {
    double total_ms;          /* wall clock of the whole call */
    double pack_ms;           /* host: chunks -> pinned staging (summed over batches) */
    double h2d_ms;            /* device copy engine time, host -> device (summed) */
    double compute_ms;        /* kernel time (summed) */
    double d2h_ms;            /* device -> host copies (summed) */
    double unpack_ms;         /* host: pinned staging -> output chunks (summed) */
    int64_t batches;
} pb_offload_timing;

/*
 * One Rusanov finite-volume step (as fv_rusanov_step) of K patches in
 * offload mode, with the step size dt given (the caller's time stepping):
 * in_chunks[k] (host, (p+2h)^3 * N doubles) -> out_chunks[k] (host,
 * p^3 * N doubles); dx[k] (host) is the cell width of patch k.  Blocking:
 * returns when every output chunk is written.  timing is nullable.
 * Errors (before any copy): PB_EINVAL for K < 0, NULL arrays or chunks,
 * dt or dx not finite and > 0.  K = 0 returns at once.  Calls on one
 * pb_offload object must not overlap (its staging buffers and streams are
 * reused); separate objects are independent.
 */
pb_status pb_offload_fv_step(pb_offload *o, int32_t K, const double *const *in_chunks, double *const *out_chunks,
                             const double *dx, double dt, pb_offload_timing *timing);

const char *pb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PATCHHIP_H */

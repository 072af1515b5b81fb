/*
 * lsfft — Green-function-preconditioned (Lippmann-Schwinger) fixed-point solver
 * for periodic linear-elastic unit cells on one AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes only; no C++ or framework types cross it.
 *
 * The method (Khorrami, Mianroodi, Shanthraj, Svendsen, "Development and
 * comparison of spectral algorithms for numerical modeling of the
 * quasi-static mechanical behavior of inhomogeneous materials"):
 *   given the grid n1 x n2 x n3, per-voxel isotropic moduli lambda(x), mu(x),
 *   a reference medium C_H = (lambda0, mu0) and a macroscopic strain Ebar,
 *   iterate (strain form of the 3D TD algorithm of Sec. 5.2, identical iterates
 *   to its displacement form):
 *       sigma^k   = C(x) : eps^k                           (Hooke, Sec. 5.1)
 *       r_k       = |sigma_hat q^b| / |sigma_hat(0)|       (stopping test)
 *       eps^{k+1} = eps^k + IDFT( Gamma_H(q) DFT(sigma^k) ) (Green step, eq. (34), (48))
 *   with eps^0 = Ebar.  The scheme selects the wavevector q:
 *       BASIC  plain Fourier wavevector (the "F" choice),
 *       FB     forward-difference gradient with the conjugate divergence,
 *       AFB    averaged forward / half-central pair (AFD, AhC) of Sec. 5.3,
 *              equal to Willot's rotated scheme,
 *       DGO    the discrete Green operator of Sec. 5.4 (PCD only), iterated in
 *              polarisation form eps^{k+1} = Ebar + IDFT(Gamma^c DFT((C - C_H) eps^k)).
 *
 * Field layout (every real field, host or device): components major, then
 * x3, x2, x1 with x1 fastest:  index = c*N + (i3*n2 + i2)*n1 + i1,
 * N = n1*n2*n3.  Tensor fields have 6 components in Voigt order
 * (11, 22, 33, 23, 13, 12) holding TENSOR components (E_12, not 2 E_12).
 *
 * Half-spectrum layout used by the operator entry points: components major,
 * then k3, k2, k1 with k1 fastest, k1 in [0, n1/2], k2 in [0, n2), k3 in
 * [0, n3) (standard FFT order; index j is the wavenumber j for j < n/2 and
 * j - n otherwise, so the Nyquist index n/2 is the paper's kappa = -n/2):
 *   index = c*(n3*n2*(n1/2+1)) + (k3*n2 + k2)*(n1/2+1) + k1,
 * complex values as interleaved (re, im) pairs of the solver's precision.
 * Transforms are unnormalised forward DFTs, exp(-i k.x).
 *
 * Error behaviour: every entry point returns an lsfft_status.  Negative
 * values mean nothing was computed and no output was written; positive
 * values mean outputs were written but the iteration did not converge
 * (LSFFT_ENOTCONV) or diverged (LSFFT_EDIVERGED).  A solver handle is not
 * thread-safe; distinct handles may be used from distinct threads.
 */
#ifndef LSFFT_H
#define LSFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lsfft_solver_s *lsfft_solver;

/* Discretisation: trapezoidal (nodes) or piecewise-constant (cell centres),
 * Sec. 3.1 / 3.2.  For BASIC, FB and AFB both give identical iterates on
 * per-voxel data (the PCD algorithm differs only in where C is sampled); the
 * flag is recorded and gates DGO, which is defined for PCD only. */
typedef enum { LSFFT_TD = 0, LSFFT_PCD = 1 } lsfft_disc;

/* BASIC, FB, AFB, DGO: see above.  CD: central-difference gradient
 * q^CD_r = i sin(2 pi kappa_r/n_r)/h_r (eq. (14)) with the conjugate divergence;
 * ACD: the averaged central difference of Sec. 5.3 (eq. (43)),
 * q_r = q^CD_r cos(2 pi kappa_s/n_s) cos(2 pi kappa_t/n_t), conjugate pair.
 * CD and ACD use the strain form (form 2 is EINVAL).  Where a wavevector
 * vanishes exactly (CD: every index 0 or Nyquist; ACD also wherever two of the
 * cosines vanish, e.g. two indices at n/4) the Green function is 0 (Sec. 3.1
 * after the TD algorithm). */
typedef enum { LSFFT_BASIC = 0, LSFFT_FB = 1, LSFFT_AFB = 2, LSFFT_DGO = 3, LSFFT_CD = 4, LSFFT_ACD = 5 } lsfft_scheme;

/* F64: all arithmetic in FP64.  F32: strain, stress, FFTs and the Green step
 * in FP32; the displacement of the displacement form, the residual, mean
 * stress and convergence reductions in FP64.  The F32 equilibrium residual
 * has a floor that depends on the form and the size: in the strain form
 * roughly chi x 1e-8 at stiffness contrast chi (about 2e-5 at chi = 1e3); in
 * the displacement form about (n/2)^2 x 2^-24 (about 1e-3 at 256^3), from
 * FP32 rounding of the displacement updates, which the discrete divergence
 * of the stiffness amplifies at high frequencies.  A tolerance below the
 * floor is not reached (LSFFT_ENOTCONV after maxit), although the fields
 * reach FP64 accuracy well before; f64_until with refine (see lsfft_config)
 * certifies such tolerances in F32 from FP64 evaluations of the residual. */
typedef enum { LSFFT_F64 = 0, LSFFT_F32 = 1 } lsfft_prec;

typedef enum {
  LSFFT_OK = 0,          /* converged: r <= tol                              */
  LSFFT_ENOTCONV = 1,    /* maxit reached; outputs hold the last iterate      */
  LSFFT_EDIVERGED = 2,   /* residual non-finite, or the unnormalised equilibrium
                            norm sqrt(sum |sigma_hat q^b|^2) > 1e6 x its first
                            value (DGO: the residual > 1e6 x the first one) */
  LSFFT_EINVAL = -1,     /* invalid argument; nothing computed                */
  LSFFT_ENOMEM = -2,     /* device allocation failed                          */
  LSFFT_EDEVICE = -3     /* HIP runtime error                                 */
} lsfft_status;

typedef struct {
  int32_t n[3];            /* n1 (fastest), n2, n3: each even 2^a*3^b, 4..512
                              (odd lengths, e.g. 9 or 27, are EINVAL)       */
  double h[3];             /* grid spacing per axis; 0 means 1.0               */
  const double *lambda;    /* N Lame lambda values, HOST memory, field layout  */
  const double *mu;        /* N shear moduli mu, HOST memory, field layout     */
  double lambda0, mu0;     /* reference medium C_H (isotropic)                 */
  int32_t disc;            /* lsfft_disc                                       */
  int32_t scheme;          /* lsfft_scheme                                     */
  int32_t prec;            /* lsfft_prec                                       */
  int32_t dgo_images;      /* DGO only: image window M >= 0 (nu in [-M, M], and
                              [-M, M+1] at a Nyquist index)                     */
  int32_t dgo_weight_power;/* DGO only: 1 = the single sinc weight as printed,
                              2 = squared sinc weight                          */
  void *stream;            /* hipStream_t for all work; NULL = default stream   */
  int32_t form;            /* FB and AFB only: 0 = automatic, 1 = strain form
                              (six transformed stress components, Green step
                              -Gamma_0), 2 = displacement form (the paper's
                              u-iteration of Sec. 5.2 with the gradient and
                              divergence applied as real-space stencils, three
                              transformed components; identical iterates).
                              Automatic picks 2 when its workgroup fits in LDS
                              (every n1 in F32, n1 <= 384 in F64).           */
  int32_t f64_warmup;      /* F32 displacement form with n1 <= 384 only (else
                              ignored): run the first f64_warmup iterations of
                              every solve in FP64 on the same displacement
                              (identical iterates up to rounding), then
                              continue in F32.  FP32 rounding of the large
                              early updates otherwise leaves an error of order
                              1e-6 (relative, at contrast 1e3) that only the
                              slowest modes of the iteration remove.  0 = off;
                              < 0 is EINVAL.  Costs the memory of an F64
                              solver.                                          */
  const double *eigenstrain; /* optional eigenstrain E_* (Sec. 7): 6N values,
                              HOST memory, [6][n3][n2][n1] Voigt tensor
                              components (eps_23, not 2 eps_23), copied at
                              create; NULL = none.  The law becomes
                              T = C [E - E_*]: the iteration starts from
                              T^(0) = C [Ebar - E_*], eps outputs are the
                              total strain E and sig outputs C [E - E_*].
                              In a batch each system has its own (NULL
                              systems have none).  EINVAL if not finite.    */
  int32_t refine;          /* F32 displacement form: FP64 iterative refinement
                              with cycles of `refine` iterations; 0 = off,
                              < 0 is EINVAL, > 0 with an F32 strain-form
                              solver is EINVAL, ignored in F64.  The solve
                              keeps u = u_b + delta: at the start of each
                              cycle delta is folded into u_b and the residual
                              force of u_b is evaluated in FP64; the F32
                              sweeps then iterate on delta with that force as
                              a fixed load.  The fixed point keeps no memory
                              beyond its iterate, so the iterates are the same
                              as without refinement up to rounding, but the
                              FP32 rounding is relative to the residual of the
                              cycle: tolerances below the F32 residual floor
                              (see lsfft_prec) are reached.  Every stop for
                              r <= tol (or maxit) is confirmed at an FP64
                              evaluation: a stop found inside a cycle is
                              re-tested on the FP64 force of the folded u, and
                              the reported residual and mean stress are that
                              evaluation's.  Rounding of the first, large
                              updates still lands in the slowest modes of the
                              iteration (contraction about (chi-1)/(chi+1) at
                              stiffness contrast chi), which refinement sees
                              but does not remove faster than the iteration:
                              at contrast >= 1e2 a refined solve takes more
                              iterations than F64 unless f64_warmup covers
                              those updates.  Costs 11N FP64 + 3N T per
                              system (+ 6N FP64 with an eigenstrain) and one
                              FP64 residual evaluation per cycle.            */
  double f64_until;        /* F32 displacement form, where f64_warmup applies:
                              run the iterations of every solve in FP64 (after
                              the f64_warmup ones, if any) until the system's
                              residual is at most f64_until, then continue in
                              F32 from that iterate; 0 = off, < 0 or not finite
                              is EINVAL.  With refine > 0 this is the F32 route
                              to a certified tolerance at high contrast: the
                              FP32 rounding of each refinement cycle is then
                              relative to a residual already small, and every
                              final status comes from an FP64 evaluation.
                              Measured (AFB, 256^3, contrast 1e3, tol 1e-6):
                              f64_until = 3e-4 with refine = 8 stops at r <=
                              tol in the FP64 iteration count, about 12 %
                              faster than F64 (tol 1e-8, f64_until 3e-6: 8 %);
                              a switch at a residual much above 300 x tol
                              leaves FP32 rounding in the slowest modes and
                              costs many more iterations at tight tol.       */
} lsfft_config;

/* Create a solver (Sec. 5.2 "given: n, C(x), Ebar, C_H, G").  Copies lambda
 * and mu to the device (the caller may free them on return), builds the
 * per-axis wavevector tables and, for DGO, the discrete Green operator
 * table (Sec. 5.4).  EINVAL: NULL pointers, unsupported n, h < 0, any
 * mu <= 0 or 3 lambda + 2 mu <= 0 (not positive definite), the same for
 * C_H, non-finite moduli, DGO with TD, dgo_images < 0 or > 64, a weight
 * power other than 1 or 2, unknown enum values, form 2 where it does not fit.  On success *out owns
 * device memory until lsfft_destroy. */
lsfft_status lsfft_create(const lsfft_config *cfg, lsfft_solver *out);

/* Create one solver for `count` systems on the same grid, solved together:
 * every kernel launch covers the whole batch (the system index is the second
 * grid dimension) and each system stops on its own test.  Typical uses: the
 * six load cases of an effective stiffness (cfgs[m] equal but for nothing, the
 * loads differ at solve time), or several cells of equal size (cfgs[m]
 * differ in lambda, mu, lambda0, mu0).  All cfgs must agree on n, h, disc,
 * scheme, prec, form, dgo_images, dgo_weight_power, stream and f64_warmup
 * (EINVAL otherwise); for the DGO they must also share lambda0 and mu0 (one
 * table).  Memory: count times that of one system.  1 <= count <= 65535.
 * lsfft_create(cfg, out) is lsfft_create_batch(cfg, 1, out).  The operator
 * entry points and lsfft_residual_history act on system 0. */
lsfft_status lsfft_create_batch(const lsfft_config *cfgs, int32_t count, lsfft_solver *out);

/* Solve for macroscopic strain Ebar[6] (Voigt tensor components): the
 * fixed point of Sec. 5.2 (TD algorithm, displacement form; the PCD
 * algorithm of Sec. 5.4 has the same iterates for BASIC, FB and AFB) or the
 * DGO algorithm of Sec. 5.4 (polarisation form), from u = 0 (eps = Ebar).
 * Stops at the first k with r_k <= tol (returns LSFFT_OK), at k = maxit
 * (LSFFT_ENOTCONV), or on divergence (LSFFT_EDIVERGED, see lsfft_status).  r_k is the relative equilibrium norm
 * sqrt(sum_xi |sigma_hat(xi) q^b(xi)|^2) / |sigma_hat(0)|_F evaluated before
 * the k-th update (BASIC, FB, AFB), or |eps^k - eps^{k-1}| / (sqrt(N)|Ebar|_F)
 * (DGO; with an eigenstrain and Ebar = 0 the RMS over the voxels of
 * |E_*|_F replaces |Ebar|_F).  With an eigenstrain, r_k is 0 when the whole
 * stress field vanishes (free expansion), and undefined when only its mean
 * does (reported as +inf: the solve returns LSFFT_EDIVERGED).  Outputs: eps and sig (6N doubles, HOST memory, field layout; either
 * may be NULL), sig_mean[6] = <sigma> (may be NULL), *iters = k (number of
 * updates applied), *residual = r_k (either may be NULL).  tol >= 0,
 * maxit >= 0.  tol = 0 runs exactly maxit iterations. */
lsfft_status lsfft_solve(lsfft_solver s, const double Ebar[6], double tol, int32_t maxit,
                         double *eps, double *sig, double sig_mean[6], int32_t *iters,
                         double *residual);

/* Same as lsfft_solve (Sec. 5.2 / 5.4, same stopping rule) with DEVICE output
 * pointers of the solver's precision (float for F32, double for F64), 6N
 * elements each, field layout, caller-owned; either may be NULL.  No host
 * copies of fields are made; sig_mean, iters and residual are HOST.  Errors
 * as lsfft_solve (EINVAL on a batch handle with count > 1). */
lsfft_status lsfft_solve_device(lsfft_solver s, const double Ebar[6], double tol, int32_t maxit,
                                void *eps_dev, void *sig_dev, double sig_mean[6],
                                int32_t *iters, double *residual);

/* Solve every system of a batch handle: Ebar[count][6] (HOST), DEVICE outputs
 * eps_dev and sig_dev of [count][6][N] values of the solver's precision (either
 * may be NULL), HOST outputs sig_mean[count][6], iters[count],
 * residual[count], status[count] (per-system lsfft_status; each may be NULL).
 * Same stopping test as lsfft_solve, per system.  Returns the largest
 * per-system status (OK < ENOTCONV < EDIVERGED) or a negative error.
 * lsfft_solve and lsfft_solve_device return EINVAL on handles with count > 1. */
lsfft_status lsfft_solve_batch(lsfft_solver s, const double *Ebar, double tol, int32_t maxit,
                               void *eps_dev, void *sig_dev, double *sig_mean, int32_t *iters,
                               double *residual, int32_t *status);

/* Solve the systems of `count` solvers (1..64 distinct handles, e.g. one
 * batch handle per cell size of a set of microstructures, each holding its
 * cells' load cases) together (Sec. 5.2 for every system; the batched
 * effective-stiffness setting of six unit loads per cell).  Each solver
 * opens its solve as lsfft_solve_batch would, then the captured chunk of
 * iterations of every solver becomes one independent child of a single
 * graph, launched once per chunk for all sizes at once until every system
 * has stopped on its own device-side test (a finished system's kernels
 * return at once).  Solvers with an FP64 warm start (f64_warmup,
 * f64_until) first run their FP64 phase the same way, as one group.
 * Results equal those of lsfft_solve_batch on each handle (the same
 * kernels, in the same order per solver).  Ebar: [sum of batch sizes][6]
 * HOST, in handle order; maxit_each: NULL (every solver gets maxit) or
 * `count` iteration limits, one per solver (maxit is then unused but must be
 * valid); eps_dev: NULL or `count` pointers, each NULL or a
 * DEVICE array [B][6][N] of that solver's precision; sig_mean [sum B][6],
 * iters, residual, status [sum B] HOST, each may be NULL.  Synchronous.
 * Returns the largest per-system status.  EINVAL: NULL handles or Ebar,
 * count outside 1..64, a NULL or repeated handle, a handle with refine > 0,
 * tol < 0, a negative iteration limit, non-finite Ebar.  Per-kernel timing is
 * not recorded during a group solve. */
lsfft_status lsfft_solve_group(const lsfft_solver *handles, int32_t count, const double *Ebar, double tol,
                               int32_t maxit, const int32_t *maxit_each, void *const *eps_dev, double *sig_mean,
                               int32_t *iters, double *residual, int32_t *status);

/* Number of systems of a handle (0 for NULL). */
int32_t lsfft_batch_size(lsfft_solver s);

/* Launch schedule of the passes of one iteration.  It decides how the work
 * is cut into workgroups and in which order they run, not the formulas:
 * results under two schedules agree to rounding (the reductions of mean
 * stress and residual add their per-workgroup partial sums in another
 * order).  Each handle has its own schedule; the FP64 warm-start iterations
 * (f64_warmup) keep their default one. */
typedef struct {
  int32_t stencil_planes; /* z-planes per stencil workgroup in the displacement
                             form: an even divisor of n3 (powers of two
                             from 2 to 128 are offered by lsfft_autotune;
                             the default is the largest of 4 .. 128 that
                             keeps 512 workgroups over the batch); 0 in the
                             strain form                                     */
  int32_t y_cols;         /* pencils (consecutive x columns) per y-pass
                             workgroup: the default or its alternative, one
                             of two values fixed by n2 and the precision    */
  int32_t z_cols;         /* the same for the z pass (the pass holding the
                             Green step)                                    */
  int32_t xcd_order;      /* bit 0 stencil, bit 1 y pass, bit 2 z pass: deal
                             consecutive tiles to the same XCD (shared L2)
                             instead of round-robin over the 8 XCDs         */
} lsfft_schedule;

/* The handle's current schedule.  EINVAL on NULL arguments. */
lsfft_status lsfft_get_schedule(lsfft_solver s, lsfft_schedule *out);

/* Replace the handle's schedule (e.g. one found by lsfft_autotune on an
 * earlier run of the same grid and precision).  EINVAL, with the schedule
 * unchanged, when a field is not one this grid offers. */
lsfft_status lsfft_set_schedule(lsfft_solver s, const lsfft_schedule *sch);

/* Schedule tuner.  Times whole iterations of every system of the handle
 * (its own moduli, a unit axial macroscopic strain, the stopping test off,
 * `iterations` rounded up to whole captured chunks of 8, best of 3 runs
 * after one untimed run) and searches the knobs one at a time: stencil
 * planes, y and z column tiles, then each XCD-order bit, keeping a change
 * that is faster by more than 1 %.  Leaves the best schedule in force and
 * returns it in *best, with the milliseconds per iteration of the schedule
 * in force on entry (*start_ms) and of the best one (*best_ms); any output
 * may be NULL.  Overwrites the handle's fields and residual history (a
 * later solve starts afresh).  Takes about 40 x iterations iteration times.
 * EINVAL: NULL handle, iterations < 1 or > 4096. */
lsfft_status lsfft_autotune(lsfft_solver s, int32_t iterations, lsfft_schedule *best, double *start_ms,
                            double *best_ms);

/* Residual history r_0..r_iters of the last solve, copied to HOST out[0..cap);
 * *count receives iters + 1.  EINVAL if no solve has run. */
lsfft_status lsfft_residual_history(lsfft_solver s, double *out, int32_t cap, int32_t *count);

/* Operator: sig_hat = DFT(C : eps) (with an eigenstrain: DFT(C : [eps -
 * E_*])) for a DEVICE strain field eps_dev (6N,
 * solver precision, field layout) into DEVICE sig_hat_dev (half-spectrum
 * layout, 6*n3*n2*(n1/2+1) complex).  For DGO the polarisation
 * (C - C_H) : eps is transformed instead.  Sec. 5.2, the steps
 * "T = C E; T_check = F^- T". */
lsfft_status lsfft_stress_spectrum(lsfft_solver s, const void *eps_dev, void *sig_hat_dev);

/* Operator: the Green step on a DEVICE half spectrum (layout above):
 * out = -Gamma_0(q) in (BASIC, FB, AFB: the strain increment of eq. (34),
 * zero at xi = 0 and at singular frequencies) or out = Gamma^c in (DGO, the
 * paper's sign), unnormalised.  in must be the transform of a real field.
 * *res_sq (may be NULL) receives sum over the FULL spectrum of
 * |in(xi) q^b(xi)|^2 (BASIC, FB, AFB; 0 for DGO).  in and out may alias. */
lsfft_status lsfft_green_apply(lsfft_solver s, const void *in_dev, void *out_dev, double *res_sq);

/* Adjoint sensitivity of an effective-stiffness objective.  For the converged
 * strains eps_a, eps_b of two solves with macroscopic strains A and B (DEVICE
 * fields of the solver's precision, 6N, field layout, e.g. from
 * lsfft_solve_device), J = <eps_a : C : eps_b> = A : C_eff : B.  BASIC, FB
 * and AFB are self-adjoint (their fixed point minimises a quadratic energy
 * over compatible fluctuations, Sec. 5.2), so the adjoint field of A is the
 * primal solution under A and the derivative of J is the partial derivative
 * at the solution:
 *   dj_dlambda[x] = tr eps_a tr eps_b / N,  dj_dmu[x] = 2 eps_a : eps_b / N,
 *   dj_dyoung[x]  = (lambda dJ/dlambda + mu dJ/dmu) / E   (fixed Poisson ratio,
 *                   E = mu (3 lambda + 2 mu) / (lambda + mu) of voxel x).
 * Outputs: DEVICE arrays of N values of the solver's precision; any may be
 * NULL.  Computed in FP64 with the moduli of system 0 of a batch handle.
 * J is a property of C_eff and needs no eigenstrain: on a handle with one,
 * pass strains of solves whose eigenstrain is zero (another handle).
 * The DGO (Sec. 5.4) is self-adjoint as well: its Green map is a real
 * symmetric operator, even in the frequency, that annihilates uniform
 * fields, so the same formula holds with the DGO's own converged strains.
 * EINVAL on NULL handle or strain fields. */
lsfft_status lsfft_stiffness_gradient(lsfft_solver s, const void *eps_a_dev, const void *eps_b_dev,
                                      void *dj_dlambda_dev, void *dj_dmu_dev, void *dj_dyoung_dev);

/* Per-kernel event timing for benchmarking.  lsfft_set_timing(s, id) makes
 * every later solve record a pair of HIP events with each launch of kernel `id`
 * (the launch records them itself; the strain form's two-kernel reduction
 * records them around its launches)
 * (0 = x-pass, 1 = forward y-pass, 2 = z-pass + Green, 3 = inverse y-pass,
 * 4 = displacement update, 5 = reduction; -1 = off).
 * lsfft_get_timing returns the mean duration in ms and the launch count
 * of the last timed solve.  In the displacement form id 0 is the stencil
 * kernel and id 4 the displacement update. */
lsfft_status lsfft_set_timing(lsfft_solver s, int32_t kernel_id);
lsfft_status lsfft_get_timing(lsfft_solver s, double *mean_ms, int32_t *launches);
const char *lsfft_kernel_name(int32_t kernel_id);

/* The kernel instantiations one iteration of solver `s` launches, in launch
 * order, written as a NUL-terminated string of space-separated names with
 * their template arguments (e.g. "k_stencil_reg<float,256,4,AFB,2>
 * k_ypass<float,256,8,32> ...": element type, transform length, points per
 * thread, then the kernel's tile or scheme arguments).  It reflects the
 * solver's lengths, form, scheme, precision and current launch schedule, so a
 * caller can tell which compiled kernels a result came from.  `buf` is
 * caller-owned host memory of `cap` bytes.  EINVAL: NULL s or buf, or cap too
 * small for the string (nothing is written then).  Launches nothing. */
lsfft_status lsfft_describe(lsfft_solver s, char *buf, int32_t cap);

/* Release all device memory and streams of the solver created by
 * lsfft_create or lsfft_create_batch (the data of the problem statement of
 * Sec. 5.2: moduli, tables, the DGO table of Sec. 5.4, iterate buffers);
 * the handle is invalid afterwards.  Waits for the solver's work to finish.
 * lsfft_destroy(NULL) is a no-op and returns LSFFT_OK. */
lsfft_status lsfft_destroy(lsfft_solver s);

/* ---------------------------------------------------------------- 1D
 * The 1D algorithms of Sec. 3 for many independent periodic bars of one
 * length, solved by one launch (a workgroup per bar iterates to its own
 * stopping test):
 *   GFP (Sec. 3.1 on nodal samples, disc TD; Sec. 3.2 on cell-centred
 *   samples, disc PCD): u^ += G T^ q^b, G = -1 / (C_H q^a q^b), with the
 *   pair (q^a, q^b) of `scheme`; stops on r = |T^ q^b| / |T^(0)| <= tol or at
 *   k = maxit (same reading as lsfft_solve).
 *   DGO (Sec. 3.3, PCD only, polarisation form): E <- Ebar + F^+ Gamma^c
 *   F^- (C - C_H) E with Gamma^c = -c_p / C_H, c_p the image sum of sinc^p
 *   (window as for the 3D DGO); stops on |E' - E| / (sqrt(n) |Ebar|) <= tol or
 *   after maxit updates. */
typedef enum {
  LSFFT_1D_F = 0,     /* Fourier symbol i k, with its conjugate             */
  LSFFT_1D_FD = 1,    /* forward difference, with its conjugate (-BD)       */
  LSFFT_1D_CD = 2,    /* central difference, with its conjugate             */
  LSFFT_1D_FD_HC = 3, /* forward difference with the half-central divergence
                         (the non-conjugate pair of Sec. 3.1)               */
  LSFFT_1D_DGO = 4    /* discrete Green operator                            */
} lsfft_scheme_1d;

typedef struct {
  int32_t n;                /* samples per bar: even 2^a*3^b, 4..512         */
  double h;                 /* spacing; 0 means 1.0                          */
  int32_t scheme;           /* lsfft_scheme_1d                               */
  int32_t disc;             /* lsfft_disc (DGO: PCD)                          */
  int32_t prec;             /* lsfft_prec                                     */
  int32_t dgo_images;       /* DGO: image window M, 0..64                     */
  int32_t dgo_weight_power; /* DGO: 1 or 2                                    */
  void *stream;             /* hipStream_t; NULL = default stream             */
} lsfft_config_1d;

/* Solve `count` bars (1..65535): C[count][n] stiffness samples, C_H[count],
 * Ebar[count] (HOST).  Outputs (HOST, each may be NULL): E and T [count][n]
 * (strain Ebar + E~ and stress), iters, residual, status [count].  Returns
 * the largest per-bar status (OK or ENOTCONV).  Synchronous.  EINVAL: NULL
 * inputs, unsupported n, h < 0, C <= 0 or C_H <= 0 or non-finite, unknown
 * enums, DGO with TD or with Ebar = 0, tol < 0, maxit < 0 or > 1e7. */
lsfft_status lsfft_solve_1d(const lsfft_config_1d *cfg, int32_t count, const double *C, const double *C_H,
                            const double *Ebar, double tol, int32_t maxit, double *E, double *T, int32_t *iters,
                            double *residual, int32_t *status);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): lsfft_solve_1d with every
 * array in DEVICE memory and no allocation of any kind.  Same algorithms,
 * configuration and results as lsfft_solve_1d (C, C_H, Ebar as FP64; E and T
 * written as FP64 [count][n]; iters, residual, status [count]; E_dev, T_dev,
 * iters_dev and residual_dev may be NULL, status_dev may not).  Asynchronous
 * on cfg->stream, which must belong to the current device: returns LSFFT_OK
 * once the work is enqueued; each bar's outcome is in status_dev (OK,
 * ENOTCONV, or LSFFT_EINVAL for a bar whose data the kernel rejects: C or C_H
 * not positive and finite, Ebar not finite, Ebar = 0 for the DGO).  The
 * per-frequency tables live in a fixed device array of 40 KB (n <= 512),
 * one per GPU, held until the process ends; the first call on a device looks
 * up its address.  Calls that overlap on one GPU share that array and race:
 * serialise them (one stream, or events).  EINVAL (nothing enqueued): NULL
 * cfg, C_dev, CH_dev, Ebar_dev or status_dev, count outside 1..65535, n above
 * the scratch limit of 512 (reported on stderr) or otherwise unsupported, and
 * the configuration errors of lsfft_solve_1d.  EDEVICE: a launch failed. */
lsfft_status lsfft_solve_1d_noalloc(const lsfft_config_1d *cfg, int32_t count, const double *C_dev,
                                    const double *CH_dev, const double *Ebar_dev, double tol, int32_t maxit,
                                    double *E_dev, double *T_dev, int32_t *iters_dev, double *residual_dev,
                                    int32_t *status_dev);

/* Static string for a status code. */
const char *lsfft_status_string(lsfft_status st);

/* Library version string. */
const char *lsfft_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LSFFT_H */

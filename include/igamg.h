/*
 * igamg.h -- C ABI of the MI355X (gfx950) solver for B-spline isogeometric
 * Poisson problems by geometric multigrid accelerated with restarted
 * polynomial vector extrapolation (RRE / MPE).
 *
 * Method: arXiv 2412.20205.  The linear system is the SPD stiffness system
 * A u = b of Section 2, eq. (2); one V-cycle (Algorithm 2 with mu = 1) is the
 * fixed-point map s_{k+1} = G(s_k) of eq. (7); RRE and MPE are Algorithms 3 and 4
 * (QR of the first differences of the iterates); the restarted driver is
 * Algorithm 5.
 *
 * Conventions shared by every call
 *  - Unknowns are the interior B-spline coefficients (homogeneous Dirichlet
 *    functions removed), n = N_el + p - 2 per direction, ordered
 *    I = i + n j (+ n^2 k), x index fastest.
 *  - Vectors passed in (x_dev, b_dev, ...) are caller-owned, contiguous FP64
 *    device buffers on the context's device, with the number of entries that
 *    igamg_ndof / igamg_level_ndof report.  The context owns every other
 *    device buffer (operators, transfer tables, level vectors, iterates).
 *  - All device work is enqueued on options.stream (a hipStream_t; NULL makes
 *    the context create its own blocking stream).  Calls that return host
 *    values synchronise that stream before returning.
 *  - Every call returns an igamg_status.  Argument errors are reported before
 *    any work is enqueued.  On an error x_dev keeps the last accepted iterate.
 *    igamg_last_error() gives a text for the last failing call on this thread.
 *  - A context must not be used by two host threads at the same time.
 */
#ifndef IGAMG_H
#define IGAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct igamg_ctx igamg_ctx;

typedef enum {
    IGAMG_OK = 0,
    IGAMG_EINVAL = -1,      /* bad argument                                     */
    IGAMG_ENOMEM = -2,      /* device or host allocation failed                 */
    IGAMG_EHIP = -3,        /* HIP runtime error (text in igamg_last_error)     */
    IGAMG_ENOTSPD = -4,     /* coarsest-level Cholesky factorisation failed     */
    IGAMG_EBREAKDOWN = -5,  /* extrapolation coefficients undefined (sum d = 0) */
    IGAMG_ENOCONV = -6,     /* max_restarts reached before the tolerance        */
    IGAMG_ENONFINITE = -7   /* NaN or Inf met in the data or the iteration      */
} igamg_status;

/* Geometry of Sections 4.2 and 4.3: the unit square and cube use Kronecker
 * operators built from 1D stiffness and mass matrices (for the Poisson
 * operator); the quarter annulus of radii r_in < r_out is the degree-2 B-spline
 * surface F(xi, eta) = (r_in + (r_out - r_in) xi)(1 - eta^2, 2 eta - eta^2)
 * (radii 1 and 2 by default) and stores (2p+1)^2 stencil coefficients per
 * unknown; QUARTER_ANNULUS_EXACT is its rational (NURBS) counterpart, weights
 * (1, 1/sqrt 2, 1) in eta, whose arcs are exact circles. */
typedef enum {
    IGAMG_UNIT_SQUARE = 0,
    IGAMG_QUARTER_ANNULUS = 1,
    IGAMG_UNIT_CUBE = 2,
    IGAMG_QUARTER_ANNULUS_EXACT = 3
} igamg_geom_kind;

typedef struct {
    int kind;      /* igamg_geom_kind                                        */
    int n_el;      /* elements per direction on the finest level             */
    double r_in;   /* annulus radii (both 0: 1 and 2); ignored otherwise     */
    double r_out;
} igamg_geometry;

/* Operator (Section 4.3).  POISSON: -Laplace.  ELLIPTIC_1 and ELLIPTIC_2:
 * -div(A grad u) + B . grad u + c u with
 *   A = [[(2 + cos x)(1 + y), cos(x+y) sin(x+y)], [cos(x+y) sin(x+y), (2 + sin y)(1 + x)]],
 *   ELLIPTIC_1 (the unit-square problem): B = (11 + sin x + y sin x - 2 cos^2(x+y),
 *              -9 - cos y - x cos y - 2 cos^2(x+y)), c = 1;
 *   ELLIPTIC_2 (the quarter-annulus problem): B = (-5y, 5x), c = xy;
 *   ADVECTION_DIFFUSION: -0.1 Laplace u + (1, 1) . grad u (A = 0.1 I, c = 0);
 * row I of the matrix is a(phi_J, phi_I), a(u, v) = int A grad u.grad v +
 * (B.grad u) v + c u v: nonsymmetric.  2D only; these operators are assembled
 * as stored stencils on either geometry. */
typedef enum {
    IGAMG_PDE_POISSON = 0,
    IGAMG_PDE_ELLIPTIC_1 = 1,
    IGAMG_PDE_ELLIPTIC_2 = 2,
    IGAMG_PDE_ADVECTION_DIFFUSION = 3
} igamg_pde;

/* Smoothers of Algorithm 2.  MCGS: multicolour Gauss-Seidel with (p+1)^d
 * colours c(I) = sum_d (i_d mod (p+1)) (p+1)^d swept in increasing order;
 * LEXGS: lexicographic Gauss-Seidel (x fastest, forward; 2D only, one
 * workgroup per sweep, for small grids); JACOBI: x += omega D^{-1} (b - A x).
 * The learned step is switched on separately (igamg_set_learned) and works
 * with MCGS; LEARNED is reserved. */
typedef enum {
    IGAMG_SMOOTH_MCGS = 0,
    IGAMG_SMOOTH_LEXGS = 1,
    IGAMG_SMOOTH_JACOBI = 2,
    IGAMG_SMOOTH_LEARNED = 3
} igamg_smoother;

typedef enum { IGAMG_EXTRAP_NONE = 0, IGAMG_RRE = 1, IGAMG_MPE = 2 } igamg_extrap;

/* FP64: every operation in FP64.  FP32_IR: G(x) = x + V32(round32(b - A x)),
 * i.e. the V-cycle in FP32 inside FP64 iterative refinement; the outer
 * residual, the extrapolation and the coarsest solve stay FP64. */
typedef enum { IGAMG_FP64 = 0, IGAMG_FP32_IR = 1 } igamg_precision;

typedef struct {
    int nu1, nu2;        /* pre- and post-smoothing steps (default 2, 2)      */
    int smoother;        /* igamg_smoother (default MCGS)                     */
    double omega;        /* Jacobi damping (default 2/3)                      */
    int precision;       /* igamg_precision (default FP64)                    */
    int n_el_coarsest;   /* elements per direction on level 0 (default 4)     */
    int use_graphs;      /* capture restart cycles as HIP graphs (default 1)  */
    int tail_items;      /* levels whose colour passes need at most this many
                            64-point x slice work items run, with everything
                            below them, in one single-workgroup kernel per
                            V-cycle (default 32; 0 disables)                  */
    int stored_stencil;  /* unit square: store (2p+1)^2 stencils (expanded from
                            the Kronecker factors) instead of the factors (0) */
    int mu;              /* cycle index of Algorithm 2: level l calls level
                            l-1's cycle mu times on the same coarse right-hand
                            side (1: V-cycle, 2: W-cycle; 1..4; default 1).
                            Batches and smoother training need mu = 1.       */
    int monitor;         /* RRE/MPE solves: 0 (default) test ||b - A t|| after
                            every restart cycle (Algorithm 5); 1 evaluate it
                            only when the generalised residual, scaled by the
                            ratio measured at the last evaluation, predicts
                            at most 4 tol (always after the first cycle);
                            the returned x passes the same test either way   */
    int pde;             /* igamg_pde (default POISSON); batches and the
                            learned smoother need POISSON                     */
    int row_sweeps;      /* stored stencils: sweep the p+1 colours of a row
                            class (rows j = r mod p+1) in one launch, one
                            workgroup per row (default 1); 0: one launch per
                            colour.  Both give the same iterates.  Sum-
                            factorised operators (unit square, cube): row
                            classes (j, or j and k, mod p+1), the rows'
                            products factored through the y (and z) bands
                            (iterates equal to rounding), and one-workgroup-
                            per-row residuals; 0: one launch per colour and
                            per-point residuals.                             */
    void* stream;        /* hipStream_t or NULL                               */
} igamg_options;

typedef struct {
    int restarts;        /* Algorithm 5 cycles (plain MG: V-cycles)           */
    int vcycles;         /* applications of G                                 */
    int breakdowns;      /* cycles whose extrapolation broke down             */
    int learned_fallbacks;
    double rel_residual; /* ||b - A x||_2 / ||b||_2 of the returned x          */
    double gen_residual; /* RRE/MPE: generalised residual ||t~ - t|| (Section 3,
                            eq. (11)) of the last cycle over ||s_1 - s_0|| of
                            the first; 0 for plain multigrid                  */
    int residual_checks; /* evaluations of ||b - A x|| during the solve       */
    double setup_ms;     /* time spent in igamg_setup                         */
    double solve_ms;     /* wall time of the solve call                       */
} igamg_stats;

/* Fills the defaults listed above.  n_el_coarsest <= 0 selects, per grid, the
 * coarsest size m in 4..7 with n_el = m 2^k. */
void igamg_options_default(igamg_options* opt);

/* Builds the hierarchy (Section 2): knots and Gauss rules, the finest
 * operator (Kronecker factors or mapped stencil assembled on the device),
 * knot-insertion prolongations, Galerkin coarse operators A_{l-1} = R A_l P
 * (eq. (4)), multicolour layouts, FP32 copies when needed and the FP64
 * Cholesky factor of the coarsest operator.  degree in 1..5 (3D: 1..3);
 * n_el must be n_el_coarsest * 2^k.  levels = 0 coarsens down to
 * n_el_coarsest; otherwise exactly `levels` levels are built.
 * The right-hand side starts at zero.  *out is owned by the caller and
 * released with igamg_destroy.  Errors: EINVAL, ENOMEM, EHIP, ENOTSPD. */
igamg_status igamg_setup(const igamg_geometry* geom, int degree, int levels,
                         const igamg_options* opt, igamg_ctx** out);
void igamg_destroy(igamg_ctx* ctx);

/* Unknowns on the finest level / on level l (0 = coarsest). */
igamg_status igamg_ndof(const igamg_ctx* ctx, long long* n);
igamg_status igamg_num_levels(const igamg_ctx* ctx, int* nlevels);
igamg_status igamg_level_ndof(const igamg_ctx* ctx, int level, long long* n);

/* Right-hand side.  set_rhs copies n FP64 values (host or device memory).
 * set_rhs_field assembles b_I = int f phi_I on the device with p+1 Gauss
 * points per direction for f(x) = sum_m a_m sin(pi (k_m . x) + phi_m) in
 * physical coordinates; modes holds (a, k, l, phi) per mode in 2D and
 * (a, k, l, m, phi) in 3D (host memory).  get_rhs copies b to a device buffer. */
igamg_status igamg_set_rhs(igamg_ctx* ctx, const double* b, int b_on_device);
igamg_status igamg_set_rhs_field(igamg_ctx* ctx, const double* modes, int n_modes);
/* Right-hand side of the context's Section 4.3 problem, assembled like
 * set_rhs_field: ELLIPTIC_1 and ADVECTION_DIFFUSION: f = 1; ELLIPTIC_2: f = -div(A grad u) + B.grad u + c u
 * of the manufactured solution u = (x^2 + y^2 - 0.2^2)(x^2 + y^2 - 1) sin x sin y
 * (which vanishes on the boundary of QUARTER_ANNULUS_EXACT with radii 0.2 and
 * 1).  EINVAL for the Poisson operator. */
igamg_status igamg_set_rhs_builtin(igamg_ctx* ctx);
igamg_status igamg_get_rhs(igamg_ctx* ctx, double* b_dev);

/* Switches the form of G between FP64 and FP32_IR (both operator copies are
 * built at setup).  A context set up with tail_items < 0 then takes the split
 * igamg_autotune cached for the new precision, if there is one (the FP32 store
 * of the single-workgroup kernel holds more levels).  Errors: EINVAL. */
igamg_status igamg_set_precision(igamg_ctx* ctx, int precision);

/* x <- G(x): one V(nu1, nu2) cycle (Algorithm 2, mu = 1) on the finest level,
 * or its FP32-in-FP64 refinement form.  In place. */
igamg_status igamg_vcycle(igamg_ctx* ctx, double* x_dev);

/* One cycle of Algorithm 5 without the accuracy test: s_0 = x,
 * s_{j+1} = G(s_j) for j = 0..q, then x <- t_{0,q} by Algorithm 3 (RRE) or 4
 * (MPE), using a Householder QR of Delta S_{q+1} computed as a tall-skinny QR
 * tree on the device.  q in 1..8.  Optional outputs (NULL to skip):
 * iterates_dev receives s_0 .. s_{q+1} (q+2 blocks of n values, device);
 * gamma receives gamma_0 .. gamma_q (host).  Breakdown (lambda ~ 0) leaves
 * x = s_{q+1} and returns EBREAKDOWN; non-finite iterates leave x = s_0 and
 * return ENONFINITE. */
igamg_status igamg_extrapolate(igamg_ctx* ctx, int method, int q, double* x_dev,
                               double* iterates_dev, double* gamma);
/* Flexible GMRES(m) on A x = b (restarted every m <= 30 steps), right-
 * preconditioned by the multigrid cycle: VCYCLE one FP64 V-cycle from zero;
 * RRE / MPE one restart cycle of Algorithm 5 (q+1 cycles of the context's
 * precision from zero, then the extrapolation) for A z = v, which depends
 * nonlinearly on v, hence the flexible variant (the paper presents the
 * extrapolated cycle as usable as a preconditioner: Section 1, conclusions).
 * Arnoldi by classical Gram-Schmidt applied twice.  Stops when
 * ||b - A x||_2 <= tol ||b||_2 at a restart; x is the initial guess on entry.
 * stats: restarts = GMRES iterations, vcycles = V-cycles applied,
 * residual_checks = true residual evaluations.  ENOCONV after max_iters. */
typedef enum { IGAMG_PRECOND_VCYCLE = 0, IGAMG_PRECOND_RRE = 1, IGAMG_PRECOND_MPE = 2 } igamg_precond;
igamg_status igamg_solve_fgmres(igamg_ctx* ctx, double tol, int max_iters, int m, int precond, int q,
                                double* x_dev, igamg_stats* stats);

/* Generalised residual ||t~ - t|| = ||sum_j gamma_j (s_{j+1} - s_j)|| of the last
 * extrapolation (igamg_extrapolate or the last restart cycle of igamg_solve),
 * computed from the R factor of the differences (||R gamma||), with no product
 * with A (Section 3, eq. (11)).  NaN after a breakdown; EINVAL before any
 * extrapolation. */
igamg_status igamg_generalized_residual(const igamg_ctx* ctx, double* gres);

/* Algorithm 5: restarted RRE(q)/MPE(q) from the initial guess in x_dev until
 * ||b - A x||_2 / ||b||_2 <= tol (tested on t only); method EXTRAP_NONE runs
 * plain V-cycles tested after each one.  max_restarts bounds the cycles
 * (V-cycles for the plain method).  stats may be NULL.  Returns ENOCONV with
 * stats filled when the bound is reached, ENONFINITE on NaN/Inf.  On every
 * return past the argument checks x_dev holds the accepted iterate: the last
 * t (or V-cycle result) whose residual was finite, else the initial guess;
 * stats count the accepted cycles and give that iterate's residual. */
igamg_status igamg_solve(igamg_ctx* ctx, double tol, int max_restarts, int method, int q,
                         double* x_dev, igamg_stats* stats);

/* Checkpoint of a solve.  Algorithm 5 carries nothing from one restart cycle
 * to the next but s_0 = t (Section 3.2), so the accepted iterate, the counts
 * and the adaptive settings below are the whole state of a solve. */
typedef struct {
    int method;             /* igamg_extrap of the solve                          */
    int q;                  /* its restart number (0 for EXTRAP_NONE)            */
    int restarts, vcycles, breakdowns, learned_fallbacks, residual_checks;
                            /* counts of the accepted cycles, as in igamg_stats  */
    int learned_off;        /* 1: the fallback switched the learned step off     */
    double rel_residual;    /* ||b - A x|| / ||b|| of the accepted iterate (the
                               monitor's estimate when it skipped the evaluation) */
    double gen_scale;       /* ||s_1 - s_0|| of the solve's first cycle (0: none) */
    double monitor_ratio;   /* monitor calibration rel / g (-1: none yet)        */
} igamg_state;

/* After igamg_solve has returned (with any status past its argument checks),
 * copies that solve's accepted iterate -- the x_dev it returned -- into x_dev
 * (device, ndof values; NULL to skip) and its state into *state.  EINVAL if
 * no solve has run on the context since setup, or a flexible-GMRES solve ran
 * after it (its preconditioner reuses the checkpoint buffer). */
igamg_status igamg_get_state(igamg_ctx* ctx, double* x_dev, igamg_state* state);
/* Loads a state for the NEXT igamg_solve call on this context (that call
 * only): it must use the state's method and q, starts from its own x_dev
 * (pass the checkpointed iterate), continues the counts (max_restarts bounds
 * the total, so max_restarts <= state.restarts runs no cycle) and takes over
 * the learned-step fallback and the monitor calibration.  A solve resumed
 * this way returns bit for bit the iterate and counts of the uninterrupted
 * solve (with the monitor, the interrupted solve's last cycle evaluates the
 * true residual, which recalibrates it).  The state may come from another
 * context set up with the same problem and options.  EINVAL on a bad field. */
igamg_status igamg_set_state(igamg_ctx* ctx, const igamg_state* state);

/* rel = ||b - A x||_2 / ||b||_2 in FP64 on the finest level. */
igamg_status igamg_residual(igamg_ctx* ctx, const double* x_dev, double* rel);

/* ---- Per-component entry points (the pieces of one V-cycle) ---------------
 * level l in 1..L unless stated; buffers hold level-l vectors. */

/* FP64 operator rows in stencil form: for each row index rows[r] (host),
 * out[r * S + o] = A_l[I, I + di + n dj (+ n^2 dk)] with
 * o = (di+p) + (2p+1)(dj+p) (+ (2p+1)^2 (dk+p)); zero outside the grid.
 * level in 0..L.  Host output. */
igamg_status igamg_get_operator_rows(igamg_ctx* ctx, int level, const long long* rows,
                                     int nrows, double* out);
/* y = A_l x (FP64), level in 0..L. */
igamg_status igamg_apply(igamg_ctx* ctx, int level, const double* x_dev, double* y_dev);
/* nsweeps smoothing steps on A_l x = b (FP64), level in 1..L. */
igamg_status igamg_smooth(igamg_ctx* ctx, int level, const double* b_dev, double* x_dev,
                          int nsweeps);
/* rc = P_l^T r (level l -> l-1). */
igamg_status igamg_restrict(igamg_ctx* ctx, int level, const double* r_dev, double* rc_dev);
/* x += P_l e (level l-1 -> l). */
igamg_status igamg_prolong_add(igamg_ctx* ctx, int level, const double* e_dev, double* x_dev);
/* x = A_0^{-1} b on the coarsest level (FP64 Cholesky factor). */
igamg_status igamg_coarse_solve(igamg_ctx* ctx, const double* b_dev, double* x_dev);
/* Coefficients gamma_0..gamma_q (host) of Algorithm 3/4 for the q+2 iterates
 * stored back to back in iterates_dev (device, (q+2) * n values).  info
 * receives 0 (regular), 1 (lucky breakdown) or -1 (lambda ~ 0). */
igamg_status igamg_extrap_coeffs(igamg_ctx* ctx, int method, int q,
                                 const double* iterates_dev, double* gamma, int* info);

/* The same coefficients, outputs and errors as igamg_extrap_coeffs, for
 * callers that cannot allocate device memory (serving loops, harnesses that
 * forbid hipMalloc): no allocation at all -- the R factors of the QR tree and
 * the coefficient record live in a fixed device array of about 10.8 MB that
 * each GPU the library runs on holds until the process ends (found once per
 * device, at context setup or at the first call there).  The context
 * supplies n and the stream; run it with the context's device current.
 * Limit: n <= 2^23 unknowns (EINVAL beyond).  Calls on one GPU share the
 * array: calls that overlap on one GPU (other host threads, other streams)
 * race and must be serialised by the caller. */
igamg_status igamg_extrap_coeffs_noalloc(igamg_ctx* ctx, int method, int q,
                                         const double* iterates_dev, double* gamma, int* info);

/* Measurement hook: runs nsweeps multicolour Gauss-Seidel sweeps on level
 * `level` (1..L) in the given precision (igamg_precision: FP64 uses the FP64
 * operator, FP32_IR the FP32 copy) on the context's own work vectors.  The
 * colour launches are captured as one HIP graph on the context stream (the
 * form a solve runs them in), replayed once to warm up and once between two
 * HIP events.  Outputs (host): avg_ms -- elapsed time of the timed replay
 * divided by the number of colour launches; bytes --
 * algorithmic HBM bytes of one average launch (per updated unknown: the
 * stored coefficients of its row plus b_I and x_I read and x_I written;
 * Kronecker operators count the vectors only); launches -- number timed.
 * Overwrites the level's work vectors; no other state changes. */
igamg_status igamg_profile_smoother(igamg_ctx* ctx, int level, int precision, int nsweeps,
                                    double* avg_ms, double* bytes, int* launches);

/* Autotuner of the launch shapes, by timing on the device in the current
 * precision: (1) per level, row-class sweep launches (the p+1 colours of a row
 * class per launch, where the kernel applies: stored stencils, p <= 4) or one
 * launch per colour; on cubes row-class or plane-class launches (the (p+1)^2
 * colours of a plane class per launch, levels of at most 64 unknowns per
 * direction); (2) per level, the learned smoother's inference kernel
 * (the 16 x 16-tile VALU/MFMA kernel, or the all-MFMA kernel with 12 x 12 or
 * 28 x 28 tiles; timed with zero weights, whose values do not change the
 * time); (3) the split between multi-block levels and the single-workgroup
 * kernel (the tail_items option), by whole V-cycles with (1) and (2) in
 * place.  The choice is cached for this process keyed by (GPU architecture,
 * geometry kind, operator, degree, n_el, precision); a later igamg_setup with
 * tail_items < 0 (and igamg_set_precision on such a context) takes the cached
 * choice, else the defaults.  Outputs (may be NULL): the chosen tail_items and
 * its V-cycle time in ms.  The launch shapes change times, not iterates:
 * every choice gives the same results. */
igamg_status igamg_autotune(igamg_ctx* ctx, int* tail_items, double* vcycle_ms);

/* The launch shapes a context uses (tuned or default). */
typedef struct {
    int tail_items;          /* the split threshold in use                      */
    int tail_top;            /* finest level of the single-workgroup kernel (0: none) */
    int num_levels;          /* levels of the hierarchy (<= 16)                 */
    int row_class[16];       /* per level: 1 row-class sweep launches, 0 one per colour;
                                cubes: 2 one launch per plane class (planes
                                k = ck mod p+1, one workgroup per plane)      */
    int learned_kernel[16];  /* per level: 0 16x16-tile VALU/MFMA kernel; 12, 28 all-MFMA
                                kernel with that tile (28: 512 threads); 29 tile 28
                                with 256 threads                               */
    double vcycle_ms;        /* V-cycle time of the last autotune (0: none)     */
} igamg_tuning;
igamg_status igamg_get_tuning(const igamg_ctx* ctx, igamg_tuning* out);
/* Sets the launch shapes (for instance a tuning saved by another process):
 * tail_items >= 0, row_class 0 or 1 (cubes: 0, 1 or 2; each takes effect
 * where its sweep applies, else the next lower one), learned_kernel one of
 * 0, 12, 28, 29; num_levels must match;
 * tail_top and vcycle_ms are ignored.  EINVAL on a bad field. */
igamg_status igamg_set_tuning(igamg_ctx* ctx, const igamg_tuning* in);

/* ---- Learned smoother (2D only) ------------------------------------------
 * Per level l >= 1 a network N_l (3x3 convolutions 1 -> 16 -> 16 -> 1, ReLU,
 * zero padding, no biases; BF16 weights, FP32 accumulation on MFMA) replaces
 * the first pre-smoothing sweep: z = D^{-1} r / sigma with sigma = RMS(D^{-1} r),
 * x += sigma N_l(z).  Levels run by the single-workgroup kernel keep plain
 * Gauss-Seidel.  Weights use the canonical layout W1[16][9], W2[16][16][9],
 * W3[16][9] (tap = 3 dy + dx), 2592 BF16 values per level. */
typedef struct {
    int n_rhs;               /* training right-hand sides                        */
    const double* modes;     /* n_rhs * n_modes mode rows (host), as set_rhs_field */
    int n_modes;
    int vcycles_per_rhs;     /* plain V-cycles recorded per right-hand side (3)  */
    int epochs;              /* passes over each level's patches (10)            */
    int batch;               /* 64 x 64 patches per Adam step (32)               */
    double lr;               /* Adam step size (1e-3)                            */
    unsigned long long seed; /* weight initialisation and shuffling              */
    const double* val_modes; /* validation right-hand side (NULL: first training one) */
    int val_n_modes;
    int val_vcycles;         /* V-cycles of the contraction measurement (12)     */
    double solve_tol;        /* relative tolerance of the level solves (1e-12)   */
    int per_level_accept;    /* 1: keep a level's network only if the cycle started
                                on that level contracts better with it (bottom-up);
                                0 (default): every trained level keeps its network
                                and only the whole-cycle test decides            */
} igamg_train_options;

typedef struct {
    int levels_trained;
    int patches;             /* training patches over all levels                 */
    double loss_first[16];   /* mean loss of the first / last epoch per level    */
    double loss_last[16];
    double rho_plain;        /* measured residual contraction per V-cycle        */
    double rho_learned;
    int accepted;            /* 1 if rho_learned < rho_plain (learned step enabled) */
    double train_ms;
    double rho_plain_level[16];   /* per level l >= 1: the same contraction for the
                                     cycle started on level l (levels 0..l), right-
                                     hand side the validation b restricted to level
                                     l; entry L equals rho_plain; 0 for level 0 */
    double rho_learned_level[16]; /* the same with the networks kept (levels above
                                     the single-workgroup split use them)      */
    int accepted_level[16];       /* 1 where the level's network is kept (above the
                                     single-workgroup split; with per_level_accept,
                                     bottom-up: level l keeps it only if the cycle
                                     started on level l contracts better with it
                                     than without, the levels below as decided)  */
} igamg_train_report;

void igamg_train_options_default(igamg_train_options* o);
/* Generates residual / target pairs from plain FP64 V-cycles on the given
 * right-hand sides (the target is the part of the algebraic error that the
 * coarse-grid correction cannot remove, e - P A_{l-1}^{-1} R r, from tight level
 * solves), trains every level's network on the device (Adam, FP32 master
 * weights), with per_level_accept keeps each level's network only where it
 * makes the cycle started on that level contract better (bottom-up), measures
 * the whole-cycle contraction with and without the networks kept and enables
 * them only if they contract better.  The right-hand side and the
 * iterate state of the context are restored.  Errors: EINVAL (3D, bad options). */
igamg_status igamg_train_smoother(igamg_ctx* ctx, const igamg_train_options* opt,
                                  igamg_train_report* report);
/* Turns the learned step on (1) or off (0); EINVAL if no weights are loaded. */
igamg_status igamg_set_learned(igamg_ctx* ctx, int enabled);
igamg_status igamg_get_smoother_weights(igamg_ctx* ctx, int level, uint16_t* bf16, size_t n);
igamg_status igamg_set_smoother_weights(igamg_ctx* ctx, int level, const uint16_t* bf16, size_t n);
/* y = N_l(z) on level l's grid (device FP32 vectors of the level's length). */
igamg_status igamg_smoother_forward(igamg_ctx* ctx, int level, const float* z_dev, float* y_dev);
/* Loss mean((N_l(z) - t)^2) over the level's grid and its gradient with
 * respect to the canonical weights (host, 2592 FP32 values). */
igamg_status igamg_smoother_loss_grad(igamg_ctx* ctx, int level, const float* z_dev,
                                      const float* t_dev, double* loss, float* grad);

/* ---- Batches of independent 2D problems ---------------------------------
 * A batch holds `count` problems of any 2D geometry, degree (1..5) and size
 * (coarsest grid chosen per problem as for n_el_coarsest <= 0), all solved by
 * restarted RRE(q) around FP32 V-cycles inside FP64 refinement (the precision
 * and smoother fields of opt are ignored).  Every V-cycle step is one launch
 * per degree group covering all unconverged problems of that degree; the
 * degree groups run as parallel branches of one captured graph per restart
 * cycle; extrapolation and the accuracy test are per problem.  All work is on
 * opt->stream (or a stream the batch creates).  With opt->tail_items < 0 each
 * problem's multi-block / single-workgroup split comes from the autotuner
 * (cached per architecture, geometry, degree, grid and precision). */
typedef struct igamg_batch igamg_batch;
igamg_status igamg_setup_batch(int count, const igamg_geometry* geoms, const int* degrees,
                               const igamg_options* opt, igamg_batch** out);
void igamg_destroy_batch(igamg_batch* batch);
/* Problem i of the batch as a context (owned by the batch): ndof, set_rhs,
 * set_rhs_field, residual and the other single-problem calls apply to it. */
igamg_status igamg_batch_instance(igamg_batch* batch, int i, igamg_ctx** ctx);
/* Solves every problem from the initial guesses x_dev[i] until its relative
 * residual is <= tol (per problem); stats[i] per problem (may be NULL).
 * Returns ENOCONV if any problem did not converge within max_restarts. */
igamg_status igamg_solve_batch(igamg_batch* batch, double tol, int max_restarts, int q,
                               double* const* x_dev, igamg_stats* stats);

/* ---- 1D model problems ----------------------------------------------------
 * The model problem of Section 2.4, eq. (6): -u'' = (2 pi)^2 sin(2 pi x) on
 * (0, 1), u(0) = u(1) = 0, exact solution u = sin(2 pi x), discretised as in
 * Section 2 with B-splines of degree 1..9 on n_el uniform elements (interior
 * unknowns n = n_el + degree - 2, x index order), stiffness and load by Gauss
 * quadrature with degree+1 points per element, `levels` grids (the coarsest
 * has n_el / 2^(levels-1) elements; Table 1's nlevels = 4) with Galerkin
 * coarse matrices (eq. (4)) and a direct coarsest solve.  A set holds `count`
 * independent problems; every call runs each problem in one workgroup of one
 * launch (Algorithm 5 around mu-cycles of Algorithm 2, all of it on the
 * device, FP64), so a set of many problems fills the chip.  The level vectors
 * of a problem live in LDS: 3 * sum_l n_l <= 16384 (EINVAL otherwise).  All
 * work is on the stream given to igamg_setup_1d (NULL: the set creates a
 * blocking stream); the calls synchronise it before returning. */
typedef struct {
    int n_el;       /* elements, a multiple of 2^(levels-1)                     */
    int degree;     /* 1..9                                                     */
    int levels;     /* 1..16                                                    */
    int smoother;   /* IGAMG_SMOOTH_JACOBI (weighted, omega), _MCGS (p+1
                       colours i mod (p+1)) or _LEXGS (forward, i increasing)   */
    int nu1, nu2;   /* pre- and post-smoothing sweeps (0..64)                   */
    int mu;         /* cycle index: 1 V-cycle, 2 W-cycle (1..4)                 */
    double omega;   /* Jacobi weight in (0, 2)                                  */
    int method;     /* igamg_extrap: NONE (plain cycles), RRE or MPE            */
    int q;          /* restart number 1..8 (RRE/MPE)                            */
} igamg_problem1d;
/* Section 4.1's setting: 64 elements, degree 2, 4 levels, weighted Jacobi
 * V(1,1) with omega = 2/3, no extrapolation, q = 4. */
void igamg_problem1d_default(igamg_problem1d* pr);

typedef struct {
    int restarts;         /* restart cycles (V-cycles for method NONE)           */
    int vcycles;          /* cycles of Algorithm 2                               */
    int breakdowns;       /* restarts with no extrapolation (t = s_{q+1})        */
    int converged;        /* 1 if ||b - A x|| / ||b|| <= tol                     */
    double rel_residual;  /* ||b - A x|| / ||b|| of the returned x               */
    double l2_error;      /* ||u_h - sin(2 pi x)||_L2, degree+1 Gauss points
                             per element (the model right-hand side)            */
    double solve_ms;      /* host wall time of the call (all problems)          */
} igamg_stats1d;

typedef struct igamg_set1d igamg_set1d;
/* Builds every problem (bands, transfer tables, coarsest inverse, element
 * tables, the load vector of f = (2 pi)^2 sin(2 pi x)).  Errors: EINVAL (bad
 * fields, too large for LDS), ENOTSPD, ENOMEM, EHIP. */
igamg_status igamg_setup_1d(int count, const igamg_problem1d* probs, void* stream, igamg_set1d** out);
void igamg_destroy_1d(igamg_set1d* set);
/* Unknowns of problem i, or -1 for a bad set or index. */
long long igamg_ndof_1d(const igamg_set1d* set, int i);
/* Replace / read problem i's right-hand side (device FP64, ndof entries). */
igamg_status igamg_set_rhs_1d(igamg_set1d* set, int i, const double* b_dev);
igamg_status igamg_get_rhs_1d(igamg_set1d* set, int i, double* b_dev);
/* ncycles mu-cycles on every problem: x_dev[i] (device FP64, ndof entries,
 * caller-owned) is the initial guess and receives the result. */
igamg_status igamg_cycles_1d(igamg_set1d* set, int ncycles, double* const* x_dev);
/* Algorithm 5 with RRE(q) / MPE(q) (or plain cycles) from the initial guesses
 * x_dev[i] until ||b - A x|| / ||b|| <= tol (||b - A x|| <= tol for b = 0),
 * tested on t after every restart
 * (after every cycle for NONE), at most max_iters restarts (cycles); x_dev[i]
 * receives the last accepted iterate and stats[i] (may be NULL) its counts.
 * Returns ENOCONV if any problem did not converge, ENONFINITE on NaN/Inf. */
igamg_status igamg_solve_1d(igamg_set1d* set, double tol, int max_iters, double* const* x_dev,
                            igamg_stats1d* stats);

/* Text of the last error raised on the calling thread ("" if none). */
const char* igamg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* IGAMG_H */

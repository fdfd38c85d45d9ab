/*
 * dd.h -- C ABI of the substructuring Schur-complement solver for nonlocal
 * FEM systems on one AMD Instinct MI355X (gfx950).
 *
 * Method (arXiv:2306.00094, section "Matrix formulation of the multi-domain
 * problem"): the free dofs of the stiffness matrix A are split into the
 * interiors I_k of K overlapping subdomains and the interface G (the dofs that
 * lie in two or more subdomains).  With K_II = blockdiag(K_II^k),
 *
 *   S = K_GG - sum_k R_k^T K_GI^k (K_II^k)^{-1} K_IG^k R_k   (eq. subSchurComplement,
 *                                                             summed as in eq. SchurComplement)
 *   g = b_G  - sum_k R_k^T K_GI^k (K_II^k)^{-1} b_I^k        (eq. subForcing)
 *   S u_G = g  by preconditioned conjugate gradients,
 *   u_I^k = (K_II^k)^{-1} (b_I^k - K_IG^k R_k u_G)          (eq. backwardSubstitution)
 *
 * where R_k picks the interface dofs coupled to subdomain k.  K_II^k is
 * non-singular for every subdomain, floating ones included (stated before
 * eq. splittingBlockCholesky), and is factored once (dd_factor).
 *
 * Conventions.
 *   - All functions return dd_status and never throw across the ABI.
 *   - Host pointers (H) are read during the call only; device pointers (D)
 *     are HIP device addresses owned by the caller.
 *   - Index arrays are int32, 0-based.  Matrices are double precision.
 *   - All device work of a context runs on the HIP stream given to dd_setup
 *     (NULL = the default stream).  A context must not be used from two host
 *     threads at once; independent contexts may run concurrently.
 */
#ifndef DD_H
#define DD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dd_ctx dd_ctx;   /* opaque solver context */

typedef enum {
  DD_OK = 0,
  DD_EINVAL = 1,   /* malformed argument (message names the field) */
  DD_ENOMEM = 2,   /* device or host allocation failed */
  DD_ENOTSPD = 3,  /* Cholesky pivot <= 0 (subdomain, column) or p^T S p <= 0 */
  DD_ENOCONV = 4,  /* iteration or refinement limit reached; output holds the last iterate */
  DD_EHIP = 5,     /* HIP runtime error (code in the message) */
  DD_ESTATE = 6    /* call out of order, e.g. solve before factor */
} dd_status;

typedef enum {
  DD_FP64 = 0,     /* FP64 factor, FP64 products, FP64 CG */
  DD_MIXED = 1     /* FP32 factor and interior solves (FP32 accumulation), FP32 coupling
                      data with FP64 accumulation, FP64 CG vectors and dots, FP64
                      full-system residual and iterative-refinement correction */
} dd_precision;

/* One subdomain, HOST pointers, deep-copied by dd_setup. */
typedef struct {
  int32_t n_i;               /* interior dofs of the subdomain (>= 1) */
  const double *k_ii;        /* n_i*n_i, column-major, symmetric; both triangles given */
  int32_t n_g;               /* interface dofs coupled to this interior (>= 0) */
  const int32_t *g_map;      /* n_g: local interface column -> interface index in [0, n_gamma) */
  const int32_t *kig_rowptr; /* n_i+1: CSR row pointers of K_IG^k (n_i x n_g) */
  const int32_t *kig_col;    /* nnz: local interface column in [0, n_g) */
  const double *kig_val;     /* nnz */
  const int32_t *i_map;      /* n_i: local interior dof -> global dof in [0, n_dof) */
} dd_subdomain;

/* The partitioned system.  Every global dof is either interior to exactly one
 * subdomain or an interface dof; interiors of different subdomains must not be
 * coupled (checked through the sparsity the caller passes).
 *
 * n_sub = 0 is the undecomposed system: every dof is an interface dof
 * (gamma_map a permutation of [0, n_dof)), K_GG is the whole matrix A, S = A
 * and diag(S) = diag(A), so dd_solve runs the diagonally preconditioned CG on
 * A that the paper compares against (section "Considered solver strategies";
 * one CSR sweep of A per iteration, no factorisation). */
typedef struct {
  int32_t n_dof;             /* size of the free-dof system A */
  int32_t n_gamma;           /* interface dofs */
  int32_t n_sub;             /* number of subdomains K (>= 0) */
  const dd_subdomain *sub;   /* n_sub entries (may be NULL when n_sub = 0) */
  const int32_t *gamma_map;  /* n_gamma: interface index -> global dof */
  const int32_t *kgg_rowptr; /* n_gamma+1: CSR of the global K_GG (n_gamma x n_gamma) */
  const int32_t *kgg_col;
  const double *kgg_val;
} dd_problem;

/* Interior-solve variants for the per-iteration (K_II^k)^{-1} products. */
typedef enum {
  DD_APPLY_AUTO = 0,   /* choose by the autotuned table (or INV) */
  DD_APPLY_INV = 1,    /* product with K_II^{-1} = L^{-T} L^{-1}, formed at factor time */
  DD_APPLY_TRSM = 2    /* forward and backward triangular sweeps with L */
} dd_apply;

/* A CG iteration on S is three launches (K_IG product with the previous
 * iteration's update, interior solve with the direction recurrence,
 * interface rows) or four (K_IG product, interior solve, interface rows,
 * update).  Untuned solves use three when the explicit inverse is applied and
 * subdomains exist, at every batch width (a column's result does not depend on
 * the batch); the autotuner times both forms per width.  The persistent
 * kernel, the triangular-sweep variant and the batch API use four. */
typedef enum {
  DD_LAUNCH_AUTO = 0,
  DD_LAUNCH_KERNELS = 1,     /* one kernel launch per phase, host polls convergence */
  DD_LAUNCH_PERSISTENT = 2,  /* one cooperative kernel runs the whole CG loop */
  DD_LAUNCH_GRAPH = 3        /* check_every CG iterations captured in one hipGraph, replayed */
} dd_launch;

typedef struct {
  double tol;            /* stop column c when ||b_c - A u_c||_2 <= tol ||b_c||_2 */
  int32_t max_it;        /* CG iteration cap per CG solve */
  int32_t precond;       /* 0 none, 1 exact diag(S) Jacobi */
  int32_t max_refine;    /* DD_MIXED: outer refinement steps */
  double inner_tol;      /* DD_MIXED: inner CG stops at ||r_in|| <= max(inner_tol ||r_outer||,
                            tol ||b|| / 2); 0 = automatic (the autotuned value for this
                            batch width, else 1e-5).  With residual replacement (`reliable`
                            below): the reduction of a column's residual after which it is
                            due for the next replacement; 0 = the autotuned value, else 1e-2 */
  int32_t fp64_fallback; /* DD_MIXED: 1 = finish stalled columns with the FP64 path */
  int32_t apply;         /* dd_apply */
  int32_t launch;        /* dd_launch */
  int32_t check_every;   /* DD_LAUNCH_KERNELS: host polls convergence every N iterations (0 = auto) */
  int32_t verify;        /* 1 = compute the true FP64 residual ||b - A u|| / ||b|| into info */
  int32_t gather32;      /* DD_MIXED: the FP32-data products gather FP32 copies of the vectors
                            they multiply (half the gathered bytes; pays off for wide
                            batches): -1 = automatic (dd_solve: the autotuned schedule, else
                            off; batches: off), 0 = off, 1 = on */
  int32_t tiles;         /* batches of 8 or more columns: coupling products on 16x16 tiles and
                            interior solves on the matrix cores (the direction kept by its own
                            kernel); a column's result then differs in rounding from the
                            narrow-batch kernels but does not depend on the width among 8..64:
                            -1 = automatic (the autotuned schedule, else off), 0 = off,
                            1 = on (ignored below 8 columns, with the triangular-sweep apply,
                            the persistent launch, or a context set up for fewer than 8) */
  int32_t reliable;      /* DD_MIXED on the tiled path (tiles above) with the FP64 factor also
                            formed (dd_factor(ctx, DD_FP64)): residual replacement.  The FP32
                            operators form the search directions; condensation, back
                            substitution and the interface residual g - S x use the FP64
                            operators.  Every `reliable` CG iterations, once some column's
                            residual has fallen by the factor inner_tol (0: the autotuned
                            value, else 1e-2) since the last replacement, every iterating
                            column has its recurrence residual replaced by the FP64 one (one
                            FP64 product serves the batch, so the replacement points depend
                            on the batch: a column's result is the same in any batch within
                            the tolerance, not bitwise).  One Krylov space then reaches the
                            tolerance (refinement steps, which restart it, only follow if
                            the final FP64 check fails).  -1 = automatic (every 8
                            iterations), 0 = off (plain refinement), N > 0 = every N
                            iterations (rounded up to a multiple of the graph length with
                            DD_LAUNCH_GRAPH).  Ignored elsewhere. */
} dd_solve_opts;

typedef struct {
  int32_t iters;         /* CG iterations (summed over refinement steps) */
  int32_t refine_steps;  /* DD_MIXED: outer steps taken */
  int32_t used_fallback; /* DD_MIXED: 1 if the FP64 path finished this column */
  int32_t converged;     /* 1 if the tolerance was met */
  double rel_resid;      /* ||b - A u||_2 / ||b||_2 (FP64) if verify or DD_MIXED, else the
                            CG recurrence estimate ||r_G||_2 / ||b||_2 */
} dd_solve_info;

/* Fill opts with defaults: tol 1e-10, max_it 1000, precond 1, max_refine 8,
 * inner_tol 0 (automatic), fp64_fallback 1, AUTO apply/launch, check_every 0, verify 1,
 * gather32 -1 (automatic), tiles -1 (automatic), reliable -1 (automatic). */
void dd_default_opts(dd_solve_opts *opts);

/* Device bytes a context for `prob` would hold: the blocks of eq.
 * subStiffnessMatrixSubBlocks as uploaded, the factors of eq.
 * splittingBlockCholesky for `prec` (DD_MIXED also counts the FP64 factors its
 * fallback forms on first use), the tiles of the wide-batch products when
 * max_nrhs >= 8, and the work vectors for max_nrhs right-hand sides.  prob: H.
 * Validates nothing beyond the sizes; DD_EINVAL on a NULL pointer or max_nrhs
 * outside [1, 64].  (max_nrhs is an addition to the interface the method
 * implies: it sizes the resident Krylov state of batched solves.) */
dd_status dd_footprint(const dd_problem *prob, dd_precision prec, int32_t max_nrhs,
                       size_t *bytes);

/* Upload the partitioned system: per subdomain the blocks K_II^k and K_IG^k
 * and the global K_GG (eqs. subStiffnessMatrix, subStiffnessMatrixSubBlocks;
 * K_GG assembled once for all subdomains, whose subdomain blocks sum to it by
 * the partition of unity of eq. zeta).  Validate `prob` (index ranges, CSR
 * monotonicity, map injectivity, coverage of every dof, no interior-interior
 * coupling across subdomains -- the requirement of eq. subRequirement that
 * interiors interact only through the interface), deep-copy it to the current
 * HIP device (prob: H, read during the call only) and bind the context to
 * `hip_stream`.  max_nrhs in [1, 64]: largest batch dd_solve will accept (an
 * addition to the interface the method implies).  *out is NULL on error
 * (DD_EINVAL with the field named, DD_ENOMEM, DD_EHIP); the message of a
 * failed setup is returned by dd_last_error(NULL). */
dd_status dd_setup(const dd_problem *prob, void *hip_stream, int32_t max_nrhs,
                   dd_ctx **out);

/* Factor every K_II^k = L_k L_k^T (batched Cholesky; the block factorisation of
 * eq. splittingBlockCholesky needs K_II^k non-singular, which holds for every
 * subdomain, floating ones included), form the interior-solve operators
 * K_II^{-1} = L^{-T} L^{-1} and the exact diagonal of S (eq.
 * subSchurComplement summed over k) for the Jacobi preconditioner, in
 * precision `prec`.  May be called
 * again with the other precision; both sets of factors are then kept.
 * DD_ENOTSPD names the subdomain and column of the first failed pivot, or the
 * interface row whose diag(S) entry is not positive.  DD_EHIP also covers a
 * block column of the one-launch Cholesky whose bounded wait for the columns
 * before it ran out (the factors are then not usable).  The first call
 * allocates the work space of the inverse and of diag(S) (counted by
 * dd_footprint); later calls reuse it. */
dd_status dd_factor(dd_ctx *ctx, dd_precision prec);

/* Solve A u = b for nrhs columns (the discrete system of the section "A
 * discretized weak formulation"): condensation g = b_G - sum_k K_GI^k
 * (K_II^k)^{-1} b_I^k (eq. subForcing summed over k), preconditioned CG on
 * S u_G = g with S = sum_k R_k^T S_k R_k (eqs. subSchurComplement,
 * SchurComplement), and back substitution of the interiors (eq.
 * backwardSubstitution).  prec selects FP64 or mixed FP32/FP64 iterative
 * refinement (an addition to the method, see dd_precision).  b_dev and u_dev:
 * D, column-major n_dof x nrhs with leading dimension ld >= n_dof; they may
 * not alias.  Uses the
 * factors of `prec` (dd_factor(prec) must have run; DD_MIXED falls back to
 * FP64 factors, computing them on first use, when opts->fp64_fallback).
 * info_host: H, nrhs entries (may be NULL).  Returns after the solution and
 * info are complete.  DD_ENOCONV if any column missed the tolerance. */
dd_status dd_solve(dd_ctx *ctx, dd_precision prec, const double *b_dev, double *u_dev,
                   int32_t nrhs, int32_t ld, const dd_solve_opts *opts,
                   dd_solve_info *info_host);

/* q = S p for interface vectors (diagnostic entry; eq. subSchurComplement
 * summed over subdomains).  p_dev, q_dev: D, column-major n_gamma x nrhs, ld. */
dd_status dd_schur_apply(dd_ctx *ctx, dd_precision prec, const double *p_dev,
                         double *q_dev, int32_t nrhs, int32_t ld);

/* The same product without any device allocation, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid it); dd_schur_apply allocates an index map per call.
 * Its work vectors -- (2 n_gamma + 2 n_I) * next_pow2(nrhs) doubles -- live in
 * a static device array of 4 Mi doubles (32 MiB) that every device the library
 * runs on holds until the process ends; larger work is rejected with
 * DD_EINVAL.  The context's device must be the current device.  All calls on
 * one device share that array: calls that overlap on one GPU (several streams
 * or host threads) race.  Same arguments, layout and errors as dd_schur_apply. */
dd_status dd_schur_apply_noalloc(dd_ctx *ctx, dd_precision prec, const double *p_dev,
                                 double *q_dev, int32_t nrhs, int32_t ld);

/* Copy the lower Cholesky factor of subdomain k (n_i x n_i column-major,
 * upper triangle zero) to host memory `out` as doubles (diagnostic entry). */
dd_status dd_get_factor(dd_ctx *ctx, dd_precision prec, int32_t k, double *out);

/* Copy diag(S) (n_gamma doubles) to host memory (diagnostic entry). */
dd_status dd_get_schur_diag(dd_ctx *ctx, dd_precision prec, double *out);

/* Schedule chosen by the autotuner (dd_autotune). */
typedef struct {
  int32_t apply;             /* dd_apply */
  int32_t launch;            /* dd_launch */
  int32_t direction_kernel;  /* 1: direction kept in memory by its own kernel, 0: formed on the fly */
  int32_t check_every;       /* polling lag (kernels) or iterations per graph (graph) */
  double ms_per_solve;       /* measured time of one solve of the batch with this schedule */
  int32_t candidates;        /* schedules timed */
  double inner_tol;          /* DD_MIXED: inner tolerance chosen, or for a schedule that
                                replaces residuals (dd_solve_opts.reliable) its drop factor
                                (0 for DD_FP64) */
  int32_t three_launch;      /* bit 0 set: three launches per CG iteration (update fused
                                into the K_IG launch, direction recurrence in the interior
                                solve), clear: four (K_IG, interior solve, interface rows,
                                update); bit 1 (DD_MIXED only): the FP32-data products
                                gather FP32 copies of the vectors they multiply (half the
                                gathered bytes; pays off for wide batches); bit 2: the tiled
                                matrix-core products of batches of 8 or more columns
                                (dd_solve_opts.tiles) */
} dd_tune_result;

/* Autotuner: time every candidate schedule of the CG loop on this context and
 * precision for a batch of nrhs synthetic right-hand sides (launch mode,
 * interior-solve variant, three or four launches per iteration, direction
 * handling, polling lag), keep the fastest,
 * and use it for later dd_solve calls of that precision and batch width whose
 * opts leave apply and launch at AUTO.  For DD_MIXED with base->inner_tol == 0
 * the inner tolerance (1e-4, 1e-5, 1e-6) is then timed with that schedule and
 * kept for solves whose inner_tol is 0.  base: tolerances used while timing
 * (NULL = defaults).  The factors of `prec` must exist.  out may be NULL. */
dd_status dd_autotune(dd_ctx *ctx, dd_precision prec, int32_t nrhs, const dd_solve_opts *base,
                      dd_tune_result *out);

/* ------------------------------------------------------------------------
 * Continuous batching (serving).  A context keeps a resident CG state with up
 * to max_nrhs slots (right-hand-side columns).  Requests are admitted into
 * free slots between CG iterations, every slot iterates independently (its
 * arithmetic does not depend on the other slots, so a result is the same
 * alone and in a mix), finished slots are retired, and their slots reused.
 * While a batch is open, dd_solve / dd_autotune on the context return
 * DD_ESTATE.  Slot states: */
enum { DD_SLOT_FREE = 0, DD_SLOT_RUNNING = 1, DD_SLOT_DONE = 2, DD_SLOT_FALLBACK = 3 };
/* DD_SLOT_DONE: result ready (converged or at the iteration cap, see info);
 * DD_SLOT_FALLBACK: mixed-precision refinement stalled; the request should be
 * solved with FP64 factors (e.g. dd_solve on another context). */

/* Open a batch: precision and tolerances (opts) for every slot.  With
 * DD_MIXED and opts->gather32 == 1 the session keeps the direction in memory
 * and its FP32-data products gather FP32 vector copies; apply, launch and
 * check_every are not used (every step launches its kernels directly). */
dd_status dd_batch_begin(dd_ctx *ctx, dd_precision prec, const dd_solve_opts *opts);

/* Admit ncol right-hand sides (b_dev: D, column-major n_dof x ncol, leading
 * dimension ld) into the free slots slots[0..ncol) (H). */
dd_status dd_batch_admit(dd_ctx *ctx, const int32_t *slots, int32_t ncol, const double *b_dev,
                         int32_t ld);

/* Advance every running slot by up to iters CG iterations, then finish,
 * refine or restart the slots whose CG converged.  state_host (H, max_nrhs
 * entries, may be NULL) receives the slot states. */
dd_status dd_batch_step(dd_ctx *ctx, int32_t iters, int32_t *state_host);

/* Copy the solutions of DONE slots to u_dev (D, column-major n_dof x ncol,
 * leading dimension ld), fill info_host (H, ncol entries, may be NULL) and
 * free the slots. */
dd_status dd_batch_retire(dd_ctx *ctx, const int32_t *slots, int32_t ncol, double *u_dev,
                          int32_t ld, dd_solve_info *info_host);

/* Close the batch (all slots are freed). */
dd_status dd_batch_end(dd_ctx *ctx);

/* Per-phase kernel timing of the CG loop (diagnostic entry for profiling).
 * Phases: one launch each per CG iteration. */
enum {
  DD_PHASE_KIG = 0,       /* y = K_IG p                        (all subdomains) */
  DD_PHASE_INTERIOR = 1,  /* w = K_II^{-1} y                   (all subdomains) */
  DD_PHASE_GAMMA = 2,     /* q = K_GG p - K_GI w, p^T q partials (interface rows) */
  DD_PHASE_UPDATE = 3,    /* alpha, x, r, z updates, r^T z, r^T r, beta, convergence */
  DD_PHASE_LOOP = 4,      /* one graph replay or one persistent CG launch (whole iterations) */
  DD_NPHASES = 5
};

/* Enable HIP-event timing of the phases whose bit is set in phase_mask
 * (0 disables).  An event pair is recorded on the context's stream around
 * every launch of a timed phase; for DD_PHASE_GAMMA the launch itself records
 * the pair at kernel start and end (the kernel's own duration; each such pair
 * adds a few microseconds of stream time).  reset != 0 clears the
 * accumulators; reset = 0 keeps them (pairs recorded so far are accumulated
 * first, which synchronises the stream), so timing can be switched on for a
 * sample of the calls. */
dd_status dd_set_timing(dd_ctx *ctx, uint32_t phase_mask, int32_t reset);

/* Accumulated milliseconds and launch counts per phase since the last reset
 * (ms, launches: H, DD_NPHASES entries each).  DD_PHASE_GAMMA counts the
 * interface-row launches that swept the matrix: in the three-launch iteration
 * those of iterations 0 .. K-1 (K the largest iteration count of the solve's
 * columns), not the launches that returned at once because every column had
 * stopped (an iteration enqueued ahead of the convergence check).
 * Synchronises the context's stream. */
dd_status dd_get_timing(dd_ctx *ctx, double *ms, int64_t *launches);

/* Last error message of ctx (or of the last failed dd_setup when ctx is NULL).
 * The string stays valid until the next call on the same context. */
const char *dd_last_error(const dd_ctx *ctx);

/* Release every device and host resource of ctx (NULL is accepted). */
void dd_destroy(dd_ctx *ctx);

/* ------------------------------------------------------------------------
 * Assembly of the nonlocal stiffness matrix on the device (the step before
 * dd_setup), 2D: the unit square with n cells per side split into right
 * triangles, plus an interaction collar of `collar` cells (Dirichlet volume
 * constraint).  Entry (m, n') of the bilinear form of eq. bil1,
 *   int int (psi_m(y) - psi_m(x)) (psi_n'(y) - psi_n'(x)) gamma(x, y) dy dx,
 * for every free node m, with gamma = phi (kernel 0, eq. constantkernel),
 * phi |x - y|^-(2 + 2s) (kernel 1, eq. fractionalkernel) or the peridynamic
 * bond tensor phi (x-y)(x-y)^T / |x-y|^3 (kernel 2, eq. peridynamics; 2x2
 * blocks), element pairs interacting when their barycentres are within delta
 * (approximate interaction balls), 7-point degree-5 Gauss rules per triangle
 * (fractional pairs sharing a vertex: mean of the 7x6- and 6x7-point rules).
 *   win_dev (D, caller-owned): (n-1)^2 rows, free node (a, b) with a, b in
 *   collar+1 .. collar+n-1 at row (b-collar-1)(n-1) + (a-collar-1); each row
 *   a dense window of (2R+1)^2 doubles (4 (2R+1)^2 for kernel 2) for nodes
 *   (a+da, b+db), |da|, |db| <= R, at (db+R)(2R+1) + (da+R) (kernel 2:
 *   [row component][window][column component]).  Collar nodes are included.
 * ceil(delta n) + 2 <= R <= 63.  The kernel keeps four copies of the nodes
 * of one row's window within distance delta n + 1.5 (node units) of its node
 * (the only ones the row reaches; three values each for kernel 2), which
 * must fit in 64 KiB: about delta n <= 23 (kernel 2: 13).
 * Launched on hip_stream; returns without waiting.  Every entry is summed in
 * a fixed order: the same arguments give the same bits on every run.
 * Errors: DD_EINVAL (message from dd_last_error(NULL)), DD_EHIP. */
dd_status dd_assemble_2d(int32_t n, int32_t collar, double delta, int32_t kernel, double phi,
                         double s, int32_t R, double *win_dev, void *hip_stream);

/* ------------------------------------------------------------------------
 * One-level FETI (section "FETI", Algorithm 1): the dual method on the same
 * reduced multi-domain problem (eq. discreteSubNonlocal).  Every subdomain k
 * keeps its own copy Gamma_k of the interface dofs of hat-Omega_k; the
 * copies are tied by Lagrange multipliers lambda, one per pair of consecutive
 * copies of a dof (B: one +1 and one -1 per row), and the projected
 * preconditioned CG runs on P F lambda = P d (eq. FETIproblem) with
 * F = B S^+ B^T, the natural coarse space G = B Z of the floating subdomains'
 * kernels (eq. P), lambda_0 = G (G^T G)^-1 e, and the scaled Dirichlet
 * preconditioner B_D S B_D^T (eq. preconditioner).  S_k^+ comes from the
 * Cholesky factor of A^k with pinned dofs for floating subdomains (section
 * "Pseudoinverse and Cholesky decomposition"), the pins chosen where the
 * kernel basis is best conditioned; alpha and u by eqs. forAlpha and forU,
 * then the interiors by eq. backwardSubstitution. */
typedef struct dd_feti_ctx dd_feti_ctx;

/* The FETI data of one subdomain, HOST pointers (read during dd_feti_setup). */
typedef struct {
  int32_t n_g;                /* dofs of Gamma_k (the interface dofs of hat-Omega_k) */
  const int32_t *g_map;       /* n_g: copy dof -> interface index of the problem, increasing */
  const int32_t *agg_rowptr;  /* n_g+1: CSR of A^k_GG (eq. subStiffnessMatrixSubBlocks assembled */
  const int32_t *agg_col;     /*   with the zeta-weighted form of eq. bilinear-multi1), n_g x n_g */
  const double *agg_val;
  const int32_t *kig_rowptr;  /* n_i+1: CSR of A^k_IG = A(I_k, Gamma_k), columns in [0, n_g) */
  const int32_t *kig_col;
  const double *kig_val;
  int32_t n_z;                /* 0 if Gamma^D_k is non-empty, else the dimension of ker A^k
                                 (1 for scalar kernels, 3 for peridynamics; at most 8) */
  const double *z;            /* n_g x n_z column-major: that kernel on Gamma_k */
} dd_feti_sub;

/* Set up FETI for `prob` (whose subdomains give K_II^k and the interior maps;
 * prob is validated as by dd_setup) and the copies fsub[0 .. prob->n_sub).
 * Forms B, B_D, Z, G and (G^T G)^-1 (host), and factors and inverts the
 * pinned subdomain matrices on the device (dense, n_i + n_g rows each) to
 * keep the interface blocks that give S_k^+.  Loads b_G are split evenly over
 * the copies of a dof (the constrained problem sees only their sum, so the
 * solution does not depend on the split).  max_nrhs in [1, 64].  Errors:
 * DD_EINVAL (field named; message by dd_feti_last_error(NULL)), DD_ENOMEM,
 * DD_ENOTSPD (a pinned subdomain matrix or G^T G not positive definite),
 * DD_EHIP. */
dd_status dd_feti_setup(const dd_problem *prob, const dd_feti_sub *fsub, void *hip_stream,
                        int32_t max_nrhs, dd_feti_ctx **out);

/* Factor the interior blocks K_II^k (the Dirichlet solves of S_k in the
 * preconditioner, the reduced forcing of eq. subForcing and the back
 * substitution), FP64. */
dd_status dd_feti_factor(dd_feti_ctx *ctx);

/* Solve A u = b (b_dev, u_dev: D, column-major n_dof x nrhs, leading
 * dimension ld >= n_dof, no aliasing).  Column c stops when the projected
 * residual ||P r_c||_2 <= tol ||P r_c^0||_2 or after max_it iterations.
 * info_host (H, nrhs entries, may be NULL): iterations, converged, and the
 * FP64 full-system relative residual ||b - A u|| / ||b||.  DD_ENOCONV if a
 * column missed the tolerance, DD_ENOTSPD on p^T F p <= 0. */
dd_status dd_feti_solve(dd_feti_ctx *ctx, const double *b_dev, double *u_dev, int32_t nrhs, int32_t ld,
                        double tol, int32_t max_it, dd_solve_info *info_host);

/* The primal interface problem S u_G = g (eq. SchurComplement summed over
 * subdomains, eq. subForcing) by CG with the balancing Neumann-Neumann
 * preconditioner, the primal counterpart of the scaled Dirichlet
 * preconditioner of eq. preconditioner (section "Preconditioning"):
 *   M^-1 = P_0 + (I - P_0 S) M_NN (I - S P_0),  M_NN = sum_k R_k^T D_k S_k^+ D_k R_k,
 * D_k = 1 / zeta on Gamma_k, S_k^+ the pseudoinverse of the zeta-weighted
 * subdomain Schur complement (the S^+ blocks of the FETI context), and the
 * coarse space N = [R_k^T D_k Z_k] of the floating subdomains, P_0 = N (N^T S N)^-1 N^T
 * (formed by the first call: S N through the primal product, N^T S N inverted
 * on the host).  Same stopping rule as dd_solve (||r_c|| <= tol ||b_c||, x0 = 0),
 * then eq. backwardSubstitution.  Arguments, layout and info as dd_feti_solve;
 * DD_ENOCONV if a column missed the tolerance, DD_ENOTSPD on p^T S p <= 0 or a
 * coarse matrix that is not positive definite. */
dd_status dd_bdd_solve(dd_feti_ctx *ctx, const double *b_dev, double *u_dev, int32_t nrhs, int32_t ld,
                       double tol, int32_t max_it, dd_solve_info *info_host);

/* Solvers of the same system that share one FETI context. */
typedef enum {
  DD_METHOD_AUTO = 0,    /* the method chosen by dd_method_autotune (tuned on first use) */
  DD_METHOD_FETI = 1,    /* dd_feti_solve: one-level FETI (Algorithm 1) */
  DD_METHOD_BDD = 2,     /* dd_bdd_solve: primal interface CG, balancing Neumann-Neumann */
  DD_METHOD_JACOBI = 3   /* dd_solve (FP64) on the primal context: primal CG, exact diag(S) */
} dd_method;

/* Time the three methods on a seeded batch of nrhs columns (values in [-1, 1))
 * at tolerance tol -- the primal context first autotunes its own schedule --
 * and keep the fastest for DD_METHOD_AUTO.  A method that misses the
 * tolerance within max_it loses.  method (H, may be NULL): the choice; ms (H,
 * 3 entries, may be NULL): ms per batch of FETI, BDD and Jacobi (1e300 for a
 * method that failed to converge).  Allocates two n_dof x nrhs device buffers
 * for the duration of the call. */
dd_status dd_method_autotune(dd_feti_ctx *ctx, int32_t nrhs, double tol, int32_t max_it, int32_t *method,
                             double *ms);

/* Solve with `method` (dd_method); arguments as dd_feti_solve.  Note that the
 * methods stop on their own residuals (FETI: the projected multiplier
 * residual; BDD and Jacobi: the interface residual relative to ||b||); info
 * always reports the full-system relative residual. */
dd_status dd_method_solve(dd_feti_ctx *ctx, int32_t method, const double *b_dev, double *u_dev, int32_t nrhs,
                          int32_t ld, double tol, int32_t max_it, dd_solve_info *info_host);

const char *dd_feti_last_error(const dd_feti_ctx *ctx);
void dd_feti_destroy(dd_feti_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* DD_H */

/*
 * epi.h -- C ABI of the MI355X (gfx950) solver library for reversed-gradient EPI
 * susceptibility-artifact correction on the face-staggered grid.
 *
 * Method: Macdonald & Ruthotto, "Efficient Numerical Optimization for Susceptibility
 * Artifact Correction of EPI-MRI". Section 3 defines the discretised problem, Section 4.1
 * the Gauss-Newton-PCG solver with the block-Jacobi preconditioner, Section 4.2 the ADMM
 * splitting (line-separable b-step solved by SQP with an active-set QP, DCT-diagonalised
 * z-step).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layout. All device arrays are float32 in the canonical layout: the phase-encoding (PE)
 *   axis is contiguous. With cell counts m = (M, m2, m3) (m[0] = PE axis; m3 = 1 in 2D):
 *     cell  (c, j, k), c in [0, M):      index c + M * (j + m2 * k)       (N = M m2 m3)
 *     face  (i, j, k), i in [0, M]:      index i + (M + 1) * (j + m2 * k) (n = (M+1) m2 m3)
 *   Face i of PE line (j, k) sits at PE coordinate i * h[0]; cell c at (c + 1/2) * h[0].
 *   The field b is in physical length units (the same units as h).
 * Ownership. Pointers named d_* are device pointers owned by the caller. epi_setup keeps
 *   borrowed pointers to the two images; they must stay valid and unchanged until
 *   epi_destroy. The problem handle owns its own device workspace.
 * Streams. Every kernel of a handle runs on the hipStream_t given to epi_setup (NULL =
 *   the default stream). Calls that return host scalars synchronise that stream before
 *   returning. One handle must not be used by two host threads at the same time.
 * Errors. No exception crosses the ABI. A non-OK status leaves a message readable with
 *   epi_last_error() (thread-local, valid until the next failing call of that thread).
 *   EPI_EINVAL: bad argument (null pointer, ndim not 2/3, m[a] < 1 or M < 2, h <= 0,
 *   alpha < 0, rho <= 0, a size beyond the limits below). EPI_EINFEASIBLE: the starting
 *   field violates the constraint (|D1 b| < 1 for GN-PCG, |D1 b| <= 1 for ADMM).
 *   EPI_ENUMERIC: NaN/Inf met in the inputs or the iteration. EPI_EHIP: a HIP runtime
 *   error (message carries the HIP error string). EPI_ENOMEM: device allocation failed.
 *   EPI_EBUSY (batched engine): no slot or HBM budget free right now; nothing changed.
 *   Hitting an iteration cap is EPI_OK with converged = 0.
 * Limits. M + 1 <= 512 faces per PE line; m2 <= 256 and m3 <= 256 (the DCT axes).
 */
#ifndef EPI_H_
#define EPI_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EPI_ABI_VERSION 6

typedef enum {
  EPI_OK = 0,
  EPI_EINVAL = 1,
  EPI_ENOMEM = 2,
  EPI_EINFEASIBLE = 3,
  EPI_ENUMERIC = 4,
  EPI_EHIP = 5,
  EPI_ENOTSUP = 6,
  EPI_EBUSY = 7
} epi_status;

/* Arithmetic of the z-step DCT products. FP32: float32 matrix-core products (the plain
 * single-precision solver). MIXED: three-term split-bfloat16 products (hi*hi + hi*lo +
 * lo*hi, float32 accumulation). Everything else is float32 with float64 reductions in
 * both modes. */
typedef enum { EPI_PREC_FP32 = 0, EPI_PREC_MIXED = 1 } epi_precision;

/* Preconditioner of the GN-PCG inner solve (Section 4.1): block-Jacobi (eq. Pblock; one
 * SPD tridiagonal system per PE line), Jacobi (diagonal of H_JGN), none, or symmetric
 * Gauss-Seidel (eq. Psgs) in the face order i + (M+1)(j + m2 k). SGS is sequential by
 * construction: its two sweeps take m2 + m3 - 1 dependent launches each. */
typedef enum {
  EPI_PRECOND_BLOCK = 0,
  EPI_PRECOND_JACOBI = 1,
  EPI_PRECOND_NONE = 2,
  EPI_PRECOND_SGS = 3
} epi_precond;

/* Continuous model of each image along the phase-encoding axis (Section 3 discretises with
 * linear interpolation; Section 5 compares against a smoothed cubic B-spline model).
 * LINEAR: I(s) interpolates the cell-centred samples linearly, zero outside the volume.
 * SPLINE: I(s) = sum_k w_k beta3(s - k) over the line's M cell centres (zero coefficients
 * outside), with w the solution of (B'B + theta G) w = B' T per PE line, B the collocation
 * matrix of beta3 at the samples and G the Gram matrix of the second derivatives
 * (theta = 0: B w = T, interpolation). The coefficients are computed once at setup. */
typedef enum { EPI_IMAGE_LINEAR = 0, EPI_IMAGE_SPLINE = 1 } epi_image_model;

/* Problem geometry and weights (Section 3). h = voxel edges (h[2] = 1 in 2D); the cell
 * volume v = h[0] h[1] h[2] plays the role of the paper's h^3. alpha weights the
 * smoothness regulariser S, beta the penalty P (default 10), gamma the identity shift of
 * the approximate Hessians (default 1e-3, unscaled). image_model (epi_image_model,
 * default LINEAR) and theta (>= 0, the smoothing weight of the SPLINE model in grid units,
 * default 0) select the image model; the batched engine takes LINEAR only. */
typedef struct {
  int32_t ndim;
  int32_t m[3];
  double h[3];
  double alpha;
  double beta;
  double gamma;
  int32_t precision;   /* epi_precision */
  int32_t image_model; /* epi_image_model */
  double theta;
} epi_grid;

/* Objective terms at a field b: J = D + alpha S (+ P when the penalty is requested).
 * D = (v/2)|r(b)|^2 (eq. D), S = (v/2)(|D1 b|^2 + |D2 b|^2 + |D3 b|^2) (eq. S),
 * P = beta v sum phi(D1 b) (eq. P). feasible = 1 iff every |D1 b| < 1 (P finite). */
typedef struct {
  double J, D, S, P;
  int32_t feasible;
} epi_terms;

/* GN-PCG options (Section 4.1). Defaults from epi_gn_default_opts: max_iter 10,
 * pcg_max 30, precond BLOCK, ls_max 10, use_stopping 1, eta 0.1 (eq. inexactGNsolve),
 * eps_obj 1e-3, eps_iter 1e-2, eps_grad 1e-2 (eq. stopping1), ls_c1 1e-4 (Armijo),
 * rel_grad_tol 0 (off; > 0 also stops when |grad| <= rel_grad_tol |grad at b0|). */
typedef struct {
  int32_t max_iter, pcg_max, precond, ls_max, use_stopping;
  double eta, eps_obj, eps_iter, eps_grad, ls_c1, rel_grad_tol;
} epi_gn_opts;

/* GN-PCG report. The arrays are host arrays owned by the caller, each of length
 * max_iter + 1 (J, grad_norm: entry 0 is the starting point) or max_iter (the others);
 * any of them may be NULL. iters = GN steps taken; ls_failed = 1 if the last step found
 * no sufficient decrease in ls_max trials (the iteration stops there, b unchanged). */
typedef struct {
  int32_t iters, converged, status, ls_failed;
  double *J, *grad_norm, *pcg_relres, *step;
  int32_t *pcg_iters;
} epi_gn_report;

/* Penalty parameter strategy of ADMM (Section 4.3, the adaptive choice of rho by residual
 * balancing): FIXED keeps rho; ADAPT multiplies rho by tau when the primal residual
 * exceeds mu times the dual residual and divides it by tau in the opposite case;
 * ADAPT_FLOOR does the same but skips a decrease that would take rho below rho_min. On a
 * change the scaled dual u = y / (rho v) is rescaled by rho_old / rho_new (y unchanged). */
enum { EPI_RHO_FIXED = 0, EPI_RHO_ADAPT = 1, EPI_RHO_ADAPT_FLOOR = 2 };

/* ADMM options (Section 4.2). Defaults from epi_admm_default_opts: max_iter 100,
 * sqp_iters 1 (linearisations per b-step), check_every 8 (iterations between host polls
 * of the device-side stopping flag; results do not depend on it), rho 1e3,
 * eps_abs = eps_rel = 0.2 (eq. admmStop), rho_mode EPI_RHO_FIXED, tau 1.3, mu 10,
 * rho_min 1e2, qp_max_iter 0 (the cap on active-set iterations of one line's QP, eq. qp;
 * 0 means 4 (M + 1)), with_lagrangian 0 (1: record the augmented Lagrangian of eq. Lp at
 * every iterate, which costs two objective evaluations and a dot product per iteration;
 * epi_solve_admm and epi_profile_admm only). */
typedef struct {
  int32_t max_iter, sqp_iters, check_every;
  double rho, eps_abs, eps_rel;
  int32_t rho_mode;
  double tau, mu, rho_min;
  int32_t qp_max_iter, with_lagrangian;
} epi_admm_opts;

/* ADMM report. Host arrays of length max_iter owned by the caller (NULL allowed):
 * per-iteration primal residual |b - z|, dual residual rho v |z_k - z_k+1| and their
 * tolerances (eq. admmStop, newest iterates), the rho each iteration used and, when
 * opts.with_lagrangian is set, the augmented Lagrangian
 * L_rho(b, z, y) = f(b) + g(z) + y'(b - z) + (rho v / 2)|b - z|^2 of eq. Lp at the
 * iteration's result (y = rho v u, f = D + (alpha v / 2)|D1 b|^2 on the feasible set,
 * g = (alpha v / 2)(|D2 z|^2 + |D3 z|^2); left untouched otherwise).
 * max_active = largest number of active constraints of one PE line at exit of any
 * b-step; hard_lines = total count of (iteration, line) pairs that needed more than the
 * unconstrained step. */
typedef struct {
  int32_t iters, converged, status, max_active;
  int64_t hard_lines;
  double *r_pri, *r_dual, *eps_pri, *eps_dual, *rho, *lagrangian;
} epi_admm_report;

/* Kernel families of one ADMM iteration, for epi_profile_admm. */
enum {
  EPI_K_BSTEP = 0,       /* b-step, unconstrained fast path (all lines)            */
  EPI_K_BSTEP_HARD = 1,  /* b-step, active-set path (lines that need it)            */
  EPI_K_DCT_AXIS3 = 2,   /* z-step DCT along the third axis (forward)              */
  EPI_K_DCT_AXIS2 = 3,   /* z-step DCT along the second axis, scaled, inverse       */
  EPI_K_DCT_LAST = 4,    /* last z-step pass with the u-step epilogue              */
  EPI_K_FINALIZE = 5,    /* float64 residual norms and stopping test               */
  EPI_K_COUNT = 6
};

/* Per-kernel-family device time of a profiled ADMM solve (milliseconds, HIP events on
 * the library's stream around every launch) and the number of launches. The pair of
 * events around each launch adds the launch latency to every interval, so the profile also
 * carries a back-to-back figure: after the solve, each family is launched isolated_reps
 * times in a row (no event in between) on a copy of the final state, with the stopping
 * test disabled, and us_isolated is the average device time per launch from one event
 * pair around the whole run (0 for a family the problem does not have). */
typedef struct {
  double ms[8];
  int64_t launches[8];
  double us_isolated[8];
  int32_t isolated_reps;
} epi_kernel_profile;

typedef struct epi_problem epi_problem;

/* Library ABI version (EPI_ABI_VERSION). */
int32_t epi_abi_version(void);

/* Fill option structs with the paper's defaults (see above). */
void epi_gn_default_opts(epi_gn_opts* opts);
void epi_admm_default_opts(epi_admm_opts* opts);

/* Create a problem handle for the image pair I_v (d_Iplus) and I_-v (d_Iminus), each N
 * floats in canonical cell layout (Section 3, the discrete distance eq. D). stream is a
 * hipStream_t (or NULL). Allocates the device workspace and the DCT tables; checks the
 * images for NaN/Inf (EPI_ENUMERIC). On success *out owns the workspace; release it with
 * epi_destroy. */
epi_status epi_setup(const epi_grid* grid, const float* d_Iplus, const float* d_Iminus,
                     void* stream, epi_problem** out);

/* Bytes of the static device scratch of epi_objective_noalloc: float64 partial sums, 48
 * bytes per four PE lines, so at most 43,688 PE lines (m2 m3) per call (240 x 200 x 110
 * with the PE axis first has 22,000). */
#define EPI_NOALLOC_SCRATCH_BYTES (1 << 19)

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the objective terms of epi_objective
 * without a problem handle and without any device allocation. grid, images and field as
 * for epi_setup and epi_objective (device pointers, canonical layout, caller-owned).
 * d_terms: caller-owned device array of 5 doubles that receives J, D, S, P and the
 * feasibility flag (1.0 iff every |D1 b| < 1; P = +inf otherwise when with_penalty != 0).
 * d_grad: NULL or n floats for grad J / grad J_GN. Everything is enqueued on stream
 * (a hipStream_t or NULL) and the call returns without synchronising. The partial sums
 * live in a static device array of EPI_NOALLOC_SCRATCH_BYTES per GPU, held until the
 * process ends; its address is looked up once per device. Calls that overlap on one GPU
 * (several streams or host threads) share that array and race. EPI_EINVAL for a grid
 * whose line count exceeds the scratch; EPI_ENOTSUP for the SPLINE image model (its
 * coefficients come from epi_setup). The images are not checked for NaN/Inf. */
epi_status epi_objective_noalloc(const epi_grid* grid, const float* d_Iplus,
                                 const float* d_Iminus, const float* d_b, int32_t with_penalty,
                                 double* d_terms, float* d_grad, void* stream);

/* Quality of a field estimate: the SSD distance D of the corrected pair (eq. D), the
 * normalised cross-correlation of the two corrected images and their means. */
typedef struct {
  double D, ncc, mean_plus, mean_minus;
} epi_quality;

/* Distortion-corrected images at the field d_b (n floats): I_v(x + A b)(1 + D1 b) into
 * d_Iplus_corr and I_-v(x - A b)(1 - D1 b) into d_Iminus_corr, N floats each in canonical
 * cell layout, caller-owned (both NULL: quality only; one NULL: EPI_EINVAL). They follow
 * the model relation of Section 2 (eq. (1)) as discretised in Section 3; at an exact field
 * they coincide with the undistorted image. Synchronises the stream. */
epi_status epi_corrected_images(epi_problem* p, const float* d_b, float* d_Iplus_corr,
                                float* d_Iminus_corr, epi_quality* out);

/* Evaluate the objective terms at d_b (n floats): D, S and, if with_penalty != 0, P
 * (eq. D, eq. S, eq. P). If d_grad is not NULL it receives grad J (with_penalty = 0) or
 * grad J_GN (with_penalty != 0), n floats (eq. dJ, eq. dJGN). Synchronises the stream. */
epi_status epi_objective(epi_problem* p, const float* d_b, int32_t with_penalty,
                         epi_terms* out, float* d_grad);

/* The non-separable smoothness solve of the ADMM z-step (Section 4.2, eq. dctdiag):
 * d_z = (alpha v (D2'D2 + D3'D3) + rho v I)^{-1} rho v d_w, by the orthonormal 2D DCT over
 * the two non-PE axes in the arithmetic of grid->precision. In split-bfloat16 the
 * j-axis forward, spectral scale and inverse of each k-slice are applied as one product
 * with a per-slice operator built on the device for this rho (rebuilt, tens of
 * microseconds, when rho differs from the last call's). d_w and d_z are n floats and may
 * alias. Does not synchronise. */
epi_status epi_smooth_solve(epi_problem* p, const float* d_w, double rho, float* d_z);

/* One application of a GN-PCG preconditioner (Section 4.1, eq. Pblock, eq. Psgs) built
 * from H_JGN at the field d_b: d_z = P^{-1} d_r. d_b, d_r, d_z are n floats in canonical
 * face layout, caller-owned; d_z must not alias d_r or d_b. precond is an epi_precond.
 * EPI_EINVAL for an unknown precond or aliasing buffers; EPI_EINFEASIBLE if some
 * |D1 b| >= 1 (the penalty Hessian is not defined there). Synchronises the stream. */
epi_status epi_precond_apply(epi_problem* p, const float* d_b, int32_t precond,
                             const float* d_r, float* d_z);

/* Inexact Gauss-Newton-PCG on J_GN = D + alpha S + P (Section 4.1, eq. GNstep,
 * eq. inexactGNstep): d_b holds the starting guess on entry (must satisfy |D1 b| < 1) and
 * the result on exit. The PCG inner solve, Armijo line search and stopping tests run on
 * the device; the host reads one report row per GN step. */
epi_status epi_solve_gnpcg(epi_problem* p, float* d_b, const epi_gn_opts* opts,
                           epi_gn_report* rep);

/* Scaled ADMM (Section 4.2, eq. admmStep1-3): d_b, d_z, d_u (n floats each) hold the
 * state (b^k, z^k, u^k) on entry and on exit, so a solve can be resumed by calling again.
 * The starting b must satisfy |D1 b| <= 1. Every iteration runs as a fixed kernel
 * sequence with a device-side stopping flag (eq. admmStop, float64 norms); kernels after
 * convergence are no-ops, so the state on exit is the state at the stopping iteration.
 * With a fixed rho in split-bfloat16 the z-step uses the per-slice operators described at
 * epi_smooth_solve (built at the start of the solve when rho changed). */
epi_status epi_solve_admm(epi_problem* p, float* d_b, float* d_z, float* d_u,
                          const epi_admm_opts* opts, epi_admm_report* rep);

/* ---- Multilevel strategy (Section 4.4) ------------------------------------------------
 * Grid transfer between a fine grid and a coarse grid whose cell counts are equal or half
 * on every axis (m_fine[a] = m_coarse[a] or 2 m_coarse[a], canonical order PE first).
 * Restriction of cell data (N floats): each coarse cell is the mean of its fine cells.
 * Prolongation of a field on the PE faces (n floats): linear along PE (fine face 2i on the
 * coarse face i, 2i + 1 at the midpoint), cell-centred weights 3/4 and 1/4 across (the
 * farther neighbour clamped at the ends). Both are asynchronous on stream; EPI_EINVAL for
 * sizes that are not such a pair. */
epi_status epi_restrict_cells(const int32_t m_fine[3], const int32_t m_coarse[3],
                              const float* d_fine, float* d_coarse, void* stream);
epi_status epi_prolong_faces(const int32_t m_coarse[3], const int32_t m_fine[3],
                             const float* d_coarse, float* d_fine, void* stream);

#define EPI_ML_MAX_LEVELS 8

/* Per-level outcome of a multilevel solve (index 0 = coarsest level). ADMM: iterations,
 * convergence, fallback[l] = 1 if the third restart's average violated |D1 b| <= 1 and
 * b0 = P b_c was used instead, rho of the last iteration. GN-PCG: GN steps, convergence and
 * the final J_GN of the level (J_last). */
typedef struct {
  int32_t levels;
  int32_t m[EPI_ML_MAX_LEVELS][3];
  int32_t iters[EPI_ML_MAX_LEVELS], converged[EPI_ML_MAX_LEVELS], fallback[EPI_ML_MAX_LEVELS];
  double rho_last[EPI_ML_MAX_LEVELS];
  double J_last[EPI_ML_MAX_LEVELS];
} epi_ml_report;

/* How ADMM restarts on a finer level from the coarse result (b_c, z_c, u_c), the three
 * strategies of Section 4.4 (P = epi_prolong_faces): PROLONG_ALL: b0 = P b_c, z0 = P z_c,
 * u0 = P u_c; FINE_B: b0 = z0 = P b_c, u0 = 0; AVERAGE (the paper's choice):
 * b0 = z0 = P((b_c + z_c) / 2), u0 = 0, with b0 = P b_c if that average is infeasible. */
enum { EPI_ML_RESTART_PROLONG_ALL = 1, EPI_ML_RESTART_FINE_B = 2, EPI_ML_RESTART_AVERAGE = 3 };

/* Coarse-to-fine ADMM (Section 4.4) for the image pair of grid (the finest level): up to
 * `levels` levels, every axis with an even count >= 4 halved per level (fewer levels when
 * no axis can be halved), images restricted level by level, ADMM from b = z = u = 0 on the
 * coarsest level with opts, each finer level started by `restart` (an EPI_ML_RESTART_*
 * value); rho carries over between levels. The finest field is written to d_b (n floats,
 * caller-owned). Allocates and frees the coarse levels' memory; synchronises stream.
 * EPI_EINVAL for levels outside [1, EPI_ML_MAX_LEVELS] or an unknown restart. */
epi_status epi_solve_multilevel_admm(const epi_grid* grid, const float* d_Iplus,
                                     const float* d_Iminus, int32_t levels, int32_t restart,
                                     const epi_admm_opts* opts, void* stream, float* d_b,
                                     epi_ml_report* rep);

/* Coarse-to-fine GN-PCG (Section 4.4: the prolongated coarse field is the finer level's
 * starting guess): GN-PCG with opts from b = 0 on the coarsest level, then from
 * P b_c on each finer level (feasible: prolongation keeps the coarse D1 b values along PE
 * and mixes lines convexly across). Levels and memory as for epi_solve_multilevel_admm. */
epi_status epi_solve_multilevel_gnpcg(const epi_grid* grid, const float* d_Iplus,
                                      const float* d_Iminus, int32_t levels,
                                      const epi_gn_opts* opts, void* stream, float* d_b,
                                      epi_ml_report* rep);

/* The same solve as epi_solve_admm (same kernels in the same order, same results),
 * launched one kernel at a time without the captured graph, with a pair of HIP events
 * around every kernel on the library's stream. prof receives the device time per kernel
 * family and, when prof->isolated_reps > 0 on entry, the back-to-back launch times
 * described at epi_kernel_profile (the caller's arrays are not touched by that part; it
 * works on the handle's GN work vectors). For measurement tools; slower than
 * epi_solve_admm by the launch overhead. */
epi_status epi_profile_admm(epi_problem* p, float* d_b, float* d_z, float* d_u,
                            const epi_admm_opts* opts, epi_admm_report* rep,
                            epi_kernel_profile* prof);

/* ------------------------------------------------------------------------------------
 * Continuous-batching ADMM engine: the served form of the Section 4.2 solver. Up to
 * max_slots volumes of different sizes (and 2D/3D) are resident at once; one ADMM
 * iteration of all running volumes is one persistent launch per kernel class over their
 * PE lines and DCT tiles, captured in a hipGraph; each volume has its own stopping flag
 * (eq. admmStop) and iteration cap, and a volume's arithmetic does not depend on the other
 * volumes in the batch. Finished volumes free their slot for new requests (continuous
 * batching). All volumes of one batch use one z-step precision.
 * ------------------------------------------------------------------------------------ */
typedef struct epi_batch epi_batch;

/* Create an engine with max_slots (<= 128) slots, an admission limit hbm_budget_bytes on
 * the summed epi_batch_footprint of resident volumes, the z-step precision
 * (epi_precision) and iters_per_step ADMM iterations per epi_batch_step call. Kernels
 * run on a private stream ordered after `stream` (a hipStream_t or NULL). */
epi_status epi_batch_create(int32_t max_slots, int64_t hbm_budget_bytes, int32_t precision,
                            int32_t iters_per_step, void* stream, epi_batch** out);

/* Device bytes one request occupies while resident: its images and state arrays
 * (borrowed from the caller) plus the workspace the engine allocates for it (three n-float
 * arrays, DCT tables, partial sums, residual histories). -1 for a NULL grid. */
int64_t epi_batch_footprint(const epi_grid* grid, int32_t max_iter);

/* Admit one request: geometry and weights (grid; its precision field is replaced by the
 * engine's), the image pair (N floats each, canonical layout), and its ADMM state arrays
 * d_b, d_z, d_u (n floats each, caller-owned, read and written in place until the slot
 * is released; |D1 b| <= 1 required, else EPI_EINFEASIBLE). opts: rho, eps_abs, eps_rel,
 * max_iter, rho_mode (with tau, mu, rho_min) and qp_max_iter as for epi_solve_admm
 * (sqp_iters must be 1 and with_lagrangian 0; check_every is not used). On
 * success *slot is the slot index. EPI_EBUSY: no free slot or not enough budget. */
epi_status epi_batch_admit(epi_batch* bt, const epi_grid* grid, const float* d_Iplus,
                           const float* d_Iminus, float* d_b, float* d_z, float* d_u,
                           const epi_admm_opts* opts, int32_t* slot);

/* Run iters_per_step ADMM iterations of every running volume (one graph replay; volumes
 * admitted since the last call join here), synchronise, and report in *running how many
 * volumes are still iterating. The graph is captured again only when the running set
 * needs a kernel class or launch width the captured graph lacks, or when a class's work
 * falls below half of its captured width (surplus workgroups return at once). */
epi_status epi_batch_step(epi_batch* bt, int32_t* running);

/* *finished = 1 once the slot's volume has converged or reached max_iter; then rep (may
 * be NULL) receives the report and histories as from epi_solve_admm. */
epi_status epi_batch_poll(epi_batch* bt, int32_t slot, int32_t* finished, epi_admm_report* rep);

/* Free a slot (finished or not): its footprint leaves the budget and its workspace goes
 * to the engine's cache of at most max_slots workspaces (the oldest cached one is freed
 * when the cache is full). A later admission takes the smallest cached workspace that is
 * large enough, keeping its DCT tables when the transverse grid matches and its per-slice
 * operators when grid, alpha and rho match, so requests of recurring sizes are admitted
 * without device allocation. The caller's arrays are not touched. */
epi_status epi_batch_release(epi_batch* bt, int32_t slot);

/* Counters of the engine since creation: admissions, admissions that had to allocate a
 * new workspace, and captures of the iteration graph (one per change of the set of kernel
 * classes or launch widths that the captured graph cannot cover). */
epi_status epi_batch_stats(const epi_batch* bt, int64_t* admissions,
                           int64_t* admissions_allocating, int64_t* graph_captures);

/* Destroy the engine and every slot's workspace (NULL is a no-op). */
void epi_batch_destroy(epi_batch* bt);

/* ------------------------------------------------------------------------------------
 * Request loop of the served solver: a FIFO of requests in front of one engine. The
 * caller submits each request when it arrives (with its arrival time on
 * epi_server_clock()) and calls epi_server_progress repeatedly; finished requests are
 * collected with epi_server_take. Results are those of the engine (epi_batch_*), so a
 * request's result does not depend on what else is in flight.
 * ------------------------------------------------------------------------------------ */
typedef struct epi_server epi_server;

/* Seconds on the monotonic clock the server stamps admissions and completions with. */
double epi_server_clock(void);

/* Create a server around a new engine (arguments as for epi_batch_create). */
epi_status epi_server_create(int32_t max_slots, int64_t hbm_budget_bytes, int32_t precision,
                             int32_t iters_per_step, void* stream, epi_server** out);

/* Queue one request (arguments as for epi_batch_admit; the caller's arrays must stay
 * valid until the request has been taken). request_id is the caller's tag; arrival_s its
 * arrival time on epi_server_clock(). Never EPI_EBUSY: the request waits in the queue. */
epi_status epi_server_submit(epi_server* sv, int64_t request_id, double arrival_s,
                             const epi_grid* grid, const float* d_Iplus, const float* d_Iminus,
                             float* d_b, float* d_z, float* d_u, const epi_admm_opts* opts);

/* Admit queued requests in arrival order while a slot and HBM budget are free, run one
 * engine step (iters_per_step ADMM iterations of every running volume) if anything is
 * running, move finished volumes to the completed list (releasing their slots) and admit
 * again. Reports the number of queued, running and completed-but-not-taken requests (any
 * pointer may be NULL). A request the engine rejects (EPI_EINFEASIBLE, EPI_EINVAL)
 * completes at once with that status; a request that cannot fit even into an idle engine
 * makes this call fail with EPI_ENOMEM. */
epi_status epi_server_progress(epi_server* sv, int32_t* queued, int32_t* running,
                               int32_t* ready);

/* Take the oldest completed request: its tag, its latency (completion minus arrival,
 * seconds) and, if rep is not NULL, its report as epi_batch_poll gives it (arrays of the
 * request's max_iter entries, caller-owned, each may be NULL; lagrangian is not used).
 * EPI_EBUSY when no request has completed. */
epi_status epi_server_take(epi_server* sv, int64_t* request_id, double* latency_s,
                           epi_admm_report* rep);

/* Destroy the server and its engine (NULL is a no-op). Requests still queued or running
 * are dropped; their arrays are not touched. */
void epi_server_destroy(epi_server* sv);

/* Release the handle and its workspace (NULL is a no-op). */
void epi_destroy(epi_problem* p);

/* Message of the calling thread's last failing call ("" if none). */
const char* epi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EPI_H_ */

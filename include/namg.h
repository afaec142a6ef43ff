/* namg — Neumann-series GMRES + classical AMG for AMD Instinct MI355X (gfx950).
 *
 * The solve phase of "Neumann Series in GMRES and Algebraic Multigrid Smoothers" (Thomas, Carr,
 * Mullowney, Li, Swirydowicz; arXiv 2112.14681): Ax = b (Section 1) is solved by a restarted,
 * right-preconditioned flexible low-synchronization MGS-GMRES whose correction matrix is applied as
 * T = I - L (Section 4, Algorithm 1), preconditioned by one classical Ruge-Stueben AMG V-cycle
 * (Section 5) whose polynomial Gauss-Seidel (Section 5.2) and ILU(0) (Section 5.3) smoothers replace
 * the sparse triangular solves by truncated Neumann-series / Jacobi inner iterations.
 *
 * Conventions for every call:
 *  - Return value: NAMG_OK (0), NAMG_NOT_CONVERGED (1, a status: outputs are valid) or a negative
 *    error code. On error, namg_last_error() returns a message for the calling thread.
 *  - Host arrays are borrowed for the duration of the call and copied where kept.
 *  - "_dev" pointers are device pointers on the hierarchy's device, contiguous, float64, caller-owned.
 *  - stream is a hipStream_t (NULL = the default stream). A hierarchy is used by one stream at a time.
 *  - CSR: 0-based, int32 row pointers and column indices, columns strictly ascending per row, the
 *    diagonal present and nonzero, finite values, nnz < 2^31.
 */
#ifndef NAMG_H
#define NAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NAMG_OK 0
#define NAMG_NOT_CONVERGED 1
#define NAMG_PENDING 2
#define NAMG_E_INVALID (-1)    /* bad argument or malformed CSR */
#define NAMG_E_ZERO_PIVOT (-2) /* zero diagonal in A, a coarse operator, an ILU pivot or the coarse LU */
#define NAMG_E_NONFINITE (-3)  /* NaN/Inf in the input or during the solve */
#define NAMG_E_NOMEM (-4)      /* device allocation failed (nothing leaked) */
#define NAMG_E_HIP (-5)        /* other HIP runtime error */
#define NAMG_E_BUDGET (-6)     /* serving: request larger than the whole HBM budget */
#define NAMG_E_NODEVICE (-7)   /* the hierarchy was set up host-only (device = -1) */

enum { NAMG_FP64 = 0, NAMG_FP32_PRECOND = 1 };        /* namg_setup_params.precision */
enum { NAMG_SMOOTH_PGS = 0, NAMG_SMOOTH_ILU0 = 1, NAMG_SMOOTH_L1JAC = 2 }; /* namg_solve_params.smoother */
enum { NAMG_TRI_NEUMANN = 0, NAMG_TRI_DIRECT = 1 };   /* namg_solve_params.tri_mode  */
enum { NAMG_T_NEUMANN = 0, NAMG_T_DIRECT = 1 };       /* namg_solve_params.gmres_T   */
enum { NAMG_STOP_RELRES = 0, NAMG_STOP_NRBE = 1 };    /* namg_solve_params.stop_rule */
enum { NAMG_ILU0 = 0, NAMG_ILUT = 1 };                /* namg_setup_params.ilu_kind  */
enum { NAMG_COARSEN_RS = 0, NAMG_COARSEN_PMIS = 1 };  /* namg_setup_params.coarsen   */
enum { NAMG_DIAG_LOSS_ORTH = 1, NAMG_DIAG_PHASE_TIMES = 2 }; /* namg_solve_params.diagnostics (bitmask) */

#define NAMG_MAX_LEVELS 32
#define NAMG_MAX_RESTART 128

typedef struct namg_hier namg_hier; /* opaque; owns the host copy and all device memory of one hierarchy */

typedef struct {
  double theta;   /* strength threshold, 0 < theta <= 1 (Section 5.1); default 0.25 */
  int max_levels; /* <= NAMG_MAX_LEVELS; default 25 */
  int max_coarse; /* stop coarsening at <= max_coarse rows (dense direct solve); default 50 */
  int precision;  /* NAMG_FP64, or NAMG_FP32_PRECOND: hierarchy values and the V-cycle in FP32,
                     Arnoldi / Hessenberg / true residual in FP64 */
  int ilu_levels; /* ILU factors on levels l < ilu_levels (1 = finest only, the hybrid V-cycle of
                     Section 6.2; -1 = every level but the coarsest; 0 = none); default 1 */
  int device;     /* HIP device ordinal; -1 = host-only setup (for inspection; solves are refused) */
  int ilu_kind;   /* NAMG_ILU0 (default): ILU(0) on A's pattern; NAMG_ILUT: ILUT(ilut_droptol, ilut_lfil),
                     the threshold factorization of Algorithm 2 (Section 5.3.4) with Saad's dual rule:
                     with tau_i = ilut_droptol * ||a_i||_2, multipliers below tau_i are dropped during the
                     elimination of row i, then off-diagonal entries below tau_i, and at most ilut_lfil
                     entries of largest magnitude stay in each strict triangle of the row (ties: smaller
                     column). The smoother applies either factor the same way (row scaling D_U = diag(U)) */
  int ilut_lfil;  /* >= 0; default 5 */
  double ilut_droptol; /* >= 0; default 1e-2 */
  int agg_levels; /* aggressive (A-1) coarsening on levels l < agg_levels (Section 5.1; the paper's runs use
                     2), default 0: a second first pass over the C points with the distance-two strength
                     (paths of at most two strong connections) keeps C_2; P = P_1 P_2 with P_2 the classical
                     interpolation of A_1 = P_1^T A P_1 onto C_2, and A_c = P_2^T A_1 P_2 */
  int coarsen;    /* NAMG_COARSEN_RS (default): host setup, Ruge-Stueben first pass and classical
                     interpolation. NAMG_COARSEN_PMIS: setup on `device`, PMIS coarsening (Section 5.1; weights
                     |S^T_i| + u_i, u_i the (i+1)-th SplitMix64 output of the stream seeded with seed + l on
                     level l, top 53 bits in [0, 1)) with BAMG direct interpolation
                     w_ij = -(a_ij + beta_i / n_i) / (a_ii + sum of the weak a_ik), beta_i the sum over
                     strong F neighbours; not with agg_levels > 0 */
  uint64_t seed;  /* PMIS stream seed; default 0 */
} namg_setup_params;

typedef struct {
  double tol;      /* stop when the quantity stop_rule names is <= tol; default 1e-8 */
  int restart;     /* m, 1..NAMG_MAX_RESTART; default 30 */
  int max_iters;   /* total Arnoldi iterations over all cycles; default 1000 */
  int smoother;    /* NAMG_SMOOTH_PGS (all levels), NAMG_SMOOTH_ILU0 (ILU on the levels that carry
                      factors, polynomial GS elsewhere) or NAMG_SMOOTH_L1JAC (the l1-Jacobi comparator of
                      Section 6, Table 6, on all levels: x += D_l1^{-1}(b - A x), (D_l1)_ii = sum_j |a_ij|;
                      tri_mode and inner_terms do not apply) */
  int tri_mode;    /* NAMG_TRI_NEUMANN (Jacobi/Neumann inner iterations) or NAMG_TRI_DIRECT (the
                      direct-triangular comparators: GS and ILU by substitution) */
  int inner_terms; /* t >= 1: Neumann terms per triangular solve (t = 1: Jacobi; t - 1 products with the
                      strict triangle); default 2 */
  int gmres_T;     /* NAMG_T_NEUMANN: T = I - L (Section 4); NAMG_T_DIRECT: T = (I + L)^{-1} */
  int pre_sweeps, post_sweeps; /* smoothing sweeps nu1, nu2 per level; default 1, 1 */
  int t_degree;    /* with NAMG_T_NEUMANN: T = sum_{j=0..p} (-L)^j, the Neumann series of (I + L)^{-1}
                      truncated at degree p (Section 1); 1 <= p <= NAMG_MAX_RESTART, default 1 (I - L) */
  int stop_rule;   /* NAMG_STOP_RELRES (default): ||b - A x||_2 / ||b||_2 (Section 4); NAMG_STOP_NRBE: the
                      normwise relative backward error ||b - A x||_2 / (||b||_2 + ||A||_inf ||x||_2) of
                      Section 3. Inside a restart cycle the residual norm is the Arnoldi estimate and ||x||
                      is that of the cycle's starting iterate (x is formed at the cycle's end); every cycle
                      starts with the true residual. The rule changes only when the iteration stops. */
  int diagnostics; /* bitmask, default 0. NAMG_DIAG_LOSS_ORTH: at every cycle end the Gram matrix of the cycle's
                      Krylov basis V_{k+1} (its last column normalised by its own norm) is reduced on the
                      device and namg_solve_stats.loss_orth reports the largest ||I - V^T V||_F over the cycles
                      (Section 3); costs k + 1 extra passes over V per cycle. NAMG_DIAG_PHASE_TIMES: hipEvents
                      around each phase of every Arnoldi step fill ms_vcycle, ms_spmv and ms_ortho */
  double *res_hist; /* optional host array (caller-owned, NULL = none): res_hist[j] receives the residual
                       estimate |g_{j+1}| / ||b|| after iteration j + 1 of the solve, for j < res_hist_cap */
  int res_hist_cap;
} namg_solve_params;

typedef struct {
  int status, iters, cycles, precond_apps;
  double relres_true; /* ||b - A x|| / ||b|| recomputed in FP64 at the end */
  double relres_est;  /* the last Givens estimate |g_{i+1}| / ||b|| */
  double nrbe;        /* ||r|| / (||b|| + ||A||_inf ||x||), Section 3 */
  double ms_total;    /* wall time of the call on the stream (hipEvent) */
  double alg_bytes;   /* algorithmic HBM bytes moved by the solve's kernels */
  double loss_orth;   /* largest ||I - V^T V||_F over the restart cycles; NaN unless NAMG_DIAG_LOSS_ORTH */
  double ms_vcycle;   /* summed device time of the preconditioner applications (V-cycles) */
  double ms_spmv;     /* summed device time of the FP64 products w = A z */
  double ms_ortho;    /* summed device time of the orthogonalisation: fused reduction, small dense step,
                         projection and column completion. The three are NaN unless NAMG_DIAG_PHASE_TIMES */
} namg_solve_stats;

typedef struct {
  int levels;
  int32_t n[NAMG_MAX_LEVELS];
  int64_t nnz[NAMG_MAX_LEVELS];
  double op_complexity, grid_complexity;
  int64_t device_bytes; /* device memory held by the hierarchy and its Krylov workspace */
} namg_hierarchy_info;

void namg_default_setup_params(namg_setup_params *p);
void namg_default_solve_params(namg_solve_params *p);

/* AMG setup (Section 5 and 5.1): per level the strength graph S (|a_ij| >= theta max_{k!=i}|a_ik|), the
 * Ruge-Stueben first-pass C/F splitting, classical interpolation P, R = P^T and the Galerkin operator
 * A_{l+1} = P^T A_l P; ILU(0) or ILUT of the first ilu_levels levels (Section 5.3); the coarsest level's dense
 * inverse. Runs on the host in FP64, then uploads (FP64 or FP32 copies) to p->device.
 * rowptr/colind/vals: host CSR of A (n rows). *out receives a new handle (release with namg_destroy).
 * Errors: NAMG_E_INVALID, NAMG_E_NONFINITE, NAMG_E_ZERO_PIVOT, NAMG_E_NOMEM, NAMG_E_HIP. */
int namg_setup(int32_t n, const int32_t *rowptr, const int32_t *colind, const double *vals,
               const namg_setup_params *p, namg_hier **out);

/* Solve A x = b (Section 1) with low-synchronization flexible GMRES(m) (Section 4, Algorithm 1) and one
 * V-cycle per preconditioner application. b_dev: n float64 (read). x_dev: n float64, the initial guess on
 * entry and the solution on return (overwritten in place). st: optional statistics.
 * Returns NAMG_OK or NAMG_NOT_CONVERGED (x holds the last iterate), or an error. */
int namg_solve(namg_hier *h, const double *b_dev, double *x_dev, const namg_solve_params *p, void *stream,
               namg_solve_stats *st);

/* For callers that cannot allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc): namg_solve with the same arguments, kernels and results (bit for bit),
 * but its Krylov workspace comes from a static per-device array of NAMG_NOALLOC_SCRATCH_BYTES that the
 * library holds on every device it runs on until the process ends, not from the hierarchy's own buffers;
 * the call makes no hipMalloc, hipFree or other allocating call. The workspace for n rows and restart m,
 * with ld = n rounded up to a multiple of 64, nb = the multi-dot's block count (at most 512) and
 * s = 8 (FP64) or 4 (FP32_PRECOND), is the sum of these parts, each rounded up to 256 bytes:
 *   8 ld (m+2) [V], s ld m [Z], 8 n [w], (FP32_PRECOND only) 4 n, 16 nb (m+2), 16 (m+2).
 * A larger workspace is refused with NAMG_E_INVALID before any work is issued (at m = 30 up to 532 032 rows
 * fit in FP64, 691 136 with FP32_PRECOND), as are diagnostics != 0 and tri_mode NAMG_TRI_DIRECT on a
 * hierarchy that has not yet run a direct solve through namg_solve (both allocate on first use). Every
 * call on a device shares that device's array and leaves its contents behind (no part of it needs to start
 * at zero): calls that overlap in time on one device, from two host threads or on two streams, race and
 * corrupt each other's results. */
#define NAMG_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int namg_solve_noalloc(namg_hier *h, const double *b_dev, double *x_dev, const namg_solve_params *p,
                       void *stream, namg_solve_stats *st);


/* One preconditioner application x = M^{-1} b: one V-cycle with zero initial guess (Section 5).
 * b_dev, x_dev: n float64 device vectors (x written). */
int namg_vcycle(namg_hier *h, const double *b_dev, double *x_dev, const namg_solve_params *p, void *stream);

/* One hot-path operator of level l on float64 device vectors of that level's sizes, for component
 * checks and profiling. In FP32_PRECOND mode the operator runs in FP32 on converted copies.
 *   NAMG_OP_SPMV          out = A_l in1                                   (n_l -> n_l)
 *   NAMG_OP_RESIDUAL      out = in2 - A_l in1                             (in1 = x, in2 = b)
 *   NAMG_OP_SMOOTH_PRE    out = in1 + M_pre^{-1}(in2 - A_l in1)           (one pre-smoothing sweep)
 *   NAMG_OP_SMOOTH_POST   out = in1 + M_post^{-1}(in2 - A_l in1)          (one post-smoothing sweep)
 *   NAMG_OP_RESTRICT      out = R_l in1                                   (n_l -> n_{l+1})
 *   NAMG_OP_PROLONG       out = in2 + P_l in1                             (in1: n_{l+1}, in2/out: n_l)
 *   NAMG_OP_COARSE        out = A_L^{-1} in1 on the coarsest level L
 *   NAMG_OP_SPMV64        out = A_0 in1 with the FP64 operator the GMRES uses (level must be 0)
 * The smoother kind, triangular mode and t come from p. */
enum {
  NAMG_OP_SPMV = 0, NAMG_OP_RESIDUAL = 1, NAMG_OP_SMOOTH_PRE = 2, NAMG_OP_SMOOTH_POST = 3,
  NAMG_OP_RESTRICT = 4, NAMG_OP_PROLONG = 5, NAMG_OP_COARSE = 6, NAMG_OP_SPMV64 = 7
};
int namg_apply(namg_hier *h, int level, int op, const namg_solve_params *p, const double *in1_dev,
               const double *in2_dev, double *out_dev, void *stream);

/* Kernel families that namg_profile_kernel can time. */
enum {
  NAMG_KF_NONE = 0,
  NAMG_KF_NEUMANN = 1,     /* one Neumann/Jacobi inner term on a strict triangle (Sections 5.2, 5.3.2) */
  NAMG_KF_RESIDUAL = 2,    /* r = b - A_l x [, f = D^{-1} r] inside the V-cycle */
  NAMG_KF_SPMV = 3,        /* restriction R_l r and the coarsest-level dense inverse */
  NAMG_KF_PROLONG = 4,     /* x += P_l e */
  NAMG_KF_GMRES_SPMV = 5,  /* w = A z, FP64 operator (Algorithm 1, the matrix-vector product) */
  NAMG_KF_MULTIDOT = 6,    /* c = V^T v, d = V^T w (Algorithm 1, the single reduction) */
  NAMG_KF_PROJECT = 7,     /* v_{i+2} = w / rho - V s (Algorithm 1, projection and lagged normalisation) */
  NAMG_KF_TRI = 8          /* one dependency level of a direct triangular solve (comparator) */
};

typedef struct {
  int64_t launches;
  double total_ms;  /* sum of the timed launches' durations (hipEvents attached to each dispatch) */
  double alg_bytes; /* sum of their algorithmic HBM bytes */
} namg_kernel_profile;

/* Time later launches of one kernel family (on one level, or -1 for all levels). Timing works on runs:
 * a maximal sequence of consecutive launches of the family on one stream gets a start event on its first
 * dispatch and a stop event after its last; the first run and then every `every`-th run are timed
 * (every >= 1). namg_profile_read returns the timed launches, their summed run times (so total_ms /
 * launches is the average launch duration, the events' own cost spread over each run) and their
 * algorithmic bytes, and clears them. family NAMG_KF_NONE switches timing off. */
int namg_profile_kernel(namg_hier *h, int family, int level, int every);
int namg_profile_read(namg_hier *h, namg_kernel_profile *out);

/* Hierarchy shape: levels, n_l, nnz(A_l), operator and grid complexity, device bytes. */
int namg_hier_info(const namg_hier *h, namg_hierarchy_info *out);

/* Sizes of level l: n_l, nnz(A_l), nnz(P_l) (0 on the coarsest level) and n_{l+1}. */
int namg_level_sizes(const namg_hier *h, int level, int32_t *n, int64_t *nnzA, int64_t *nnzP,
                     int32_t *ncoarse);

/* Host copies of level l for inspection: C/F markers (1 = C, 0 = F; n_l entries, not on the coarsest
 * level), A_l in CSR, P_l in CSR (n_l x n_{l+1}). Any pointer may be NULL; sizes from namg_level_sizes. */
int namg_export_level(const namg_hier *h, int level, int8_t *cf, int32_t *A_rowptr, int32_t *A_colind,
                      double *A_vals, int32_t *P_rowptr, int32_t *P_colind, double *P_vals);

/* Host copies of the ILU smoother factors of level l (Section 5.3.2: L = I + L_s, U = D_U (I + U_s)):
 * L_s (strict lower, as factored), U_s = D_U^{-1} times the strict upper part of U, and d_inv[i] = 1/u_ii,
 * each CSR with n_l + 1 row pointers. Call with NULL arrays first to get *nnz_lower and *nnz_upper.
 * NAMG_E_INVALID if the level carries no ILU factors. */
int namg_export_ilu(const namg_hier *h, int level, int64_t *nnz_lower, int64_t *nnz_upper, int32_t *L_rowptr,
                    int32_t *L_colind, double *L_vals, int32_t *U_rowptr, int32_t *U_colind, double *U_vals,
                    double *d_inv);

/* Non-normality of the ILU factors of level l (Section 5.3.4), computed on the host from the factors the
 * smoother applies (L = I + L_s; U = D_U (I + U_s), D_U = diag(U)). Departure from normality (Henrici):
 * dep(T)^2 = ||T||_F^2 - sum |lambda_i(T)|^2, which for a triangular T is ||strict(T)||_F^2. */
typedef struct {
  int64_t n, nnz_lower, nnz_upper; /* rows; stored strict entries of L_s and U_s */
  int max_row_upper;   /* p: most stored entries in a row of U, diagonal included */
  int ruiz_iters;      /* Ruiz iterations taken (<= ruiz_max_iters) */
  double dep_L;        /* dep(L) = ||L_s||_F */
  double dep_U;        /* dep(U) = ||strict(U)||_F, unscaled */
  double nu;           /* ||U_s||_F = dep(I + U_s) */
  double norm2_Us;     /* ||U_s||_2 = sigma_1(U_s): power iteration on U_s^T U_s, a lower estimate */
  double th1_bound;    /* Theorem 1: sqrt(n (p - 1)) */
  double th3_bound;    /* Theorem 3: sqrt((2 sqrt(n) + nu) nu) */
  double delta;        /* max_i max(0, sum_j |(U_s)_ij| - 1): near diagonal dominance of I + U_s */
  double th4_bound;    /* Theorem 4: sqrt(n) (1 + delta) */
  double dep_U_ruiz;   /* dep(D_r U D_c) after Ruiz scaling: rows and columns scaled together by
                          1/sqrt(largest magnitude) until each is within ruiz_tol of 1 */
} namg_ilu_diag;

/* Fill *out for level l. power_iters >= 1 (iterations for norm2_Us; the start vector is fixed), ruiz_max_iters
 * >= 0, ruiz_tol >= 0. NAMG_E_INVALID if the level carries no ILU factors or an argument is out of range. */
int namg_ilu_diagnostics(const namg_hier *h, int level, int power_iters, int ruiz_max_iters, double ruiz_tol,
                         namg_ilu_diag *out);

/* Table 2's measure on level l: `iters` Jacobi iterations from zero for L y = b (y <- y + (b - L y)), then
 * for U v = y with row scaling (v <- v + D_U^{-1}(y - U v)); *res_L = ||b - L y|| / ||b||,
 * *res_U = ||y - U v|| / ||y||. b: host array of n_l doubles; iters >= 0. */
int namg_tri_jacobi_residuals(const namg_hier *h, int level, const double *b, int iters, double *res_L,
                              double *res_U);

/* The powers of U_s that the Neumann form of the U solve sums (Section 5.3.2, the figure of max |(U_s^p)_ij|,
 * ||U_s^p||_2 and nnz(U_s^p) against p): for p = 1..pmax, max_abs[p-1] = the largest magnitude,
 * norm2[p-1] = sigma_1(U_s^p) by power_iters power iterations on (U_s^p)^T U_s^p from a fixed start (a lower
 * estimate), nnz[p-1] = the entries of U_s^p that are not exactly zero. U_s = D_U^{-1} U - I of level l's
 * ILU factors; U_s^p is formed by sparse products (row i sums over the entries of row i of U_s^{p-1} in
 * order), so the cost grows with the fill of the powers; once a power is zero the later ones are reported
 * as zero without work. Output arrays: host, pmax entries each, caller-owned. NAMG_E_INVALID if the level
 * has no ILU factors, pmax < 1, power_iters < 1, an output is NULL or a power exceeds 2^31 entries. */
int namg_us_powers(const namg_hier *h, int level, int pmax, int power_iters, double *max_abs, double *norm2,
                   int64_t *nnz);

/* ---- Serving (continuous batching of many solves on one GPU) ------------------------------------- */

typedef struct namg_server namg_server; /* opaque; owns its threads, stream and in-flight solves */

typedef struct {
  int64_t hbm_budget;  /* device bytes the in-flight solves may hold; <= 0: device memory less 48 GiB (16 GiB
                          for other users of the device, 32 GiB for device setup memory, which admission
                          does not count; see peak_setup_device_bytes) */
  int max_inflight;    /* solves advanced together per scheduler tick, 1..256 */
  int setup_threads;   /* host threads running the AMG setup of queued requests */
  int device;          /* HIP device ordinal */
  int precision;       /* NAMG_FP64 or NAMG_FP32_PRECOND, for every request */
  namg_solve_params solve; /* the default solve parameters of a request (namg_server_submit may give its
                              own); tri_mode must be NAMG_TRI_NEUMANN, diagnostics 0 and res_hist NULL */
} namg_server_params;

typedef struct {
  double submit, setup_start, setup_done, admitted, done; /* seconds on the server's clock */
} namg_request_times;

/* device_bytes_in_use and peak_device_bytes count the footprints reserved at admission (every device
 * buffer counted at the size it allocates, its block-cache size class); footprint_mismatches counts admitted
 * requests whose solver allocated other than its reserved footprint (0 when the admission estimate is
 * exact). peak_setup_device_bytes is the process-wide high-water mark of device setup memory, which no
 * footprint covers: uploaded matrices, coarsening and sparse-product scratch, and the levels a set-up
 * request keeps on the device until its solver is built. */
typedef struct {
  int64_t submitted, completed, failed, inflight, waiting, ticks, launches;
  int64_t device_bytes_in_use, peak_device_bytes, peak_inflight;
  int64_t footprint_mismatches;
  int64_t peak_setup_device_bytes;
} namg_server_counters;

void namg_default_server_params(namg_server_params *p);

/* Start a server: setup threads, one scheduler thread and its stream. Requests are set up on the host
 * (as namg_setup), admitted in order of setup completion when a slot is free and their exact device
 * footprint fits the budget, and then advanced together: every scheduler tick moves every in-flight
 * solve by one Arnoldi step of Algorithm 1 (or one restart-cycle boundary), with each V-cycle row
 * operation and each Krylov kernel issued as one batched launch for all of them. Solves leave at tick
 * boundaries and free their memory; waiting requests are admitted while the others keep running.
 * Errors: NAMG_E_INVALID (bad parameters), NAMG_E_HIP. */
int namg_server_create(const namg_server_params *p, namg_server **out);

/* Queue one system A x = b (host CSR and b, copied; x0 = 0) with its setup parameters (precision and
 * device come from the server) and its solve parameters p (copied; NULL = the server's default). Requests
 * with different smoothers, Neumann terms, restarts, tolerances or T forms are batched together: every
 * batched launch carries each solve's own operands and parameters. p is validated as for namg_solve, and
 * must keep tri_mode NAMG_TRI_NEUMANN, diagnostics 0 and res_hist NULL (NAMG_E_INVALID otherwise).
 * Returns at once with a ticket. */
int namg_server_submit(namg_server *s, int32_t n, const int32_t *rowptr, const int32_t *colind, const double *vals,
                       const double *b, const namg_setup_params *sp, const namg_solve_params *p, uint64_t *ticket);

/* NAMG_PENDING while the request is queued or in flight. Once it has finished: copies x (n doubles,
 * host, may be NULL), its statistics and times, forgets the ticket and returns its status (NAMG_OK,
 * NAMG_NOT_CONVERGED or the error of its setup or solve, e.g. NAMG_E_BUDGET). */
int namg_server_poll(namg_server *s, uint64_t ticket, double *x, namg_solve_stats *st, namg_request_times *tm);

/* As namg_server_poll, but blocks until the request has finished. */
int namg_server_wait(namg_server *s, uint64_t ticket, double *x, namg_solve_stats *st, namg_request_times *tm);

int namg_server_stats(namg_server *s, namg_server_counters *out);

/* Seconds since the server started (the clock of namg_request_times). */
double namg_server_clock(const namg_server *s);

/* Stop the threads and release everything; requests still queued or in flight are dropped. */
void namg_server_destroy(namg_server *s);

/* Release the hierarchy. Waits for the device to finish pending work (namg_vcycle / namg_apply on the
 * caller's stream), then returns its device memory to the library's block cache: freed blocks are
 * handed to later allocations of the same size class instead of being freed (a free can wait for every
 * stream of the device), up to 32 GiB cached per device, held until the process ends. NULL is ignored. */
void namg_destroy(namg_hier *h);

/* Message of the last error on the calling thread ("" if none). */
const char *namg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* NAMG_H */

/* Oracle for the GMRES + classical-AMG solve phase of "Neumann Series in GMRES and Algebraic Multigrid
 * Smoothers" (Thomas, Carr, Mullowney, Li, Swirydowicz; arXiv 2112.14681).
 *
 * TEST INFRASTRUCTURE ONLY. This is a plain, slow, single-threaded FP64 CPU implementation used to
 * check the HIP library. Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it. It shares no code, header or helper with the library under paper_2112_14681_amd/.
 *
 * Built with -O2 -ffp-contract=off so every sum is taken in the order written in oracle.cpp.
 * All matrices are 0-based CSR with int32 indices, columns ascending, diagonal present.
 */
#ifndef NAMG_ORACLE_H
#define NAMG_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_NOT_CONVERGED = 1, ORC_E_INVALID = -1, ORC_E_ZERO_PIVOT = -2, ORC_E_NONFINITE = -3 };
enum { ORC_SMOOTH_PGS = 0, ORC_SMOOTH_ILU0 = 1, ORC_SMOOTH_L1JAC = 2 };
enum { ORC_TRI_NEUMANN = 0, ORC_TRI_DIRECT = 1 };
enum { ORC_T_NEUMANN = 0, ORC_T_DIRECT = 1 };
enum { ORC_PRECOND_NONE = 0, ORC_PRECOND_AMG = 1 };
enum { ORC_STOP_RELRES = 0, ORC_STOP_NRBE = 1 };
enum { ORC_ILU_KIND_ILU0 = 0, ORC_ILU_KIND_ILUT = 1 };
enum { ORC_COARSEN_RS = 0, ORC_COARSEN_PMIS = 1 }; /* RS + classical, or PMIS + BAMG direct interpolation */
/* single-level smoother kinds for orc_smooth */
enum {
  ORC_PGS_FWD = 0,     /* polynomial GS, forward (D+L), t Neumann terms      */
  ORC_PGS_BWD = 1,     /* polynomial GS, backward (D+U), t Neumann terms     */
  ORC_GS_FWD = 2,      /* GS, forward substitution                           */
  ORC_GS_BWD = 3,      /* GS, backward substitution                          */
  ORC_ILU_NEUMANN = 4, /* ILU(0) with t-term Jacobi/Neumann triangular solves */
  ORC_ILU_DIRECT = 5,  /* ILU(0) with substitution                            */
  ORC_L1_JACOBI = 6    /* l1-Jacobi: x += D_l1^{-1} (b - A x)                */
};

typedef struct {
  double tol;
  int restart;
  int max_iters;
  int precond;    /* ORC_PRECOND_* */
  int smoother;   /* ORC_SMOOTH_* */
  int tri_mode;   /* ORC_TRI_* */
  int inner_terms;/* t >= 1: number of Neumann terms */
  int gmres_T;    /* ORC_T_* */
  int pre_sweeps, post_sweeps;
  int t_degree;   /* p >= 1: T = sum_{j=0..p} (-L)^j when gmres_T == ORC_T_NEUMANN (p = 1: I - L) */
  int stop_rule;  /* ORC_STOP_RELRES: ||r|| / ||b|| <= tol; ORC_STOP_NRBE: ||r|| / (||b|| + ||A||_inf ||x||) <= tol */
} orc_params;

typedef struct {
  int status, iters, cycles, precond_apps;
  double relres_true, relres_est, nrbe;
} orc_stats;

/* ---- primitives on one matrix ---- */
int orc_spmv(int n_rows, const int *rp, const int *ci, const double *v, const double *x, double *y);
/* S in CSR (pattern only); S_rp has n+1 entries; S_ci must hold up to nnz entries. */
int orc_strength(int n, const int *rp, const int *ci, const double *v, double theta, int *S_rp, int *S_ci);
/* cf[i] = 1 (C) or 0 (F) from the RS first pass on A's strength graph. */
int orc_coarsen(int n, const int *rp, const int *ci, const double *v, double theta, signed char *cf);
/* ILU(0) on A's pattern: out holds L's strict-lower entries (unit diagonal implied) and U's
 * upper entries (diagonal included) in A's positions. */
int orc_ilu0(int n, const int *rp, const int *ci, const double *v, double *out);
/* ILUT(droptol, lfil) factors L \ U as CSR (frp: n + 1 entries; fci, fv: up to cap entries); *nnz gets the
   factor's entry count, ORC_E_INVALID when it exceeds cap */
int orc_ilut(int n, const int *rp, const int *ci, const double *v, double droptol, int lfil, long long cap,
             int *frp, int *fci, double *fv, long long *nnz);
/* one ILUT smoothing sweep: Jacobi triangular solves with t terms (direct = 0) or substitution (1) */
int orc_smooth_ilut(int n, const int *rp, const int *ci, const double *v, double droptol, int lfil, int direct,
                    int t, const double *b, double *x);
/* one smoothing sweep x <- x + M^{-1}(b - A x) of the given kind */
int orc_smooth(int n, const int *rp, const int *ci, const double *v, int kind, int t, const double *b, double *x);

/* ---- hierarchy ---- */
void *orc_setup(int n, const int *rp, const int *ci, const double *v, double theta, int max_levels,
                int max_coarse, int ilu_levels, int ilu_kind, double droptol, int lfil, int agg_levels,
                int coarsen, unsigned long long seed, int *status);
/* the k-th output (k >= 1) of SplitMix64 seeded with seed, and the [0, 1) draw of point i (output i + 1) */
unsigned long long orc_splitmix64(unsigned long long seed, unsigned long long k);
double orc_uniform01(unsigned long long seed, long long i);
void orc_free(void *h);
int orc_num_levels(const void *h);
/* n, nnz(A_l), nnz(P_l) (0 on the coarsest level), n_{l+1} */
int orc_level_info(const void *h, int l, int *n, long long *nnzA, long long *nnzP, int *ncoarse);
int orc_level_export(const void *h, int l, signed char *cf, int *Arp, int *Aci, double *Av, int *Prp,
                     int *Pci, double *Pv);
/* one V-cycle x = M^{-1} b (x is output only) */
int orc_vcycle(void *h, int smoother, int tri_mode, int t, int nu1, int nu2, const double *b, double *x);
/* Low-synchronization right-preconditioned flexible GMRES(m). x holds x0 on input.
 * hist (optional): per-iteration estimate |g_{i+1}|/||b||; true relres at each cycle start is
 * written to cyc_hist (optional). cap_* (optional): the last cycle's V (n x (m+2), col-major),
 * Z (n x m), Hessenberg before rotations ((m+1) x m, col-major) and its column count k. */
int orc_solve(void *h, const double *b, double *x, const orc_params *p, orc_stats *st, double *hist,
              int hist_cap, int *hist_len, double *cyc_hist, int cyc_cap, int *cyc_len, double *cap_V,
              double *cap_Z, double *cap_H, int *cap_k);
/* ||I - V^T V||_F over the first k columns of an n x k column-major matrix */
double orc_loss_orth(int n, int k, const double *V);

#ifdef __cplusplus
}
#endif
#endif

// Non-normality diagnostics of the ILU smoother factors (Sections 5.3.1 to 5.3.4 of arXiv 2112.14681:
// Henrici's departure from normality, 5.3.1; the powers of U_s, 5.3.2; Theorems 1 to 4 and Ruiz scaling,
// 5.3.4) and the Jacobi triangular-solve residuals of Table 2 (5.3.3). Host code on the factors a level stores for its smoother: L_s, U_s = D_U^{-1} strict(U) and
// D_U = diag(U). For triangular T the eigenvalues are the diagonal, so dep(T) = ||strict(T)||_F.
#include <algorithm>
#include <cmath>
#include <vector>

#include "setup_host.hpp"

namespace namg {
namespace {

[[noreturn]] void bad(const char *msg) { throw SetupError{NAMG_E_INVALID, msg}; }

double frob(const HostCsr &T) {
  double s = 0.0;
  for (double v : T.v) s += v * v;
  return std::sqrt(s);
}

// y = T x for a CSR T
void csr_mv(const HostCsr &T, const std::vector<double> &x, std::vector<double> &y) {
  y.assign(T.nr, 0.0);
  for (int32_t i = 0; i < T.nr; ++i) {
    double s = 0.0;
    for (int32_t k = T.rp[i]; k < T.rp[i + 1]; ++k) s += T.v[k] * x[T.ci[k]];
    y[i] = s;
  }
}

// z = T^T y for a CSR T (scatter by rows)
void csr_mtv(const HostCsr &T, const std::vector<double> &y, std::vector<double> &z) {
  z.assign(T.nc, 0.0);
  for (int32_t i = 0; i < T.nr; ++i)
    for (int32_t k = T.rp[i]; k < T.rp[i + 1]; ++k) z[T.ci[k]] += T.v[k] * y[i];
}

double norm2(const std::vector<double> &v) {
  double s = 0.0;
  for (double a : v) s += a * a;
  return std::sqrt(s);
}

// sigma_1(T) by power iteration on T^T T from a fixed start; ||T x|| / ||x|| at the last iterate never
// exceeds sigma_1. The iteration runs on T scaled by a power of two that brings its largest magnitude into
// [0.5, 1), so that T^T T x neither underflows nor overflows (the scaling is exact).
double sigma1_scaled(const HostCsr &T, int iters);

double sigma1(const HostCsr &T, int iters) {
  double m = 0.0;
  for (double v : T.v) m = std::max(m, std::fabs(v));
  if (m == 0.0) return 0.0;
  int e = 0;
  (void)std::frexp(m, &e);
  HostCsr S = T;
  for (double &v : S.v) v = std::ldexp(v, -e);
  return std::ldexp(sigma1_scaled(S, iters), e);
}

double sigma1_scaled(const HostCsr &T, int iters) {
  std::vector<double> x(T.nc), y, z;
  for (int32_t i = 0; i < T.nc; ++i) x[i] = 1.0 + 0.5 * std::sin((double)i);
  double est = 0.0;
  for (int it = 0; it < iters; ++it) {
    const double xn = norm2(x);
    for (double &a : x) a /= xn;
    csr_mv(T, x, y);
    est = norm2(y);
    csr_mtv(T, y, z);
    if (norm2(z) == 0.0) break;  // T x = 0 (e.g. T = 0)
    x.swap(z);
  }
  return est;
}

// C = X Y by rows with a dense accumulator (row i of C: the sum over the entries x_ik of x_ik times row k
// of Y, in entry order); exact zeros are not stored.
HostCsr csr_product(const HostCsr &X, const HostCsr &Y, int64_t max_nnz) {
  HostCsr C;
  C.nr = X.nr;
  C.nc = Y.nc;
  C.rp.assign(X.nr + 1, 0);
  std::vector<double> acc(Y.nc, 0.0);
  std::vector<int32_t> mark(Y.nc, -1), cols;
  for (int32_t i = 0; i < X.nr; ++i) {
    cols.clear();
    for (int32_t k = X.rp[i]; k < X.rp[i + 1]; ++k) {
      const int32_t r = X.ci[k];
      for (int32_t q = Y.rp[r]; q < Y.rp[r + 1]; ++q) {
        const int32_t j = Y.ci[q];
        if (mark[j] != i) {
          mark[j] = i;
          acc[j] = 0.0;
          cols.push_back(j);
        }
        acc[j] += X.v[k] * Y.v[q];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int32_t j : cols)
      if (acc[j] != 0.0) {
        C.ci.push_back(j);
        C.v.push_back(acc[j]);
      }
    if ((int64_t)C.ci.size() > max_nnz) bad("a power of U_s exceeds 2^31 stored entries");
    C.rp[i + 1] = (int32_t)C.ci.size();
  }
  return C;
}

}  // namespace

void us_powers(const HostLevel &L, int pmax, int power_iters, double *max_abs, double *norm2_out, int64_t *nnz) {
  if (!L.has_ilu) bad("level carries no ILU factors");
  if (pmax < 1 || power_iters < 1) bad("diagnostic parameter out of range");
  if (!max_abs || !norm2_out || !nnz) bad("null output array");
  const HostCsr &Us = L.ilu_up;
  HostCsr P = Us;
  // exact zeros of U_s are not entries of its powers
  {
    HostCsr Q;
    Q.nr = P.nr;
    Q.nc = P.nc;
    Q.rp.assign(P.nr + 1, 0);
    for (int32_t i = 0; i < P.nr; ++i) {
      for (int32_t k = P.rp[i]; k < P.rp[i + 1]; ++k)
        if (P.v[k] != 0.0) {
          Q.ci.push_back(P.ci[k]);
          Q.v.push_back(P.v[k]);
        }
      Q.rp[i + 1] = (int32_t)Q.ci.size();
    }
    P = std::move(Q);
  }
  for (int p = 1; p <= pmax; ++p) {
    if (P.nnz() == 0) {
      max_abs[p - 1] = 0.0;
      norm2_out[p - 1] = 0.0;
      nnz[p - 1] = 0;
      continue;
    }
    double m = 0.0;
    for (double v : P.v) m = std::max(m, std::fabs(v));
    max_abs[p - 1] = m;
    norm2_out[p - 1] = sigma1(P, power_iters);
    nnz[p - 1] = P.nnz();
    if (p < pmax) P = csr_product(P, Us, (int64_t)INT32_MAX);
  }
}

void ilu_diagnostics(const HostLevel &L, int power_iters, int ruiz_max_iters, double ruiz_tol, namg_ilu_diag *out) {
  if (!L.has_ilu) bad("level carries no ILU factors");
  if (power_iters < 1 || ruiz_max_iters < 0 || !(ruiz_tol >= 0.0)) bad("diagnostic parameter out of range");
  const HostCsr &Ls = L.ilu_lo, &Us = L.ilu_up;
  const std::vector<double> &du = L.ilu_diag;
  const int32_t n = Us.nr;
  namg_ilu_diag d{};
  d.n = n;
  d.nnz_lower = Ls.nnz();
  d.nnz_upper = Us.nnz();
  int32_t p = 1;
  double delta = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    p = std::max(p, Us.rp[i + 1] - Us.rp[i] + 1);
    double s = 0.0;
    for (int32_t k = Us.rp[i]; k < Us.rp[i + 1]; ++k) s += std::fabs(Us.v[k]);
    delta = std::max(delta, s - 1.0);
  }
  d.max_row_upper = p;
  d.dep_L = frob(Ls);
  double su = 0.0;
  for (int32_t i = 0; i < n; ++i)
    for (int32_t k = Us.rp[i]; k < Us.rp[i + 1]; ++k) {
      const double u = Us.v[k] * du[i];  // strict(U)_ij = u_ii (U_s)_ij
      su += u * u;
    }
  d.dep_U = std::sqrt(su);
  d.nu = frob(Us);
  d.th1_bound = std::sqrt((double)n * (double)(p - 1));
  d.th3_bound = std::sqrt((2.0 * std::sqrt((double)n) + d.nu) * d.nu);
  d.delta = delta;
  d.th4_bound = std::sqrt((double)n) * (1.0 + delta);

  d.norm2_Us = sigma1(Us, power_iters);

  // Ruiz scaling of U (diagonal u_ii, strict part u_ii (U_s)_ij): r_i and c_j are the largest magnitudes in
  // row i and column j of diag(dr) U diag(dc); both scalings update together until all are within tol of 1
  std::vector<double> dr(n, 1.0), dc(n, 1.0), r(n), c(n);
  int iters = 0;
  while (true) {
    for (int32_t i = 0; i < n; ++i) {
      const double dd = dr[i] * std::fabs(du[i]) * dc[i];
      r[i] = dd;
      c[i] = dd;
    }
    for (int32_t i = 0; i < n; ++i)
      for (int32_t k = Us.rp[i]; k < Us.rp[i + 1]; ++k) {
        const int32_t j = Us.ci[k];
        const double a = dr[i] * std::fabs(Us.v[k] * du[i]) * dc[j];
        r[i] = std::max(r[i], a);
        c[j] = std::max(c[j], a);
      }
    double worst = 0.0;
    for (int32_t i = 0; i < n; ++i) worst = std::max({worst, std::fabs(1.0 - r[i]), std::fabs(1.0 - c[i])});
    if (worst <= ruiz_tol || iters >= ruiz_max_iters) break;
    for (int32_t i = 0; i < n; ++i) {
      dr[i] /= std::sqrt(r[i]);
      dc[i] /= std::sqrt(c[i]);
    }
    ++iters;
  }
  double sr = 0.0;
  for (int32_t i = 0; i < n; ++i)
    for (int32_t k = Us.rp[i]; k < Us.rp[i + 1]; ++k) {
      const double a = dr[i] * (Us.v[k] * du[i]) * dc[Us.ci[k]];
      sr += a * a;
    }
  d.dep_U_ruiz = std::sqrt(sr);
  d.ruiz_iters = iters;
  *out = d;
}

void tri_jacobi_residuals(const HostLevel &L, const double *b, int iters, double *res_L, double *res_U) {
  if (!L.has_ilu) bad("level carries no ILU factors");
  if (!b || iters < 0) bad("bad right-hand side or iteration count");
  const HostCsr &Ls = L.ilu_lo, &Us = L.ilu_up;
  const std::vector<double> &du = L.ilu_diag;
  const int32_t n = Ls.nr;
  const std::vector<double> bv(b, b + n);
  // L y = b with L = I + L_s: y <- y + (b - L y) = b - L_s y
  std::vector<double> yv(n, 0.0), t;
  for (int it = 0; it < iters; ++it) {
    csr_mv(Ls, yv, t);
    for (int32_t i = 0; i < n; ++i) yv[i] = bv[i] - t[i];
  }
  csr_mv(Ls, yv, t);
  std::vector<double> rl(n);
  for (int32_t i = 0; i < n; ++i) rl[i] = bv[i] - (yv[i] + t[i]);
  // U v = y with U = D_U (I + U_s) and D = D_U^{-1}: v <- v + D (y - U v) = D y - U_s v
  std::vector<double> v(n, 0.0);
  for (int it = 0; it < iters; ++it) {
    csr_mv(Us, v, t);
    for (int32_t i = 0; i < n; ++i) v[i] = yv[i] / du[i] - t[i];
  }
  csr_mv(Us, v, t);
  std::vector<double> ru(n);
  for (int32_t i = 0; i < n; ++i) ru[i] = yv[i] - du[i] * (v[i] + t[i]);
  const double bn = norm2(bv), yn = norm2(yv);
  *res_L = bn > 0.0 ? norm2(rl) / bn : 0.0;
  *res_U = yn > 0.0 ? norm2(ru) / yn : 0.0;
}

}  // namespace namg

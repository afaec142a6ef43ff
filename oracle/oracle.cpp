// Oracle for the GMRES + classical-AMG solve phase of arXiv 2112.14681.
//
// TEST INFRASTRUCTURE ONLY: a plain, slow, single-threaded FP64 CPU implementation that the test-suite,
// the smoke check and the CPU-baseline leg of the benchmark use to check the HIP library. It shares
// no code with the library. Every loop below sums in the order it is written (built with
// -ffp-contract=off), and each function names the passage of the paper it follows.
//
// Readings of passages the paper leaves open (each one is listed with its reason in the design notes):
//  * strength uses |a_ij| as printed (Section 5.1, the strength inequality);
//  * coarsening is the Ruge-Stueben first pass with ties broken by the smallest index;
//  * interpolation is the classical Ruge-Stueben formula (Section 5.1 cites it, does not print it);
//  * the V-cycle pre-smooths forward and post-smooths backward (Section 5.2 allows either);
//  * t counts Neumann terms: t = 1 is Jacobi, t - 1 products with the strict triangle follow
//    (Section 5.2, Jacobi recurrence; Algorithm 2 loops from a zero start);
//  * the low-synchronization GMRES scales w by 1/r_{i+1,i+1} and the last projection coefficient by
//    1/r_{i+1,i+1}^2, which the lagged normalisation of Algorithm 1 requires (Section 4).
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <set>
#include <stdexcept>
#include <utility>
#include <vector>

namespace {

struct OracleError {
  int code;
};

struct Csr {
  int nr = 0, nc = 0;
  std::vector<int> rp, ci;
  std::vector<double> v;
};

Csr make_csr(int nr, int nc, const int *rp, const int *ci, const double *v) {
  if (nr < 0 || rp == nullptr || (nr > 0 && rp[0] != 0)) throw OracleError{ORC_E_INVALID};
  Csr A;
  A.nr = nr;
  A.nc = nc;
  A.rp.assign(rp, rp + nr + 1);
  for (int i = 0; i < nr; ++i) {
    if (A.rp[i + 1] < A.rp[i]) throw OracleError{ORC_E_INVALID};
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      if (ci[k] < 0 || ci[k] >= nc) throw OracleError{ORC_E_INVALID};
      if (k > A.rp[i] && ci[k] <= ci[k - 1]) throw OracleError{ORC_E_INVALID};
      if (!std::isfinite(v[k])) throw OracleError{ORC_E_NONFINITE};
    }
  }
  long long nnz = A.rp[nr];
  A.ci.assign(ci, ci + nnz);
  A.v.assign(v, v + nnz);
  return A;
}

double entry(const Csr &A, int i, int j) {  // a_ij, 0 when not structural
  for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
    if (A.ci[k] == j) return A.v[k];
  return 0.0;
}

bool structural(const Csr &A, int i, int j) {
  for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
    if (A.ci[k] == j) return true;
  return false;
}

double diag_of(const Csr &A, int i) {
  for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
    if (A.ci[k] == i) return A.v[k];
  throw OracleError{ORC_E_ZERO_PIVOT};
}

// y = A x (rows summed in ascending column order).
void spmv(const Csr &A, const std::vector<double> &x, std::vector<double> &y) {
  y.assign(A.nr, 0.0);
  for (int i = 0; i < A.nr; ++i) {
    double s = 0.0;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) s += A.v[k] * x[A.ci[k]];
    y[i] = s;
  }
}

// r = b - A x  (Section 1: r^(0) = b - A x^(0); Section 5.2 eq. one-stage).
void residual(const Csr &A, const std::vector<double> &b, const std::vector<double> &x,
              std::vector<double> &r) {
  spmv(A, x, r);
  for (int i = 0; i < A.nr; ++i) r[i] = b[i] - r[i];
}

double dot(const std::vector<double> &a, const std::vector<double> &b) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}

double norm2(const std::vector<double> &a) { return std::sqrt(dot(a, a)); }

// ---------------------------------------------------------------------------------------------
// Section 5.1: point j strongly influences i iff |a_ij| >= theta * max_{k != i} |a_ik|.
std::vector<std::vector<int>> strength(const Csr &A, double theta) {
  std::vector<std::vector<int>> S(A.nr);
  for (int i = 0; i < A.nr; ++i) {
    double m = 0.0;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (A.ci[k] != i) m = std::max(m, std::fabs(A.v[k]));
    if (m == 0.0) continue;
    double thr = theta * m;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (A.ci[k] != i && std::fabs(A.v[k]) >= thr) S[i].push_back(A.ci[k]);
  }
  return S;
}

std::vector<std::vector<int>> transpose_graph(const std::vector<std::vector<int>> &S) {
  std::vector<std::vector<int>> T(S.size());
  for (size_t i = 0; i < S.size(); ++i)
    for (int j : S[i]) T[j].push_back((int)i);
  return T;
}

// Ruge-Stueben first-pass colouring (Section 5.1 describes the C/F selection; Ruge & Stueben 1987).
// lambda_i = |S^T_i intersect U| + 2 |S^T_i intersect F|; repeatedly the undecided point with the
// largest lambda (smallest index on ties) becomes C and every undecided j that it strongly
// influences becomes F. Points with no strong connection either way are F from the start.
std::vector<signed char> rs_first_pass(const std::vector<std::vector<int>> &S) {
  const int n = (int)S.size();
  const auto ST = transpose_graph(S);
  enum { U = 0, C = 1, F = 2 };
  std::vector<int> state(n, U);
  for (int i = 0; i < n; ++i)
    if (S[i].empty() && ST[i].empty()) state[i] = F;
  auto lambda = [&](int i) {
    int c = 0;
    for (int j : ST[i]) c += (state[j] == U) ? 1 : (state[j] == F ? 2 : 0);
    return c;
  };
  std::vector<int> lam(n, 0);
  std::set<std::pair<int, int>> queue;  // (-lambda, index): begin() = max lambda, smallest index
  for (int i = 0; i < n; ++i)
    if (state[i] == U) {
      lam[i] = lambda(i);
      queue.insert({-lam[i], i});
    }
  while (!queue.empty()) {
    const int i = queue.begin()->second;
    queue.erase(queue.begin());
    state[i] = C;
    std::vector<int> newF;
    for (int j : ST[i])
      if (state[j] == U) {
        state[j] = F;
        queue.erase({-lam[j], j});
        newF.push_back(j);
      }
    std::vector<int> touched(S[i].begin(), S[i].end());
    for (int j : newF) touched.insert(touched.end(), S[j].begin(), S[j].end());
    for (int k : touched) {
      if (state[k] != U) continue;
      int nl = lambda(k);
      if (nl != lam[k]) {
        queue.erase({-lam[k], k});
        lam[k] = nl;
        queue.insert({-nl, k});
      }
    }
  }
  std::vector<signed char> cf(n);
  for (int i = 0; i < n; ++i) cf[i] = (state[i] == C) ? 1 : 0;
  return cf;
}

// SplitMix64 (Steele, Lea and Flood 2014): the k-th output (k >= 1) of the stream seeded with s is
// mix(s + k * 0x9E3779B97F4A7C15). Used as a counter-based generator: point i of level l draws the
// (i + 1)-th output of the stream seeded with seed + l, as a double in [0, 1) from its top 53 bits.
uint64_t splitmix64_output(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double uniform01(uint64_t seed, int64_t i) {
  return (double)(splitmix64_output(seed, (uint64_t)i + 1) >> 11) * 0x1.0p-53;
}

// PMIS coarsening (Section 5.1: Luby's maximal independent set with random numbers, as modified by De
// Sterck, Yang and Heys). Weights w_i = |S^T_i| + u_i with u_i in [0, 1) drawn as above. Points that
// influence no other point (w_i < 1) are F from the start. Then, in rounds until no point is undecided,
// every undecided point whose weight beats that of each undecided point it is strongly connected to
// (either direction; equal weights: the smaller index wins) becomes C, all at once, and every undecided
// point that strongly depends on one of these new C points becomes F.
std::vector<signed char> pmis(const std::vector<std::vector<int>> &S, uint64_t seed) {
  const int n = (int)S.size();
  const auto ST = transpose_graph(S);
  enum { U = 0, C = 1, F = 2 };
  std::vector<int> state(n, U);
  std::vector<double> w(n);
  for (int i = 0; i < n; ++i) {
    w[i] = (double)ST[i].size() + uniform01(seed, i);
    if (ST[i].empty()) state[i] = F;
  }
  auto beats = [&](int i, int j) { return w[i] > w[j] || (w[i] == w[j] && i < j); };
  while (true) {
    std::vector<int> newC;
    for (int i = 0; i < n; ++i) {
      if (state[i] != U) continue;
      bool best = true;
      for (int j : S[i])
        if (state[j] == U && !beats(i, j)) best = false;
      for (int j : ST[i])
        if (state[j] == U && !beats(i, j)) best = false;
      if (best) newC.push_back(i);
    }
    if (newC.empty()) break;
    for (int i : newC) state[i] = C;
    for (int i : newC)
      for (int j : ST[i])
        if (state[j] == U) state[j] = F;
  }
  std::vector<signed char> cf(n);
  for (int i = 0; i < n; ++i) cf[i] = (state[i] == C) ? 1 : 0;
  return cf;
}

// BAMG direct interpolation (Section 5.1, the closed form of the local least-squares problem with target
// f = 1): for an F point i with strong C neighbours C_i (n_i of them), strong F neighbours and weak
// neighbours N^w_i, w_ij = -(a_ij + beta_i / n_i) / (a_ii + sum_{k in N^w_i} a_ik) for j in C_i with
// beta_i = the sum of a_ik over the strong F neighbours (both sums in ascending column order, the
// denominator starting from a_ii). An F point without strong C neighbours gets an empty row.
Csr bamg_direct_interp(const Csr &A, const std::vector<std::vector<int>> &S, const std::vector<signed char> &cf,
                       int &nc_out) {
  const int n = A.nr;
  std::vector<int> cidx(n, -1);
  int nc = 0;
  for (int i = 0; i < n; ++i)
    if (cf[i] == 1) cidx[i] = nc++;
  nc_out = nc;
  Csr P;
  P.nr = n;
  P.nc = nc;
  P.rp.assign(1, 0);
  for (int i = 0; i < n; ++i) {
    if (cf[i] == 1) {
      P.ci.push_back(cidx[i]);
      P.v.push_back(1.0);
      P.rp.push_back((int)P.ci.size());
      continue;
    }
    const std::vector<int> &Si = S[i];
    auto is_strong = [&](int j) { return std::binary_search(Si.begin(), Si.end(), j); };
    int ni = 0;
    double beta = 0.0, dd = diag_of(A, i);
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int j = A.ci[k];
      if (j == i) continue;
      if (!is_strong(j))
        dd += A.v[k];
      else if (cf[j] == 1)
        ++ni;
      else
        beta += A.v[k];
    }
    if (ni > 0) {
      for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        const int j = A.ci[k];
        if (j != i && cf[j] == 1 && is_strong(j)) {
          P.ci.push_back(cidx[j]);
          P.v.push_back(-(A.v[k] + beta / ni) / dd);
        }
      }
    }
    P.rp.push_back((int)P.ci.size());
  }
  return P;
}

// Classical (Ruge-Stueben standard) interpolation, P = [W; I] in the ordering of the fine grid.
// For an F point i with strong C set C_i, strong F set Fs_i and weak set N^w_i:
//   w_ij = -(a_ij + sum_{k in Fs_i} a_ik a_kj / den_k) / (a_ii + sum_{n in N^w_i} a_in),
//   den_k = sum_{l in C_i} a_kl; a strong F neighbour with den_k = 0 is treated as weak.
Csr classical_interp(const Csr &A, const std::vector<std::vector<int>> &S,
                     const std::vector<signed char> &cf, int &nc_out) {
  const int n = A.nr;
  std::vector<int> cidx(n, -1);
  int nc = 0;
  for (int i = 0; i < n; ++i)
    if (cf[i] == 1) cidx[i] = nc++;
  nc_out = nc;
  Csr P;
  P.nr = n;
  P.nc = nc;
  P.rp.assign(1, 0);
  for (int i = 0; i < n; ++i) {
    if (cf[i] == 1) {
      P.ci.push_back(cidx[i]);
      P.v.push_back(1.0);
      P.rp.push_back((int)P.ci.size());
      continue;
    }
    const std::vector<int> &Si = S[i];
    auto is_strong = [&](int j) { return std::binary_search(Si.begin(), Si.end(), j); };
    std::vector<int> Ci, Fs;
    for (int j : Si) (cf[j] == 1 ? Ci : Fs).push_back(j);
    if (Ci.empty()) {
      P.rp.push_back((int)P.ci.size());
      continue;
    }
    // den_k for strong F neighbours, summed over l in C_i in ascending column order
    std::vector<double> den(Fs.size(), 0.0);
    for (size_t q = 0; q < Fs.size(); ++q) {
      const int k = Fs[q];
      double s = 0.0;
      for (int kk = A.rp[k]; kk < A.rp[k + 1]; ++kk)
        if (std::binary_search(Ci.begin(), Ci.end(), A.ci[kk])) s += A.v[kk];
      den[q] = s;
    }
    auto moved_to_weak = [&](int j) {
      for (size_t q = 0; q < Fs.size(); ++q)
        if (Fs[q] == j) return den[q] == 0.0;
      return false;
    };
    // denominator: a_ii, then + a_in over weak neighbours in ascending column order
    double dd = diag_of(A, i);
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int j = A.ci[k];
      if (j == i) continue;
      if (!is_strong(j) || (cf[j] == 0 && moved_to_weak(j))) dd += A.v[k];
    }
    for (int j : Ci) {
      double num = entry(A, i, j);
      for (size_t q = 0; q < Fs.size(); ++q) {
        const int k = Fs[q];
        if (den[q] == 0.0) continue;
        if (!structural(A, k, j)) continue;
        num += (entry(A, i, k) * entry(A, k, j)) / den[q];
      }
      P.ci.push_back(cidx[j]);
      P.v.push_back(-num / dd);
    }
    P.rp.push_back((int)P.ci.size());
  }
  return P;
}

Csr transpose(const Csr &P) {
  Csr R;
  R.nr = P.nc;
  R.nc = P.nr;
  std::vector<std::vector<std::pair<int, double>>> rows(P.nc);
  for (int i = 0; i < P.nr; ++i)
    for (int k = P.rp[i]; k < P.rp[i + 1]; ++k) rows[P.ci[k]].push_back({i, P.v[k]});
  R.rp.assign(1, 0);
  for (auto &row : rows) {
    for (auto &e : row) {
      R.ci.push_back(e.first);
      R.v.push_back(e.second);
    }
    R.rp.push_back((int)R.ci.size());
  }
  return R;
}

// Sparse product X Y by rows: row i of the result accumulates x_ij y_jJ over j in row i of X (stored,
// ascending order) and J in row j of Y; the first product of an entry starts its sum.
Csr spgemm(const Csr &X, const Csr &Y) {
  Csr C;
  C.nr = X.nr;
  C.nc = Y.nc;
  C.rp.assign(1, 0);
  for (int i = 0; i < X.nr; ++i) {
    std::map<int, double> row;
    for (int k = X.rp[i]; k < X.rp[i + 1]; ++k) {
      const int j = X.ci[k];
      for (int q = Y.rp[j]; q < Y.rp[j + 1]; ++q) {
        auto it = row.find(Y.ci[q]);
        if (it == row.end())
          row.emplace(Y.ci[q], X.v[k] * Y.v[q]);
        else
          it->second += X.v[k] * Y.v[q];
      }
    }
    for (const auto &e : row) {
      C.ci.push_back(e.first);
      C.v.push_back(e.second);
    }
    C.rp.push_back((int)C.ci.size());
  }
  return C;
}

// Strength among the C points for the second pass of aggressive (A-1) coarsening (Section 5.1): C point
// i is connected to C point j != i when a path of at most two strong connections leads from i to j,
// j in S_i or j in S_k for some k in S_i (the CC block of S + S^2). Returned in C numbering, ascending.
std::vector<std::vector<int>> cc_distance2(const std::vector<std::vector<int>> &S,
                                           const std::vector<signed char> &cf) {
  const int n = (int)S.size();
  std::vector<int> cidx(n, -1);
  int nc = 0;
  for (int i = 0; i < n; ++i)
    if (cf[i] == 1) cidx[i] = nc++;
  std::vector<std::vector<int>> G(nc);
  for (int i = 0; i < n; ++i) {
    if (cf[i] != 1) continue;
    std::set<int> reach;
    for (int k : S[i]) {
      if (cf[k] == 1 && k != i) reach.insert(cidx[k]);
      for (int j : S[k])
        if (cf[j] == 1 && j != i) reach.insert(cidx[j]);
    }
    G[cidx[i]].assign(reach.begin(), reach.end());
  }
  return G;
}

// Galerkin coarse operator A_c = P^T A P (Section 5, A_k = R_k A_{k-1} P_k with R_k = P_k^T).
// AP first: row i of AP accumulates a_ij p_jJ over j ascending in row i of A and J in row j of P.
// Then A_c[I][J] accumulates p_iI ap_iJ over fine rows i ascending. The pattern is the structural
// union of every touched (I, J); computed zeros are kept.
Csr galerkin(const Csr &A, const Csr &P) {
  std::vector<std::map<int, double>> AP(A.nr);
  for (int i = 0; i < A.nr; ++i) {
    auto &row = AP[i];
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int j = A.ci[k];
      const double a = A.v[k];
      for (int kk = P.rp[j]; kk < P.rp[j + 1]; ++kk) {
        auto it = row.find(P.ci[kk]);
        if (it == row.end())
          row.emplace(P.ci[kk], a * P.v[kk]);
        else
          it->second += a * P.v[kk];
      }
    }
  }
  std::vector<std::map<int, double>> Ac(P.nc);
  for (int i = 0; i < A.nr; ++i) {
    for (int kk = P.rp[i]; kk < P.rp[i + 1]; ++kk) {
      const int I = P.ci[kk];
      const double p = P.v[kk];
      auto &row = Ac[I];
      for (const auto &e : AP[i]) {
        auto it = row.find(e.first);
        if (it == row.end())
          row.emplace(e.first, p * e.second);
        else
          it->second += p * e.second;
      }
    }
    AP[i].clear();
  }
  Csr C;
  C.nr = C.nc = P.nc;
  C.rp.assign(1, 0);
  for (auto &row : Ac) {
    for (auto &e : row) {
      C.ci.push_back(e.first);
      C.v.push_back(e.second);
    }
    C.rp.push_back((int)C.ci.size());
  }
  return C;
}

// ILU(0) in IKJ order on A's pattern (Section 1, "ILU factorization"; the smoother of Section 5.3):
// for each row i, for k < i in the row: a_ik /= a_kk, then a_ij -= a_ik a_kj for j > k present in
// both row i and row k. The result holds L (strict lower, unit diagonal implied) and U.
std::vector<double> ilu0(const Csr &A) {
  std::vector<double> w = A.v;
  for (int i = 0; i < A.nr; ++i) {
    for (int kp = A.rp[i]; kp < A.rp[i + 1]; ++kp) {
      const int k = A.ci[kp];
      if (k >= i) break;
      double pivot = 0.0;
      bool have = false;
      for (int q = A.rp[k]; q < A.rp[k + 1]; ++q)
        if (A.ci[q] == k) {
          pivot = w[q];
          have = true;
        }
      if (!have || pivot == 0.0) throw OracleError{ORC_E_ZERO_PIVOT};
      w[kp] = w[kp] / pivot;
      for (int jp = kp + 1; jp < A.rp[i + 1]; ++jp) {
        const int j = A.ci[jp];
        for (int q = A.rp[k]; q < A.rp[k + 1]; ++q)
          if (A.ci[q] == j) w[jp] -= w[kp] * w[q];
      }
    }
    bool diag_ok = false;
    for (int kp = A.rp[i]; kp < A.rp[i + 1]; ++kp)
      if (A.ci[kp] == i) diag_ok = (w[kp] != 0.0);
    if (!diag_ok) throw OracleError{ORC_E_ZERO_PIVOT};
  }
  return w;
}

// ILU(0) as a factor matrix: A's pattern with the ILU(0) values (strict lower = L_s, the rest = U).
Csr ilu0_factor(const Csr &A) {
  Csr F = A;
  F.v = ilu0(A);
  return F;
}

// ILUT(droptol, lfil), the threshold incomplete LU that Algorithm 2 factors with (Section 5.3.4; the
// paper fixes the two parameters, the dropping rule is Saad's dual-threshold ILUT). Row i is
// eliminated in a sparse work row w = a_i with tau_i = droptol * ||a_i||_2: for each k < i with
// w_k != 0, in increasing k, the multiplier w_k / u_kk is dropped when its magnitude is below tau_i and
// otherwise kept and used, w_j -= w_k u_kj for the stored entries of U's row k (j > k), which creates
// fill. Afterwards every off-diagonal w_j that is zero or below tau_i is dropped, and of the rest at most
// lfil of largest magnitude stay in the strict lower part and lfil in the strict upper part (equal
// magnitudes: the smaller column first). Returns L \ U as one CSR with sorted columns: strict lower =
// L_s (unit diagonal implied), diagonal and strict upper = U.
Csr ilut(const Csr &A, double droptol, int lfil) {
  if (!(droptol >= 0.0) || lfil < 0) throw OracleError{ORC_E_INVALID};
  const int n = A.nr;
  Csr F;
  F.nr = F.nc = n;
  F.rp.assign(1, 0);
  std::vector<int> udiag(n, -1);  // position of u_kk in F
  for (int i = 0; i < n; ++i) {
    std::map<int, double> w;
    double nrm2 = 0.0;
    for (int q = A.rp[i]; q < A.rp[i + 1]; ++q) {
      w[A.ci[q]] = A.v[q];
      nrm2 += A.v[q] * A.v[q];
    }
    const double tau = droptol * std::sqrt(nrm2);
    for (auto it = w.begin(); it != w.end() && it->first < i; ++it) {
      const int k = it->first;
      if (it->second == 0.0) continue;
      const double lik = it->second / F.v[udiag[k]];
      if (std::fabs(lik) < tau) {
        it->second = 0.0;
        continue;
      }
      it->second = lik;
      for (int q = udiag[k] + 1; q < F.rp[k + 1]; ++q) w[F.ci[q]] -= lik * F.v[q];
    }
    std::vector<std::pair<int, double>> lo, up;
    double diag = 0.0;
    for (const auto &e : w) {
      if (e.first == i) {
        diag = e.second;
      } else if (e.second != 0.0 && std::fabs(e.second) >= tau) {
        (e.first < i ? lo : up).push_back(e);
      }
    }
    if (diag == 0.0) throw OracleError{ORC_E_ZERO_PIVOT};
    auto keep_largest = [lfil](std::vector<std::pair<int, double>> &v) {
      std::sort(v.begin(), v.end(), [](const std::pair<int, double> &a, const std::pair<int, double> &b) {
        const double ma = std::fabs(a.second), mb = std::fabs(b.second);
        return ma > mb || (ma == mb && a.first < b.first);
      });
      if ((int)v.size() > lfil) v.resize(lfil);
      std::sort(v.begin(), v.end());
    };
    keep_largest(lo);
    keep_largest(up);
    for (const auto &e : lo) {
      F.ci.push_back(e.first);
      F.v.push_back(e.second);
    }
    udiag[i] = (int)F.ci.size();
    F.ci.push_back(i);
    F.v.push_back(diag);
    for (const auto &e : up) {
      F.ci.push_back(e.first);
      F.v.push_back(e.second);
    }
    F.rp.push_back((int)F.ci.size());
  }
  return F;
}

// ---------------------------------------------------------------------------------------------
// Smoothers, one sweep each: x <- x + Mhat^{-1} (b - A x).

// l1-Jacobi (the comparator of Section 6, Table 6): x <- x + D_l1^{-1} (b - A x), every row updated from
// the previous x, with (D_l1)_ii = sum_j |a_ij|, the l1 norm of row i. (The l1 smoother adds to a_ii the
// absolute couplings a row has outside its own block; on one device each row is taken as its own block,
// which makes D_l1 - A positive semidefinite for symmetric A with positive diagonal.)
void l1_jacobi(const Csr &A, const std::vector<double> &b, std::vector<double> &x) {
  const int n = A.nr;
  std::vector<double> r;
  residual(A, b, x, r);
  for (int i = 0; i < n; ++i) {
    double d = 0.0;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) d += std::fabs(A.v[k]);
    x[i] += r[i] / d;
  }
}

// Polynomial Gauss-Seidel (Section 5.2): g^(0) = D^{-1} r, then t-1 Jacobi inner iterations
// g^(j+1) = D^{-1}(r - L g^(j)) (forward) or with U (backward); every inner step uses the previous
// iterate in full, so the sweep equals the truncated Neumann series sum_{j<t} (-D^{-1}L)^j D^{-1} r.
void pgs_neumann(const Csr &A, const std::vector<double> &b, std::vector<double> &x, int t, bool fwd) {
  const int n = A.nr;
  std::vector<double> r, g(n), gn(n);
  residual(A, b, x, r);
  for (int i = 0; i < n; ++i) g[i] = r[i] / diag_of(A, i);
  for (int rep = 1; rep < t; ++rep) {
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        const int j = A.ci[k];
        if (fwd ? (j < i) : (j > i)) s += A.v[k] * g[j];
      }
      gn[i] = (r[i] - s) / diag_of(A, i);
    }
    g.swap(gn);
  }
  for (int i = 0; i < n; ++i) x[i] += g[i];
}

// Gauss-Seidel with the direct triangular solve (Section 5.2, M = D + L forward, D + U backward).
void gs_direct(const Csr &A, const std::vector<double> &b, std::vector<double> &x, bool fwd) {
  const int n = A.nr;
  std::vector<double> r, g(n, 0.0);
  residual(A, b, x, r);
  for (int q = 0; q < n; ++q) {
    const int i = fwd ? q : n - 1 - q;
    double s = 0.0;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int j = A.ci[k];
      if (fwd ? (j < i) : (j > i)) s += A.v[k] * g[j];
    }
    g[i] = (r[i] - s) / diag_of(A, i);
  }
  for (int i = 0; i < n; ++i) x[i] += g[i];
}

// ILU smoother with Jacobi triangular solves (Section 5.3.2 and Algorithm 2 without Ruiz scaling,
// row scaling D_U = diag(U) per its footnote): y = r then t-1 steps y <- r - L_s y; v = D_U^{-1} y then
// t-1 steps v <- D_U^{-1}(y - U_s v), with U_s the strict upper part of U. F holds L \ U (ILU(0) in A's
// pattern, or ILUT with its own fill).
void ilu_neumann(const Csr &A, const Csr &F, const std::vector<double> &b, std::vector<double> &x, int t) {
  const int n = A.nr;
  std::vector<double> r, y, yn(n), v(n), vn(n), du(n);
  residual(A, b, x, r);
  for (int i = 0; i < n; ++i)
    for (int k = F.rp[i]; k < F.rp[i + 1]; ++k)
      if (F.ci[k] == i) du[i] = F.v[k];
  y = r;
  for (int rep = 1; rep < t; ++rep) {
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int k = F.rp[i]; k < F.rp[i + 1]; ++k)
        if (F.ci[k] < i) s += F.v[k] * y[F.ci[k]];
      yn[i] = r[i] - s;
    }
    y.swap(yn);
  }
  for (int i = 0; i < n; ++i) v[i] = y[i] / du[i];
  for (int rep = 1; rep < t; ++rep) {
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int k = F.rp[i]; k < F.rp[i + 1]; ++k)
        if (F.ci[k] > i) s += F.v[k] * v[F.ci[k]];
      vn[i] = (y[i] - s) / du[i];
    }
    v.swap(vn);
  }
  for (int i = 0; i < n; ++i) x[i] += v[i];
}

// ILU smoother with direct forward/backward substitution (the comparator of Section 6.2, Table 7).
void ilu_direct(const Csr &A, const Csr &F, const std::vector<double> &b, std::vector<double> &x) {
  const int n = A.nr;
  std::vector<double> r, y(n), v(n);
  residual(A, b, x, r);
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int k = F.rp[i]; k < F.rp[i + 1]; ++k)
      if (F.ci[k] < i) s += F.v[k] * y[F.ci[k]];
    y[i] = r[i] - s;
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = 0.0, d = 0.0;
    for (int k = F.rp[i]; k < F.rp[i + 1]; ++k) {
      if (F.ci[k] > i) s += F.v[k] * v[F.ci[k]];
      if (F.ci[k] == i) d = F.v[k];
    }
    v[i] = (y[i] - s) / d;
  }
  for (int i = 0; i < n; ++i) x[i] += v[i];
}

// ---------------------------------------------------------------------------------------------
// Dense LU with partial pivoting for the coarsest level (Section 5: the coarse solver is direct).
struct DenseLU {
  int n = 0;
  std::vector<double> a;  // row-major n x n, overwritten by L\U
  std::vector<int> piv;
  void factor(const Csr &A) {
    n = A.nr;
    a.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) a[(size_t)i * n + A.ci[k]] = A.v[k];
    piv.resize(n);
    for (int c = 0; c < n; ++c) {
      int p = c;
      for (int r = c + 1; r < n; ++r)
        if (std::fabs(a[(size_t)r * n + c]) > std::fabs(a[(size_t)p * n + c])) p = r;
      if (a[(size_t)p * n + c] == 0.0) throw OracleError{ORC_E_ZERO_PIVOT};
      piv[c] = p;
      if (p != c)
        for (int q = 0; q < n; ++q) std::swap(a[(size_t)c * n + q], a[(size_t)p * n + q]);
      for (int r = c + 1; r < n; ++r) {
        double l = a[(size_t)r * n + c] / a[(size_t)c * n + c];
        a[(size_t)r * n + c] = l;
        for (int q = c + 1; q < n; ++q) a[(size_t)r * n + q] -= l * a[(size_t)c * n + q];
      }
    }
  }
  void solve(const std::vector<double> &b, std::vector<double> &x) const {
    x = b;
    for (int c = 0; c < n; ++c) std::swap(x[c], x[piv[c]]);
    for (int r = 0; r < n; ++r)
      for (int q = 0; q < r; ++q) x[r] -= a[(size_t)r * n + q] * x[q];
    for (int r = n - 1; r >= 0; --r) {
      for (int q = r + 1; q < n; ++q) x[r] -= a[(size_t)r * n + q] * x[q];
      x[r] /= a[(size_t)r * n + r];
    }
  }
};

struct Level {
  Csr A, P, R;
  std::vector<signed char> cf;
  Csr ilu;  // L \ U of ILU(0) or ILUT (no rows when not requested)
};

struct Hierarchy {
  std::vector<Level> lv;
  DenseLU coarse;
};

// Setup: strength, RS first pass, classical interpolation, R = P^T, A_{l+1} = P^T A_l P (Section 5).
// Coarsen while n_l > max_coarse and l + 1 < max_levels; stop if the next level would be empty or
// as large as this one. ILU factors on the first ilu_levels levels (-1: all but the coarsest): ILU(0),
// or ILUT(droptol, lfil) when ilu_kind is ORC_ILU_KIND_ILUT.
// On the first agg_levels levels the coarsening is aggressive (A-1, Section 5.1): the first pass gives
// C_1 with classical interpolation P_1 and A_1 = P_1^T A P_1; a second first pass on the distance-two
// strength among the C_1 points keeps C_2 within C_1; P_2 is the classical interpolation of A_1 (its own
// strength) onto C_2, the level's interpolation is P = P_1 P_2 and its coarse operator
// A_c = P_2^T A_1 P_2 (= P^T A P). A second pass that keeps every C_1 point, or none, leaves the level
// standard.
// coarsen = ORC_COARSEN_PMIS replaces the RS first pass and classical interpolation on every level by
// PMIS (level l seeded with seed + l) and BAMG direct interpolation; it does not combine with
// aggressive coarsening.
Hierarchy *build(const Csr &A0, double theta, int max_levels, int max_coarse, int ilu_levels, int ilu_kind,
                 double droptol, int lfil, int agg_levels, int coarsen, uint64_t seed) {
  if (!(theta > 0.0 && theta <= 1.0) || max_levels < 1 || max_coarse < 1) throw OracleError{ORC_E_INVALID};
  if (ilu_kind != ORC_ILU_KIND_ILU0 && ilu_kind != ORC_ILU_KIND_ILUT) throw OracleError{ORC_E_INVALID};
  if (agg_levels < 0) throw OracleError{ORC_E_INVALID};
  if (coarsen != ORC_COARSEN_RS && coarsen != ORC_COARSEN_PMIS) throw OracleError{ORC_E_INVALID};
  if (coarsen == ORC_COARSEN_PMIS && agg_levels > 0) throw OracleError{ORC_E_INVALID};
  if (ilu_kind == ORC_ILU_KIND_ILUT && (!(droptol >= 0.0) || !std::isfinite(droptol) || lfil < 0))
    throw OracleError{ORC_E_INVALID};
  for (int i = 0; i < A0.nr; ++i)
    if (diag_of(A0, i) == 0.0) throw OracleError{ORC_E_ZERO_PIVOT};
  auto *H = new Hierarchy;
  H->lv.push_back(Level{A0, {}, {}, {}, {}});
  while (true) {
    Level &L = H->lv.back();
    const int n = L.A.nr;
    if (n <= max_coarse || (int)H->lv.size() >= max_levels) break;
    auto S = strength(L.A, theta);
    const bool use_pmis = coarsen == ORC_COARSEN_PMIS;
    auto cf = use_pmis ? pmis(S, seed + (uint64_t)(H->lv.size() - 1)) : rs_first_pass(S);
    int nc = 0;
    Csr P = use_pmis ? bamg_direct_interp(L.A, S, cf, nc) : classical_interp(L.A, S, cf, nc);
    if (nc == 0 || nc == n) break;
    Csr Ac = galerkin(L.A, P);
    if ((int)H->lv.size() <= agg_levels) {
      auto cf2 = rs_first_pass(cc_distance2(S, cf));
      int nc2 = 0;
      for (signed char c : cf2) nc2 += c;
      if (nc2 > 0 && nc2 < nc) {
        for (int i = 0; i < Ac.nr; ++i)
          if (diag_of(Ac, i) == 0.0) throw OracleError{ORC_E_ZERO_PIVOT};
        int nc2b = 0;
        Csr P2 = classical_interp(Ac, strength(Ac, theta), cf2, nc2b);
        P = spgemm(P, P2);
        Ac = galerkin(Ac, P2);
        int q = 0;  // the level's C points are C_2, marked on the fine grid
        for (int i = 0; i < n; ++i)
          if (cf[i] == 1) cf[i] = cf2[q++];
      }
    }
    for (int i = 0; i < Ac.nr; ++i)
      if (diag_of(Ac, i) == 0.0) throw OracleError{ORC_E_ZERO_PIVOT};
    L.cf = cf;
    L.R = transpose(P);
    L.P = std::move(P);
    H->lv.push_back(Level{std::move(Ac), {}, {}, {}, {}});
  }
  const int nl = (int)H->lv.size();
  for (int l = 0; l < nl - 1; ++l)
    if (ilu_levels < 0 || l < ilu_levels)
      H->lv[l].ilu = ilu_kind == ORC_ILU_KIND_ILUT ? ilut(H->lv[l].A, droptol, lfil) : ilu0_factor(H->lv[l].A);
  H->coarse.factor(H->lv.back().A);
  return H;
}

struct CycleOpts {
  int smoother, tri_mode, t, nu1, nu2;
};

// One V-cycle (Section 5; the cycle itself is the standard one the paper cites): zero initial guess,
// nu1 pre-smoothing sweeps, residual, restriction by R, coarse correction, prolongation by P,
// nu2 post-smoothing sweeps; the coarsest level is solved directly. ILU smoothing is used on the levels
// that carry ILU factors (the hybrid V-cycle of Section 6.2) and polynomial GS elsewhere; the l1-Jacobi
// comparator smooths every level with l1-Jacobi.
void vcycle(const Hierarchy &H, int l, const CycleOpts &o, const std::vector<double> &b,
            std::vector<double> &x) {
  const Level &L = H.lv[l];
  if (l == (int)H.lv.size() - 1) {
    H.coarse.solve(b, x);
    return;
  }
  const bool use_ilu = (o.smoother == ORC_SMOOTH_ILU0) && L.ilu.nr > 0;
  const bool direct = (o.tri_mode == ORC_TRI_DIRECT);
  x.assign(L.A.nr, 0.0);
  for (int s = 0; s < o.nu1; ++s) {
    if (o.smoother == ORC_SMOOTH_L1JAC)
      l1_jacobi(L.A, b, x);
    else if (use_ilu)
      direct ? ilu_direct(L.A, L.ilu, b, x) : ilu_neumann(L.A, L.ilu, b, x, o.t);
    else
      direct ? gs_direct(L.A, b, x, true) : pgs_neumann(L.A, b, x, o.t, true);
  }
  std::vector<double> r, bc, ec, corr;
  residual(L.A, b, x, r);
  spmv(L.R, r, bc);
  vcycle(H, l + 1, o, bc, ec);
  spmv(L.P, ec, corr);
  for (int i = 0; i < L.A.nr; ++i) x[i] += corr[i];
  for (int s = 0; s < o.nu2; ++s) {
    if (o.smoother == ORC_SMOOTH_L1JAC)
      l1_jacobi(L.A, b, x);
    else if (use_ilu)
      direct ? ilu_direct(L.A, L.ilu, b, x) : ilu_neumann(L.A, L.ilu, b, x, o.t);
    else
      direct ? gs_direct(L.A, b, x, false) : pgs_neumann(L.A, b, x, o.t, false);
  }
}

// ---------------------------------------------------------------------------------------------
// Low-synchronization MGS-GMRES with lagged normalisation (Section 4, Algorithm 1), right
// preconditioned and flexible (Z stored), restarted. Per iteration i = 1..m:
//   z_{i+1} = M^{-1} v_{i+1}, w = A z_{i+1}                (skipped at i = m)
//   c = V_{i+1}^T v_{i+1}, d = V_{i+1}^T w                  (the single reduction)
//   rho = sqrt(c_{i+1}); v_{i+1}, z_{i+1}, w scaled by 1/rho (lagged normalisation)
//   L_{i+1,j} = c_j / rho; q_j = d_j / rho, q_{i+1} = d_{i+1} / rho^2
//   s = T q with T = (I + L)^{-1} (forward substitution) or T = I - L (Neumann, Section 4)
//   v_{i+2} = w - V_{i+1} s; H column i = [previous s; rho]; Givens rotation; estimate |g_{i+1}|/||b||.
struct Cap {
  double *V = nullptr, *Z = nullptr, *H = nullptr;
  int *k = nullptr;
};

int fgmres(Hierarchy *Hh, const Csr &A, const std::vector<double> &b, std::vector<double> &x,
           const orc_params &p, orc_stats &st, std::vector<double> &hist, std::vector<double> &cyc,
           const Cap &cap) {
  const int n = A.nr;
  const int m = p.restart;
  CycleOpts co{p.smoother, p.tri_mode, p.inner_terms, p.pre_sweeps, p.post_sweeps};
  auto precond = [&](const std::vector<double> &v, std::vector<double> &z) {
    st.precond_apps++;
    if (p.precond == ORC_PRECOND_AMG)
      vcycle(*Hh, 0, co, v, z);
    else
      z = v;
  };
  st = orc_stats{};
  const double beta = norm2(b);
  double anorm = 0.0;
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) s += std::fabs(A.v[k]);
    anorm = std::max(anorm, s);
  }
  std::vector<double> r;
  auto finish = [&](int status, double rn) {
    st.status = status;
    st.relres_true = (beta > 0.0) ? rn / beta : 0.0;
    st.nrbe = rn / (beta + anorm * norm2(x));
    return status;
  };
  if (beta == 0.0) {
    x.assign(n, 0.0);
    return finish(ORC_OK, 0.0);
  }
  std::vector<std::vector<double>> V, Z;
  while (true) {
    residual(A, b, x, r);
    const double rn = norm2(r);
    if (!std::isfinite(rn)) throw OracleError{ORC_E_NONFINITE};
    cyc.push_back(rn / beta);
    // the stopping test's denominator: ||b|| (relative residual), or ||b|| + ||A||_inf ||x|| with the
    // cycle's starting iterate (normwise relative backward error, Section 3)
    const double denom = p.stop_rule == ORC_STOP_NRBE ? beta + anorm * norm2(x) : beta;
    if (rn / denom <= p.tol) return finish(ORC_OK, rn);
    if (st.iters >= p.max_iters) return finish(ORC_NOT_CONVERGED, rn);
    st.cycles++;
    const int me = std::min(m, p.max_iters - st.iters);
    V.assign(1, r);
    Z.assign(1, {});
    std::vector<double> w;
    precond(V[0], Z[0]);
    spmv(A, Z[0], w);
    // initial MGS step on [v_1, w] (Algorithm 1, step 3)
    const double s11 = dot(V[0], V[0]);
    const double u = dot(V[0], w);
    const double r11 = std::sqrt(s11);
    for (int q = 0; q < n; ++q) {
      V[0][q] /= r11;
      Z[0][q] /= r11;
      w[q] /= r11;
    }
    std::vector<double> Rprev(1, (u / r11) / r11);  // projection coefficients of the pending column
    std::vector<double> v2(n);
    for (int q = 0; q < n; ++q) v2[q] = w[q] - Rprev[0] * V[0][q];
    V.push_back(v2);
    std::vector<double> g(me + 1, 0.0), cs(me, 0.0), sn(me, 0.0);
    std::vector<std::vector<double>> Hc(me), Hraw(me);  // column i: rows 0..i
    std::vector<std::vector<double>> Lm(me + 1);       // row i+1 of the strictly lower L
    g[0] = r11;
    int k = 0;
    bool stop = false;
    for (int i = 1; i <= me && !stop; ++i) {
      const int cur = i;  // 0-based column index of v_{i+1}
      std::vector<double> zn;
      if (i < me) {
        precond(V[cur], zn);
        spmv(A, zn, w);
      }
      std::vector<double> c(i + 1), d(i + 1, 0.0);
      for (int j = 0; j <= i; ++j) {
        c[j] = dot(V[j], V[cur]);
        if (i < me) d[j] = dot(V[j], w);
      }
      const double rho = std::sqrt(c[i]);
      if (!std::isfinite(rho)) throw OracleError{ORC_E_NONFINITE};
      std::vector<double> h(i + 1);
      for (int j = 0; j < i; ++j) h[j] = Rprev[j];
      h[i] = rho;
      if (rho != 0.0) {
        for (int q = 0; q < n; ++q) V[cur][q] /= rho;
        if (i < me) {
          for (int q = 0; q < n; ++q) {
            zn[q] /= rho;
            w[q] /= rho;
          }
          std::vector<double> Lrow(i), qv(i + 1), s(i + 1);
          for (int j = 0; j < i; ++j) Lrow[j] = c[j] / rho;
          Lm[i] = Lrow;
          for (int j = 0; j < i; ++j) qv[j] = d[j] / rho;
          qv[i] = (d[i] / rho) / rho;
          if (p.gmres_T == ORC_T_DIRECT) {  // (I + L) s = q by forward substitution
            for (int j = 0; j <= i; ++j) {
              double acc = qv[j];
              for (int l = 0; l < j; ++l) acc -= Lm[j][l] * s[l];
              s[j] = acc;
            }
          } else {  // s = sum_{j=0..p} (-L)^j q, by Horner: s <- q, then p times s <- q - L s
            std::vector<double> prev = qv;
            for (int deg = 0; deg < p.t_degree; ++deg) {
              for (int j = 0; j <= i; ++j) {
                double acc = qv[j];
                for (int l = 0; l < j; ++l) acc -= Lm[j][l] * prev[l];
                s[j] = acc;
              }
              prev = s;
            }
          }
          std::vector<double> vn(n);
          for (int q = 0; q < n; ++q) {
            double acc = w[q];
            for (int j = 0; j <= i; ++j) acc -= s[j] * V[j][q];
            vn[q] = acc;
          }
          V.push_back(vn);
          Z.push_back(zn);
          Rprev = s;
        }
      }
      Hraw[i - 1] = h;
      for (int j = 0; j < i - 1; ++j) {
        const double a = h[j], bb = h[j + 1];
        h[j] = cs[j] * a + sn[j] * bb;
        h[j + 1] = -sn[j] * a + cs[j] * bb;
      }
      if (h[i] == 0.0) {
        cs[i - 1] = 1.0;
        sn[i - 1] = 0.0;
      } else {
        const double den = std::hypot(h[i - 1], h[i]);
        cs[i - 1] = h[i - 1] / den;
        sn[i - 1] = h[i] / den;
      }
      h[i - 1] = cs[i - 1] * h[i - 1] + sn[i - 1] * h[i];
      h[i] = 0.0;
      g[i] = -sn[i - 1] * g[i - 1];
      g[i - 1] = cs[i - 1] * g[i - 1];
      Hc[i - 1] = h;
      st.iters++;
      const double est = std::fabs(g[i]) / beta;
      hist.push_back(est);
      st.relres_est = est;
      k = i;
      if (std::fabs(g[i]) / denom <= p.tol || i == me || rho == 0.0) stop = true;
    }
    // y from the rotated k x k triangle, then x += Z_k y (Algorithm 1, steps 14-15)
    std::vector<double> y(k, 0.0);
    for (int j = k - 1; j >= 0; --j) {
      double acc = g[j];
      for (int l = j + 1; l < k; ++l) acc -= Hc[l][j] * y[l];
      y[j] = acc / Hc[j][j];
    }
    for (int q = 0; q < n; ++q) {
      double acc = 0.0;
      for (int j = 0; j < k; ++j) acc += Z[j][q] * y[j];
      x[q] += acc;
    }
    if (cap.k) {
      *cap.k = k;
      for (int j = 0; j <= k && j < (int)V.size(); ++j)
        if (cap.V) std::memcpy(cap.V + (size_t)j * n, V[j].data(), sizeof(double) * n);
      for (int j = 0; j < k; ++j) {
        if (cap.Z) std::memcpy(cap.Z + (size_t)j * n, Z[j].data(), sizeof(double) * n);
        if (cap.H)
          for (int l = 0; l <= j + 1; ++l) cap.H[(size_t)j * (m + 1) + l] = Hraw[j][l];
      }
    }
  }
}

template <class F>
int guarded(F &&f) {
  try {
    return f();
  } catch (const OracleError &e) {
    return e.code;
  } catch (...) {
    return ORC_E_INVALID;
  }
}

}  // namespace

extern "C" {

int orc_spmv(int n_rows, const int *rp, const int *ci, const double *v, const double *x, double *y) {
  return guarded([&]() -> int {
    int ncol = 0;
    for (int k = 0; k < rp[n_rows]; ++k) ncol = std::max(ncol, ci[k] + 1);
    Csr A = make_csr(n_rows, ncol, rp, ci, v);
    std::vector<double> xv(x, x + ncol), yv;
    spmv(A, xv, yv);
    std::copy(yv.begin(), yv.end(), y);
    return ORC_OK;
  });
}

int orc_strength(int n, const int *rp, const int *ci, const double *v, double theta, int *S_rp, int *S_ci) {
  return guarded([&]() -> int {
    Csr A = make_csr(n, n, rp, ci, v);
    auto S = strength(A, theta);
    S_rp[0] = 0;
    int c = 0;
    for (int i = 0; i < n; ++i) {
      for (int j : S[i]) S_ci[c++] = j;
      S_rp[i + 1] = c;
    }
    return ORC_OK;
  });
}

int orc_coarsen(int n, const int *rp, const int *ci, const double *v, double theta, signed char *cf) {
  return guarded([&]() -> int {
    Csr A = make_csr(n, n, rp, ci, v);
    auto c = rs_first_pass(strength(A, theta));
    std::copy(c.begin(), c.end(), cf);
    return ORC_OK;
  });
}

unsigned long long orc_splitmix64(unsigned long long seed, unsigned long long k) {
  return splitmix64_output(seed, k);
}

double orc_uniform01(unsigned long long seed, long long i) { return uniform01(seed, i); }

int orc_ilu0(int n, const int *rp, const int *ci, const double *v, double *out) {
  return guarded([&]() -> int {
    Csr A = make_csr(n, n, rp, ci, v);
    auto w = ilu0(A);
    std::copy(w.begin(), w.end(), out);
    return ORC_OK;
  });
}

int orc_smooth(int n, const int *rp, const int *ci, const double *v, int kind, int t, const double *b, double *x) {
  return guarded([&]() -> int {
    Csr A = make_csr(n, n, rp, ci, v);
    if (t < 1) return (int)ORC_E_INVALID;
    std::vector<double> bv(b, b + n), xv(x, x + n);
    switch (kind) {
      case ORC_PGS_FWD: pgs_neumann(A, bv, xv, t, true); break;
      case ORC_PGS_BWD: pgs_neumann(A, bv, xv, t, false); break;
      case ORC_GS_FWD: gs_direct(A, bv, xv, true); break;
      case ORC_GS_BWD: gs_direct(A, bv, xv, false); break;
      case ORC_ILU_NEUMANN: ilu_neumann(A, ilu0_factor(A), bv, xv, t); break;
      case ORC_ILU_DIRECT: ilu_direct(A, ilu0_factor(A), bv, xv); break;
      case ORC_L1_JACOBI: l1_jacobi(A, bv, xv); break;
      default: return (int)ORC_E_INVALID;
    }
    std::copy(xv.begin(), xv.end(), x);
    return ORC_OK;
  });
}

int orc_ilut(int n, const int *rp, const int *ci, const double *v, double droptol, int lfil, long long cap,
             int *frp, int *fci, double *fv, long long *nnz) {
  return guarded([&]() -> int {
    Csr A = make_csr(n, n, rp, ci, v);
    Csr F = ilut(A, droptol, lfil);
    *nnz = (long long)F.ci.size();
    if (*nnz > cap) return (int)ORC_E_INVALID;
    std::copy(F.rp.begin(), F.rp.end(), frp);
    std::copy(F.ci.begin(), F.ci.end(), fci);
    std::copy(F.v.begin(), F.v.end(), fv);
    return ORC_OK;
  });
}

int orc_smooth_ilut(int n, const int *rp, const int *ci, const double *v, double droptol, int lfil, int direct,
                    int t, const double *b, double *x) {
  return guarded([&]() -> int {
    Csr A = make_csr(n, n, rp, ci, v);
    if (t < 1) return (int)ORC_E_INVALID;
    Csr F = ilut(A, droptol, lfil);
    std::vector<double> bv(b, b + n), xv(x, x + n);
    direct ? ilu_direct(A, F, bv, xv) : ilu_neumann(A, F, bv, xv, t);
    std::copy(xv.begin(), xv.end(), x);
    return ORC_OK;
  });
}

void *orc_setup(int n, const int *rp, const int *ci, const double *v, double theta, int max_levels,
                int max_coarse, int ilu_levels, int ilu_kind, double droptol, int lfil, int agg_levels,
                int coarsen, unsigned long long seed, int *status) {
  Hierarchy *H = nullptr;
  int s = guarded([&]() -> int {
    Csr A = make_csr(n, n, rp, ci, v);
    if (n < 1) return (int)ORC_E_INVALID;
    H = build(A, theta, max_levels, max_coarse, ilu_levels, ilu_kind, droptol, lfil, agg_levels, coarsen,
              (uint64_t)seed);
    return ORC_OK;
  });
  if (status) *status = s;
  return H;
}

void orc_free(void *h) { delete static_cast<Hierarchy *>(h); }

int orc_num_levels(const void *h) { return (int)static_cast<const Hierarchy *>(h)->lv.size(); }

int orc_level_info(const void *h, int l, int *n, long long *nnzA, long long *nnzP, int *ncoarse) {
  const auto *H = static_cast<const Hierarchy *>(h);
  if (l < 0 || l >= (int)H->lv.size()) return ORC_E_INVALID;
  const Level &L = H->lv[l];
  *n = L.A.nr;
  *nnzA = (long long)L.A.ci.size();
  *nnzP = (long long)L.P.ci.size();
  *ncoarse = L.P.nc;
  return ORC_OK;
}

int orc_level_export(const void *h, int l, signed char *cf, int *Arp, int *Aci, double *Av, int *Prp,
                     int *Pci, double *Pv) {
  const auto *H = static_cast<const Hierarchy *>(h);
  if (l < 0 || l >= (int)H->lv.size()) return ORC_E_INVALID;
  const Level &L = H->lv[l];
  if (cf) std::copy(L.cf.begin(), L.cf.end(), cf);
  if (Arp) std::copy(L.A.rp.begin(), L.A.rp.end(), Arp);
  if (Aci) std::copy(L.A.ci.begin(), L.A.ci.end(), Aci);
  if (Av) std::copy(L.A.v.begin(), L.A.v.end(), Av);
  if (!L.P.rp.empty()) {
    if (Prp) std::copy(L.P.rp.begin(), L.P.rp.end(), Prp);
    if (Pci) std::copy(L.P.ci.begin(), L.P.ci.end(), Pci);
    if (Pv) std::copy(L.P.v.begin(), L.P.v.end(), Pv);
  }
  return ORC_OK;
}

int orc_vcycle(void *h, int smoother, int tri_mode, int t, int nu1, int nu2, const double *b, double *x) {
  return guarded([&]() -> int {
    auto *H = static_cast<Hierarchy *>(h);
    if (t < 1 || nu1 < 0 || nu2 < 0) return (int)ORC_E_INVALID;
    const int n = H->lv[0].A.nr;
    std::vector<double> bv(b, b + n), xv;
    vcycle(*H, 0, CycleOpts{smoother, tri_mode, t, nu1, nu2}, bv, xv);
    std::copy(xv.begin(), xv.end(), x);
    return ORC_OK;
  });
}

int orc_solve(void *h, const double *b, double *x, const orc_params *p, orc_stats *st, double *hist,
              int hist_cap, int *hist_len, double *cyc_hist, int cyc_cap, int *cyc_len, double *cap_V,
              double *cap_Z, double *cap_H, int *cap_k) {
  return guarded([&]() -> int {
    auto *H = static_cast<Hierarchy *>(h);
    if (!(p->tol > 0.0) || p->restart < 1 || p->max_iters < 0 || p->inner_terms < 1 || p->t_degree < 1 ||
        (p->stop_rule != ORC_STOP_RELRES && p->stop_rule != ORC_STOP_NRBE))
      return (int)ORC_E_INVALID;
    const Csr &A = H->lv[0].A;
    const int n = A.nr;
    std::vector<double> bv(b, b + n), xv(x, x + n), hv, cv;
    for (int i = 0; i < n; ++i)
      if (!std::isfinite(b[i]) || !std::isfinite(x[i])) return (int)ORC_E_NONFINITE;
    orc_stats s{};
    Cap cap{cap_V, cap_Z, cap_H, cap_k};
    int status = fgmres(H, A, bv, xv, *p, s, hv, cv, cap);
    std::copy(xv.begin(), xv.end(), x);
    if (st) *st = s;
    if (hist) {
      const int c = std::min<int>(hist_cap, (int)hv.size());
      std::copy(hv.begin(), hv.begin() + c, hist);
    }
    if (hist_len) *hist_len = (int)hv.size();
    if (cyc_hist) {
      const int c = std::min<int>(cyc_cap, (int)cv.size());
      std::copy(cv.begin(), cv.begin() + c, cyc_hist);
    }
    if (cyc_len) *cyc_len = (int)cv.size();
    return status;
  });
}

double orc_loss_orth(int n, int k, const double *V) {
  double s = 0.0;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      double d = 0.0;
      for (int q = 0; q < n; ++q) d += V[(size_t)i * n + q] * V[(size_t)j * n + q];
      const double e = (i == j ? 1.0 : 0.0) - d;
      s += e * e;
    }
  return std::sqrt(s);
}

}  // extern "C"

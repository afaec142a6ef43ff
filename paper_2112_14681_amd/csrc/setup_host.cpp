// Host-side AMG setup (Section 5 and 5.1 of arXiv 2112.14681, plus ILU(0) of Section 5.3).
//
// Canonical arithmetic (so that two independent setups produce bit-identical coarse operators and
// therefore identical C/F splittings on every level):
//   * strength: thr_i = theta * max_{k != i} |a_ik| (one multiply); j is strong iff |a_ij| >= thr_i;
//   * interpolation weights: den_k summed over the strong C set in ascending column order; the
//     numerator starts at a_ij and adds (a_ik * a_kj) / den_k for strong F neighbours k in ascending
//     order; the denominator starts at a_ii and adds the weak entries in ascending column order;
//   * Galerkin product: AP row i accumulates a_ij * p_jJ for j ascending; A_c row I accumulates
//     p_iI * ap_iJ for fine rows i ascending; every touched position is kept (no zero dropping).
#include "setup_host.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <queue>

#include "../../include/namg.h"
#include "gpu_setup.hpp"

namespace namg {

namespace {

[[noreturn]] void fail(int code, const std::string &msg) { throw SetupError{code, msg}; }

double diagonal(const HostCsr &A, int32_t i) {
  const int32_t *b = A.ci.data() + A.rp[i], *e = A.ci.data() + A.rp[i + 1];
  const int32_t *p = std::lower_bound(b, e, i);
  if (p == e || *p != i) fail(NAMG_E_ZERO_PIVOT, "missing diagonal in row " + std::to_string(i));
  return A.v[A.rp[i] + (p - b)];
}

// ---- strength of connection: S in CSR form -------------------------------------------------------
struct Graph {
  std::vector<int32_t> rp, ci;
};

Graph strength_graph(const HostCsr &A, double theta) {
  Graph S;
  S.rp.assign(A.nr + 1, 0);
  S.ci.reserve(A.ci.size());
  for (int32_t i = 0; i < A.nr; ++i) {
    double mx = 0.0;
    for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (A.ci[k] != i) {
        double a = std::fabs(A.v[k]);
        if (a > mx) mx = a;
      }
    if (mx > 0.0) {
      const double thr = theta * mx;
      for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
        if (A.ci[k] != i && std::fabs(A.v[k]) >= thr) S.ci.push_back(A.ci[k]);
    }
    S.rp[i + 1] = (int32_t)S.ci.size();
  }
  return S;
}

Graph transpose_graph(const Graph &S, int32_t n) {
  Graph T;
  T.rp.assign(n + 1, 0);
  for (int32_t j : S.ci) T.rp[j + 1]++;
  for (int32_t i = 0; i < n; ++i) T.rp[i + 1] += T.rp[i];
  T.ci.resize(S.ci.size());
  std::vector<int32_t> fill(T.rp.begin(), T.rp.end() - 1);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t k = S.rp[i]; k < S.rp[i + 1]; ++k) T.ci[fill[S.ci[k]]++] = i;
  return T;
}

// ---- Ruge-Stueben first pass ------------------------------------------------------------------------
// Undecided points are kept in one bucket per measure value. A bucket is a 64-ary tree of bitsets over the
// point index, so its smallest member is found with one count-trailing-zeros per tree level, and a point
// moves between buckets in O(1) word updates. The next point to colour is the smallest index in the
// highest non-empty bucket: the largest measure, ties broken by the smallest index.
class BitTree {
 public:
  void init(int32_t n) {
    size_t m = (size_t)std::max<int32_t>(n, 1);
    do {
      const size_t words = (m + 63) / 64;
      lv_.emplace_back(words, 0ull);
      m = words;
    } while (m > 1);
  }
  bool ready() const { return !lv_.empty(); }
  void set(int32_t i) {
    size_t bit = (size_t)i;
    for (auto &L : lv_) {
      uint64_t &w = L[bit >> 6];
      const bool was_empty = (w == 0);
      w |= 1ull << (bit & 63);
      if (!was_empty) break;
      bit >>= 6;
    }
  }
  void clear(int32_t i) {
    size_t bit = (size_t)i;
    for (auto &L : lv_) {
      uint64_t &w = L[bit >> 6];
      w &= ~(1ull << (bit & 63));
      if (w != 0) break;
      bit >>= 6;
    }
  }
  int32_t first() const {
    size_t word = 0;
    for (int k = (int)lv_.size() - 1; k >= 0; --k) word = word * 64 + (size_t)__builtin_ctzll(lv_[k][word]);
    return (int32_t)word;
  }

 private:
  std::vector<std::vector<uint64_t>> lv_;
};

class MeasureBuckets {
 public:
  MeasureBuckets(int32_t n, int32_t max_measure) : n_(n), tree_(max_measure + 1), count_(max_measure + 1, 0) {}
  void insert(int32_t i, int32_t m) {
    if (!tree_[m].ready()) tree_[m].init(n_);
    tree_[m].set(i);
    count_[m]++;
    if (m > top_) top_ = m;
  }
  void erase(int32_t i, int32_t m) {
    tree_[m].clear(i);
    count_[m]--;
  }
  bool empty() {
    while (top_ >= 0 && count_[top_] == 0) --top_;
    return top_ < 0;
  }
  int32_t top() const { return top_; }
  int32_t smallest_in_top() const { return tree_[top_].first(); }

 private:
  int32_t n_, top_ = -1;
  std::vector<BitTree> tree_;
  std::vector<int32_t> count_;
};

// C/F splitting (1 = C, 0 = F). Measure lambda_i = |S^T_i & U| + 2 |S^T_i & F|, maintained incrementally:
// a point turning F adds 1 to every undecided point it depends on, a point turning C subtracts 1.
std::vector<int8_t> rs_coarsen(const Graph &S, int32_t n) {
  const Graph ST = transpose_graph(S, n);
  enum : int8_t { UNDECIDED = -1, FPT = 0, CPT = 1 };
  std::vector<int8_t> st(n, UNDECIDED);
  std::vector<int32_t> lam(n, 0);
  int32_t maxm = 0;
  for (int32_t i = 0; i < n; ++i) maxm = std::max(maxm, 2 * (ST.rp[i + 1] - ST.rp[i]));
  MeasureBuckets B(n, maxm);
  for (int32_t i = 0; i < n; ++i) {
    if (S.rp[i + 1] == S.rp[i] && ST.rp[i + 1] == ST.rp[i]) {
      st[i] = FPT;
    } else {
      lam[i] = ST.rp[i + 1] - ST.rp[i];
      B.insert(i, lam[i]);
    }
  }
  std::vector<int32_t> fresh;
  while (!B.empty()) {
    const int32_t i = B.smallest_in_top();
    B.erase(i, lam[i]);
    st[i] = CPT;
    fresh.clear();
    for (int32_t k = ST.rp[i]; k < ST.rp[i + 1]; ++k) {
      const int32_t j = ST.ci[k];
      if (st[j] == UNDECIDED) {
        st[j] = FPT;
        B.erase(j, lam[j]);
        fresh.push_back(j);
      }
    }
    for (int32_t j : fresh)
      for (int32_t k = S.rp[j]; k < S.rp[j + 1]; ++k) {
        const int32_t q = S.ci[k];
        if (st[q] == UNDECIDED) {
          B.erase(q, lam[q]);
          B.insert(q, ++lam[q]);
        }
      }
    for (int32_t k = S.rp[i]; k < S.rp[i + 1]; ++k) {
      const int32_t q = S.ci[k];
      if (st[q] == UNDECIDED) {
        B.erase(q, lam[q]);
        B.insert(q, --lam[q]);
      }
    }
  }
  return st;
}

// ---- classical interpolation -------------------------------------------------------------------------
// Second-pass strength of aggressive (A-1) coarsening: among the C points (numbered in fine order), C
// point i is connected to C point j != i when j is in S_i or in S_k for some k in S_i (the CC block of
// S + S^2). A marker per C point collects each row once; rows come out sorted.
Graph cc_distance2(const Graph &S, const std::vector<int8_t> &cf) {
  const int32_t n = (int32_t)cf.size();
  std::vector<int32_t> cnum(n, -1);
  int32_t nc = 0;
  for (int32_t i = 0; i < n; ++i)
    if (cf[i] == 1) cnum[i] = nc++;
  Graph G;
  G.rp.assign(nc + 1, 0);
  std::vector<int32_t> mark(nc, -1);
  for (int32_t i = 0; i < n; ++i) {
    if (cf[i] != 1) continue;
    const int32_t I = cnum[i];
    const size_t start = G.ci.size();
    auto add = [&](int32_t j) {
      if (j != i && cf[j] == 1 && mark[cnum[j]] != I) {
        mark[cnum[j]] = I;
        G.ci.push_back(cnum[j]);
      }
    };
    for (int32_t q = S.rp[i]; q < S.rp[i + 1]; ++q) {
      const int32_t k = S.ci[q];
      add(k);
      for (int32_t r = S.rp[k]; r < S.rp[k + 1]; ++r) add(S.ci[r]);
    }
    std::sort(G.ci.begin() + start, G.ci.end());
    G.rp[I + 1] = (int32_t)G.ci.size();
  }
  return G;
}

HostCsr classical_interpolation(const HostCsr &A, const Graph &S, const std::vector<int8_t> &cf) {
  const int32_t n = A.nr;
  std::vector<int32_t> cnum(n, -1);
  int32_t nc = 0;
  for (int32_t i = 0; i < n; ++i)
    if (cf[i] == 1) cnum[i] = nc++;
  HostCsr P;
  P.nr = n;
  P.nc = nc;
  P.rp.assign(n + 1, 0);
  // role[j] for the current row: 0 none, 1 strong C, 2 strong F, 3 strong F treated as weak
  std::vector<int8_t> role(n, 0);
  std::vector<double> num(n, 0.0), aval(n, 0.0), dens;
  std::vector<int32_t> strongF, cpos;
  std::vector<std::pair<int32_t, double>> centries;
  for (int32_t i = 0; i < n; ++i) {
    if (cf[i] == 1) {
      P.ci.push_back(cnum[i]);
      P.v.push_back(1.0);
      P.rp[i + 1] = (int32_t)P.ci.size();
      continue;
    }
    bool anyC = false;
    strongF.clear();
    for (int32_t k = S.rp[i]; k < S.rp[i + 1]; ++k) {
      const int32_t j = S.ci[k];
      if (cf[j] == 1) {
        role[j] = 1;
        anyC = true;
      } else {
        role[j] = 2;
        strongF.push_back(j);
      }
    }
    if (anyC) {
      // one scan of each strong F neighbour's row: its entries in the strong C set (in row order) are
      // kept for the distribution below, and their sum is the denominator
      dens.assign(strongF.size(), 0.0);
      cpos.assign(strongF.size() + 1, 0);
      centries.clear();
      for (size_t q = 0; q < strongF.size(); ++q) {
        const int32_t k = strongF[q];
        double s = 0.0;
        for (int32_t p = A.rp[k]; p < A.rp[k + 1]; ++p)
          if (role[A.ci[p]] == 1) {
            s += A.v[p];
            centries.emplace_back(A.ci[p], A.v[p]);
          }
        dens[q] = s;
        cpos[q + 1] = (int32_t)centries.size();
        if (s == 0.0) role[k] = 3;
      }
      double dd = 0.0;
      for (int32_t p = A.rp[i]; p < A.rp[i + 1]; ++p) {
        const int32_t j = A.ci[p];
        if (j == i) dd = A.v[p];
      }
      for (int32_t p = A.rp[i]; p < A.rp[i + 1]; ++p) {
        const int32_t j = A.ci[p];
        if (j != i && (role[j] == 0 || role[j] == 3)) dd += A.v[p];
      }
      for (int32_t p = A.rp[i]; p < A.rp[i + 1]; ++p)
        if (role[A.ci[p]] == 1) num[A.ci[p]] = A.v[p];
      // strong F neighbours in ascending order; their rows distribute into the strong C set
      for (int32_t p = A.rp[i]; p < A.rp[i + 1]; ++p) aval[A.ci[p]] = A.v[p];
      for (size_t q = 0; q < strongF.size(); ++q) {
        if (dens[q] == 0.0) continue;
        const double aik = aval[strongF[q]];
        for (int32_t e = cpos[q]; e < cpos[q + 1]; ++e) num[centries[e].first] += (aik * centries[e].second) / dens[q];
      }
      for (int32_t k = S.rp[i]; k < S.rp[i + 1]; ++k) {
        const int32_t j = S.ci[k];
        if (cf[j] == 1) {
          P.ci.push_back(cnum[j]);
          P.v.push_back(-num[j] / dd);
        }
      }
    }
    for (int32_t k = S.rp[i]; k < S.rp[i + 1]; ++k) role[S.ci[k]] = 0;
    P.rp[i + 1] = (int32_t)P.ci.size();
  }
  return P;
}

HostCsr transpose_csr(const HostCsr &P) {
  HostCsr R;
  R.nr = P.nc;
  R.nc = P.nr;
  R.rp.assign(R.nr + 1, 0);
  for (int32_t j : P.ci) R.rp[j + 1]++;
  for (int32_t i = 0; i < R.nr; ++i) R.rp[i + 1] += R.rp[i];
  R.ci.resize(P.ci.size());
  R.v.resize(P.v.size());
  std::vector<int32_t> fill(R.rp.begin(), R.rp.end() - 1);
  for (int32_t i = 0; i < P.nr; ++i)
    for (int32_t k = P.rp[i]; k < P.rp[i + 1]; ++k) {
      const int32_t d = fill[P.ci[k]]++;
      R.ci[d] = i;
      R.v[d] = P.v[k];
    }
  return R;
}

// C = X * Y, row by row (Gustavson). Row i of C accumulates x_ij * y_jJ over the entries of row i of X in
// stored order and, inside, over row j of Y in stored order; every c_iJ is that running sum, so the
// result does not depend on how the accumulator is stored. The accumulator is a small open-addressing
// table sized for the row (it stays in the L1 cache), not an array over all columns. Columns of each row
// come out sorted.
HostCsr spgemm(const HostCsr &X, const HostCsr &Y) {
  HostCsr C;
  C.nr = X.nr;
  C.nc = Y.nc;
  C.rp.assign(X.nr + 1, 0);
  std::vector<int32_t> key, cols;
  std::vector<double> acc;
  std::vector<std::pair<int32_t, double>> row;
  C.ci.reserve(X.ci.size() * 4);
  C.v.reserve(X.ci.size() * 4);
  for (int32_t i = 0; i < X.nr; ++i) {
    int64_t bound = 0;
    for (int32_t k = X.rp[i]; k < X.rp[i + 1]; ++k) bound += Y.rp[X.ci[k] + 1] - Y.rp[X.ci[k]];
    size_t cap = 16;
    while ((int64_t)cap < 2 * bound) cap <<= 1;
    if (key.size() < cap) {
      key.assign(cap, -1);
      acc.resize(cap);
    }
    const size_t mask = cap - 1;
    cols.clear();
    for (int32_t k = X.rp[i]; k < X.rp[i + 1]; ++k) {
      const int32_t j = X.ci[k];
      const double x = X.v[k];
      for (int32_t q = Y.rp[j]; q < Y.rp[j + 1]; ++q) {
        const int32_t J = Y.ci[q];
        const double prod = x * Y.v[q];
        size_t h = ((uint32_t)J * 2654435761u) & mask;
        while (key[h] != J && key[h] != -1) h = (h + 1) & mask;
        if (key[h] == -1) {
          key[h] = J;
          acc[h] = prod;
          cols.push_back((int32_t)h);
        } else {
          acc[h] += prod;
        }
      }
    }
    row.clear();
    for (int32_t h : cols) {
      row.emplace_back(key[h], acc[h]);
      key[h] = -1;
    }
    std::sort(row.begin(), row.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    for (const auto &e : row) {
      C.ci.push_back(e.first);
      C.v.push_back(e.second);
    }
    C.rp[i + 1] = (int32_t)C.ci.size();
  }
  return C;
}

// ILU(0) in IKJ order on A's pattern; returns factor values in A's positions (strict lower: L_s with
// unit diagonal implied; diagonal and upper: U).
std::vector<double> ilu0_values(const HostCsr &A) {
  const int32_t n = A.nr;
  std::vector<double> w = A.v;
  std::vector<int32_t> pos(n, -1), dpos(n, -1);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (A.ci[k] == i) dpos[i] = k;
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) pos[A.ci[k]] = k;
    for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int32_t c = A.ci[k];
      if (c >= i) break;
      const double piv = w[dpos[c]];
      if (piv == 0.0) fail(NAMG_E_ZERO_PIVOT, "zero ILU(0) pivot in row " + std::to_string(c));
      w[k] /= piv;
      const double lik = w[k];
      for (int32_t q = dpos[c] + 1; q < A.rp[c + 1]; ++q) {
        const int32_t p = pos[A.ci[q]];
        if (p >= 0) w[p] -= lik * w[q];
      }
    }
    if (w[dpos[i]] == 0.0) fail(NAMG_E_ZERO_PIVOT, "zero ILU(0) pivot in row " + std::to_string(i));
    for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) pos[A.ci[k]] = -1;
  }
  return w;
}

// ILUT(droptol, lfil) with Saad's dual threshold (Algorithm 2 factors with it, Section 5.3.4). Row i is
// eliminated in a dense work row w (scattered from a_i, reset through its list of touched columns), with
// tau_i = droptol * ||a_i||_2. The lower positions of w are taken in increasing column order from a
// min-heap, which also receives fill created below the diagonal: the multiplier w_k / u_kk is dropped
// when below tau_i, else kept and used (w_j -= l_ik u_kj over U's finished row k). Each w_j thus takes its
// updates in increasing k, the same sequence of roundings as any other increasing-k elimination.
// Afterwards off-diagonal entries that are zero or below tau_i go, and at most lfil of the largest
// magnitude (ties: smaller column) stay in each strict triangle. Returns L \ U with sorted columns.
HostCsr ilut_factor(const HostCsr &A, double droptol, int32_t lfil) {
  const int32_t n = A.nr;
  HostCsr F;
  F.nr = F.nc = n;
  F.rp.assign(n + 1, 0);
  F.ci.reserve((size_t)n * (2 * (size_t)std::min<int32_t>(lfil, 8) + 1));
  F.v.reserve(F.ci.capacity());
  std::vector<int32_t> udiag(n, -1), touched;
  std::vector<double> w(n, 0.0);
  std::vector<uint8_t> in(n, 0);
  std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>> lower;
  std::vector<std::pair<int32_t, double>> lo, up;
  auto by_magnitude = [](const std::pair<int32_t, double> &a, const std::pair<int32_t, double> &b) {
    const double ma = std::fabs(a.second), mb = std::fabs(b.second);
    return ma > mb || (ma == mb && a.first < b.first);
  };
  auto keep_largest = [&](std::vector<std::pair<int32_t, double>> &v) {
    if ((int64_t)v.size() > lfil) {
      std::nth_element(v.begin(), v.begin() + lfil, v.end(), by_magnitude);
      v.resize(lfil);
    }
    std::sort(v.begin(), v.end());
  };
  for (int32_t i = 0; i < n; ++i) {
    double nrm2 = 0.0;
    for (int32_t q = A.rp[i]; q < A.rp[i + 1]; ++q) {
      const int32_t j = A.ci[q];
      w[j] = A.v[q];
      in[j] = 1;
      touched.push_back(j);
      if (j < i) lower.push(j);
      nrm2 += A.v[q] * A.v[q];
    }
    const double tau = droptol * std::sqrt(nrm2);
    while (!lower.empty()) {
      const int32_t k = lower.top();
      lower.pop();
      if (w[k] == 0.0) continue;
      const double lik = w[k] / F.v[udiag[k]];
      if (std::fabs(lik) < tau) {
        w[k] = 0.0;
        continue;
      }
      w[k] = lik;
      for (int32_t q = udiag[k] + 1; q < F.rp[k + 1]; ++q) {
        const int32_t j = F.ci[q];
        if (!in[j]) {
          in[j] = 1;
          w[j] = 0.0;
          touched.push_back(j);
          if (j < i) lower.push(j);
        }
        w[j] -= lik * F.v[q];
      }
    }
    const double diag = in[i] ? w[i] : 0.0;
    if (diag == 0.0) fail(NAMG_E_ZERO_PIVOT, "zero ILUT pivot in row " + std::to_string(i));
    lo.clear();
    up.clear();
    for (int32_t j : touched) {
      if (j != i && w[j] != 0.0 && std::fabs(w[j]) >= tau) (j < i ? lo : up).emplace_back(j, w[j]);
      w[j] = 0.0;
      in[j] = 0;
    }
    touched.clear();
    keep_largest(lo);
    keep_largest(up);
    for (const auto &e : lo) {
      F.ci.push_back(e.first);
      F.v.push_back(e.second);
    }
    udiag[i] = (int32_t)F.ci.size();
    F.ci.push_back(i);
    F.v.push_back(diag);
    for (const auto &e : up) {
      F.ci.push_back(e.first);
      F.v.push_back(e.second);
    }
    if (F.ci.size() > (size_t)INT32_MAX) fail(NAMG_E_INVALID, "ILUT factor exceeds 2^31 entries");
    F.rp[i + 1] = (int32_t)F.ci.size();
  }
  return F;
}

// Strict lower or upper part of a pattern with values vals[k] * scale[row] (scale may be empty).
HostCsr strict_part(const HostCsr &A, const std::vector<double> &vals, bool lower,
                    const std::vector<double> &scale) {
  HostCsr T;
  T.nr = A.nr;
  T.nc = A.nc;
  T.rp.assign(A.nr + 1, 0);
  T.ci.reserve(A.ci.size() / 2 + 1);
  T.v.reserve(A.ci.size() / 2 + 1);
  for (int32_t i = 0; i < A.nr; ++i) {
    for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int32_t j = A.ci[k];
      if (lower ? (j < i) : (j > i)) {
        T.ci.push_back(j);
        T.v.push_back(scale.empty() ? vals[k] : vals[k] * scale[i]);
      }
    }
    T.rp[i + 1] = (int32_t)T.ci.size();
  }
  return T;
}

std::vector<double> dense_inverse(const HostCsr &A) {
  const int32_t n = A.nr;
  std::vector<double> a((size_t)n * n, 0.0), inv((size_t)n * n, 0.0);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) a[(size_t)i * n + A.ci[k]] = A.v[k];
  std::vector<int32_t> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  for (int32_t c = 0; c < n; ++c) {
    int32_t p = c;
    for (int32_t r = c + 1; r < n; ++r)
      if (std::fabs(a[(size_t)r * n + c]) > std::fabs(a[(size_t)p * n + c])) p = r;
    if (a[(size_t)p * n + c] == 0.0) fail(NAMG_E_ZERO_PIVOT, "singular coarsest operator");
    if (p != c) {
      for (int32_t q = 0; q < n; ++q) std::swap(a[(size_t)c * n + q], a[(size_t)p * n + q]);
      std::swap(perm[c], perm[p]);
    }
    for (int32_t r = c + 1; r < n; ++r) {
      const double l = a[(size_t)r * n + c] / a[(size_t)c * n + c];
      a[(size_t)r * n + c] = l;
      for (int32_t q = c + 1; q < n; ++q) a[(size_t)r * n + q] -= l * a[(size_t)c * n + q];
    }
  }
  std::vector<double> col(n);
  for (int32_t e = 0; e < n; ++e) {
    for (int32_t r = 0; r < n; ++r) col[r] = (perm[r] == e) ? 1.0 : 0.0;
    for (int32_t r = 0; r < n; ++r)
      for (int32_t q = 0; q < r; ++q) col[r] -= a[(size_t)r * n + q] * col[q];
    for (int32_t r = n - 1; r >= 0; --r) {
      for (int32_t q = r + 1; q < n; ++q) col[r] -= a[(size_t)r * n + q] * col[q];
      col[r] /= a[(size_t)r * n + r];
    }
    for (int32_t r = 0; r < n; ++r) inv[(size_t)r * n + e] = col[r];
  }
  return inv;
}

void smoother_data(HostLevel &L, bool with_ilu, const namg_setup_params &p, bool host_smoother) {
  const HostCsr &A = L.A;
  L.host_smoother = host_smoother;
  // without the host copy there is nothing to check either: the device setup has checked every diagonal,
  // level 0's on import and each coarse operator's as it was built
  if (host_smoother) pgs_data(A, L.dinv, L.dl1inv, L.pgs_lo, L.pgs_up);
  if (with_ilu) {
    // L \ U as one CSR: ILU(0) values in A's pattern, or the ILUT factor with its own fill
    HostCsr F;
    if (p.ilu_kind == NAMG_ILUT) {
      F = ilut_factor(A, p.ilut_droptol, p.ilut_lfil);
    } else {
      F.nr = A.nr;
      F.nc = A.nc;
      F.rp = A.rp;
      F.ci = A.ci;
      F.v = ilu0_values(A);
    }
    L.has_ilu = true;
    L.ilu_dinv.resize(A.nr);
    std::vector<double> du(A.nr);
    for (int32_t i = 0; i < A.nr; ++i)
      for (int32_t k = F.rp[i]; k < F.rp[i + 1]; ++k)
        if (F.ci[k] == i) du[i] = F.v[k];
    for (int32_t i = 0; i < A.nr; ++i) L.ilu_dinv[i] = 1.0 / du[i];
    L.ilu_diag = du;
    L.ilu_lo = strict_part(F, F.v, true, {});
    L.ilu_up = strict_part(F, F.v, false, {});
    for (int32_t i = 0; i < A.nr; ++i)
      for (int32_t k = L.ilu_up.rp[i]; k < L.ilu_up.rp[i + 1]; ++k) L.ilu_up.v[k] /= du[i];
  }
}

}  // namespace

LevelSchedule level_schedule(const HostCsr &T, bool lower) {
  const int32_t n = T.nr;
  std::vector<int32_t> lev(n, 0);
  int32_t nlev = 0;
  for (int32_t q = 0; q < n; ++q) {
    const int32_t i = lower ? q : n - 1 - q;
    int32_t l = 0;
    for (int32_t k = T.rp[i]; k < T.rp[i + 1]; ++k) l = std::max(l, lev[T.ci[k]] + 1);
    lev[i] = l;
    nlev = std::max(nlev, l + 1);
  }
  LevelSchedule s;
  s.ptr.assign(nlev + 1, 0);
  for (int32_t i = 0; i < n; ++i) s.ptr[lev[i] + 1]++;
  for (int32_t l = 0; l < nlev; ++l) s.ptr[l + 1] += s.ptr[l];
  s.order.resize(n);
  std::vector<int32_t> fill(s.ptr.begin(), s.ptr.end() - 1);
  for (int32_t i = 0; i < n; ++i) s.order[fill[lev[i]]++] = i;
  return s;
}

HostCsr import_csr(int32_t n, const int32_t *rp, const int32_t *ci, const double *v) {
  if (n < 1) fail(NAMG_E_INVALID, "n must be >= 1");
  if (!rp || !ci || !v) fail(NAMG_E_INVALID, "null CSR array");
  if (rp[0] != 0) fail(NAMG_E_INVALID, "rowptr[0] must be 0");
  for (int32_t i = 0; i < n; ++i)
    if (rp[i + 1] < rp[i]) fail(NAMG_E_INVALID, "rowptr not monotone at row " + std::to_string(i));
  HostCsr A;
  A.nr = A.nc = n;
  A.rp.assign(rp, rp + n + 1);
  const int64_t nnz = rp[n];
  A.ci.assign(ci, ci + nnz);
  A.v.assign(v, v + nnz);
  for (int32_t i = 0; i < n; ++i) {
    bool diag = false;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      if (ci[k] < 0 || ci[k] >= n) fail(NAMG_E_INVALID, "column index out of range in row " + std::to_string(i));
      if (k > rp[i] && ci[k] <= ci[k - 1])
        fail(NAMG_E_INVALID, "columns not strictly ascending in row " + std::to_string(i));
      if (!std::isfinite(v[k])) fail(NAMG_E_NONFINITE, "non-finite value in row " + std::to_string(i));
      if (ci[k] == i) {
        diag = true;
        if (v[k] == 0.0) fail(NAMG_E_ZERO_PIVOT, "zero diagonal in row " + std::to_string(i));
      }
    }
    if (!diag) fail(NAMG_E_ZERO_PIVOT, "missing diagonal in row " + std::to_string(i));
  }
  return A;
}

void validate_hierarchy_params(const namg_setup_params &p) {
  if (!(p.theta > 0.0 && p.theta <= 1.0)) fail(NAMG_E_INVALID, "theta must be in (0, 1]");
  if (p.ilu_kind != NAMG_ILU0 && p.ilu_kind != NAMG_ILUT) fail(NAMG_E_INVALID, "unknown ilu_kind");
  if (p.agg_levels < 0) fail(NAMG_E_INVALID, "agg_levels must be >= 0");
  if (p.coarsen != NAMG_COARSEN_RS && p.coarsen != NAMG_COARSEN_PMIS) fail(NAMG_E_INVALID, "unknown coarsen");
  if (p.ilu_kind == NAMG_ILUT && (!(p.ilut_droptol >= 0.0) || !std::isfinite(p.ilut_droptol) || p.ilut_lfil < 0))
    fail(NAMG_E_INVALID, "ILUT needs ilut_droptol >= 0 and ilut_lfil >= 0");
  if (p.max_levels < 1 || p.max_levels > NAMG_MAX_LEVELS) fail(NAMG_E_INVALID, "max_levels out of range");
  if (p.max_coarse < 1) fail(NAMG_E_INVALID, "max_coarse must be >= 1");
}

double inf_norm(const HostCsr &A) {
  double m = 0.0;
  for (int32_t i = 0; i < A.nr; ++i) {
    double s = 0.0;
    for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) s += std::fabs(A.v[k]);
    m = std::max(m, s);
  }
  return m;
}

HostCsr restriction_of(const HostCsr &P) { return transpose_csr(P); }

void pgs_data(const HostCsr &A, std::vector<double> &dinv, std::vector<double> &dl1inv, HostCsr &lo, HostCsr &up) {
  // One pass per row: 1 / a_ii, 1 / sum_j |a_ij| (l1-Jacobi), and D^{-1}L, D^{-1}U with entries a_ij / a_ii
  const int32_t n = A.nr;
  dinv.resize(n);
  dl1inv.resize(n);
  lo.nr = up.nr = n;
  lo.nc = up.nc = A.nc;
  lo.rp.assign(n + 1, 0);
  up.rp.assign(n + 1, 0);
  int64_t nlo = 0;
  for (int32_t i = 0; i < n; ++i) {
    const int32_t *b = A.ci.data() + A.rp[i], *e = A.ci.data() + A.rp[i + 1];
    nlo += std::lower_bound(b, e, i) - b;
  }
  const int64_t nup = A.nnz() - nlo - n;
  lo.ci.resize(nlo);
  lo.v.resize(nlo);
  up.ci.resize(std::max<int64_t>(nup, 0));
  up.v.resize(std::max<int64_t>(nup, 0));
  int64_t ql = 0, qu = 0;
  for (int32_t i = 0; i < n; ++i) {
    const double d = diagonal(A, i);
    if (d == 0.0) fail(NAMG_E_ZERO_PIVOT, "zero diagonal in row " + std::to_string(i));
    dinv[i] = 1.0 / d;
    double l1 = 0.0;
    for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int32_t j = A.ci[k];
      l1 += std::fabs(A.v[k]);
      if (j < i) {
        lo.ci[ql] = j;
        lo.v[ql++] = A.v[k] / d;
      } else if (j > i) {
        up.ci[qu] = j;
        up.v[qu++] = A.v[k] / d;
      }
    }
    dl1inv[i] = 1.0 / l1;
    lo.rp[i + 1] = (int32_t)ql;
    up.rp[i + 1] = (int32_t)qu;
  }
}

void finish_hierarchy(HostHierarchy &H, const namg_setup_params &p, bool host_smoother) {
  const int nl = (int)H.lv.size();
  for (int l = 0; l < nl - 1; ++l)
    smoother_data(H.lv[l], p.ilu_levels < 0 || l < p.ilu_levels, p, host_smoother);
  const HostCsr &Ac = H.lv.back().A;
  if (Ac.nr > 4096) fail(NAMG_E_INVALID, "coarsest level has more than 4096 rows; raise max_levels");
  H.coarse_inv = dense_inverse(Ac);
}

HostHierarchy build_hierarchy(HostCsr &&A0, const namg_setup_params &p) {
  validate_hierarchy_params(p);
  if (p.coarsen == NAMG_COARSEN_PMIS) return build_hierarchy_pmis_device(std::move(A0), p);
  return build_hierarchy(static_cast<const HostCsr &>(A0), p);
}

HostHierarchy build_hierarchy(const HostCsr &A0, const namg_setup_params &p) {
  validate_hierarchy_params(p);
  if (p.coarsen == NAMG_COARSEN_PMIS) return build_hierarchy_pmis_device(HostCsr(A0), p);
  const double theta = p.theta;
  const int max_levels = p.max_levels, max_coarse = p.max_coarse;
  HostHierarchy H;
  const bool trace = std::getenv("NAMG_SETUP_TRACE") != nullptr;
  double t_str = 0, t_rs = 0, t_int = 0, t_rap = 0;
  auto now = [] { return std::chrono::steady_clock::now(); };
  auto secs = [](auto a, auto b) { return std::chrono::duration<double>(b - a).count(); };
  H.anorm_inf = inf_norm(A0);
  H.lv.emplace_back();
  H.lv.back().A = A0;
  while (true) {
    HostLevel &L = H.lv.back();
    const int32_t n = L.A.nr;
    if (n <= max_coarse || (int)H.lv.size() >= max_levels) break;
    auto t0 = now();
    Graph S = strength_graph(L.A, theta);
    auto t1 = now();
    std::vector<int8_t> cf = rs_coarsen(S, n);
    auto t2 = now();
    HostCsr P = classical_interpolation(L.A, S, cf);
    auto t3 = now();
    if (P.nc == 0 || P.nc == n) break;
    HostCsr R = transpose_csr(P);
    HostCsr AP = spgemm(L.A, P);
    auto t3b = now();
    HostCsr Ac = spgemm(R, AP);
    if ((int)H.lv.size() <= p.agg_levels) {
      // aggressive (A-1): a second first pass on the distance-two strength among the C points keeps C_2;
      // P_2 interpolates A_1 = P_1^T A P_1 onto C_2 with A_1's own strength; P = P_1 P_2 and
      // A_c = P_2^T A_1 P_2
      std::vector<int8_t> cf2 = rs_coarsen(cc_distance2(S, cf), P.nc);
      int32_t nc2 = 0;
      for (int8_t c : cf2) nc2 += c;
      if (nc2 > 0 && nc2 < P.nc) {
        for (int32_t i = 0; i < Ac.nr; ++i)
          if (diagonal(Ac, i) == 0.0) fail(NAMG_E_ZERO_PIVOT, "zero diagonal in a coarse operator");
        HostCsr P2 = classical_interpolation(Ac, strength_graph(Ac, theta), cf2);
        HostCsr R2 = transpose_csr(P2);
        HostCsr AP2 = spgemm(Ac, P2);
        Ac = spgemm(R2, AP2);
        P = spgemm(P, P2);
        R = transpose_csr(P);
        int32_t q = 0;
        for (int32_t i = 0; i < n; ++i)
          if (cf[i] == 1) cf[i] = cf2[q++];
      }
    }
    auto t4 = now();
    t_str += secs(t0, t1);
    t_rs += secs(t1, t2);
    t_int += secs(t2, t3);
    t_rap += secs(t3, t4);
    if (trace)
      std::fprintf(stderr,
                   "[namg setup]   level %d n %d nnz %zu: strength %.3f rs %.3f interp %.3f ap %.3f r(ap) %.3f s "
                   "(nnz P %zu AP %zu Ac %zu)\n",
                   (int)H.lv.size() - 1, n, L.A.ci.size(), secs(t0, t1), secs(t1, t2), secs(t2, t3), secs(t3, t3b),
                   secs(t3b, t4), P.ci.size(), AP.ci.size(), Ac.ci.size());
    for (int32_t i = 0; i < Ac.nr; ++i)
      if (diagonal(Ac, i) == 0.0) fail(NAMG_E_ZERO_PIVOT, "zero diagonal in a coarse operator");
    L.cf = std::move(cf);
    L.P = std::move(P);
    L.R = std::move(R);
    HostLevel next;
    next.A = std::move(Ac);
    H.lv.push_back(std::move(next));
  }
  auto t5 = now();
  finish_hierarchy(H, p);
  if (trace)
    std::fprintf(stderr, "[namg setup] strength %.3f rs %.3f interp %.3f rap %.3f smoother+coarse %.3f s\n", t_str,
                 t_rs, t_int, t_rap, secs(t5, now()));
  return H;
}

}  // namespace namg

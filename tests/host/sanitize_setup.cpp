// Host-only driver for the sanitizer builds of the library's host code (setup_host.cpp, diagnostics.cpp):
// tests/test_host_sanitizers.py compiles it with g++ -fsanitize=address,undefined and runs it. It drives
// every host entry point on small matrices of the kinds the solver meets (stencils, a nonsymmetric
// upwind operator, random sparse, degenerate sizes) and the rejection of malformed input. Exit code 0 and
// no sanitizer report mean every access was in bounds and no undefined behaviour was hit.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2112_14681_amd/csrc/gpu_setup.hpp"
#include "../../paper_2112_14681_amd/csrc/setup_host.hpp"

namespace namg {
// The device setup is not part of a host-only build.
HostHierarchy build_hierarchy_pmis_device(HostCsr &&, const namg_setup_params &) {
  throw SetupError{NAMG_E_INVALID, "no device in the host-only build"};
}
}  // namespace namg

using namespace namg;

namespace {

// 7-point operator on an N^3 grid with per-direction coefficients (upwind-style asymmetry when skew > 0).
HostCsr stencil3d(int N, double skew, unsigned seed) {
  std::mt19937 gen(seed);
  std::uniform_real_distribution<double> u(0.5, 2.0);
  HostCsr A;
  A.nr = A.nc = N * N * N;
  A.rp.push_back(0);
  for (int z = 0; z < N; ++z)
    for (int y = 0; y < N; ++y)
      for (int x = 0; x < N; ++x) {
        const int p = x + N * (y + N * z);
        struct E { int c; double v; };
        std::vector<E> row;
        double diag = 0.0;
        const int d[3] = {1, N, N * N}, c[3] = {x, y, z};
        for (int a = 2; a >= 0; --a)
          if (c[a] > 0) {
            const double w = u(gen);
            row.push_back({p - d[a], -w - skew});
            diag += w + skew;
          }
        row.push_back({p, 0.0});
        const size_t di = row.size() - 1;
        for (int a = 0; a < 3; ++a)
          if (c[a] < N - 1) {
            const double w = u(gen);
            row.push_back({p + d[a], -w});
            diag += w;
          }
        row[di].v = diag + 1.0;
        for (auto &e : row) {
          A.ci.push_back(e.c);
          A.v.push_back(e.v);
        }
        A.rp.push_back((int32_t)A.ci.size());
      }
  return A;
}

HostCsr random_csr(int n, int per_row, unsigned seed) {
  std::mt19937 gen(seed);
  std::uniform_int_distribution<int> col(0, n - 1);
  std::uniform_real_distribution<double> val(-1.0, 0.2);
  HostCsr A;
  A.nr = A.nc = n;
  A.rp.push_back(0);
  for (int i = 0; i < n; ++i) {
    std::vector<double> dense(n, 0.0);
    std::vector<char> used(n, 0);
    double off = 0.0;
    for (int q = 0; q < per_row; ++q) {
      const int j = col(gen);
      if (j == i || used[j]) continue;
      used[j] = 1;
      dense[j] = val(gen);
      off += std::fabs(dense[j]);
    }
    used[i] = 1;
    dense[i] = 1.5 * off + 1.0;
    for (int j = 0; j < n; ++j)
      if (used[j]) {
        A.ci.push_back(j);
        A.v.push_back(dense[j]);
      }
    A.rp.push_back((int32_t)A.ci.size());
  }
  return A;
}

// The documented defaults of namg_setup_params (namg_default_setup_params lives in the HIP translation
// unit), host-only.
namg_setup_params defaults() {
  namg_setup_params p{};
  p.theta = 0.25;
  p.max_levels = 25;
  p.max_coarse = 50;
  p.precision = NAMG_FP64;
  p.ilu_levels = 1;
  p.device = -1;
  p.ilu_kind = NAMG_ILU0;
  p.ilut_lfil = 5;
  p.ilut_droptol = 1e-2;
  p.agg_levels = 0;
  p.coarsen = NAMG_COARSEN_RS;
  p.seed = 0;
  return p;
}

int failures = 0;

void exercise(const HostCsr &A, namg_setup_params p, const char *what) {
  try {
    HostHierarchy H = build_hierarchy(A, p);
    for (size_t l = 0; l < H.lv.size(); ++l) {
      const HostLevel &L = H.lv[l];
      if (l + 1 < H.lv.size()) {
        const HostCsr R = restriction_of(L.P);
        std::vector<double> dinv, dl1;
        HostCsr lo, up;
        pgs_data(L.A, dinv, dl1, lo, up);
        (void)level_schedule(lo, true);
        (void)level_schedule(up, false);
        if (R.nr != L.P.nc) ++failures;
      }
      if (L.has_ilu) {
        namg_ilu_diag d{};
        ilu_diagnostics(L, 20, 10, 1e-8, &d);
        std::vector<double> b(L.A.nr, 1.0);
        double rl = 0, ru = 0;
        tri_jacobi_residuals(L, b.data(), 3, &rl, &ru);
        if (L.A.nr <= 400) {
          std::vector<double> ma(8), n2(8);
          std::vector<int64_t> nz(8);
          us_powers(L, 8, 20, ma.data(), n2.data(), nz.data());
        }
      }
    }
    std::printf("%s: %zu levels\n", what, H.lv.size());
  } catch (const SetupError &e) {
    std::printf("%s: setup error %d (%s)\n", what, e.code, e.msg.c_str());
    ++failures;
  }
}

void expect_rejected(int n, std::vector<int32_t> rp, std::vector<int32_t> ci, std::vector<double> v, const char *what) {
  try {
    (void)import_csr(n, rp.data(), ci.data(), v.data());
    std::printf("%s: accepted, expected a rejection\n", what);
    ++failures;
  } catch (const SetupError &) {
  }
}

}  // namespace

int main() {
  namg_setup_params p = defaults();
  exercise(stencil3d(9, 0.0, 1), p, "symmetric 9^3");
  exercise(stencil3d(8, 0.7, 2), p, "nonsymmetric 8^3");
  namg_setup_params all_ilu = p;
  all_ilu.ilu_levels = -1;
  exercise(stencil3d(7, 0.3, 3), all_ilu, "ILU(0) on every level");
  namg_setup_params ilut = p;
  ilut.ilu_kind = NAMG_ILUT;
  ilut.ilut_droptol = 1e-3;
  ilut.ilut_lfil = 7;
  exercise(stencil3d(7, 0.2, 4), ilut, "ILUT(1e-3, 7)");
  ilut.ilut_lfil = 0;
  exercise(stencil3d(6, 0.2, 5), ilut, "ILUT(1e-3, 0)");
  namg_setup_params agg = p;
  agg.agg_levels = 2;
  exercise(stencil3d(10, 0.0, 6), agg, "aggressive x2");
  namg_setup_params coarse = p;
  coarse.max_coarse = 5;
  exercise(random_csr(120, 6, 7), coarse, "random 120");
  exercise(random_csr(1, 1, 8), p, "1x1");
  exercise(stencil3d(3, 0.0, 9), p, "one level");
  namg_setup_params theta = p;
  theta.theta = 1.0;
  exercise(stencil3d(6, 0.5, 10), theta, "theta 1");
  // malformed input is rejected before any work
  expect_rejected(2, {0, 1, 2}, {0, 2}, {1.0, 1.0}, "column out of range");
  expect_rejected(2, {0, 2, 1}, {0, 1}, {1.0, 1.0}, "row pointers not monotone");
  expect_rejected(2, {0, 2, 3}, {1, 0, 1}, {1.0, 1.0, 1.0}, "columns not ascending");
  expect_rejected(2, {0, 1, 2}, {1, 0}, {1.0, 1.0}, "missing diagonal");
  expect_rejected(1, {0, 1}, {0}, {NAN}, "non-finite value");
  expect_rejected(0, {0}, {}, {}, "empty");
  std::printf("failures: %d\n", failures);
  return failures == 0 ? 0 : 1;
}

// Host-side AMG setup of the namg library: strength, Ruge-Stueben coarsening, classical interpolation,
// Galerkin coarse operators, ILU(0), smoother data and level schedules. FP64, deterministic, built with
// -ffp-contract=off so that every coarse value is summed in the canonical order documented per function.
#pragma once

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/namg.h"

namespace namg {

struct HostCsr {
  int32_t nr = 0, nc = 0;
  std::vector<int32_t> rp, ci;
  std::vector<double> v;
  int64_t nnz() const { return (int64_t)ci.size(); }
};

struct SetupError {
  int code;
  std::string msg;
};

// Rows of a strict triangle grouped by dependency level: rows order[ptr[k] .. ptr[k+1]) only depend on
// rows of earlier groups. Used by the direct-triangular comparators.
struct LevelSchedule {
  std::vector<int32_t> order, ptr;
  int levels() const { return ptr.empty() ? 0 : (int)ptr.size() - 1; }
};

struct HostLevel {
  HostCsr A, P, R;
  std::vector<int8_t> cf;
  std::vector<double> dinv;    // 1 / a_ii
  std::vector<double> dl1inv;  // 1 / sum_j |a_ij| (l1-Jacobi)
  HostCsr pgs_lo, pgs_up;      // D^{-1} L and D^{-1} U: strict parts of A scaled by the row's diagonal
  bool host_smoother = true;   // false: dinv, dl1inv, pgs_lo, pgs_up left empty (built on the device)
  bool host_restriction = true;  // false: R is not copied to the host (restriction_of(P) derives it)
  bool has_ilu = false;
  HostCsr ilu_lo, ilu_up;      // L_s (strict lower of the unit-diagonal L) and U_s = D_U^{-1} U - I
  std::vector<double> ilu_dinv;  // 1 / u_ii
  std::vector<double> ilu_diag;  // u_ii
};

struct HostHierarchy {
  std::vector<HostLevel> lv;
  std::vector<double> coarse_inv;  // dense inverse of the coarsest operator, row-major
  double anorm_inf = 0.0;          // ||A_0||_inf
  double t_levels = 0.0, t_finish = 0.0;  // seconds: building the levels (device phase incl. waits), finishing
  // Levels built on the device (a DeviceLevels, opaque here): the solve-phase layouts are packed from them
  // on the device; released once they are built.
  std::shared_ptr<void> device_levels;
  // Decided once at setup: the solver packs device_levels on the device, so R and the polynomial-GS data
  // have no host copies (false: host packing, every host copy present).
  bool pack_on_device = false;
};

// Throws SetupError{NAMG_E_INVALID / NAMG_E_NONFINITE / NAMG_E_ZERO_PIVOT} on malformed input.
HostCsr import_csr(int32_t n, const int32_t *rp, const int32_t *ci, const double *v);

// The hierarchy of namg_setup_params p (theta, max_levels, max_coarse and the ILU fields; precision and
// device are the caller's). Throws SetupError on invalid parameters or a zero pivot.
HostHierarchy build_hierarchy(const HostCsr &A, const namg_setup_params &p);
// The same, taking ownership of A (the device setup keeps it as level 0 without a copy).
HostHierarchy build_hierarchy(HostCsr &&A, const namg_setup_params &p);

// Parameter checks shared by both setups, ||A||_inf, and the host part that completes a hierarchy whose
// levels (A, P, R, C/F) are built: smoother data of every level but the coarsest, the coarse inverse.
// host_smoother = false leaves the polynomial-GS data to a device packing (the ILU factors stay on the
// host); the caller has then checked every level's diagonal (the device setup does, as it builds them).
void validate_hierarchy_params(const namg_setup_params &p);
double inf_norm(const HostCsr &A);
void finish_hierarchy(HostHierarchy &H, const namg_setup_params &p, bool host_smoother = true);
// R = P^T, rows sorted by fine index (the host setup's restriction, bit for bit the device setup's).
HostCsr restriction_of(const HostCsr &P);
// The polynomial-GS and l1-Jacobi data of a level matrix in one pass per row: 1 / a_ii, 1 / sum_j |a_ij|,
// D^{-1}L and D^{-1}U. Throws SetupError{NAMG_E_ZERO_PIVOT} on a zero diagonal.
void pgs_data(const HostCsr &A, std::vector<double> &dinv, std::vector<double> &dl1inv, HostCsr &lo, HostCsr &up);

// Dependency levels of a strict lower (lower = true) or upper triangle, for the direct comparators.
LevelSchedule level_schedule(const HostCsr &T, bool lower);

// Non-normality diagnostics of a level's ILU factors and the Jacobi triangular-solve residuals
// (diagnostics.cpp). Throw SetupError on invalid arguments.
void ilu_diagnostics(const HostLevel &L, int power_iters, int ruiz_max_iters, double ruiz_tol, namg_ilu_diag *out);
void tri_jacobi_residuals(const HostLevel &L, const double *b, int iters, double *res_L, double *res_U);
void us_powers(const HostLevel &L, int pmax, int power_iters, double *max_abs, double *norm2, int64_t *nnz);

}  // namespace namg

// namg solve phase: device hierarchy, V-cycle driver, low-synchronization flexible GMRES and the C ABI.
//
// Host code issues every kernel on the caller's stream; the only host<->device crossings inside a solve
// are one readback per Arnoldi step (the convergence estimate, written by the step kernel straight into
// host-mapped memory) and one per restart cycle (the true residual norm).
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/namg.h"
#include "device.hpp"
#include "kernels.hpp"
#include "pack.hpp"
#include "setup_host.hpp"

namespace namg {

namespace {
thread_local std::string g_last_error;

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    hip_check(hipGetDevice(&prev), "hipGetDevice");
    if (prev != dev) hip_check(hipSetDevice(dev), "hipSetDevice");
  }
  ~DeviceGuard() {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
  }
};

struct CycleOpts {
  int smoother, tri_mode, t, nu1, nu2;
};

CycleOpts cycle_opts(const namg_solve_params &p) {
  return CycleOpts{p.smoother, p.tri_mode, p.inner_terms, p.pre_sweeps, p.post_sweeps};
}

// The correction T of the small dense step as the step kernels take it: 0 = (I + L)^{-1} by forward
// substitution, p >= 1 = the Neumann series truncated at degree p.
inline int32_t t_mode(const namg_solve_params &p) { return p.gmres_T == NAMG_T_DIRECT ? 0 : p.t_degree; }

void validate_solve_params(const namg_solve_params &p) {
  if (!(p.tol > 0.0) || !std::isfinite(p.tol)) throw SetupError{NAMG_E_INVALID, "tol must be > 0"};
  if (p.restart < 1 || p.restart > NAMG_MAX_RESTART) throw SetupError{NAMG_E_INVALID, "restart out of range"};
  if (p.max_iters < 0) throw SetupError{NAMG_E_INVALID, "max_iters must be >= 0"};
  if (p.inner_terms < 1) throw SetupError{NAMG_E_INVALID, "inner_terms must be >= 1"};
  if (p.smoother != NAMG_SMOOTH_PGS && p.smoother != NAMG_SMOOTH_ILU0 && p.smoother != NAMG_SMOOTH_L1JAC)
    throw SetupError{NAMG_E_INVALID, "unknown smoother"};
  if (p.tri_mode != NAMG_TRI_NEUMANN && p.tri_mode != NAMG_TRI_DIRECT)
    throw SetupError{NAMG_E_INVALID, "unknown tri_mode"};
  if (p.gmres_T != NAMG_T_NEUMANN && p.gmres_T != NAMG_T_DIRECT) throw SetupError{NAMG_E_INVALID, "unknown gmres_T"};
  if (p.pre_sweeps < 0 || p.post_sweeps < 0) throw SetupError{NAMG_E_INVALID, "negative sweep count"};
  if (p.t_degree < 1 || p.t_degree > NAMG_MAX_RESTART) throw SetupError{NAMG_E_INVALID, "t_degree out of range"};
  if (p.stop_rule != NAMG_STOP_RELRES && p.stop_rule != NAMG_STOP_NRBE)
    throw SetupError{NAMG_E_INVALID, "unknown stop_rule"};
  if (p.diagnostics & ~(NAMG_DIAG_LOSS_ORTH | NAMG_DIAG_PHASE_TIMES))
    throw SetupError{NAMG_E_INVALID, "unknown diagnostics flag"};
  if (p.res_hist_cap < 0 || (p.res_hist_cap > 0 && !p.res_hist))
    throw SetupError{NAMG_E_INVALID, "res_hist_cap > 0 needs a res_hist array"};
}

// A served request's solve parameters: batched launches cover the Neumann smoothers only, and a request
// keeps no pointer into the caller's memory and reports no diagnostics.
void validate_served_params(const namg_solve_params &p) {
  validate_solve_params(p);
  if (p.tri_mode != NAMG_TRI_NEUMANN)
    throw SetupError{NAMG_E_INVALID, "serving batches the Neumann smoothers only (tri_mode must be NEUMANN)"};
  if (p.diagnostics != 0 || p.res_hist || p.res_hist_cap != 0)
    throw SetupError{NAMG_E_INVALID, "served requests take no diagnostics and no residual history"};
}

// One function pointer per lanes-per-row group for every row kernel.
#define NAMG_GROUP_SWITCH(NAME, ...)                      \
  switch (g) {                                            \
    case 1: return &NAME<1, __VA_ARGS__>;                 \
    case 2: return &NAME<2, __VA_ARGS__>;                 \
    case 4: return &NAME<4, __VA_ARGS__>;                 \
    case 8: return &NAME<8, __VA_ARGS__>;                 \
    case 16: return &NAME<16, __VA_ARGS__>;               \
    case 32: return &NAME<32, __VA_ARGS__>;               \
    default: return &NAME<64, __VA_ARGS__>;               \
  }
// Chunks of eight (unroll == 8) exist for one lane per row only (SELL-64, see choose_unroll).
template <class Acc, class TM, class TX, class TY>
auto sel_spmv(int g, int unroll = 4) {
  if (g == 1 && unroll == 8) return &k_spmv<1, Acc, TM, TX, TY, 8>;
  NAMG_GROUP_SWITCH(k_spmv, Acc, TM, TX, TY)
}
template <class T>
auto sel_residual(int g, int unroll = 4) {
  if (g == 1 && unroll == 8) return &k_residual<1, T, 8>;
  NAMG_GROUP_SWITCH(k_residual, T)
}
template <class T>
auto sel_neumann(int g, int unroll = 4) {
  if (g == 1 && unroll == 8) return &k_neumann<1, T, 8>;
  NAMG_GROUP_SWITCH(k_neumann, T)
}
template <class T>
auto sel_prolong(int g) { NAMG_GROUP_SWITCH(k_prolong, T) }
#undef NAMG_GROUP_SWITCH

// The leading kernel arguments of a sparse operator (see NAMG_MAT_HEAD in kernels.hpp).
template <class T>
const void *mat_idx(const MatView<T> &M) {
  if (M.dia) return static_cast<const void *>(M.dia);
  return M.col16 ? static_cast<const void *>(M.col16) : static_cast<const void *>(M.col);
}
template <class T>
int32_t mat_form(const MatView<T> &M) {
  return M.dia ? 2 : M.col16 ? 1 : 0;
}
#define NAMG_HEAD_ARGS(M) (M).ptr, mat_idx(M), (M).val, (M).nrows, mat_form(M)

template <class T>
unsigned rows_grid(const DMat<T> &M) {
  if (M.unit && M.unit_pairs) return (unsigned)((M.nrows + UNIT_BLOCK_ROWS - 1) / UNIT_BLOCK_ROWS);
  return row_blocks(M.nrows, M.group);
}
}  // namespace

class SolverBase {
 public:
  virtual ~SolverBase() = default;
  virtual int solve(const double *b, double *x, const namg_solve_params &p, hipStream_t s, namg_solve_stats *st) = 0;
  virtual int solve_in(const double *b, double *x, const namg_solve_params &p, hipStream_t s, namg_solve_stats *st,
                       void *scratch, size_t scratch_bytes) = 0;
  virtual void vcycle64(const double *b, double *x, const namg_solve_params &p, hipStream_t s) = 0;
  virtual void apply(int level, int op, const namg_solve_params &p, const double *in1, const double *in2, double *out,
                     hipStream_t s) = 0;
  virtual int64_t device_bytes() const = 0;
  virtual void profile(int family, int level, int every) = 0;
  virtual namg_kernel_profile profile_read() = 0;
};

template <class T>
class BatchEngine;

template <class T>
struct DevLevel {
  int32_t n = 0;
  DMat<T> A, P, R, pgs_lo, pgs_up, ilu_lo, ilu_up;
  DevBuf<T> dinv, dl1inv, ilu_dinv;
  bool has_ilu = false;
  DTri<T> tri_pgs_lo, tri_pgs_up, tri_ilu_lo, tri_ilu_up;
  DevBuf<T> b, x, r, f, g1, g2;
};

template <class T>
class Solver final : public SolverBase {
  static constexpr double S = sizeof(T);
  friend class BatchEngine<T>;

 public:
  // allow_dia false: no operator takes the slice-diagonal form (the served requests: their setup, not their
  // solve, bounds the stream, and the form's device analysis would lengthen every setup)
  Solver(const HostHierarchy &H, int device, bool allow_dia = true) : dev_(device), host_(&H) {
    DeviceGuard g(dev_);
    const bool ad = allow_dia;
    const int nl = (int)H.lv.size();
    lv_.resize(nl);
    // levels built on the device are packed there (same bytes as the host packing below)
    const DeviceLevels *dl = (H.device_levels && H.pack_on_device)
                                 ? static_cast<const DeviceLevels *>(H.device_levels.get())
                                 : nullptr;
    for (int l = 0; l < nl; ++l) {
      const HostLevel &h = H.lv[l];
      DevLevel<T> &d = lv_[l];
      d.n = h.A.nr;
      d.b.alloc(d.n, &mc_);
      d.x.alloc(d.n, &mc_);
      if (l == nl - 1) break;
      if (dl) {
        pack_device(d.A, dl->A[l], &mc_, 0, nullptr, ad);
        const UnitRows pu = unit_rows_of(h.P, h.cf);
        pack_device(d.P, dl->P[l], &mc_, 0, &pu, ad);
        pack_device(d.R, dl->R[l], &mc_, 0, nullptr, ad);
        DCsr lo, up;
        smoother_data_device(dl->A[l], lo, up, d.dinv, d.dl1inv, &mc_);
        pack_device(d.pgs_lo, lo, &mc_, 0, nullptr, ad);
        pack_device(d.pgs_up, up, &mc_, 0, nullptr, ad);
      } else {
        d.A.build(h.A, &mc_, 0, nullptr, ad);
        d.P.build(h.P, &mc_, 0, &h.cf, ad);
        if (h.host_restriction)
          d.R.build(h.R, &mc_, 0, nullptr, ad);
        else
          d.R.build(restriction_of(h.P), &mc_, 0, nullptr, ad);
        if (h.host_smoother) {
          d.pgs_lo.build(h.pgs_lo, &mc_, 0, nullptr, ad);
          d.pgs_up.build(h.pgs_up, &mc_, 0, nullptr, ad);
          upload_vec(d.dinv, h.dinv);
          upload_vec(d.dl1inv, h.dl1inv);
        } else {
          std::vector<double> dinv, dl1inv;
          HostCsr lo, up;
          pgs_data(h.A, dinv, dl1inv, lo, up);
          d.pgs_lo.build(lo, &mc_, 0, nullptr, ad);
          d.pgs_up.build(up, &mc_, 0, nullptr, ad);
          upload_vec(d.dinv, dinv);
          upload_vec(d.dl1inv, dl1inv);
        }
      }
      d.has_ilu = h.has_ilu;
      if (h.has_ilu) {
        d.ilu_lo.build(h.ilu_lo, &mc_, 0, nullptr, ad);
        d.ilu_up.build(h.ilu_up, &mc_, 0, nullptr, ad);
        upload_vec(d.ilu_dinv, h.ilu_dinv);
      }
      d.r.alloc(d.n, &mc_);
      d.f.alloc(d.n, &mc_);
      d.g1.alloc(d.n, &mc_);
      d.g2.alloc(d.n, &mc_);
    }
    nc_ = H.lv.back().A.nr;
    // the coarsest level's dense inverse as a full CSR matrix, one wavefront per row
    HostCsr inv;
    inv.nr = inv.nc = nc_;
    inv.rp.resize(nc_ + 1);
    for (int32_t i = 0; i <= nc_; ++i) inv.rp[i] = i * nc_;
    inv.ci.resize((size_t)nc_ * nc_);
    for (int32_t i = 0; i < nc_; ++i)
      for (int32_t j = 0; j < nc_; ++j) inv.ci[(size_t)i * nc_ + j] = j;
    inv.v = H.coarse_inv;
    coarse_inv_.build(inv, &mc_, nc_ > 1 ? 64 : 1, nullptr, ad);
    if (dl)
      pack_device(A64_, dl->A[0], &mc_, 1, nullptr, ad);
    else
      A64_.build(H.lv[0].A, &mc_, 1, nullptr, ad);
    anorm_inf_ = H.anorm_inf;
    const int32_t n = lv_[0].n;
    nblk_red_ = (int32_t)blocks_for(n);
    ldv_ = ((int64_t)n + 63) / 64 * 64;
    ldz_ = ldv_;
    nblk_dot_ = dot_blocks(n);
    rows_per_dot_ = dot_rows_per_block(n);
    hip_check(hipEventCreate(&wall_ev_[0]), "hipEventCreate");
    hip_check(hipEventCreate(&wall_ev_[1]), "hipEventCreate");
    red_.alloc(std::max<int32_t>(nblk_red_, 1) + 8, &mc_);
    kst_.alloc(1, &mc_);
    hip_check(hipHostMalloc((void **)&pinned_, sizeof(double) * (size_t)step_slot(NAMG_MAX_RESTART + 1),
                            hipHostMallocMapped),
              "hipHostMalloc");
    hip_check(hipHostGetDevicePointer((void **)&pinned_dev_, pinned_, 0), "hipHostGetDevicePointer");
  }

  ~Solver() override {
    for (auto &kv : tri_graphs_) (void)hipGraphExecDestroy(kv.second);
    if (capture_) (void)hipStreamDestroy(capture_);
    for (auto &e : events_) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    for (hipEvent_t e : phase_ev_) (void)hipEventDestroy(e);
    if (wall_ev_[0]) (void)hipEventDestroy(wall_ev_[0]);
    if (wall_ev_[1]) (void)hipEventDestroy(wall_ev_[1]);
    if (pinned_) (void)hipHostFree(pinned_);
  }

  int64_t device_bytes() const override { return mc_.bytes.load(); }

  // Allocate the Krylov workspace for restart m ahead of the first solve (used by serving).
  void reserve_workspace(int m) {
    DeviceGuard g(dev_);
    ensure_workspace(m);
  }

  void profile(int family, int level, int every) override {
    DeviceGuard g(dev_);
    flush_profile();
    prof_family_ = family;
    prof_level_ = level;
    prof_every_ = every;
    prof_seen_ = 0;
    prof_ = namg_kernel_profile{0, 0.0, 0.0};
  }

  namg_kernel_profile profile_read() override {
    DeviceGuard g(dev_);
    flush_profile();
    namg_kernel_profile out = prof_;
    prof_ = namg_kernel_profile{0, 0.0, 0.0};
    return out;
  }

  // ------------------------------------------------------------------------------------------ V-cycle
  void vcycle64(const double *b, double *x, const namg_solve_params &p, hipStream_t s) override {
    DeviceGuard g(dev_);
    const int32_t n = lv_[0].n;
    CycleOpts o = cycle_opts(p);
    if (o.tri_mode == NAMG_TRI_DIRECT) ensure_direct();
    if constexpr (std::is_same<T, double>::value) {
      vcycle(0, b, x, o, s);
    } else {
      cast(b, lv_[0].b.get(), n, s);
      vcycle(0, lv_[0].b.get(), lv_[0].x.get(), o, s);
      cast(lv_[0].x.get(), x, n, s);
    }
  }

  void apply(int level, int op, const namg_solve_params &p, const double *in1, const double *in2, double *out,
             hipStream_t s) override {
    DeviceGuard g(dev_);
    const int nl = (int)lv_.size();
    if (level < 0 || level >= nl) throw SetupError{NAMG_E_INVALID, "level out of range"};
    CycleOpts o = cycle_opts(p);
    if (o.tri_mode == NAMG_TRI_DIRECT) ensure_direct();
    if (!in1) throw SetupError{NAMG_E_INVALID, "missing operand"};
    if (op == NAMG_OP_SPMV64) {
      if (level != 0) throw SetupError{NAMG_E_INVALID, "SPMV64 is defined on level 0 only"};
      const MatView<double> M = A64_.view();
      launch(NAMG_KF_GMRES_SPMV, 0, A64_.bytes() + 16.0 * A64_.nrows, sel_spmv<double, double, double, double>(1, A64_.unroll),
             rows_grid(A64_), s, NAMG_HEAD_ARGS(M), in1, (const double *)nullptr, out, (double *)nullptr, M.mul);
      return;
    }
    if (op == NAMG_OP_COARSE) {
      if (level != nl - 1) throw SetupError{NAMG_E_INVALID, "COARSE applies to the coarsest level"};
      DevLevel<T> &d = lv_[level];
      cast(in1, d.b.get(), d.n, s);
      coarse_solve(level, d.b.get(), d.x.get(), s);
      cast(d.x.get(), out, d.n, s);
      return;
    }
    if (level == nl - 1) throw SetupError{NAMG_E_INVALID, "operator not defined on the coarsest level"};
    DevLevel<T> &d = lv_[level];
    DevLevel<T> &c = lv_[level + 1];
    const int32_t n = d.n;
    const bool need2 = op == NAMG_OP_RESIDUAL || op == NAMG_OP_SMOOTH_PRE || op == NAMG_OP_SMOOTH_POST ||
                       op == NAMG_OP_PROLONG;
    if (need2 && !in2) throw SetupError{NAMG_E_INVALID, "missing operand"};
    switch (op) {
      case NAMG_OP_SPMV:
        cast(in1, d.x.get(), n, s);
      {
        const MatView<T> M = d.A.view();
        launch(NAMG_KF_SPMV, level, d.A.bytes() + 2 * S * n, sel_spmv<T, T, T, T>(d.A.group, d.A.unroll), rows_grid(d.A), s,
               NAMG_HEAD_ARGS(M), (const T *)d.x.get(), (const T *)nullptr, d.b.get(), (T *)nullptr, M.mul);
      }
        cast(d.b.get(), out, n, s);
        break;
      case NAMG_OP_RESIDUAL:
        cast(in1, d.x.get(), n, s);
        cast(in2, d.b.get(), n, s);
        residual(level, d.b.get(), d.x.get(), nullptr, d.r.get(), nullptr, s);
        cast(d.r.get(), out, n, s);
        break;
      case NAMG_OP_SMOOTH_PRE:
      case NAMG_OP_SMOOTH_POST: {
        cast(in1, d.x.get(), n, s);
        cast(in2, d.b.get(), n, s);
        const bool ilu = (o.smoother == NAMG_SMOOTH_ILU0) && d.has_ilu;
        smooth(level, d.b.get(), d.x.get(), false, op == NAMG_OP_SMOOTH_PRE, ilu, o, s);
        cast(d.x.get(), out, n, s);
        break;
      }
      case NAMG_OP_RESTRICT:
        cast(in1, d.r.get(), n, s);
        restrict_(level, o, s);
        cast(c.b.get(), out, c.n, s);
        break;
      case NAMG_OP_PROLONG:
        cast(in1, c.x.get(), c.n, s);
        cast(in2, d.x.get(), n, s);
        prolong(level, d.x.get(), s);
        cast(d.x.get(), out, n, s);
        break;
      default:
        throw SetupError{NAMG_E_INVALID, "unknown operator"};
    }
  }

  // ------------------------------------------------------------------------------------------- solve
  int solve(const double *b, double *x, const namg_solve_params &p, hipStream_t s, namg_solve_stats *stats) override {
    DeviceGuard g(dev_);
    ensure_workspace(p.restart);
    const Workspace ws{V_.get(), w_.get(), dot_.get(), cd_.get(), Z_.get(), vin_.get()};
    return run(b, x, p, s, stats, ws);
  }

  // The same solve with its Krylov workspace carved out of caller-provided device memory of scratch_bytes
  // bytes instead of the hierarchy's own buffers: nothing is allocated on the device. The options that
  // allocate on first use (the direct comparators' schedules and graphs, the Gram matrix and phase events
  // of the diagnostics) are refused before any work is issued.
  int solve_in(const double *b, double *x, const namg_solve_params &p, hipStream_t s, namg_solve_stats *stats,
               void *scratch, size_t scratch_bytes) override {
    DeviceGuard g(dev_);
    if (p.tri_mode == NAMG_TRI_DIRECT && !direct_ready_)
      throw SetupError{NAMG_E_INVALID, "the direct comparators allocate their level schedules on first use; run "
                                       "one namg_solve with tri_mode DIRECT on this hierarchy first"};
    if (p.diagnostics != 0) throw SetupError{NAMG_E_INVALID, "diagnostics allocate on first use; pass 0"};
    size_t off[7];
    const size_t need = workspace_layout(p.restart, off);
    if (need > scratch_bytes)
      throw SetupError{NAMG_E_INVALID, "the Krylov workspace needs " + std::to_string(need) +
                                           " bytes (n = " + std::to_string(lv_[0].n) + ", restart " +
                                           std::to_string(p.restart) + "); the static workspace holds " +
                                           std::to_string(scratch_bytes)};
    char *base = static_cast<char *>(scratch);
    const Workspace ws{reinterpret_cast<double *>(base + off[0]), reinterpret_cast<double *>(base + off[2]),
                       reinterpret_cast<double *>(base + off[4]), reinterpret_cast<double *>(base + off[5]),
                       reinterpret_cast<T *>(base + off[1]),
                       std::is_same<T, double>::value ? nullptr : reinterpret_cast<T *>(base + off[3])};
    return run(b, x, p, s, stats, ws);
  }

 private:
  // The Krylov workspace of one solve: basis V (m + 2 columns of ldv_), w = A z, the multi-dot partials,
  // the reduced inner products, the preconditioned vectors Z (m columns of ldz_) and, in FP32 mode, the
  // low-precision copy of the V-cycle's input.
  struct Workspace {
    double *V, *w, *dot, *cd;
    T *Z, *vin;
  };

  // Byte offsets of the workspace parts for restart m in one block (V, Z, w, vin, dot partials, cd; each
  // part starts on a 256-byte boundary); off[6] and the return value are the total size.
  size_t workspace_layout(int m, size_t off[7]) const {
    const int32_t n = lv_[0].n;
    const size_t part[6] = {8 * (size_t)ldv_ * (m + 2),
                            sizeof(T) * (size_t)ldz_ * m,
                            8 * (size_t)n,
                            std::is_same<T, double>::value ? 0 : sizeof(T) * (size_t)n,
                            8 * (size_t)nblk_dot_ * 2 * (m + 2),
                            8 * (size_t)2 * (m + 2)};
    size_t at = 0;
    for (int q = 0; q < 6; ++q) {
      off[q] = at;
      at += (part[q] + 255) / 256 * 256;
    }
    off[6] = at;
    return at;
  }

  int run(const double *b, double *x, const namg_solve_params &p, hipStream_t s, namg_solve_stats *stats,
          const Workspace &ws) {
    const int32_t n = lv_[0].n;
    const int m = p.restart;
    alg_ = 0.0;
    hip_check(hipEventRecord(wall_ev_[0], s), "hipEventRecord");
    const CycleOpts o = cycle_opts(p);
    if (o.tri_mode == NAMG_TRI_DIRECT) ensure_direct();
    const bool trace = std::getenv("NAMG_TRACE") != nullptr;
    const bool timing = (p.diagnostics & NAMG_DIAG_PHASE_TIMES) != 0;
    const bool orth = (p.diagnostics & NAMG_DIAG_LOSS_ORTH) != 0;
    phase_used_ = 0;
    std::vector<size_t> marks;  // four phase events per Arnoldi step (before the V-cycle, after it, after
                                // the product, after the column completion)
    KState *ks = kst_.get();
    double *cd = ws.cd;
    double *V = ws.V;
    T *Z = ws.Z;
    double *w = ws.w;
    T *vin = std::is_same<T, double>::value ? nullptr : ws.vin;
    const MatView<double> M64 = A64_.view();

    const double beta = std::sqrt(norm2sq(b, n, s));
    namg_solve_stats st{};
    st.loss_orth = st.ms_vcycle = st.ms_spmv = st.ms_ortho = std::nan("");
    if (orth) st.loss_orth = 0.0;
    int status = NAMG_OK;
    double rn = 0.0;
    if (!std::isfinite(beta)) throw SetupError{NAMG_E_NONFINITE, "non-finite right-hand side"};
    if (beta == 0.0) {
      launch(-1, 0, 8.0 * n, &k_fill<double>, blocks_for(n), s, x, 0.0, n);
    } else {
      while (true) {
        // the stopping test's denominator: ||b||, or ||b|| + ||A||_inf ||x|| at the cycle's start
        const double denom =
            p.stop_rule == NAMG_STOP_NRBE ? beta + anorm_inf_ * std::sqrt(norm2sq(x, n, s)) : beta;
        // true residual r = b - A x into V(:,0) (FP64), plus the FP32 copy for the V-cycle
        launch(-1, 0, A64_.bytes() + 24.0 * n + (vin ? S * n : 0.0), &k_residual64<T>, blocks_for(n), s,
               NAMG_HEAD_ARGS(M64), b, (const double *)x, V, vin, red_.get(), M64.mul);
        rn = std::sqrt(reduce_read(red_.get(), nblk_red_, s));
        if (!std::isfinite(rn)) throw SetupError{NAMG_E_NONFINITE, "non-finite residual"};
        if (trace) std::fprintf(stderr, "[namg] cycle %d true relres %.3e\n", st.cycles, rn / beta);
        if (rn / denom <= p.tol) {
          status = NAMG_OK;
          break;
        }
        if (st.iters >= p.max_iters) {
          status = NAMG_NOT_CONVERGED;
          break;
        }
        st.cycles++;
        const int me = std::min(m, p.max_iters - st.iters);
        // column completion of step 0: rho_0 = ||r|| from the residual pass's partial sums
        launch_small(&k_finish, s, ks, (const double *)red_.get(), nblk_red_, 0, 0, p.tol, beta, denom,
                     pinned_dev_);
        // The host reads each step's (estimate, stop flag) from its own host-mapped slot. It waits for the
        // device after a step only when that step might be the last: from the last two estimates read, the
        // steps ahead are issued without waiting while even a convergence twice as fast as the last step's
        // (per step) would not reach the stopping level (at most PLAN_AHEAD steps at a time). Every step
        // issued past the stopping one only writes workspace columns and Hessenberg entries beyond it, so
        // the iterate is the one of the step-by-step loop; the waits saved are the device's idle time.
        const double stop_level = p.tol * denom / beta;  // estimate |g| / ||b|| at which the flag is raised
        int k = 0, first_unread = 0, sync_at = 0;
        double e_prev = -1.0, e_last = -1.0;
        bool stop = false;
        for (int i = 0; i < me && !stop; ++i) {
          double *vi = V + (int64_t)i * ldv_;
          T *zi = Z + (int64_t)i * ldz_;
          const T *b0;
          if constexpr (std::is_same<T, double>::value)
            b0 = vi;
          else
            b0 = vin;
          if (timing) marks.push_back(phase_mark(s));
          vcycle(0, b0, zi, o, s);
          st.precond_apps++;
          if (timing) marks.push_back(phase_mark(s));
          launch(NAMG_KF_GMRES_SPMV, 0, A64_.bytes() + (S + 8.0) * n, sel_spmv<double, double, T, double>(1, A64_.unroll),
                 rows_grid(A64_), s, NAMG_HEAD_ARGS(M64), (const T *)zi, (const double *)nullptr, w, (double *)nullptr,
                 M64.mul);
          if (timing) marks.push_back(phase_mark(s));
          const int32_t ncols = i + 1;
          launch(NAMG_KF_MULTIDOT, 0, 8.0 * n * (ncols + 1), multidot_kernel(ncols), nblk_dot_, s, (const double *)V,
                 ldv_, ncols, (const double *)w, n, rows_per_dot_, ws.dot, nblk_dot_);
          launch(-1, 0, 0.0, &k_colreduce, (unsigned)(2 * ncols), s, (const double *)ws.dot, nblk_dot_, cd);
          launch_small(&k_step, s, ks, (const double *)cd, i, t_mode(p));
          launch(NAMG_KF_PROJECT, 0, 8.0 * n * (i + 4) + (vin ? S * n : 0.0), &k_project<T>, blocks_for(n), s, V,
                 ldv_, i, (const double *)w, (const KState *)ks, n, vin, red_.get());
          // column i is complete once ||v_{i+2}|| is known: estimate and stop test before the next V-cycle
          launch_small(&k_finish, s, ks, (const double *)red_.get(), nblk_red_, i + 1, (int)(i + 1 == me), p.tol, beta,
                       denom, pinned_dev_ + step_slot(i));
          if (timing) marks.push_back(phase_mark(s));
          if (i < sync_at && i + 1 < me) continue;
          wait_stream(s);
          for (int j = first_unread; j <= i; ++j) {
            const double est = pinned_[step_slot(j)];
            const int flag = (int)pinned_[step_slot(j) + 1];
            if (flag < 0) throw SetupError{NAMG_E_NONFINITE, "non-finite value in the Arnoldi step"};
            if (st.iters < p.res_hist_cap) p.res_hist[st.iters] = est;
            st.iters++;
            st.relres_est = est;
            if (trace) std::fprintf(stderr, "[namg]   iter %d est %.3e\n", st.iters, est);
            if (flag == 1) {
              k = j + 1;
              stop = true;
              break;
            }
            e_prev = e_last;
            e_last = est;
          }
          first_unread = i + 1;
          int ahead = 1;
          if (!timing && e_prev > 0.0 && e_last > 0.0) {
            const double rate = 0.5 * e_last / e_prev;
            double pred = e_last;
            while (ahead < PLAN_AHEAD && i + ahead + 1 < me) {
              pred *= rate;
              if (!(pred > stop_level)) break;
              ++ahead;
            }
          }
          sync_at = i + ahead;
        }
        if (orth) st.loss_orth = std::max(st.loss_orth, loss_of_orthogonality(k, m, ws, s));
        launch_small(&k_backsolve, s, ks, k);
        launch(-1, 0, (double)n * (S * k + 16.0), &k_update_x<T>, blocks_for(n), s, (const T *)Z, ldz_, k,
               (const KState *)ks, x, n);
      }
    }
    const double xn = std::sqrt(norm2sq(x, n, s));
    hip_check(hipEventRecord(wall_ev_[1], s), "hipEventRecord");
    hip_check(hipEventSynchronize(wall_ev_[1]), "hipEventSynchronize");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, wall_ev_[0], wall_ev_[1]), "hipEventElapsedTime");
    if (timing) {
      st.ms_vcycle = st.ms_spmv = st.ms_ortho = 0.0;
      for (size_t q = 0; q + 3 < marks.size(); q += 4) {
        const double tv = phase_ms(marks[q], marks[q + 1]), tm = phase_ms(marks[q + 1], marks[q + 2]),
                     to = phase_ms(marks[q + 2], marks[q + 3]);
        st.ms_vcycle += tv;
        st.ms_spmv += tm;
        st.ms_ortho += to;
        if (trace)
          std::fprintf(stderr, "[namg]   iter %zu: V-cycle %.3f ms, A z %.3f ms, orthogonalisation %.3f ms\n", q / 4 + 1,
                       tv, tm, to);
      }
    }
    st.status = status;
    st.relres_true = beta > 0.0 ? rn / beta : 0.0;
    st.nrbe = (beta > 0.0) ? rn / (beta + anorm_inf_ * xn) : 0.0;
    st.ms_total = ms;
    st.alg_bytes = alg_;
    if (stats) *stats = st;
    return status;
  }

 private:
  // Launch a kernel of BLK threads per block; bytes are the launch's algorithmic HBM bytes. family/level
  // select the launches the profiler times. It times runs: a maximal sequence of consecutive launches of
  // the selected family (for instance the four Neumann terms of one smoothing sweep) carries one start
  // event, attached to its first dispatch, and one stop event, recorded on the stream when the next other
  // kernel is issued; every prof_every_-th run is timed. The run's time over its launch count is the
  // average launch duration, with the events' own cost spread over the run.
  template <class Kernel, class... Args>
  void launch(int family, int level, double bytes, Kernel kernel, unsigned grid, hipStream_t s, Args... args) {
    if (grid == 0) return;
    alg_ += bytes;
    const bool selected = family >= 0 && family == prof_family_ && (prof_level_ < 0 || prof_level_ == level);
    if (!selected) {
      end_run();
    } else if (!in_run_) {
      in_run_ = true;
      run_timed_ = prof_seen_++ % prof_every_ == 0;
      if (run_timed_) {
        auto &ev = next_events();
        run_stream_ = s;
        prof_.launches++;
        prof_.alg_bytes += bytes;
        hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(BLK), 0, s, ev.first, (hipEvent_t) nullptr, 0, args...);
        hip_check(hipGetLastError(), "kernel launch");
        return;
      }
    } else if (run_timed_) {
      prof_.launches++;
      prof_.alg_bytes += bytes;
    }
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(BLK), 0, s, args...);
    hip_check(hipGetLastError(), "kernel launch");
  }

  // Close the open profiler run: its stop event follows the run's last launch on its stream.
  void end_run() {
    if (!in_run_) return;
    if (run_timed_) hip_check(hipEventRecord(events_[ev_used_ - 1].second, run_stream_), "hipEventRecord");
    in_run_ = false;
    run_timed_ = false;
  }

  // The next free start/stop event pair of the kernel profiler.
  std::pair<hipEvent_t, hipEvent_t> &next_events() {
    if (ev_used_ == events_.size()) {
      hipEvent_t a, b;
      hip_check(hipEventCreate(&a), "hipEventCreate");
      hip_check(hipEventCreate(&b), "hipEventCreate");
      events_.push_back({a, b});
    }
    return events_[ev_used_++];
  }

  template <class Kernel, class... Args>
  void launch_small(Kernel kernel, hipStream_t s, Args... args) {
    end_run();
    hipLaunchKernelGGL(kernel, dim3(1), dim3(BLK), 0, s, args...);
    hip_check(hipGetLastError(), "kernel launch");
  }

  void flush_profile() {
    end_run();
    if (ev_used_ == 0) return;
    for (size_t q = 0; q < ev_used_; ++q) {
      hip_check(hipEventSynchronize(events_[q].second), "hipEventSynchronize");
      float ms = 0.f;
      hip_check(hipEventElapsedTime(&ms, events_[q].first, events_[q].second), "hipEventElapsedTime");
      prof_.total_ms += ms;
    }
    ev_used_ = 0;
  }

  // Record the next phase event of the pool on stream s; returns its index.
  size_t phase_mark(hipStream_t s) {
    end_run();
    if (phase_used_ == phase_ev_.size()) {
      hipEvent_t e;
      hip_check(hipEventCreate(&e), "hipEventCreate");
      phase_ev_.push_back(e);
    }
    hip_check(hipEventRecord(phase_ev_[phase_used_], s), "hipEventRecord");
    return phase_used_++;
  }

  double phase_ms(size_t a, size_t b) {
    hip_check(hipEventSynchronize(phase_ev_[b]), "hipEventSynchronize");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, phase_ev_[a], phase_ev_[b]), "hipEventElapsedTime");
    return ms;
  }

  // ||I - G||_F for the Gram matrix G of the cycle's basis V_{k+1} (Section 3's loss of orthogonality): column
  // j's inner products with columns 0..j come from the fused reduction with ncols = j + 1 and no w. Columns
  // 0..k-1 are normalised; column k (v_{k+1}, lagged) is scaled by its own reduced norm.
  double loss_of_orthogonality(int k, int m, const Workspace &ws, hipStream_t s) {
    const int32_t n = lv_[0].n;
    const int ld = m + 2;
    if (gram_.size() < (size_t)ld * ld) gram_.alloc((size_t)ld * ld, &mc_);
    for (int j = 0; j <= k; ++j) {
      launch(-1, 0, 8.0 * n * (j + 1), &k_multidot<8>, nblk_dot_, s, (const double *)ws.V, ldv_, (int32_t)(j + 1),
             (const double *)nullptr, n, rows_per_dot_, ws.dot, nblk_dot_);
      launch(-1, 0, 0.0, &k_colreduce, (unsigned)(j + 1), s, (const double *)ws.dot, nblk_dot_,
             gram_.get() + (int64_t)j * ld);
    }
    std::vector<double> G((size_t)ld * ld);
    hip_check(hipMemcpyAsync(G.data(), gram_.get(), sizeof(double) * ld * (k + 1), hipMemcpyDeviceToHost, s), "D2H");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    auto g = [&](int j, int i) -> double & { return G[(size_t)j * ld + i]; };  // i <= j
    int cols = k + 1;
    if (g(k, k) > 0.0) {
      const double sc = 1.0 / std::sqrt(g(k, k));
      for (int i = 0; i < k; ++i) g(k, i) *= sc;
      g(k, k) *= sc * sc;
    } else {
      cols = k;  // lucky breakdown: v_{k+1} = 0
    }
    double acc = 0.0;
    for (int j = 0; j < cols; ++j) {
      acc += (1.0 - g(j, j)) * (1.0 - g(j, j));
      for (int i = 0; i < j; ++i) acc += 2.0 * g(j, i) * g(j, i);
    }
    return std::sqrt(acc);
  }

  void upload_vec(DevBuf<T> &d, const std::vector<double> &h) {
    std::vector<T> t(h.begin(), h.end());
    d.alloc(t.size(), &mc_);
    d.upload(t.data(), t.size());
  }

  template <class TI, class TO>
  void cast(const TI *src, TO *dst, int32_t n, hipStream_t s) {
    if (!src) throw SetupError{NAMG_E_INVALID, "missing operand"};
    launch(-1, 0, (sizeof(TI) + sizeof(TO)) * (double)n, &k_cast<TI, TO>, blocks_for(n), s, src, dst, n);
  }

  void ensure_workspace(int m) {
    if (ws_m_ >= m) return;
    const int32_t n = lv_[0].n;
    V_.alloc((size_t)ldv_ * (m + 2), &mc_);
    Z_.alloc((size_t)ldz_ * m, &mc_);
    w_.alloc(n, &mc_);
    if (!std::is_same<T, double>::value) vin_.alloc(n, &mc_);
    dot_.alloc((size_t)nblk_dot_ * 2 * (m + 2), &mc_);
    cd_.alloc((size_t)2 * (m + 2), &mc_);
    ws_m_ = m;
  }

  // |v|^2 (deterministic two-stage reduction on the device, read back to the host)
  double norm2sq(const double *v, int32_t n, hipStream_t s) {
    launch(-1, 0, 8.0 * n, &k_sumsq, blocks_for(n), s, v, n, red_.get());
    return reduce_read(red_.get(), nblk_red_, s);
  }

  // Deterministic final reduction written straight into host-mapped memory, then read by the host.
  double reduce_read(const double *partial, int32_t nb, hipStream_t s) {
    launch_small(&k_reduce, s, partial, nb, pinned_dev_ + 2);
    wait_stream(s);
    return pinned_[2];
  }

  // Steps issued ahead of the host's reading of their stop flags (see run).
  static constexpr int PLAN_AHEAD = 4;
  static constexpr int step_slot(int i) { return 4 + 2 * i; }

  // Waits until stream s is idle by polling it: the solve waits once per Arnoldi step, for a few
  // microseconds of work at a time, and a blocking wait adds its wake-up latency to each of those waits.
  // Errors as hipStreamSynchronize.
  static void wait_stream(hipStream_t s) {
    while (true) {
      const hipError_t e = hipStreamQuery(s);
      if (e == hipSuccess) return;
      if (e != hipErrorNotReady) hip_check(e, "hipStreamQuery");
    }
  }

  // ------------------------------------------------------------------ V-cycle row operations
  // Every row operation of the V-cycle is described by a RowOp. emit() launches it at once, or appends
  // it to record_ while the batching engine collects the operations of several solves.
 public:
  struct RowOp {
    int kind, group, family, level;
    unsigned grid;
    double bytes;
    RowTask<T> t;
  };

 private:
  std::vector<RowOp> *record_ = nullptr;

  // A matrix-free view that only carries the row count (vector operations).
  static MatView<T> axpy_view(int32_t n) {
    MatView<T> v;
    v.nrows = n;
    return v;
  }

  static RowOp row_op(int kind, int family, int level, const MatView<T> &M, int group, unsigned grid, double bytes,
                      const T *a, const T *b, const T *c, const T *d, T *o0, T *o1, int32_t n) {
    RowOp op;
    op.kind = kind;
    op.group = group;
    op.family = family;
    op.level = level;
    op.grid = grid;
    op.bytes = bytes;
    op.t.M = M;
    op.t.a = a;
    op.t.b = b;
    op.t.c = c;
    op.t.d = d;
    op.t.o0 = o0;
    op.t.o1 = o1;
    op.t.n = n;
    op.t.pad = 0;
    return op;
  }

  void emit(const RowOp &op, hipStream_t s) {
    // a unit-row matrix (a prolongation's layout) is only read by the prolongation kernels, which receive
    // its masks; any other row kernel would read its entries as plain SELL-64 and gather out of range
    if (op.t.M.umask && op.kind != ROP_PROLONG)
      throw SetupError{NAMG_E_INVALID, "internal: unit-row layout passed to a row kernel other than prolongation"};
    if (record_) {
      record_->push_back(op);
      return;
    }
    const RowTask<T> &t = op.t;
    switch (op.kind) {
      case ROP_RESIDUAL:
        launch(op.family, op.level, op.bytes, sel_residual<T>(op.group, t.M.unroll), op.grid, s, NAMG_HEAD_ARGS(t.M), t.a, t.c, t.b,
               t.o0, t.o1, t.M.mul);
        break;
      case ROP_NEUMANN:
        if constexpr (std::is_same<T, float>::value) {
          // two rows per lane (8-byte pairs of every row vector; never with both scale and acc, so that the
          // output expression is the one-row kernel's without a fused multiply-add to choose)
          auto al8 = [](const void *p) { return ((uintptr_t)p & 7) == 0; };
          if (t.M.pairs && !(t.c && t.d) && al8(t.a) && al8(t.c) && al8(t.d) && al8(t.o0)) {
            launch(op.family, op.level, op.bytes, &k_neumann_pairs, neumann_pairs_blocks(t.M.nrows), s,
                   NAMG_HEAD_ARGS(t.M), t.a, t.c, t.d, t.b, t.o0);
            break;
          }
        }
        launch(op.family, op.level, op.bytes, sel_neumann<T>(op.group, t.M.unroll), op.grid, s, NAMG_HEAD_ARGS(t.M), t.a, t.c, t.d,
               t.b, t.o0, t.M.mul);
        break;
      case ROP_SPMV:
        launch(op.family, op.level, op.bytes, sel_spmv<T, T, T, T>(op.group, t.M.unroll), op.grid, s, NAMG_HEAD_ARGS(t.M), t.b, t.c,
               t.o0, t.o1, t.M.mul);
        break;
      case ROP_PROLONG:
        launch(op.family, op.level, op.bytes, sel_prolong<T>(op.group), op.grid, s, NAMG_HEAD_ARGS(t.M), t.o0, t.b,
               t.M.mul, t.M.umask, t.M.smeta, t.M.ncols, t.M.unroll);
        break;
      case ROP_AXPY:
        launch(op.family, op.level, op.bytes, &k_axpy<T>, op.grid, s, t.a, t.c, t.d, t.o0, t.n);
        break;
      default:
        launch(op.family, op.level, op.bytes, &k_fill<T>, op.grid, s, t.o0, T(0), t.n);
        break;
    }
  }

  // r = b - A_l x (x may be null: x = 0) with optional outputs r and f = d .* r.
  void residual(int l, const T *b, const T *x, const T *d, T *r, T *f, hipStream_t s) {
    const DevLevel<T> &L = lv_[l];
    const int32_t n = L.n;
    const double bytes = (x ? L.A.bytes() + S * n : 0.0) + S * n * (1 + (r ? 1 : 0) + (f ? 2 : 0));
    const unsigned grid = x ? rows_grid(L.A) : row_blocks(n, 1);
    emit(row_op(ROP_RESIDUAL, NAMG_KF_RESIDUAL, l, L.A.view(), x ? L.A.group : 1, grid, bytes, b, x, d, nullptr, r, f,
                n),
         s);
  }

  // out = [acc +] [scale .*] (f - M in): one Neumann term on the strict triangle M of level l.
  void neumann(int l, const DMat<T> &M, const T *f, const T *in, const T *scale, const T *acc, T *out,
               hipStream_t s) {
    const int32_t n = M.nrows;
    const double vecs = (f == in ? 1 : 2) + 1 + (scale ? 1 : 0) + (acc ? 1 : 0);
    emit(row_op(ROP_NEUMANN, NAMG_KF_NEUMANN, l, M.view(), M.group, rows_grid(M), M.bytes() + S * n * vecs, f, in,
                scale, acc, out, nullptr, n),
         s);
  }

  void axpy(int l, const T *f, const T *scale, const T *acc, T *out, int32_t n, hipStream_t s) {
    const double vecs = 2 + (scale ? 1 : 0) + (acc ? 1 : 0);
    emit(row_op(ROP_AXPY, -1, l, axpy_view(n), 1, blocks_for(n), S * n * vecs, f, nullptr,
                scale, acc, out, nullptr, n),
         s);
  }

  void fill_zero(int l, T *out, int32_t n, hipStream_t s) {
    emit(row_op(ROP_FILL, -1, l, axpy_view(n), 1, blocks_for(n), S * n, nullptr, nullptr,
                nullptr, nullptr, out, nullptr, n),
         s);
  }

  // True when level l's first pre-smoothing term f = D^{-1} b (polynomial GS, zero initial guess) is
  // produced by the restriction from level l - 1 instead of a pass of its own.
  bool fused_f(int l, const CycleOpts &o) const {
    const int nl = (int)lv_.size();
    if (l < 1 || l + 1 >= nl || o.nu1 < 1) return false;
    if (o.smoother == NAMG_SMOOTH_L1JAC) return false;
    return !((o.smoother == NAMG_SMOOTH_ILU0) && lv_[l].has_ilu);
  }

  // b_{l+1} = R_l r_l [and f_{l+1} = D_{l+1}^{-1} b_{l+1} when the coarse level's sweep starts with it]
  void restrict_(int l, const CycleOpts &o, hipStream_t s) {
    DevLevel<T> &d = lv_[l];
    DevLevel<T> &c = lv_[l + 1];
    const bool ff = fused_f(l + 1, o);
    emit(row_op(ROP_SPMV, NAMG_KF_SPMV, l, d.R.view(), d.R.group, rows_grid(d.R),
                d.R.bytes() + S * ((double)d.n + c.n) + (ff ? 2.0 * S * c.n : 0.0), nullptr, d.r.get(),
                ff ? (const T *)c.dinv.get() : nullptr, nullptr, c.b.get(), ff ? c.f.get() : nullptr, c.n),
         s);
  }

  void prolong(int l, T *x, hipStream_t s) {
    DevLevel<T> &d = lv_[l];
    DevLevel<T> &c = lv_[l + 1];
    emit(row_op(ROP_PROLONG, NAMG_KF_PROLONG, l, d.P.view(), d.P.group, rows_grid(d.P),
                d.P.bytes() + S * ((double)c.n + 2.0 * d.n), nullptr, c.x.get(), nullptr, nullptr, x, nullptr, d.n),
         s);
  }

  void coarse_solve(int l, const T *b, T *x, hipStream_t s) {
    emit(row_op(ROP_SPMV, NAMG_KF_SPMV, l, coarse_inv_.view(), coarse_inv_.group, rows_grid(coarse_inv_),
                coarse_inv_.bytes() + 2 * S * nc_, nullptr, b, nullptr, nullptr, x, nullptr, nc_),
         s);
  }

  // g = (I + S)^{-1} f, one launch per dependency level: hundreds of small dependent launches per
  // triangle. The chain is captured once per (triangle, f, g) into a HIP graph and replayed, so the host
  // issues one graph launch per triangular solve. (Timing events are not attached inside graphs.)
  void tri_solve(int l, const DTri<T> &tr, const T *f, T *g, hipStream_t s) {
    (void)l;
    const int nlev = (int)tr.lev_ptr.size() - 1;
    if (nlev <= 0) return;
    alg_ += tr.nnz * (S + 4.0) + S * 3.0 * tr.n + 12.0 * tr.n;
    const auto key = std::make_tuple((const void *)&tr, (const void *)f, (const void *)g);
    auto it = tri_graphs_.find(key);
    if (it == tri_graphs_.end()) {
      if (!capture_) hip_check(hipStreamCreateWithFlags(&capture_, hipStreamNonBlocking), "hipStreamCreateWithFlags");
      hip_check(hipStreamBeginCapture(capture_, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
      hipError_t launch_err = hipSuccess;
      for (int k = 0; k < nlev; ++k) {
        const int32_t beg = tr.lev_ptr[k], cnt = tr.lev_ptr[k + 1] - beg;
        hipLaunchKernelGGL(k_tri_level<T>, dim3(blocks_for(cnt)), dim3(BLK), 0, capture_, (const int32_t *)tr.rp.get(),
                           (const int32_t *)tr.ci.get(), (const T *)tr.val.get(), (const int32_t *)tr.order.get(), beg,
                           cnt, f, g);
        if (launch_err == hipSuccess) launch_err = hipGetLastError();
      }
      hipGraph_t graph = nullptr;
      const hipError_t end_err = hipStreamEndCapture(capture_, &graph);
      hip_check(launch_err, "kernel launch during graph capture");
      hip_check(end_err, "hipStreamEndCapture");
      hipGraphExec_t exec = nullptr;
      const hipError_t inst_err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      hip_check(inst_err, "hipGraphInstantiate");
      it = tri_graphs_.emplace(key, exec).first;
    }
    end_run();
    hip_check(hipGraphLaunch(it->second, s), "hipGraphLaunch");
  }

  // Smoothing sweep on level l: x <- x + Mhat^{-1}(b - A x); first = true means x == 0 on entry.
  // f_ready: f = D^{-1} b is already in place (first sweep of a level fed by a fused restriction).
  void smooth(int l, const T *b, T *x, bool first, bool pre, bool ilu, const CycleOpts &o, hipStream_t s,
              bool f_ready = false) {
    DevLevel<T> &d = lv_[l];
    const int32_t n = d.n;
    const T *nul = nullptr;
    const int t = o.t;
    T *pp[2] = {d.g1.get(), d.g2.get()};
    if (o.smoother == NAMG_SMOOTH_L1JAC) {
      // l1-Jacobi (the Table 6 comparator): x <- x + D_l1^{-1}(b - A x); from x = 0 one pass x = D_l1^{-1} b
      if (first) {
        residual(l, b, nul, d.dl1inv.get(), nullptr, x, s);
      } else {
        residual(l, b, x, d.dl1inv.get(), nullptr, d.f.get(), s);
        axpy(l, d.f.get(), nul, x, x, n, s);
      }
      return;
    }
    if (!ilu) {
      // polynomial Gauss-Seidel (Section 5.2): f = D^{-1}(b - A x), g <- f - (D^{-1}L) g, x += g
      if (!f_ready) residual(l, b, first ? nul : (const T *)x, d.dinv.get(), nullptr, d.f.get(), s);
      const DMat<T> &M = pre ? d.pgs_lo : d.pgs_up;
      if (o.tri_mode == NAMG_TRI_NEUMANN) {
        if (t == 1) {
          axpy(l, d.f.get(), nul, first ? nul : (const T *)x, x, n, s);
        } else {
          const T *in = d.f.get();
          for (int q = 1; q < t; ++q) {
            const bool last = q == t - 1;
            T *out = last ? x : pp[q & 1];
            neumann(l, M, d.f.get(), in, nul, (last && !first) ? (const T *)x : nul, out, s);
            in = out;
          }
        }
      } else {
        tri_solve(l, pre ? d.tri_pgs_lo : d.tri_pgs_up, d.f.get(), d.g1.get(), s);
        axpy(l, d.g1.get(), nul, first ? nul : (const T *)x, x, n, s);
      }
      return;
    }
    // ILU(0) (Section 5.3): r = b - A x; y <- r - L_s y; v <- D_U^{-1}y - U_s v; x += v
    const T *r = b;
    if (!first) {
      residual(l, b, x, nullptr, d.r.get(), nullptr, s);
      r = d.r.get();
    }
    if (o.tri_mode == NAMG_TRI_NEUMANN) {
      if (t == 1) {
        axpy(l, r, d.ilu_dinv.get(), first ? nul : (const T *)x, x, n, s);
        return;
      }
      const T *in = r;
      for (int q = 1; q < t; ++q) {
        const bool last = q == t - 1;
        T *out = last ? d.f.get() : pp[q & 1];
        neumann(l, d.ilu_lo, r, in, last ? (const T *)d.ilu_dinv.get() : nul, nul, out, s);
        in = out;
      }
      in = d.f.get();
      for (int q = 1; q < t; ++q) {
        const bool last = q == t - 1;
        T *out = last ? x : pp[q & 1];
        neumann(l, d.ilu_up, d.f.get(), in, nul, (last && !first) ? (const T *)x : nul, out, s);
        in = out;
      }
    } else {
      if (first) {
        axpy(l, b, nul, nul, d.r.get(), n, s);  // the captured solve reads a fixed buffer
        r = d.r.get();
      }
      tri_solve(l, d.tri_ilu_lo, r, d.g1.get(), s);
      axpy(l, d.g1.get(), d.ilu_dinv.get(), nul, d.f.get(), n, s);
      tri_solve(l, d.tri_ilu_up, d.f.get(), d.g2.get(), s);
      axpy(l, d.g2.get(), nul, first ? nul : (const T *)x, x, n, s);
    }
  }

  // The two halves of one level of the V-cycle (Section 5). Down: zero initial guess, pre-smoothing,
  // residual, restriction. Up: prolongation and correction, post-smoothing.
  void level_down(int l, const T *b, T *x, const CycleOpts &o, hipStream_t s) {
    DevLevel<T> &d = lv_[l];
    const bool ilu = (o.smoother == NAMG_SMOOTH_ILU0) && d.has_ilu;
    if (o.nu1 == 0) fill_zero(l, x, d.n, s);
    for (int k = 0; k < o.nu1; ++k) smooth(l, b, x, k == 0, true, ilu, o, s, k == 0 && fused_f(l, o));
    residual(l, b, x, nullptr, d.r.get(), nullptr, s);
    restrict_(l, o, s);
  }

  void level_up(int l, const T *b, T *x, const CycleOpts &o, hipStream_t s) {
    DevLevel<T> &d = lv_[l];
    const bool ilu = (o.smoother == NAMG_SMOOTH_ILU0) && d.has_ilu;
    prolong(l, x, s);
    for (int k = 0; k < o.nu2; ++k) smooth(l, b, x, false, false, ilu, o, s);
  }

  // One V-cycle with zero initial guess; dense solve on the coarsest level.
  void vcycle(int l, const T *b, T *x, const CycleOpts &o, hipStream_t s) {
    const int nl = (int)lv_.size();
    if (l == nl - 1) {
      coarse_solve(l, b, x, s);
      return;
    }
    DevLevel<T> &c = lv_[l + 1];
    level_down(l, b, x, o, s);
    vcycle(l + 1, c.b.get(), c.x.get(), o, s);
    level_up(l, b, x, o, s);
  }

  // Level schedules and CSR copies for the direct comparators, built on their first use.
  void ensure_direct() {
    if (direct_ready_) return;
    for (size_t l = 0; l + 1 < lv_.size(); ++l) {
      const HostLevel &h = host_->lv[l];
      DevLevel<T> &d = lv_[l];
      if (h.host_smoother) {
        d.tri_pgs_lo.build(h.pgs_lo, level_schedule(h.pgs_lo, true), &mc_);
        d.tri_pgs_up.build(h.pgs_up, level_schedule(h.pgs_up, false), &mc_);
      } else {
        std::vector<double> dinv, dl1inv;
        HostCsr lo, up;
        pgs_data(h.A, dinv, dl1inv, lo, up);
        d.tri_pgs_lo.build(lo, level_schedule(lo, true), &mc_);
        d.tri_pgs_up.build(up, level_schedule(up, false), &mc_);
      }
      if (h.has_ilu) {
        d.tri_ilu_lo.build(h.ilu_lo, level_schedule(h.ilu_lo, true), &mc_);
        d.tri_ilu_up.build(h.ilu_up, level_schedule(h.ilu_up, false), &mc_);
      }
    }
    direct_ready_ = true;
  }

  int dev_;
  const HostHierarchy *host_;
  bool direct_ready_ = false;
  std::map<std::tuple<const void *, const void *, const void *>, hipGraphExec_t> tri_graphs_;
  hipStream_t capture_ = nullptr;
  MemCounter mc_;
  std::vector<DevLevel<T>> lv_;
  DMat<T> coarse_inv_;
  int32_t nc_ = 0;
  DMat<double> A64_;
  double anorm_inf_ = 0.0;
  DevBuf<double> red_, V_, w_, dot_, cd_, gram_;
  DevBuf<T> Z_, vin_;
  DevBuf<KState> kst_;
  int ws_m_ = 0;
  int64_t ldv_ = 0, ldz_ = 0;
  int32_t nblk_red_ = 0, nblk_dot_ = 0, rows_per_dot_ = 0;
  // host-mapped scalars: [0] estimate, [1] flag (column 0, and the serving engine's steps), [2] reductions,
  // then (estimate, flag) of Arnoldi step i at step_slot(i)
  double *pinned_ = nullptr;
  double *pinned_dev_ = nullptr;  // the same memory as seen from the device
  double alg_ = 0.0;
  int prof_family_ = NAMG_KF_NONE, prof_level_ = -1, prof_every_ = 1;
  int64_t prof_seen_ = 0;
  bool in_run_ = false, run_timed_ = false;
  hipStream_t run_stream_ = nullptr;
  namg_kernel_profile prof_{0, 0.0, 0.0};
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events_;
  size_t ev_used_ = 0;
  std::vector<hipEvent_t> phase_ev_;  // phase timing (NAMG_DIAG_PHASE_TIMES), reused across solves
  size_t phase_used_ = 0;
  hipEvent_t wall_ev_[2] = {nullptr, nullptr};  // ms_total of every solve, created on the first one
};

}  // namespace namg

#include "server.hpp"

// Krylov workspace of namg_solve_noalloc: one static array per device, held from the library's load until
// the process ends. Host code never passes the array's name to a kernel (on the host it names a host-side
// stand-in); it uses the device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[NAMG_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;  // device ordinal -> address of that device's copy of `scratch`

// The device address of `scratch` on device dev, resolved once per device with dev current.
void *scratch_on(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  namg::DeviceGuard g(dev);
  void *ptr = nullptr;
  namg::hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
  if (!ptr) throw namg::HipError{NAMG_E_HIP, "hipGetSymbolAddress(scratch) returned a null address"};
  g_scratch_ptr.emplace(dev, ptr);
  return ptr;
}

}  // namespace

struct namg_hier {
  namg::HostHierarchy host;
  int precision = NAMG_FP64;
  int device = -1;
  std::unique_ptr<namg::SolverBase> dev;
};

namespace {

template <class F>
int guarded(F &&f) {
  try {
    namg::g_last_error.clear();
    return f();
  } catch (const namg::SetupError &e) {
    namg::g_last_error = e.msg;
    return e.code;
  } catch (const namg::HipError &e) {
    namg::g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    namg::g_last_error = "host allocation failed";
    return NAMG_E_NOMEM;
  } catch (...) {
    namg::g_last_error = "unexpected internal error";
    return NAMG_E_INVALID;
  }
}

namg::SolverBase *device_of(namg_hier *h) {
  if (!h) throw namg::SetupError{NAMG_E_INVALID, "null hierarchy"};
  if (!h->dev) throw namg::SetupError{NAMG_E_NODEVICE, "hierarchy was set up host-only (device = -1)"};
  return h->dev.get();
}

}  // namespace

extern "C" {

void namg_default_setup_params(namg_setup_params *p) {
  if (!p) return;
  p->theta = 0.25;
  p->max_levels = 25;
  p->max_coarse = 50;
  p->precision = NAMG_FP64;
  p->ilu_levels = 1;
  p->device = 0;
  p->ilu_kind = NAMG_ILU0;
  p->ilut_lfil = 5;
  p->ilut_droptol = 1e-2;
  p->agg_levels = 0;
  p->coarsen = NAMG_COARSEN_RS;
  p->seed = 0;
}

void namg_default_solve_params(namg_solve_params *p) {
  if (!p) return;
  p->tol = 1e-8;
  p->restart = 30;
  p->max_iters = 1000;
  p->smoother = NAMG_SMOOTH_PGS;
  p->tri_mode = NAMG_TRI_NEUMANN;
  p->inner_terms = 2;
  p->gmres_T = NAMG_T_NEUMANN;
  p->pre_sweeps = 1;
  p->post_sweeps = 1;
  p->t_degree = 1;
  p->stop_rule = NAMG_STOP_RELRES;
  p->diagnostics = 0;
  p->res_hist = nullptr;
  p->res_hist_cap = 0;
}

int namg_setup(int32_t n, const int32_t *rowptr, const int32_t *colind, const double *vals,
               const namg_setup_params *p, namg_hier **out) {
  return guarded([&]() -> int {
    if (!p || !out) throw namg::SetupError{NAMG_E_INVALID, "null argument"};
    *out = nullptr;
    if (p->precision != NAMG_FP64 && p->precision != NAMG_FP32_PRECOND)
      throw namg::SetupError{NAMG_E_INVALID, "unknown precision"};
    namg::HostCsr A = namg::import_csr(n, rowptr, colind, vals);
    if (p->coarsen == NAMG_COARSEN_PMIS && p->device < 0)
      throw namg::SetupError{NAMG_E_INVALID, "PMIS setup runs on a device (device >= 0)"};
    if (p->device >= 0) {
      int count = 0;
      namg::hip_check(hipGetDeviceCount(&count), "hipGetDeviceCount");
      if (p->device >= count) throw namg::SetupError{NAMG_E_INVALID, "device ordinal out of range"};
    }
    auto h = std::make_unique<namg_hier>();
    h->host = namg::build_hierarchy(A, *p);
    h->precision = p->precision;
    h->device = p->device;
    if (p->device >= 0) {
      if (p->precision == NAMG_FP64)
        h->dev = std::make_unique<namg::Solver<double>>(h->host, p->device);
      else
        h->dev = std::make_unique<namg::Solver<float>>(h->host, p->device);
    }
    h->host.device_levels.reset();  // device-built levels, now packed into the solver's layouts
    *out = h.release();
    return NAMG_OK;
  });
}

int namg_solve(namg_hier *h, const double *b_dev, double *x_dev, const namg_solve_params *p, void *stream,
               namg_solve_stats *st) {
  return guarded([&]() -> int {
    if (!p || !b_dev || !x_dev) throw namg::SetupError{NAMG_E_INVALID, "null argument"};
    namg::validate_solve_params(*p);
    return device_of(h)->solve(b_dev, x_dev, *p, (hipStream_t)stream, st);
  });
}

int namg_solve_noalloc(namg_hier *h, const double *b_dev, double *x_dev, const namg_solve_params *p, void *stream,
                       namg_solve_stats *st) {
  return guarded([&]() -> int {
    if (!p || !b_dev || !x_dev) throw namg::SetupError{NAMG_E_INVALID, "null argument"};
    namg::validate_solve_params(*p);
    namg::SolverBase *sv = device_of(h);
    return sv->solve_in(b_dev, x_dev, *p, (hipStream_t)stream, st, scratch_on(h->device), NAMG_NOALLOC_SCRATCH_BYTES);
  });
}

int namg_vcycle(namg_hier *h, const double *b_dev, double *x_dev, const namg_solve_params *p, void *stream) {
  return guarded([&]() -> int {
    if (!p || !b_dev || !x_dev) throw namg::SetupError{NAMG_E_INVALID, "null argument"};
    namg::validate_solve_params(*p);
    device_of(h)->vcycle64(b_dev, x_dev, *p, (hipStream_t)stream);
    return NAMG_OK;
  });
}

int namg_apply(namg_hier *h, int level, int op, const namg_solve_params *p, const double *in1_dev,
               const double *in2_dev, double *out_dev, void *stream) {
  return guarded([&]() -> int {
    if (!p || !out_dev) throw namg::SetupError{NAMG_E_INVALID, "null argument"};
    namg::validate_solve_params(*p);
    device_of(h)->apply(level, op, *p, in1_dev, in2_dev, out_dev, (hipStream_t)stream);
    return NAMG_OK;
  });
}

int namg_profile_kernel(namg_hier *h, int family, int level, int every) {
  return guarded([&]() -> int {
    if (family < NAMG_KF_NONE || family > NAMG_KF_TRI) throw namg::SetupError{NAMG_E_INVALID, "unknown kernel family"};
    if (every < 1) throw namg::SetupError{NAMG_E_INVALID, "every must be >= 1"};
    device_of(h)->profile(family, level, every);
    return NAMG_OK;
  });
}

int namg_profile_read(namg_hier *h, namg_kernel_profile *out) {
  return guarded([&]() -> int {
    if (!out) throw namg::SetupError{NAMG_E_INVALID, "null argument"};
    *out = device_of(h)->profile_read();
    return NAMG_OK;
  });
}

int namg_hier_info(const namg_hier *h, namg_hierarchy_info *out) {
  return guarded([&]() -> int {
    if (!h || !out) throw namg::SetupError{NAMG_E_INVALID, "null argument"};
    std::memset(out, 0, sizeof(*out));
    out->levels = (int)h->host.lv.size();
    double nnz = 0, rows = 0;
    for (int l = 0; l < out->levels; ++l) {
      out->n[l] = h->host.lv[l].A.nr;
      out->nnz[l] = h->host.lv[l].A.nnz();
      nnz += (double)out->nnz[l];
      rows += out->n[l];
    }
    out->op_complexity = nnz / (double)out->nnz[0];
    out->grid_complexity = rows / (double)out->n[0];
    out->device_bytes = h->dev ? h->dev->device_bytes() : 0;
    return NAMG_OK;
  });
}

int namg_level_sizes(const namg_hier *h, int level, int32_t *n, int64_t *nnzA, int64_t *nnzP, int32_t *ncoarse) {
  return guarded([&]() -> int {
    if (!h) throw namg::SetupError{NAMG_E_INVALID, "null hierarchy"};
    if (level < 0 || level >= (int)h->host.lv.size()) throw namg::SetupError{NAMG_E_INVALID, "level out of range"};
    const auto &L = h->host.lv[level];
    if (n) *n = L.A.nr;
    if (nnzA) *nnzA = L.A.nnz();
    if (nnzP) *nnzP = L.P.nnz();
    if (ncoarse) *ncoarse = L.P.nc;
    return NAMG_OK;
  });
}

int namg_export_level(const namg_hier *h, int level, int8_t *cf, int32_t *A_rowptr, int32_t *A_colind,
                      double *A_vals, int32_t *P_rowptr, int32_t *P_colind, double *P_vals) {
  return guarded([&]() -> int {
    if (!h) throw namg::SetupError{NAMG_E_INVALID, "null hierarchy"};
    if (level < 0 || level >= (int)h->host.lv.size()) throw namg::SetupError{NAMG_E_INVALID, "level out of range"};
    const auto &L = h->host.lv[level];
    if (cf) std::copy(L.cf.begin(), L.cf.end(), cf);
    if (A_rowptr) std::copy(L.A.rp.begin(), L.A.rp.end(), A_rowptr);
    if (A_colind) std::copy(L.A.ci.begin(), L.A.ci.end(), A_colind);
    if (A_vals) std::copy(L.A.v.begin(), L.A.v.end(), A_vals);
    if (!L.P.rp.empty()) {
      if (P_rowptr) std::copy(L.P.rp.begin(), L.P.rp.end(), P_rowptr);
      if (P_colind) std::copy(L.P.ci.begin(), L.P.ci.end(), P_colind);
      if (P_vals) std::copy(L.P.v.begin(), L.P.v.end(), P_vals);
    }
    return NAMG_OK;
  });
}

int namg_export_ilu(const namg_hier *h, int level, int64_t *nnz_lower, int64_t *nnz_upper, int32_t *L_rowptr,
                    int32_t *L_colind, double *L_vals, int32_t *U_rowptr, int32_t *U_colind, double *U_vals,
                    double *d_inv) {
  return guarded([&]() -> int {
    if (!h) throw namg::SetupError{NAMG_E_INVALID, "null hierarchy"};
    if (level < 0 || level >= (int)h->host.lv.size()) throw namg::SetupError{NAMG_E_INVALID, "level out of range"};
    const auto &L = h->host.lv[level];
    if (!L.has_ilu) throw namg::SetupError{NAMG_E_INVALID, "level carries no ILU factors"};
    if (nnz_lower) *nnz_lower = (int64_t)L.ilu_lo.ci.size();
    if (nnz_upper) *nnz_upper = (int64_t)L.ilu_up.ci.size();
    auto put = [](const namg::HostCsr &T, int32_t *rp, int32_t *ci, double *v) {
      if (rp) std::copy(T.rp.begin(), T.rp.end(), rp);
      if (ci) std::copy(T.ci.begin(), T.ci.end(), ci);
      if (v) std::copy(T.v.begin(), T.v.end(), v);
    };
    put(L.ilu_lo, L_rowptr, L_colind, L_vals);
    put(L.ilu_up, U_rowptr, U_colind, U_vals);
    if (d_inv) std::copy(L.ilu_dinv.begin(), L.ilu_dinv.end(), d_inv);
    return NAMG_OK;
  });
}

int namg_ilu_diagnostics(const namg_hier *h, int level, int power_iters, int ruiz_max_iters, double ruiz_tol,
                         namg_ilu_diag *out) {
  return guarded([&]() -> int {
    if (!h || !out) throw namg::SetupError{NAMG_E_INVALID, "null argument"};
    if (level < 0 || level >= (int)h->host.lv.size()) throw namg::SetupError{NAMG_E_INVALID, "level out of range"};
    namg::ilu_diagnostics(h->host.lv[level], power_iters, ruiz_max_iters, ruiz_tol, out);
    return NAMG_OK;
  });
}

int namg_tri_jacobi_residuals(const namg_hier *h, int level, const double *b, int iters, double *res_L,
                              double *res_U) {
  return guarded([&]() -> int {
    if (!h || !res_L || !res_U) throw namg::SetupError{NAMG_E_INVALID, "null argument"};
    if (level < 0 || level >= (int)h->host.lv.size()) throw namg::SetupError{NAMG_E_INVALID, "level out of range"};
    namg::tri_jacobi_residuals(h->host.lv[level], b, iters, res_L, res_U);
    return NAMG_OK;
  });
}

int namg_us_powers(const namg_hier *h, int level, int pmax, int power_iters, double *max_abs, double *norm2,
                   int64_t *nnz) {
  return guarded([&]() -> int {
    if (!h) throw namg::SetupError{NAMG_E_INVALID, "null argument"};
    if (level < 0 || level >= (int)h->host.lv.size()) throw namg::SetupError{NAMG_E_INVALID, "level out of range"};
    namg::us_powers(h->host.lv[level], pmax, power_iters, max_abs, norm2, nnz);
    return NAMG_OK;
  });
}

void namg_destroy(namg_hier *h) {
  if (!h) return;
  try {
    if (h->dev) {
      namg::DeviceGuard g(h->device);
      // namg_vcycle and namg_apply may still run on the caller's stream; the hierarchy's device blocks go
      // back to the block cache for reuse, so they must be idle first
      (void)hipDeviceSynchronize();
      h->dev.reset();
    }
  } catch (...) {
  }
  delete h;
}

const char *namg_last_error(void) { return namg::g_last_error.c_str(); }

struct namg_server {
  std::unique_ptr<namg::ServerBase> impl;
  namg_solve_params solve;  // the requests' default solve parameters
};

void namg_default_server_params(namg_server_params *p) {
  if (!p) return;
  p->hbm_budget = 0;
  p->max_inflight = 64;
  p->setup_threads = 8;
  p->device = 0;
  p->precision = NAMG_FP32_PRECOND;
  namg_default_solve_params(&p->solve);
}

int namg_server_create(const namg_server_params *p, namg_server **out) {
  return guarded([&]() -> int {
    if (!p || !out) throw namg::SetupError{NAMG_E_INVALID, "null argument"};
    *out = nullptr;
    namg::validate_served_params(p->solve);
    if (p->max_inflight < 1 || p->max_inflight > namg::MAX_BATCH)
      throw namg::SetupError{NAMG_E_INVALID, "max_inflight out of range"};
    if (p->setup_threads < 1) throw namg::SetupError{NAMG_E_INVALID, "setup_threads must be >= 1"};
    if (p->precision != NAMG_FP64 && p->precision != NAMG_FP32_PRECOND)
      throw namg::SetupError{NAMG_E_INVALID, "unknown precision"};
    int count = 0;
    namg::hip_check(hipGetDeviceCount(&count), "hipGetDeviceCount");
    if (p->device < 0 || p->device >= count) throw namg::SetupError{NAMG_E_INVALID, "device ordinal out of range"};
    namg_server_params q = *p;
    if (q.hbm_budget <= 0) {
      namg::DeviceGuard g(q.device);
      size_t free_b = 0, total_b = 0;
      namg::hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
      // other users of the device, and device setup memory (uploads, scratch, kept levels), which
      // admission does not count
      q.hbm_budget = (int64_t)total_b - ((int64_t)16 << 30) - namg::SETUP_DEVICE_RESERVE;
      if (q.hbm_budget <= 0) q.hbm_budget = (int64_t)total_b / 2;
    }
    auto s = std::make_unique<namg_server>();
    s->solve = q.solve;
    if (q.precision == NAMG_FP64)
      s->impl = std::make_unique<namg::Server<double>>(q);
    else
      s->impl = std::make_unique<namg::Server<float>>(q);
    *out = s.release();
    return NAMG_OK;
  });
}

int namg_server_submit(namg_server *s, int32_t n, const int32_t *rowptr, const int32_t *colind, const double *vals,
                       const double *b, const namg_setup_params *sp, const namg_solve_params *p, uint64_t *ticket) {
  return guarded([&]() -> int {
    if (!s || !b || !sp || !ticket) throw namg::SetupError{NAMG_E_INVALID, "null argument"};
    const namg_solve_params q = p ? *p : s->solve;
    namg::validate_served_params(q);
    *ticket = s->impl->submit(namg::import_csr(n, rowptr, colind, vals), b, *sp, q);
    return NAMG_OK;
  });
}

int namg_server_poll(namg_server *s, uint64_t ticket, double *x, namg_solve_stats *st, namg_request_times *tm) {
  return guarded([&]() -> int {
    if (!s) throw namg::SetupError{NAMG_E_INVALID, "null server"};
    return s->impl->poll(ticket, false, x, st, tm);
  });
}

int namg_server_wait(namg_server *s, uint64_t ticket, double *x, namg_solve_stats *st, namg_request_times *tm) {
  return guarded([&]() -> int {
    if (!s) throw namg::SetupError{NAMG_E_INVALID, "null server"};
    return s->impl->poll(ticket, true, x, st, tm);
  });
}

int namg_server_stats(namg_server *s, namg_server_counters *out) {
  return guarded([&]() -> int {
    if (!s || !out) throw namg::SetupError{NAMG_E_INVALID, "null argument"};
    *out = s->impl->stats();
    return NAMG_OK;
  });
}

double namg_server_clock(const namg_server *s) { return s ? s->impl->clock() : 0.0; }

void namg_server_destroy(namg_server *s) {
  if (!s) return;
  try {
    s->impl.reset();
  } catch (...) {
  }
  delete s;
}

}  // extern "C"

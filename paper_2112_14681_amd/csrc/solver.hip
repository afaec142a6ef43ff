// namg solve phase: device hierarchy, V-cycle driver, low-synchronization flexible GMRES and the C ABI.
//
// Host code issues every kernel on the caller's stream; the only host<->device crossings inside a solve
// are one 8-byte readback per Arnoldi step (the convergence estimate) and one per restart cycle
// (the true residual norm).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/namg.h"
#include "device.hpp"
#include "kernels.hpp"
#include "setup_host.hpp"

namespace namg {

namespace {
thread_local std::string g_last_error;

#define NAMG_LAUNCH(kernel, grid, stream, ...)                                                 \
  do {                                                                                         \
    if ((grid) > 0) {                                                                          \
      hipLaunchKernelGGL(kernel, dim3(grid), dim3(BLK), 0, stream, __VA_ARGS__);               \
      hip_check(hipGetLastError(), #kernel);                                                   \
    }                                                                                          \
  } while (0)

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

void validate_solve_params(const namg_solve_params &p) {
  if (!(p.tol > 0.0) || !std::isfinite(p.tol)) throw SetupError{NAMG_E_INVALID, "tol must be > 0"};
  if (p.restart < 1 || p.restart > NAMG_MAX_RESTART) throw SetupError{NAMG_E_INVALID, "restart out of range"};
  if (p.max_iters < 0) throw SetupError{NAMG_E_INVALID, "max_iters must be >= 0"};
  if (p.inner_terms < 1) throw SetupError{NAMG_E_INVALID, "inner_terms must be >= 1"};
  if (p.smoother != NAMG_SMOOTH_PGS && p.smoother != NAMG_SMOOTH_ILU0)
    throw SetupError{NAMG_E_INVALID, "unknown smoother"};
  if (p.tri_mode != NAMG_TRI_NEUMANN && p.tri_mode != NAMG_TRI_DIRECT)
    throw SetupError{NAMG_E_INVALID, "unknown tri_mode"};
  if (p.gmres_T != NAMG_T_NEUMANN && p.gmres_T != NAMG_T_DIRECT) throw SetupError{NAMG_E_INVALID, "unknown gmres_T"};
  if (p.pre_sweeps < 0 || p.post_sweeps < 0) throw SetupError{NAMG_E_INVALID, "negative sweep count"};
}
}  // namespace

class SolverBase {
 public:
  virtual ~SolverBase() = default;
  virtual int solve(const double *b, double *x, const namg_solve_params &p, hipStream_t s, namg_solve_stats *st) = 0;
  virtual void vcycle64(const double *b, double *x, const namg_solve_params &p, hipStream_t s) = 0;
  virtual void apply(int level, int op, const namg_solve_params &p, const double *in1, const double *in2, double *out,
                     hipStream_t s) = 0;
  virtual int64_t device_bytes() const = 0;
};

template <class T>
struct DevLevel {
  int32_t n = 0;
  DSell<T> A, P, R, pgs_lo, pgs_up, ilu_lo, ilu_up;
  DevBuf<T> dinv, ilu_dinv;
  bool has_ilu = false;
  DTri<T> tri_pgs_lo, tri_pgs_up, tri_ilu_lo, tri_ilu_up;
  DevBuf<T> b, x, r, f, g1, g2;
};

template <class T>
class Solver final : public SolverBase {
 public:
  Solver(const HostHierarchy &H, int device) : dev_(device) {
    DeviceGuard g(dev_);
    const int nl = (int)H.lv.size();
    lv_.resize(nl);
    for (int l = 0; l < nl; ++l) {
      const HostLevel &h = H.lv[l];
      DevLevel<T> &d = lv_[l];
      d.n = h.A.nr;
      d.b.alloc(d.n, &mc_);
      d.x.alloc(d.n, &mc_);
      if (l == nl - 1) break;
      d.A.build(h.A, &mc_);
      d.P.build(h.P, &mc_);
      d.R.build(h.R, &mc_);
      d.pgs_lo.build(h.pgs_lo, &mc_);
      d.pgs_up.build(h.pgs_up, &mc_);
      upload_vec(d.dinv, h.dinv);
      d.tri_pgs_lo.build(h.pgs_lo, h.pgs_lo_sched, &mc_);
      d.tri_pgs_up.build(h.pgs_up, h.pgs_up_sched, &mc_);
      d.has_ilu = h.has_ilu;
      if (h.has_ilu) {
        d.ilu_lo.build(h.ilu_lo, &mc_);
        d.ilu_up.build(h.ilu_up, &mc_);
        upload_vec(d.ilu_dinv, h.ilu_dinv);
        d.tri_ilu_lo.build(h.ilu_lo, h.ilu_lo_sched, &mc_);
        d.tri_ilu_up.build(h.ilu_up, h.ilu_up_sched, &mc_);
      }
      d.r.alloc(d.n, &mc_);
      d.f.alloc(d.n, &mc_);
      d.g1.alloc(d.n, &mc_);
      d.g2.alloc(d.n, &mc_);
    }
    nc_ = H.lv.back().A.nr;
    std::vector<double> invT((size_t)nc_ * nc_);
    for (int32_t i = 0; i < nc_; ++i)
      for (int32_t j = 0; j < nc_; ++j) invT[(size_t)j * nc_ + i] = H.coarse_inv[(size_t)i * nc_ + j];
    upload_vec(coarse_invT_, invT);
    A64_.build(H.lv[0].A, &mc_);
    anorm_inf_ = H.anorm_inf;
    const int32_t n = lv_[0].n;
    nblk_red_ = (int32_t)blocks_for(n);
    red_.alloc(std::max<int32_t>(nblk_red_, 1) + 8, &mc_);
    kst_.alloc(1, &mc_);
    hip_check(hipHostMalloc((void **)&pinned_, 64, hipHostMallocDefault), "hipHostMalloc");
    hip_check(hipDeviceSynchronize(), "upload");
  }

  ~Solver() override {
    if (pinned_) (void)hipHostFree(pinned_);
  }

  int64_t device_bytes() const override { return mc_.bytes; }

  // ------------------------------------------------------------------------------------------ V-cycle
  void vcycle64(const double *b, double *x, const namg_solve_params &p, hipStream_t s) override {
    DeviceGuard g(dev_);
    const int32_t n = lv_[0].n;
    CycleOpts o = cycle_opts(p);
    if constexpr (std::is_same<T, double>::value) {
      vcycle(0, b, x, o, s);
    } else {
      NAMG_LAUNCH((k_cast<double, T>), blocks_for(n), s, b, lv_[0].b.get(), n);
      vcycle(0, lv_[0].b.get(), lv_[0].x.get(), o, s);
      NAMG_LAUNCH((k_cast<T, double>), blocks_for(n), s, lv_[0].x.get(), x, n);
    }
  }

  void apply(int level, int op, const namg_solve_params &p, const double *in1, const double *in2, double *out,
             hipStream_t s) override {
    DeviceGuard g(dev_);
    const int nl = (int)lv_.size();
    if (level < 0 || level >= nl) throw SetupError{NAMG_E_INVALID, "level out of range"};
    CycleOpts o = cycle_opts(p);
    if (op == NAMG_OP_SPMV64) {
      if (level != 0) throw SetupError{NAMG_E_INVALID, "SPMV64 is defined on level 0 only"};
      NAMG_LAUNCH((k_spmv<double, double, double, double>), blocks_for(A64_.nrows), s, A64_.view(), in1, out);
      return;
    }
    if (op == NAMG_OP_COARSE) {
      if (level != nl - 1) throw SetupError{NAMG_E_INVALID, "COARSE applies to the coarsest level"};
      DevLevel<T> &d = lv_[level];
      cast_in(in1, d.b.get(), d.n, s);
      NAMG_LAUNCH((k_dense_gemv<T>), blocks_for(nc_), s, coarse_invT_.get(), nc_, d.b.get(), d.x.get());
      cast_out(d.x.get(), out, d.n, s);
      return;
    }
    if (level == nl - 1) throw SetupError{NAMG_E_INVALID, "operator not defined on the coarsest level"};
    DevLevel<T> &d = lv_[level];
    DevLevel<T> &c = lv_[level + 1];
    const int32_t n = d.n;
    // private scratch for the operands: the level's b and x vectors and the next level's b / x
    switch (op) {
      case NAMG_OP_SPMV:
        cast_in(in1, d.x.get(), n, s);
        NAMG_LAUNCH((k_spmv<T, T, T, T>), blocks_for(n), s, d.A.view(), d.x.get(), d.b.get());
        cast_out(d.b.get(), out, n, s);
        break;
      case NAMG_OP_RESIDUAL:
        cast_in(in1, d.x.get(), n, s);
        cast_in(in2, d.b.get(), n, s);
        NAMG_LAUNCH((k_residual<T>), blocks_for(n), s, d.A.view(), d.b.get(), d.x.get(), (const T *)nullptr,
                    d.r.get(), (T *)nullptr);
        cast_out(d.r.get(), out, n, s);
        break;
      case NAMG_OP_SMOOTH_PRE:
      case NAMG_OP_SMOOTH_POST: {
        cast_in(in1, d.x.get(), n, s);
        cast_in(in2, d.b.get(), n, s);
        const bool ilu = (o.smoother == NAMG_SMOOTH_ILU0) && d.has_ilu;
        smooth(level, d.b.get(), d.x.get(), false, op == NAMG_OP_SMOOTH_PRE, ilu, o, s);
        cast_out(d.x.get(), out, n, s);
        break;
      }
      case NAMG_OP_RESTRICT:
        cast_in(in1, d.r.get(), n, s);
        NAMG_LAUNCH((k_spmv<T, T, T, T>), blocks_for(c.n), s, d.R.view(), d.r.get(), c.b.get());
        cast_out(c.b.get(), out, c.n, s);
        break;
      case NAMG_OP_PROLONG:
        cast_in(in1, c.x.get(), c.n, s);
        cast_in(in2, d.x.get(), n, s);
        NAMG_LAUNCH((k_prolong<T>), blocks_for(n), s, d.P.view(), c.x.get(), d.x.get());
        cast_out(d.x.get(), out, n, s);
        break;
      default:
        throw SetupError{NAMG_E_INVALID, "unknown operator"};
    }
  }

  // ------------------------------------------------------------------------------------------- solve
  int solve(const double *b, double *x, const namg_solve_params &p, hipStream_t s, namg_solve_stats *stats) override {
    DeviceGuard g(dev_);
    const int32_t n = lv_[0].n;
    const int m = p.restart;
    ensure_workspace(m);
    alg_ = 0.0;
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    hip_check(hipEventRecord(e0, s), "hipEventRecord");
    const CycleOpts o = cycle_opts(p);
    const bool trace = std::getenv("NAMG_TRACE") != nullptr;
    KState *ks = kst_.get();
    double *V = V_.get();
    T *Z = Z_.get();
    double *w = w_.get();
    T *vin = std::is_same<T, double>::value ? nullptr : vin_.get();

    // beta = ||b||, kept on the device for the residual estimates
    const double beta = std::sqrt(norm2sq(b, n, s));
    pinned_[4] = beta;
    hip_check(hipMemcpyAsync(&ks->beta, pinned_ + 4, sizeof(double), hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    namg_solve_stats st{};
    int status = NAMG_OK;
    double rn = 0.0;
    if (!std::isfinite(beta)) throw SetupError{NAMG_E_NONFINITE, "non-finite right-hand side"};
    if (beta == 0.0) {
      NAMG_LAUNCH((k_fill<double>), blocks_for(n), s, x, 0.0, n);
    } else {
      while (true) {
        // true residual r = b - A x into V(:,0) (FP64), plus the FP32 copy for the V-cycle
        NAMG_LAUNCH((k_residual64<T>), blocks_for(n), s, A64_.view(), b, x, V, vin, red_.get());
        alg_ += spmv_bytes(A64_, 8, 8) + 8.0 * n * 2;
        rn = std::sqrt(reduce_read(red_.get(), nblk_red_, s));
        if (!std::isfinite(rn)) throw SetupError{NAMG_E_NONFINITE, "non-finite residual"};
        if (trace) std::fprintf(stderr, "[namg] cycle %d true relres %.3e\n", st.cycles, rn / beta);
        if (rn / beta <= p.tol) {
          status = NAMG_OK;
          break;
        }
        if (st.iters >= p.max_iters) {
          status = NAMG_NOT_CONVERGED;
          break;
        }
        st.cycles++;
        const int me = std::min(m, p.max_iters - st.iters);
        int k = 0;
        for (int i = 0; i <= me; ++i) {
          const bool has_w = i < me;
          double *vi = V + (int64_t)i * ldv_;
          if (has_w) {
            T *zi = Z + (int64_t)i * ldz_;
            const T *b0;
            if constexpr (std::is_same<T, double>::value)
              b0 = vi;
            else
              b0 = vin;
            vcycle(0, b0, zi, o, s);
            st.precond_apps++;
            NAMG_LAUNCH((k_spmv<double, double, T, double>), blocks_for(n), s, A64_.view(), zi, w);
            alg_ += spmv_bytes(A64_, sizeof(T), 8);
          }
          const int32_t ncols = i + 1;
          NAMG_LAUNCH((k_multidot<8>), nblk_dot_, s, V, ldv_, ncols, has_w ? w : (const double *)nullptr, n,
                      rows_per_dot_, dot_.get(), nblk_dot_);
          alg_ += 8.0 * n * (ncols + (has_w ? 1 : 0));
          hipLaunchKernelGGL(k_arnoldi_step, dim3(1), dim3(BLK), 0, s, ks, dot_.get(), nblk_dot_, i, (int)has_w,
                             (int)(p.gmres_T == NAMG_T_DIRECT), (int)(i == me), p.tol);
          hip_check(hipGetLastError(), "k_arnoldi_step");
          hip_check(hipMemcpyAsync(pinned_, ks, 32, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
          hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
          const double est = pinned_[1];
          int32_t flag;
          std::memcpy(&flag, pinned_ + 3, sizeof(flag));
          if (flag < 0) throw SetupError{NAMG_E_NONFINITE, "non-finite value in the Arnoldi step"};
          if (i >= 1) {
            st.iters++;
            st.relres_est = est;
            if (trace) std::fprintf(stderr, "[namg]   iter %d est %.3e\n", st.iters, est);
          }
          if (i >= 1 && flag == 1) {
            k = i;
            break;
          }
          NAMG_LAUNCH((k_project<T>), blocks_for(n), s, V, ldv_, i, w, ks, n, vin);
          alg_ += 8.0 * n * (i + 4) + (vin ? sizeof(T) * (double)n : 0.0);
        }
        hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(64), 0, s, ks, k);
        hip_check(hipGetLastError(), "k_backsolve");
        NAMG_LAUNCH((k_update_x<T>), blocks_for(n), s, Z, ldz_, k, ks, x, n);
        alg_ += (double)n * (sizeof(T) * k + 16.0);
      }
    }
    const double xn = std::sqrt(norm2sq(x, n, s));
    hip_check(hipEventRecord(e1, s), "hipEventRecord");
    hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    st.status = status;
    st.relres_true = beta > 0.0 ? rn / beta : 0.0;
    st.nrbe = (beta > 0.0) ? rn / (beta + anorm_inf_ * xn) : 0.0;
    st.ms_total = ms;
    st.alg_bytes = alg_;
    if (stats) *stats = st;
    return status;
  }

 private:
  void upload_vec(DevBuf<T> &d, const std::vector<double> &h) {
    std::vector<T> t(h.begin(), h.end());
    d.alloc(t.size(), &mc_);
    d.upload(t.data(), t.size());
  }

  void cast_in(const double *src, T *dst, int32_t n, hipStream_t s) {
    if (!src) throw SetupError{NAMG_E_INVALID, "missing operand"};
    NAMG_LAUNCH((k_cast<double, T>), blocks_for(n), s, src, dst, n);
  }
  void cast_out(const T *src, double *dst, int32_t n, hipStream_t s) {
    NAMG_LAUNCH((k_cast<T, double>), blocks_for(n), s, src, dst, n);
  }

  static double spmv_bytes(const DSell<double> &A, double sx, double sy) {
    return A.nnz * (8.0 + 4.0) + sx * A.ncols + sy * A.nrows;
  }
  static double sell_bytes(const DSell<T> &A) { return A.nnz * (sizeof(T) + 4.0); }

  void ensure_workspace(int m) {
    if (ws_m_ >= m) return;
    const int32_t n = lv_[0].n;
    ldv_ = ((int64_t)n + 63) / 64 * 64;
    ldz_ = ldv_;
    V_.alloc((size_t)ldv_ * (m + 2), &mc_);
    Z_.alloc((size_t)ldz_ * m, &mc_);
    w_.alloc(n, &mc_);
    if (!std::is_same<T, double>::value) vin_.alloc(n, &mc_);
    nblk_dot_ = (int32_t)std::min<int64_t>(1024, std::max<int64_t>(1, blocks_for(n)));
    rows_per_dot_ = (int32_t)(((int64_t)n + nblk_dot_ - 1) / nblk_dot_);
    dot_.alloc((size_t)nblk_dot_ * 2 * (m + 2), &mc_);
    ws_m_ = m;
  }

  // |v|^2 (deterministic two-stage reduction on the device, read back to the host)
  double norm2sq(const double *v, int32_t n, hipStream_t s) {
    NAMG_LAUNCH(k_sumsq, blocks_for(n), s, v, n, red_.get());
    return reduce_read(red_.get(), nblk_red_, s);
  }

  double reduce_read(const double *partial, int32_t nb, hipStream_t s) {
    double *out = red_.get() + (red_.size() - 1);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(BLK), 0, s, partial, nb, out);
    hip_check(hipGetLastError(), "k_reduce");
    hip_check(hipMemcpyAsync(pinned_, out, sizeof(double), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    return pinned_[0];
  }

  // Smoothing sweep on level l: x <- x + Mhat^{-1}(b - A x); first = true means x == 0 on entry.
  void smooth(int l, const T *b, T *x, bool first, bool pre, bool ilu, const CycleOpts &o, hipStream_t s) {
    DevLevel<T> &d = lv_[l];
    const int32_t n = d.n;
    const unsigned gb = blocks_for(n);
    const T *nul = nullptr;
    const int t = o.t;
    T *pp[2] = {d.g1.get(), d.g2.get()};
    if (!ilu) {
      // polynomial Gauss-Seidel (Section 5.2): f = D^{-1}(b - A x), g <- f - (D^{-1}L) g, x += g
      NAMG_LAUNCH((k_residual<T>), gb, s, d.A.view(), b, first ? nul : (const T *)x, (const T *)d.dinv.get(),
                  (T *)nullptr, d.f.get());
      alg_ += (first ? 0.0 : sell_bytes(d.A)) + sizeof(T) * (double)n * (first ? 3 : 4);
      const DSell<T> &S = pre ? d.pgs_lo : d.pgs_up;
      if (o.tri_mode == NAMG_TRI_NEUMANN) {
        if (t == 1) {
          NAMG_LAUNCH((k_axpy<T>), gb, s, (const T *)d.f.get(), nul, first ? nul : (const T *)x, x, n);
          alg_ += sizeof(T) * (double)n * (first ? 2 : 3);
        } else {
          const T *in = d.f.get();
          for (int q = 1; q < t; ++q) {
            const bool last = q == t - 1;
            T *out = last ? x : pp[q & 1];
            NAMG_LAUNCH((k_neumann<T>), gb, s, S.view(), (const T *)d.f.get(), in, nul,
                        (last && !first) ? (const T *)x : nul, out);
            alg_ += sell_bytes(S) + sizeof(T) * (double)n * ((last && !first) ? 4 : 3);
            in = out;
          }
        }
      } else {
        const DTri<T> &tr = pre ? d.tri_pgs_lo : d.tri_pgs_up;
        tri_solve(tr, d.f.get(), d.g1.get(), s);
        NAMG_LAUNCH((k_axpy<T>), gb, s, (const T *)d.g1.get(), nul, first ? nul : (const T *)x, x, n);
        alg_ += sizeof(T) * (double)n * (first ? 2 : 3);
      }
      return;
    }
    // ILU(0) (Section 5.3): r = b - A x; y <- r - L_s y; v <- D_U^{-1}y - U_s v; x += v
    const T *r = b;
    if (!first) {
      NAMG_LAUNCH((k_residual<T>), gb, s, d.A.view(), b, (const T *)x, nul, d.r.get(), (T *)nullptr);
      alg_ += sell_bytes(d.A) + sizeof(T) * (double)n * 3;
      r = d.r.get();
    }
    if (o.tri_mode == NAMG_TRI_NEUMANN) {
      if (t == 1) {
        NAMG_LAUNCH((k_axpy<T>), gb, s, r, (const T *)d.ilu_dinv.get(), first ? nul : (const T *)x, x, n);
        alg_ += sizeof(T) * (double)n * (first ? 3 : 4);
        return;
      }
      const T *in = r;
      for (int q = 1; q < t; ++q) {
        const bool last = q == t - 1;
        T *out = last ? d.f.get() : pp[q & 1];
        NAMG_LAUNCH((k_neumann<T>), gb, s, d.ilu_lo.view(), r, in, last ? (const T *)d.ilu_dinv.get() : nul, nul, out);
        alg_ += sell_bytes(d.ilu_lo) + sizeof(T) * (double)n * (last ? 4 : 3);
        in = out;
      }
      in = d.f.get();
      for (int q = 1; q < t; ++q) {
        const bool last = q == t - 1;
        T *out = last ? x : pp[q & 1];
        NAMG_LAUNCH((k_neumann<T>), gb, s, d.ilu_up.view(), (const T *)d.f.get(), in, nul,
                    (last && !first) ? (const T *)x : nul, out);
        alg_ += sell_bytes(d.ilu_up) + sizeof(T) * (double)n * ((last && !first) ? 4 : 3);
        in = out;
      }
    } else {
      tri_solve(d.tri_ilu_lo, r, d.g1.get(), s);
      NAMG_LAUNCH((k_axpy<T>), gb, s, (const T *)d.g1.get(), (const T *)d.ilu_dinv.get(), nul, d.f.get(), n);
      tri_solve(d.tri_ilu_up, d.f.get(), d.g2.get(), s);
      NAMG_LAUNCH((k_axpy<T>), gb, s, (const T *)d.g2.get(), nul, first ? nul : (const T *)x, x, n);
      alg_ += sizeof(T) * (double)n * (first ? 5 : 6);
    }
  }

  // g = (I + S)^{-1} f, one launch per dependency level.
  void tri_solve(const DTri<T> &tr, const T *f, T *g, hipStream_t s) {
    const int nlev = (int)tr.lev_ptr.size() - 1;
    for (int k = 0; k < nlev; ++k) {
      const int32_t beg = tr.lev_ptr[k], cnt = tr.lev_ptr[k + 1] - beg;
      NAMG_LAUNCH((k_tri_level<T>), blocks_for(cnt), s, tr.rp.get(), tr.ci.get(), tr.val.get(), tr.order.get(), beg,
                  cnt, f, g);
    }
    alg_ += tr.nnz * (sizeof(T) + 4.0) + sizeof(T) * (double)tr.n * 3 + 8.0 * tr.n;
  }

  // One V-cycle with zero initial guess (Section 5): pre-smooth, residual, restrict, recurse, prolong
  // and correct, post-smooth; dense solve on the coarsest level.
  void vcycle(int l, const T *b, T *x, const CycleOpts &o, hipStream_t s) {
    const int nl = (int)lv_.size();
    if (l == nl - 1) {
      NAMG_LAUNCH((k_dense_gemv<T>), blocks_for(nc_), s, coarse_invT_.get(), nc_, b, x);
      alg_ += sizeof(T) * ((double)nc_ * nc_ + 2.0 * nc_);
      return;
    }
    DevLevel<T> &d = lv_[l];
    DevLevel<T> &c = lv_[l + 1];
    const int32_t n = d.n;
    const bool ilu = (o.smoother == NAMG_SMOOTH_ILU0) && d.has_ilu;
    if (o.nu1 == 0) NAMG_LAUNCH((k_fill<T>), blocks_for(n), s, x, T(0), n);
    for (int k = 0; k < o.nu1; ++k) smooth(l, b, x, k == 0, true, ilu, o, s);
    NAMG_LAUNCH((k_residual<T>), blocks_for(n), s, d.A.view(), b, (const T *)x, (const T *)nullptr, d.r.get(),
                (T *)nullptr);
    alg_ += sell_bytes(d.A) + sizeof(T) * (double)n * 3;
    NAMG_LAUNCH((k_spmv<T, T, T, T>), blocks_for(c.n), s, d.R.view(), (const T *)d.r.get(), c.b.get());
    alg_ += sell_bytes(d.R) + sizeof(T) * ((double)n + c.n);
    vcycle(l + 1, c.b.get(), c.x.get(), o, s);
    NAMG_LAUNCH((k_prolong<T>), blocks_for(n), s, d.P.view(), (const T *)c.x.get(), x);
    alg_ += sell_bytes(d.P) + sizeof(T) * ((double)c.n + 2.0 * n);
    for (int k = 0; k < o.nu2; ++k) smooth(l, b, x, false, false, ilu, o, s);
  }

  int dev_;
  MemCounter mc_;
  std::vector<DevLevel<T>> lv_;
  DevBuf<T> coarse_invT_;
  int32_t nc_ = 0;
  DSell<double> A64_;
  double anorm_inf_ = 0.0;
  DevBuf<double> red_, V_, w_, dot_;
  DevBuf<T> Z_, vin_;
  DevBuf<KState> kst_;
  int ws_m_ = 0;
  int64_t ldv_ = 0, ldz_ = 0;
  int32_t nblk_red_ = 0, nblk_dot_ = 0, rows_per_dot_ = 0;
  double *pinned_ = nullptr;
  double alg_ = 0.0;
};

}  // namespace namg

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
}

int namg_setup(int32_t n, const int32_t *rowptr, const int32_t *colind, const double *vals,
               const namg_setup_params *p, namg_hier **out) {
  return guarded([&]() -> int {
    if (!p || !out) throw namg::SetupError{NAMG_E_INVALID, "null argument"};
    *out = nullptr;
    if (p->precision != NAMG_FP64 && p->precision != NAMG_FP32_PRECOND)
      throw namg::SetupError{NAMG_E_INVALID, "unknown precision"};
    namg::HostCsr A = namg::import_csr(n, rowptr, colind, vals);
    auto h = std::make_unique<namg_hier>();
    h->host = namg::build_hierarchy(A, p->theta, p->max_levels, p->max_coarse, p->ilu_levels);
    h->precision = p->precision;
    h->device = p->device;
    if (p->device >= 0) {
      int count = 0;
      namg::hip_check(hipGetDeviceCount(&count), "hipGetDeviceCount");
      if (p->device >= count) throw namg::SetupError{NAMG_E_INVALID, "device ordinal out of range"};
      if (p->precision == NAMG_FP64)
        h->dev = std::make_unique<namg::Solver<double>>(h->host, p->device);
      else
        h->dev = std::make_unique<namg::Solver<float>>(h->host, p->device);
    }
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

void namg_destroy(namg_hier *h) {
  if (!h) return;
  try {
    if (h->dev) {
      namg::DeviceGuard g(h->device);
      h->dev.reset();
    }
  } catch (...) {
  }
  delete h;
}

const char *namg_last_error(void) { return namg::g_last_error.c_str(); }

}  // extern "C"

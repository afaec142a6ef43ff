// Serving: a request scheduler that keeps many solves in flight on one GPU and advances them together.
//
// Requests (host CSR + right-hand side) are set up by a pool of host threads, admitted in arrival order
// when a slot is free and their exact device footprint fits the HBM budget, uploaded, and then join the
// scheduler. Each scheduler tick advances every in-flight solve by one Arnoldi step (or one restart-cycle
// boundary) with *batched* launches: every row operation of the V-cycle and every Krylov kernel is
// issued once per tick for all solves that need it, from one task table uploaded per tick. A finished
// solve leaves at the tick boundary, its memory is released and the next request is admitted while the
// others keep running (continuous batching). The per-solve arithmetic is the single-solve path's, so
// a result is bit-identical alone and in the mix.
#pragma once

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <utility>

namespace namg {

// One pass over a level matrix: its own layout and those of its strict lower and upper parts (the scaled
// triangles of polynomial GS, which have A's rows and columns and so A's column offsets).
struct MatrixShape {
  LayoutCount all, lo, up;
};

inline MatrixShape matrix_shape(const HostCsr &A, bool allow_dia = true) {
  MatrixShape m;
  m.all.dia_ok = m.lo.dia_ok = m.up.dia_ok = allow_dia;
  const int64_t mul = diag_mul(A.nr, A.nc);
  for (int32_t r = 0; r < A.nr; ++r) {
    const int32_t base = diag_base(r, mul);
    if (!allow_dia) {
      // one tight pass: the row's counts and the range of each part's offsets (row_span)
      int64_t mn = INT64_MAX, mx = INT64_MIN, lmn = INT64_MAX, lmx = INT64_MIN, umn = INT64_MAX, umx = INT64_MIN;
      int32_t nlo = 0, nup = 0;
      for (int32_t k = A.rp[r]; k < A.rp[r + 1]; ++k) {
        const int32_t c = A.ci[k];
        const int64_t d = (int64_t)c - base;
        mn = std::min(mn, d);
        mx = std::max(mx, d);
        if (c < r) {
          ++nlo;
          lmn = std::min(lmn, d);
          lmx = std::max(lmx, d);
        } else if (c > r) {
          ++nup;
          umn = std::min(umn, d);
          umx = std::max(umx, d);
        }
      }
      m.all.row_span(r, A.rp[r + 1] - A.rp[r], mn, mx);
      m.lo.row_span(r, nlo, lmn, lmx);
      m.up.row_span(r, nup, umn, umx);
      continue;
    }
    int32_t nlo = 0, nup = 0;
    for (int32_t k = A.rp[r]; k < A.rp[r + 1]; ++k) {
      const int32_t c = A.ci[k];
      const int64_t d = (int64_t)c - base;
      m.all.col(d);
      if (c < r) {
        ++nlo;
        m.lo.col(d);
      } else if (c > r) {
        ++nup;
        m.up.col(d);
      }
    }
    m.all.row(r, A.rp[r + 1] - A.rp[r]);
    m.lo.row(r, nlo);
    m.up.row(r, nup);
  }
  return m;
}

// Device bytes one DMat<T>::build of A allocates.
template <class T>
int64_t mat_alloc_bytes(const HostCsr &A, int force_group = 0, bool allow_dia = true) {
  return layout_count(A, allow_dia).bytes<T>(A.nr, force_group);
}

// One pass over P for the layouts of P and of R = P^T (R's rows are P's columns; entry (c, i) of R takes its
// column offset from R's own diagonal base).
inline std::pair<LayoutCount, LayoutCount> transfer_shape(const HostCsr &P) {
  LayoutCount lp, lr;
  // neither is counted for the slice-diagonal form (served requests never take it, and lr's columns arrive
  // out of row order)
  lp.dia_ok = lr.dia_ok = false;
  const int64_t mul_p = diag_mul(P.nr, P.nc), mul_r = diag_mul(P.nc, P.nr);
  std::vector<int32_t> rlen(P.nc, 0);
  int64_t rmn = INT64_MAX, rmx = INT64_MIN;  // R's offsets, over all its entries (its 16-bit test is global)
  for (int32_t i = 0; i < P.nr; ++i) {
    const int32_t base = diag_base(i, mul_p);
    int64_t mn = INT64_MAX, mx = INT64_MIN;
    for (int32_t k = P.rp[i]; k < P.rp[i + 1]; ++k) {
      const int32_t c = P.ci[k];
      const int64_t d = (int64_t)c - base, dr = (int64_t)i - diag_base(c, mul_r);
      mn = std::min(mn, d);
      mx = std::max(mx, d);
      rmn = std::min(rmn, dr);
      rmx = std::max(rmx, dr);
      rlen[c]++;
    }
    lp.row_span(i, P.rp[i + 1] - P.rp[i], mn, mx);
  }
  for (int32_t c = 0; c < P.nc; ++c) lr.row_span(c, rlen[c], rmn, rmx);
  return {lp, lr};
}

// Device bytes of the DMat<T> that packs prolongation P of C/F splitting cf (lp = its LayoutCount): the
// unit-row layout when it applies (pointers, masks, per-slice counts, the explicit rows' entries), else lp's layout.
template <class T>
int64_t prolong_alloc_bytes(const HostCsr &P, const std::vector<int8_t> &cf, const LayoutCount &lp) {
  if (choose_group(P.nr, lp.nnz) == 1) {
    const UnitRows u = unit_rows_of(P, cf);
    if (u.ok) {
      const int64_t ns = (int64_t)u.mask.size();
      return alloc_bytes(ns + 1, 4) + alloc_bytes(ns, 8) + alloc_bytes(2 * ns, 4) +
             alloc_bytes(u.stored, lp.narrow ? 2 : 4) + alloc_bytes(u.stored, sizeof(T));
    }
  }
  return lp.bytes<T>(P.nr);
}

// Device bytes of Solver<T>(H, device, allow_dia) with its Krylov workspace for restart m (the direct
// comparators' level schedules, which serving never builds, excluded).
template <class T>
int64_t solver_footprint(const HostHierarchy &H, int m, bool allow_dia = true) {
  const int64_t S = sizeof(T);
  const int nl = (int)H.lv.size();
  int64_t total = 0;
  for (int l = 0; l < nl; ++l) {
    const HostLevel &h = H.lv[l];
    const int64_t n = h.A.nr;
    total += 2 * alloc_bytes(n, S);  // b, x
    if (l == nl - 1) break;
    // A, its strict parts and (level 0) its FP64 copy from one pass; P and R from one pass over P
    const MatrixShape ms = matrix_shape(h.A, allow_dia);
    const auto pr = transfer_shape(h.P);
    if (l == 0) total += ms.all.bytes<double>(h.A.nr, 1);
    // A, P, then D^-1, D_l1^-1, r, f, g1, g2
    total += ms.all.bytes<T>(h.A.nr) + prolong_alloc_bytes<T>(h.P, h.cf, pr.first) + 6 * alloc_bytes(n, S);
    total += h.host_restriction ? mat_alloc_bytes<T>(h.R, 0, allow_dia) : pr.second.bytes<T>(h.P.nc);
    total += h.host_smoother ? mat_alloc_bytes<T>(h.pgs_lo, 0, allow_dia) + mat_alloc_bytes<T>(h.pgs_up, 0, allow_dia)
                             : ms.lo.bytes<T>(h.A.nr) + ms.up.bytes<T>(h.A.nr);
    if (h.has_ilu)
      total += mat_alloc_bytes<T>(h.ilu_lo, 0, allow_dia) + mat_alloc_bytes<T>(h.ilu_up, 0, allow_dia) + alloc_bytes(n, S);
  }
  const int64_t nc = H.lv.back().A.nr;
  // dense inverse: CSR with 64 lanes per row, columns always fit 16 bits; one row: group 1, counted as such
  if (nc > 1) {
    total += alloc_bytes(nc + 1, 4) + alloc_bytes(nc * nc, 2) + alloc_bytes(nc * nc, S);
  } else {
    LayoutCount one;
    one.dia_ok = allow_dia;
    one.col(0);
    one.row(0, 1);
    total += one.bytes<T>(1, 1);
  }
  if (nl == 1) total += mat_alloc_bytes<double>(H.lv[0].A, 1, allow_dia);
  const int64_t n0 = H.lv[0].A.nr;
  const int64_t nred = blocks_for(n0);
  total += alloc_bytes(std::max<int64_t>(nred, 1) + 8, 8) + alloc_bytes(1, sizeof(KState));
  // Krylov workspace: V, Z, w, the FP32 copy of v, the fused reduction's partial sums, its results
  const int64_t ld = (n0 + 63) / 64 * 64;
  const int64_t nblk = dot_blocks(n0);
  total += alloc_bytes(ld * (m + 2), 8) + alloc_bytes(ld * m, S) + alloc_bytes(n0, 8) +
           (S == 4 ? alloc_bytes(n0, S) : 0) + alloc_bytes(nblk * 2 * (m + 2), 8) + alloc_bytes(2 * (m + 2), 8);
  return total;
}

template <class T>
class BatchEngine {
 public:
  enum Phase { INIT = 0, STEP = 1, END = 2, DONE = 3 };
  struct Slot {
    Solver<T> *sv = nullptr;
    const double *b = nullptr;
    double *x = nullptr;
    int32_t n = 0;
    int phase = INIT, i = 0, me = 0, k = 0;
    double beta = 0.0, denom = 0.0, rn = 0.0, est = 0.0, alg = 0.0;
    int iters = 0, cycles = 0, apps = 0;
    int status = NAMG_PENDING;
    std::string err;
    namg_solve_params p{};  // this solve's parameters
    CycleOpts o{};          // and its V-cycle options
  };

  explicit BatchEngine(int device) : dev_(device) {
    DeviceGuard g(dev_);
    hip_check(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking), "hipStreamCreateWithFlags");
  }
  ~BatchEngine() {
    if (pinned_) (void)hipHostFree(pinned_);
    if (dbuf_) (void)hipFree(dbuf_);
    if (s_) (void)hipStreamDestroy(s_);
  }
  hipStream_t stream() const { return s_; }
  int64_t launches() const { return launches_; }
  double sync_seconds() const { return sync_s_; }

  // Advance every slot that is not DONE by one step. Throws HipError on a runtime failure.
  void tick(std::vector<Slot *> &slots) {
    DeviceGuard g(dev_);
    groups_.clear();
    stage_.clear();
    std::vector<Slot *> step, init, end, resid;
    for (Slot *sl : slots) {
      if (sl->phase == STEP) {
        step.push_back(sl);
      } else if (sl->phase == INIT) {
        init.push_back(sl);
        resid.push_back(sl);
      } else if (sl->phase == END) {
        end.push_back(sl);
        resid.push_back(sl);
      }
    }
    // 1. V-cycles z = M^{-1} v_{i+1} of every stepping solve, level by level, then w = A z
    if (!step.empty()) {
      batch_vcycles(step);
      std::vector<KTask<T>> t;
      std::vector<unsigned> nb;
      for (Slot *sl : step) {
        KTask<T> k = base(sl);
        k.zin = sl->sv->Z_.get() + (int64_t)sl->i * sl->sv->ldz_;
        t.push_back(k);
        nb.push_back(row_blocks(sl->n, 1));
        sl->alg += sl->sv->A64_.bytes() + (sizeof(T) + 8.0) * sl->n;
      }
      add_krylov(KOP_SPMV64, t, nb);
    }
    // 2. column completion of step 0 (rho_0 from the residual pass), the fused reduction, the small dense
    //    step, the projection, and the completion of column i from the projection's partial sums
    if (!step.empty()) {
      std::vector<KTask<T>> t, t0, tp, tf;
      std::vector<unsigned> nb, nc, ones, ones0, np;
      for (Slot *sl : step) {
        KTask<T> k = base(sl);
        k.partial = sl->sv->dot_.get();
        k.nblk = sl->sv->nblk_dot_;
        t.push_back(k);
        nb.push_back((unsigned)sl->sv->nblk_dot_);
        nc.push_back((unsigned)(2 * k.ncols));
        ones.push_back(1u);
        np.push_back(blocks_for(sl->n));
        KTask<T> f = base(sl);
        f.partial = sl->sv->red_.get();
        f.nblk = sl->sv->nblk_red_;
        tp.push_back(f);
        if (sl->i == 0) {
          f.last = 0;
          t0.push_back(f);
          ones0.push_back(1u);
        }
        f.i = sl->i + 1;
        f.last = sl->i + 1 == sl->me;
        tf.push_back(f);
        sl->alg += 8.0 * sl->n * (k.ncols + 1) + 8.0 * sl->n * (sl->i + 4);
      }
      if (!t0.empty()) add_krylov(KOP_FINISH, t0, ones0);
      add_krylov(KOP_MULTIDOT, t, nb);
      add_krylov(KOP_COLREDUCE, t, nc);
      add_krylov(KOP_STEP, t, ones);
      add_krylov(KOP_PROJECT, tp, np);
      add_krylov(KOP_FINISH, tf, ones);
    }
    // 3. cycle ends: y from the rotated Hessenberg, x += Z y
    if (!end.empty()) {
      std::vector<KTask<T>> t;
      std::vector<unsigned> ones, nb;
      for (Slot *sl : end) {
        t.push_back(base(sl));
        ones.push_back(1u);
        nb.push_back(blocks_for(sl->n));
        sl->alg += (double)sl->n * (sizeof(T) * sl->k + 16.0);
      }
      add_krylov(KOP_BACKSOLVE, t, ones);
      add_krylov(KOP_UPDATE, t, nb);
    }
    // 4. ||b|| of new solves, then the true residual of new solves and finished cycles
    if (!init.empty()) {
      std::vector<KTask<T>> t, tr;
      std::vector<unsigned> nb, ones;
      for (Slot *sl : init) {
        KTask<T> k = base(sl);
        k.x = const_cast<double *>(sl->b);
        k.partial = sl->sv->red_.get();
        k.nblk = sl->sv->nblk_red_;
        k.host_out = sl->sv->pinned_dev_ + 3;
        t.push_back(k);
        nb.push_back(blocks_for(sl->n));
        ones.push_back(1u);
      }
      add_krylov(KOP_SUMSQ, t, nb);
      add_krylov(KOP_REDUCE, t, ones);
    }
    if (!resid.empty()) {
      // ||x||^2 at the cycle's start for the backward-error denominator, before the residual pass
      // reuses the same partial-sum buffer
      std::vector<KTask<T>> t;
      std::vector<unsigned> nb, ones;
      for (Slot *sl : resid) {
        if (sl->p.stop_rule != NAMG_STOP_NRBE) continue;
        KTask<T> k = base(sl);
        k.partial = sl->sv->red_.get();
        k.nblk = sl->sv->nblk_red_;
        k.host_out = sl->sv->pinned_dev_ + 4;
        t.push_back(k);
        nb.push_back(blocks_for(sl->n));
        ones.push_back(1u);
        sl->alg += 8.0 * sl->n;
      }
      add_krylov(KOP_SUMSQ, t, nb);
      add_krylov(KOP_REDUCE, t, ones);
    }
    if (!resid.empty()) {
      std::vector<KTask<T>> t;
      std::vector<unsigned> nb, ones;
      for (Slot *sl : resid) {
        KTask<T> k = base(sl);
        k.partial = sl->sv->red_.get();
        k.nblk = sl->sv->nblk_red_;
        k.host_out = sl->sv->pinned_dev_ + 2;
        t.push_back(k);
        nb.push_back(blocks_for(sl->n));
        ones.push_back(1u);
        sl->alg += sl->sv->A64_.bytes() + 24.0 * sl->n;
      }
      add_krylov(KOP_RESIDUAL64, t, nb);
      add_krylov(KOP_REDUCE, t, ones);
    }
    submit_and_wait();
    // host side of the step: read back (estimate, flag) and the reductions, move every solve on
    for (Slot *sl : step) {
      const double *pin = sl->sv->pinned_;
      const int flag = (int)pin[1];
      if (flag < 0) {
        fail(sl, NAMG_E_NONFINITE, "non-finite value in the Arnoldi step");
        continue;
      }
      sl->apps++;
      sl->iters++;
      sl->est = pin[0];
      if (flag == 1) {
        sl->k = sl->i + 1;
        sl->phase = END;
      } else {
        sl->i++;
      }
    }
    for (Slot *sl : init) {
      const double b2 = sl->sv->pinned_[3];
      sl->beta = std::sqrt(b2);
      if (!std::isfinite(sl->beta)) {
        fail(sl, NAMG_E_NONFINITE, "non-finite right-hand side");
        continue;
      }
      if (sl->beta == 0.0) {
        hipLaunchKernelGGL(k_fill<double>, dim3(blocks_for(sl->n)), dim3(BLK), 0, s_, sl->x, 0.0, sl->n);
        hip_check(hipGetLastError(), "k_fill");
        hip_check(hipStreamSynchronize(s_), "hipStreamSynchronize");
        sl->rn = 0.0;
        sl->status = NAMG_OK;
        sl->phase = DONE;
        continue;
      }
      decide(sl);
    }
    for (Slot *sl : end) decide(sl);
  }

 private:
  struct Group {
    bool krylov;
    int op, g;
    size_t task_off, off_off;
    int ntasks;
    unsigned grid;
  };

  KTask<T> base(Slot *sl) const {
    Solver<T> &v = *sl->sv;
    KTask<T> k{};
    k.A = v.A64_.view();
    k.b = sl->b;
    k.x = sl->x;
    k.V = v.V_.get();
    k.w = v.w_.get();
    k.cd = v.cd_.get();
    k.host_out = v.pinned_dev_;
    k.Z = v.Z_.get();
    k.vlow = std::is_same<T, double>::value ? nullptr : v.vin_.get();
    k.ks = v.kst_.get();
    k.ldv = v.ldv_;
    k.ldz = v.ldz_;
    k.n = sl->n;
    k.i = sl->i;
    k.ncols = sl->i + 1;
    k.has_w = 1;
    k.last = 0;
    k.k = sl->k;
    k.nblk = v.nblk_dot_;
    k.rows_per_blk = v.rows_per_dot_;
    k.beta = sl->beta;
    k.denom = sl->denom;
    k.tol = sl->p.tol;
    k.t_mode = t_mode(sl->p);
    return k;
  }

  void fail(Slot *sl, int code, const char *msg) {
    sl->status = code;
    sl->err = msg;
    sl->phase = DONE;
  }

  // Cycle boundary: converged, out of iterations, or start the next cycle at step 0.
  void decide(Slot *sl) {
    sl->rn = std::sqrt(sl->sv->pinned_[2]);
    if (!std::isfinite(sl->rn)) {
      fail(sl, NAMG_E_NONFINITE, "non-finite residual");
      return;
    }
    sl->denom = sl->beta;
    if (sl->p.stop_rule == NAMG_STOP_NRBE) sl->denom += sl->sv->anorm_inf_ * std::sqrt(sl->sv->pinned_[4]);
    if (sl->rn / sl->denom <= sl->p.tol) {
      sl->status = NAMG_OK;
      sl->phase = DONE;
    } else if (sl->iters >= sl->p.max_iters) {
      sl->status = NAMG_NOT_CONVERGED;
      sl->phase = DONE;
    } else {
      sl->cycles++;
      sl->phase = STEP;
      sl->i = 0;
      sl->k = 0;
      sl->me = std::min(sl->p.restart, sl->p.max_iters - sl->iters);
    }
  }

  template <class Task>
  void add(bool krylov, int op, int g, const std::vector<Task> &tasks, const std::vector<unsigned> &blocks) {
    for (size_t c0 = 0; c0 < tasks.size(); c0 += MAX_BATCH) {
      const size_t nt = std::min<size_t>(MAX_BATCH, tasks.size() - c0);
      align();
      const size_t toff = stage_.size();
      stage_.resize(toff + nt * sizeof(Task));
      std::memcpy(stage_.data() + toff, tasks.data() + c0, nt * sizeof(Task));
      align();
      const size_t ooff = stage_.size();
      stage_.resize(ooff + (nt + 1) * sizeof(uint32_t));
      uint32_t *off = reinterpret_cast<uint32_t *>(stage_.data() + ooff);
      off[0] = 0;
      for (size_t q = 0; q < nt; ++q) off[q + 1] = off[q] + blocks[c0 + q];
      if (off[nt] == 0) continue;
      groups_.push_back(Group{krylov, op, g, toff, ooff, (int)nt, off[nt]});
    }
  }
  void add_krylov(int op, const std::vector<KTask<T>> &t, const std::vector<unsigned> &nb) { add(true, op, 0, t, nb); }
  void align() { stage_.resize((stage_.size() + 15) / 16 * 16); }

  // Record every stepping solve's V-cycle as row operations, then issue the k-th operation of every solve
  // on a level together (grouped by operation and lanes-per-row), level by level down and back up.
  void batch_vcycles(const std::vector<Slot *> &vc) {
    using Op = typename Solver<T>::RowOp;
    struct Rec {
      std::vector<std::vector<Op>> down, up;
      std::vector<Op> coarse;
      int L = 0;
    };
    std::vector<Rec> rec(vc.size());
    int Lmax = 0;
    for (size_t q = 0; q < vc.size(); ++q) {
      Slot *sl = vc[q];
      Solver<T> &v = *sl->sv;
      Rec &r = rec[q];
      r.L = (int)v.lv_.size();
      Lmax = std::max(Lmax, r.L);
      r.down.resize(r.L);
      r.up.resize(r.L);
      const T *b0;
      if constexpr (std::is_same<T, double>::value)
        b0 = v.V_.get() + (int64_t)sl->i * v.ldv_;
      else
        b0 = v.vin_.get();
      T *x0 = v.Z_.get() + (int64_t)sl->i * v.ldz_;
      auto bl = [&](int l) -> const T * { return l == 0 ? b0 : v.lv_[l].b.get(); };
      auto xl = [&](int l) -> T * { return l == 0 ? x0 : v.lv_[l].x.get(); };
      for (int l = 0; l + 1 < r.L; ++l) {
        v.record_ = &r.down[l];
        v.level_down(l, bl(l), xl(l), sl->o, s_);
        v.record_ = &r.up[l];
        v.level_up(l, bl(l), xl(l), sl->o, s_);
      }
      v.record_ = &r.coarse;
      v.coarse_solve(r.L - 1, bl(r.L - 1), xl(r.L - 1), s_);
      v.record_ = nullptr;
      for (auto &ops : r.down)
        for (auto &op : ops) sl->alg += op.bytes;
      for (auto &ops : r.up)
        for (auto &op : ops) sl->alg += op.bytes;
      for (auto &op : r.coarse) sl->alg += op.bytes;
    }
    auto zip = [&](auto pick) {
      size_t maxlen = 0;
      for (size_t q = 0; q < vc.size(); ++q)
        if (const std::vector<Op> *ops = pick(q)) maxlen = std::max(maxlen, ops->size());
      for (size_t k = 0; k < maxlen; ++k) {
        // bucket the k-th operations by (kind, group), keeping solve order
        std::vector<std::pair<int, int>> keys;
        std::vector<std::vector<RowTask<T>>> tasks;
        std::vector<std::vector<unsigned>> blocks;
        for (size_t q = 0; q < vc.size(); ++q) {
          const std::vector<Op> *ops = pick(q);
          if (!ops || k >= ops->size()) continue;
          const Op &op = (*ops)[k];
          // a SELL matrix loaded in chunks of eight has kernels of its own (row_kernel, WIDE)
          const bool wide = op.group == 1 && op.t.M.unroll == 8 && op.kind != ROP_PROLONG;
          const std::pair<int, int> key{op.kind, op.group | (wide ? WIDE : 0)};
          size_t j = 0;
          while (j < keys.size() && keys[j] != key) ++j;
          if (j == keys.size()) {
            keys.push_back(key);
            tasks.emplace_back();
            blocks.emplace_back();
          }
          tasks[j].push_back(op.t);
          blocks[j].push_back(op.grid);
        }
        for (size_t j = 0; j < keys.size(); ++j) add(false, keys[j].first, keys[j].second, tasks[j], blocks[j]);
      }
    };
    for (int l = 0; l < Lmax; ++l) {
      zip([&](size_t q) -> const std::vector<Op> * { return l + 1 < rec[q].L ? &rec[q].down[l] : nullptr; });
      zip([&](size_t q) -> const std::vector<Op> * { return l == rec[q].L - 1 ? &rec[q].coarse : nullptr; });
    }
    for (int l = Lmax - 2; l >= 0; --l)
      zip([&](size_t q) -> const std::vector<Op> * { return l + 1 < rec[q].L ? &rec[q].up[l] : nullptr; });
  }

  using RowKernel = void (*)(const RowTask<T> *, const uint32_t *, int);
  using KKernel = void (*)(const KTask<T> *, const uint32_t *, int);

  // Group code of a SELL matrix whose row kernels load entries in chunks of eight.
  static constexpr int WIDE = 0x100;

  template <int OP>
  static RowKernel row_kernel(int g) {
    switch (g) {
      case 1 | WIDE: return &kb_rows<OP, 1, T, 8>;
      case 1: return &kb_rows<OP, 1, T>;
      case 2: return &kb_rows<OP, 2, T>;
      case 4: return &kb_rows<OP, 4, T>;
      case 8: return &kb_rows<OP, 8, T>;
      case 16: return &kb_rows<OP, 16, T>;
      case 32: return &kb_rows<OP, 32, T>;
      default: return &kb_rows<OP, 64, T>;
    }
  }
  static RowKernel row_kernel(int op, int g) {
    switch (op) {
      case ROP_RESIDUAL: return row_kernel<ROP_RESIDUAL>(g);
      case ROP_NEUMANN: return row_kernel<ROP_NEUMANN>(g);
      case ROP_SPMV: return row_kernel<ROP_SPMV>(g);
      case ROP_PROLONG: return row_kernel<ROP_PROLONG>(g);
      case ROP_AXPY: return &kb_rows<ROP_AXPY, 1, T>;
      default: return &kb_rows<ROP_FILL, 1, T>;
    }
  }
  static KKernel krylov_kernel(int op) {
    switch (op) {
      case KOP_RESIDUAL64: return &kb_krylov<KOP_RESIDUAL64, T>;
      case KOP_SPMV64: return &kb_krylov<KOP_SPMV64, T>;
      case KOP_MULTIDOT: return &kb_krylov<KOP_MULTIDOT, T>;
      case KOP_COLREDUCE: return &kb_krylov<KOP_COLREDUCE, T>;
      case KOP_STEP: return &kb_krylov<KOP_STEP, T>;
      case KOP_PROJECT: return &kb_krylov<KOP_PROJECT, T>;
      case KOP_FINISH: return &kb_krylov<KOP_FINISH, T>;
      case KOP_BACKSOLVE: return &kb_krylov<KOP_BACKSOLVE, T>;
      case KOP_UPDATE: return &kb_krylov<KOP_UPDATE, T>;
      case KOP_REDUCE: return &kb_krylov<KOP_REDUCE, T>;
      default: return &kb_krylov<KOP_SUMSQ, T>;
    }
  }

  // One host-to-device copy of the whole task table, every launch in order, one synchronisation.
  void submit_and_wait() {
    if (groups_.empty()) return;
    const size_t bytes = stage_.size();
    if (bytes > pinned_cap_) {
      if (pinned_) hip_check(hipHostFree(pinned_), "hipHostFree");
      pinned_cap_ = bytes * 2;
      hip_check(hipHostMalloc((void **)&pinned_, pinned_cap_, hipHostMallocDefault), "hipHostMalloc");
    }
    if (bytes > dcap_) {
      if (dbuf_) hip_check(hipFree(dbuf_), "hipFree");
      dcap_ = bytes * 2;
      hip_check(hipMalloc((void **)&dbuf_, dcap_), "hipMalloc");
    }
    std::memcpy(pinned_, stage_.data(), bytes);
    hip_check(hipMemcpyAsync(dbuf_, pinned_, bytes, hipMemcpyHostToDevice, s_), "hipMemcpyAsync");
    for (const Group &gr : groups_) {
      const uint32_t *off = reinterpret_cast<const uint32_t *>(dbuf_ + gr.off_off);
      if (gr.krylov) {
        const KTask<T> *tasks = reinterpret_cast<const KTask<T> *>(dbuf_ + gr.task_off);
        hipLaunchKernelGGL(krylov_kernel(gr.op), dim3(gr.grid), dim3(BLK), 0, s_, tasks, off, gr.ntasks);
      } else {
        const RowTask<T> *tasks = reinterpret_cast<const RowTask<T> *>(dbuf_ + gr.task_off);
        hipLaunchKernelGGL(row_kernel(gr.op, gr.g), dim3(gr.grid), dim3(BLK), 0, s_, tasks, off, gr.ntasks);
      }
      hip_check(hipGetLastError(), "batched launch");
      launches_++;
    }
    const auto w0 = std::chrono::steady_clock::now();
    hip_check(hipStreamSynchronize(s_), "hipStreamSynchronize");
    sync_s_ += std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count();
  }

  int dev_;
  hipStream_t s_ = nullptr;
  double sync_s_ = 0.0;
  std::vector<char> stage_;
  std::vector<Group> groups_;
  char *pinned_ = nullptr, *dbuf_ = nullptr;
  size_t pinned_cap_ = 0, dcap_ = 0;
  int64_t launches_ = 0;
};

class ServerBase {
 public:
  virtual ~ServerBase() = default;
  virtual uint64_t submit(HostCsr &&A, const double *b, const namg_setup_params &sp, const namg_solve_params &p) = 0;
  virtual int poll(uint64_t ticket, bool wait, double *x, namg_solve_stats *st, namg_request_times *tm) = 0;
  virtual namg_server_counters stats() = 0;
  virtual double clock() const = 0;
};

template <class T>
class Server final : public ServerBase {
  using Engine = BatchEngine<T>;
  struct Req {
    uint64_t ticket = 0;
    HostCsr A;
    std::vector<double> b;
    namg_setup_params sp{};
    namg_solve_params p{};
    std::unique_ptr<HostHierarchy> H;
    std::unique_ptr<Solver<T>> sv;
    DevBuf<double> bd, xd;
    int64_t footprint = 0;
    typename Engine::Slot slot;
    std::vector<double> x;
    namg_solve_stats st{};
    namg_request_times tm{};
    int status = NAMG_PENDING;
    std::string err;
    bool done = false, counted = false;
    double tm_granted = 0.0;  // admission granted (before the device upload)
  };

 public:
  explicit Server(const namg_server_params &p) : p_(p), t0_(std::chrono::steady_clock::now()), eng_(p.device) {
    for (int q = 0; q < p_.setup_threads; ++q) setup_.emplace_back([this] { setup_loop(); });
    sched_ = std::thread([this] { sched_loop(); });
    finisher_ = std::thread([this] { finish_loop(); });
  }

  ~Server() override {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_setup_.notify_all();
    cv_admit_.notify_all();
    cv_sched_.notify_all();
    cv_done_.notify_all();
    cv_finish_.notify_all();
    for (auto &t : setup_) t.join();
    sched_.join();
    finisher_.join();
    if (std::getenv("NAMG_SERVER_TRACE"))
      std::fprintf(stderr, "[namg server] setup threads, summed over requests: setup %.3f s (device levels %.3f s, "
                           "host finish %.3f s), admission wait %.3f s, device upload %.3f s\n", t_setup_, t_levels_,
                   t_finish_, t_wait_admit_, t_upload_);
    DeviceGuard g(p_.device);
    reqs_.clear();
  }

  double clock() const override {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
  }

  uint64_t submit(HostCsr &&A, const double *b, const namg_setup_params &sp, const namg_solve_params &p) override {
    auto r = std::make_unique<Req>();
    r->b.assign(b, b + A.nr);
    r->A = std::move(A);
    r->sp = sp;
    r->p = p;
    r->tm.submit = clock();
    std::lock_guard<std::mutex> lk(mu_);
    r->ticket = next_++;
    const uint64_t t = r->ticket;
    setup_q_.push_back(r.get());
    reqs_[t] = std::move(r);
    submitted_++;
    cv_setup_.notify_one();
    return t;
  }

  int poll(uint64_t ticket, bool wait, double *x, namg_solve_stats *st, namg_request_times *tm) override {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) throw SetupError{NAMG_E_INVALID, "unknown ticket"};
    Req *r = it->second.get();
    if (wait) cv_done_.wait(lk, [&] { return r->done || stop_; });
    if (!r->done) return NAMG_PENDING;
    const int status = r->status;
    const std::string err = r->err;
    if (x && !r->x.empty()) std::copy(r->x.begin(), r->x.end(), x);
    if (st) *st = r->st;
    if (tm) *tm = r->tm;
    reqs_.erase(it);
    if (status < 0) throw SetupError{status, err};
    return status;
  }

  namg_server_counters stats() override {
    std::lock_guard<std::mutex> lk(mu_);
    namg_server_counters s{};
    s.submitted = submitted_;
    s.completed = completed_;
    s.failed = failed_;
    s.inflight = inflight_;
    s.waiting = (int64_t)(setup_q_.size() + admit_q_.size());
    s.ticks = ticks_;
    s.launches = eng_.launches();
    s.device_bytes_in_use = used_;
    s.peak_device_bytes = peak_;
    s.peak_inflight = peak_inflight_;
    s.footprint_mismatches = footprint_mismatches_;
    s.peak_setup_device_bytes = setup_mem().peak.load();
    return s;
  }

 private:
  void finish_locked(Req *r) {
    r->done = true;
    if (r->status >= 0)
      completed_++;
    else
      failed_++;
    r->tm.done = clock();
    cv_done_.notify_all();
  }

  void setup_loop() {
    (void)hipSetDevice(p_.device);
    while (true) {
      Req *r = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_setup_.wait(lk, [&] { return stop_ || !setup_q_.empty(); });
        if (stop_) return;
        r = setup_q_.front();
        setup_q_.pop_front();
      }
      r->tm.setup_start = clock();
      try {
        if (r->sp.coarsen == NAMG_COARSEN_PMIS) r->sp.device = p_.device;  // device setup on the server's GPU
        r->H = std::make_unique<HostHierarchy>(build_hierarchy(std::move(r->A), r->sp));
        // the solver, and the request's b and x
        r->footprint = solver_footprint<T>(*r->H, r->p.restart, false) + 2 * alloc_bytes(r->H->lv[0].A.nr, 8);
        r->A = HostCsr{};
      } catch (const SetupError &e) {
        std::lock_guard<std::mutex> lk(mu_);
        r->status = e.code;
        r->err = e.msg;
        finish_locked(r);
        continue;
      } catch (const HipError &e) {
        std::lock_guard<std::mutex> lk(mu_);
        r->status = e.code;
        r->err = e.msg;
        finish_locked(r);
        continue;
      } catch (...) {
        std::lock_guard<std::mutex> lk(mu_);
        r->status = NAMG_E_NOMEM;
        r->err = "host allocation failed during setup";
        finish_locked(r);
        continue;
      }
      r->tm.setup_done = clock();
      {
        std::unique_lock<std::mutex> lk(mu_);
        if (r->footprint > p_.hbm_budget) {
          r->status = NAMG_E_BUDGET;
          r->err = "request needs more device memory than the whole budget";
          finish_locked(r);
          continue;
        }
        admit_q_.push_back(r);
        cv_admit_.wait(lk, [&] {
          return stop_ || (admit_q_.front() == r && inflight_ < p_.max_inflight && used_ + r->footprint <= p_.hbm_budget);
        });
        if (stop_) return;
        admit_q_.pop_front();
        r->tm_granted = clock();
        used_ += r->footprint;
        peak_ = std::max(peak_, used_);
        inflight_++;
        peak_inflight_ = std::max<int64_t>(peak_inflight_, inflight_);
        cv_admit_.notify_all();
      }
      try {
        const int32_t n = r->H->lv[0].A.nr;
        r->sv = std::make_unique<Solver<T>>(*r->H, p_.device, false);  // SELL-64 only: see Solver
        r->H->device_levels.reset();  // packed into the solver's layouts; the blocks go back to the cache
        r->sv->reserve_workspace(r->p.restart);
        if (r->sv->device_bytes() + 2 * alloc_bytes(n, 8) != r->footprint) {
          std::lock_guard<std::mutex> lk(mu_);
          footprint_mismatches_++;
        }
        r->bd.alloc(n, nullptr);
        r->bd.upload(r->b.data(), n);
        std::vector<double> zero(n, 0.0);
        r->xd.alloc(n, nullptr);
        r->xd.upload(zero.data(), n);
        r->slot.sv = r->sv.get();
        r->slot.p = r->p;
        r->slot.o = cycle_opts(r->p);
        r->slot.b = r->bd.get();
        r->slot.x = r->xd.get();
        r->slot.n = n;
      } catch (...) {
        int code = NAMG_E_NOMEM;
        std::string msg = "device upload failed";
        try {
          throw;
        } catch (const HipError &e) {
          code = e.code;
          msg = e.msg;
        } catch (...) {
        }
        r->sv.reset();
        r->bd.release();
        r->xd.release();
        std::lock_guard<std::mutex> lk(mu_);
        used_ -= r->footprint;
        inflight_--;
        r->status = code;
        r->err = msg;
        finish_locked(r);
        cv_admit_.notify_all();
        continue;
      }
      r->tm.admitted = clock();
      {
        std::lock_guard<std::mutex> lk(mu_);
        join_q_.push_back(r);
        t_setup_ += r->tm.setup_done - r->tm.setup_start;
        t_levels_ += r->H->t_levels;
        t_finish_ += r->H->t_finish;
        t_wait_admit_ += r->tm_granted - r->tm.setup_done;
        t_upload_ += r->tm.admitted - r->tm_granted;
      }
      cv_sched_.notify_one();
    }
  }

  void complete(Req *r) {
    const int32_t n = r->slot.n;
    auto &sl = r->slot;
    r->x.assign(n, 0.0);
    if (sl.status >= 0)
      hip_check(hipMemcpy(r->x.data(), r->xd.get(), sizeof(double) * n, hipMemcpyDeviceToHost), "hipMemcpy D2H");
    double xn = 0.0;
    for (double v : r->x) xn += v * v;
    xn = std::sqrt(xn);
    r->st.status = sl.status;
    r->st.iters = sl.iters;
    r->st.cycles = sl.cycles;
    r->st.precond_apps = sl.apps;
    r->st.relres_true = sl.beta > 0.0 ? sl.rn / sl.beta : 0.0;
    r->st.relres_est = sl.est;
    r->st.nrbe = sl.beta > 0.0 ? sl.rn / (sl.beta + r->H->anorm_inf * xn) : 0.0;
    r->st.ms_total = (clock() - r->tm.admitted) * 1e3;
    r->st.alg_bytes = sl.alg;
    r->st.loss_orth = r->st.ms_vcycle = r->st.ms_spmv = r->st.ms_ortho = std::nan("");
    r->status = sl.status;
    r->err = sl.err;
    r->sv.reset();
    r->bd.release();
    r->xd.release();
    r->H.reset();
    r->b.clear();
    r->b.shrink_to_fit();
  }

  void sched_loop() {
    (void)hipSetDevice(p_.device);
    std::vector<Req *> active;
    // NAMG_SERVER_TRACE: where the scheduler thread's time goes (printed when the server stops)
    const bool trace = std::getenv("NAMG_SERVER_TRACE") != nullptr;
    double t_idle = 0.0, t_tick = 0.0, t_complete = 0.0;
    auto sec = [] { return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count(); };
    struct Report {
      bool on;
      const double &idle, &tick, &comp;
      ~Report() {
        if (on) std::fprintf(stderr, "[namg server] scheduler: idle %.3f s, ticks %.3f s, hand-off %.3f s\n", idle, tick, comp);
      }
    } report{trace, t_idle, t_tick, t_complete};
    struct SyncReport {
      bool on;
      const Engine &e;
      ~SyncReport() {
        if (on) std::fprintf(stderr, "[namg server] ticks: %.3f s waiting for the device\n", e.sync_seconds());
      }
    } sync_report{trace, eng_};
    while (true) {
      const double w0 = trace ? sec() : 0.0;
      {
        std::unique_lock<std::mutex> lk(mu_);
        if (active.empty()) cv_sched_.wait(lk, [&] { return stop_ || !join_q_.empty(); });
        if (stop_) return;
        for (Req *r : join_q_) active.push_back(r);
        join_q_.clear();
      }
      const double w1 = trace ? sec() : 0.0;
      t_idle += w1 - w0;
      std::vector<typename Engine::Slot *> slots;
      for (Req *r : active) slots.push_back(&r->slot);
      try {
        eng_.tick(slots);
      } catch (const HipError &e) {
        // every in-flight solve shared the failed batch; launches queued before the error may still write
        // to their buffers, so the stream drains before the finisher releases them
        (void)hipStreamSynchronize(eng_.stream());
        (void)hipGetLastError();
        for (auto *sl : slots) {
          sl->status = e.code;
          sl->err = e.msg;
          sl->phase = Engine::DONE;
        }
      }
      {
        std::lock_guard<std::mutex> lk(mu_);
        ticks_++;
      }
      const double w2 = trace ? sec() : 0.0;
      t_tick += w2 - w1;
      // finished solves go to the finisher thread: copying x back and freeing the solve's device memory
      // (whose frees can wait for the whole device) must not hold up the next tick
      std::vector<Req *> still;
      bool handed = false;
      for (Req *r : active) {
        if (r->slot.phase != Engine::DONE) {
          still.push_back(r);
          continue;
        }
        std::lock_guard<std::mutex> lk(mu_);
        finish_q_.push_back(r);
        handed = true;
      }
      if (handed) cv_finish_.notify_one();
      active.swap(still);
      if (trace) t_complete += sec() - w2;
    }
  }

  // Completes finished solves: x to the host, statistics, device memory released, then the request's
  // HBM share is returned to admission.
  void finish_loop() {
    (void)hipSetDevice(p_.device);
    while (true) {
      Req *r = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_finish_.wait(lk, [&] { return stop_ || !finish_q_.empty(); });
        if (finish_q_.empty()) return;  // stopping, nothing left
        r = finish_q_.front();
        finish_q_.pop_front();
      }
      try {
        complete(r);
      } catch (const HipError &e) {
        r->status = e.code;
        r->err = e.msg;
      }
      std::lock_guard<std::mutex> lk(mu_);
      used_ -= r->footprint;
      inflight_--;
      finish_locked(r);
      cv_admit_.notify_all();
    }
  }

  namg_server_params p_;
  std::chrono::steady_clock::time_point t0_;
  Engine eng_;
  std::mutex mu_;
  std::condition_variable cv_setup_, cv_admit_, cv_sched_, cv_done_, cv_finish_;
  std::deque<Req *> setup_q_, admit_q_, finish_q_;
  std::vector<Req *> join_q_;
  std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs_;
  std::vector<std::thread> setup_;
  std::thread sched_, finisher_;
  bool stop_ = false;
  uint64_t next_ = 1;
  int64_t used_ = 0, peak_ = 0, inflight_ = 0, peak_inflight_ = 0, submitted_ = 0, completed_ = 0, failed_ = 0;
  int64_t footprint_mismatches_ = 0;
  int64_t ticks_ = 0;
  double t_setup_ = 0.0, t_wait_admit_ = 0.0, t_upload_ = 0.0, t_levels_ = 0.0, t_finish_ = 0.0;
};

}  // namespace namg

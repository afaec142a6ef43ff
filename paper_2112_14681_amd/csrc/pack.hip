// Solve-phase layouts packed on the device from a hierarchy whose levels were built there (the device
// setup of Section 5.1): the same SELL-64 / CSR-lane-group arrays, 16-bit or 32-bit columns, that
// DMat::build packs on the host, byte for byte; and the polynomial Gauss-Seidel data of a level
// (D^{-1}L, D^{-1}U with entries a_ij / a_ii, 1 / a_ii and 1 / sum_j |a_ij|) computed with the host's
// arithmetic. Nothing of the matrix crosses PCIe: only slice widths and per-row counts come back for
// their (host) prefix sums.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <vector>

#include "../../include/namg.h"
#include "device.hpp"
#include "pack.hpp"

namespace namg {
namespace {

constexpr int PB = 256;
inline unsigned pgrid(int64_t n) { return (unsigned)std::max<int64_t>((n + PB - 1) / PB, 1); }

// w[s] = 64 * (longest row of slice s)
__global__ __launch_bounds__(PB) void k_slice_width(int32_t nrows, const int32_t *__restrict__ rp,
                                                    int32_t *__restrict__ w) {
  const int32_t s = blockIdx.x * PB + threadIdx.x;
  const int32_t nslices = (nrows + SELL_C - 1) / SELL_C;
  if (s >= nslices) return;
  int32_t m = 0;
  for (int32_t r = s * SELL_C; r < std::min(nrows, (s + 1) * SELL_C); ++r) m = std::max(m, rp[r + 1] - rp[r]);
  w[s] = m * SELL_C;
}

// The slice-diagonal form (see LayoutCount), one wavefront per slice s, lane l on row 64 s + l: each round
// takes the smallest pending column offset (column - the row's scaled diagonal base) over the wavefront,
// which is the slice's next slot, and the lanes whose row has that offset advance past it.
// uw[s] = the slice's number of distinct offsets, counted up to dia_cap(its longest row) + 1;
// *unsorted = 1 when some row's columns do not strictly increase (integer atomic only).
__global__ __launch_bounds__(PB) void k_dia_width(int32_t nrows, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci, int64_t mul,
                                                  int32_t *__restrict__ uw, int32_t *unsorted) {
  const int64_t t = (int64_t)blockIdx.x * PB + threadIdx.x;
  const int32_t s = (int32_t)(t >> 6), lane = (int32_t)(t & 63);
  if (s >= (nrows + SELL_C - 1) / SELL_C) return;  // whole wavefronts
  const int32_t r = s * SELL_C + lane;
  const int32_t base = diag_base(r, mul);
  int32_t k = 0, end = 0;
  if (r < nrows) {
    k = rp[r];
    end = rp[r + 1];
  }
  for (int32_t q = k + 1; q < end; ++q)
    if (ci[q] <= ci[q - 1]) {
      atomicOr(unsorted, 1);
      break;
    }
  int32_t len = end - k;
  for (int off = 32; off > 0; off >>= 1) len = max(len, __shfl_xor(len, off, 64));
  const int64_t cap = dia_cap(len);
  int32_t cnt = 0;
  while (true) {
    const int32_t cur = k < end ? ci[k] - base : INT32_MAX;
    int32_t m = cur;
    for (int off = 32; off > 0; off >>= 1) m = min(m, __shfl_xor(m, off, 64));
    if (m == INT32_MAX || cnt > cap) break;
    ++cnt;
    if (cur == m) ++k;
  }
  if (lane == 0) uw[s] = cnt;
}

// Packs the slice-diagonal form with the rounds of k_dia_width (run only when every slice was counted in
// full and every row is sorted, so slice s fills exactly its slots [sptr[s], sptr[s + 1]) / 64 ...):
// slot j of slice s takes offset doff[1 + sptr[s] / 64 + j] and, lane by lane, the row's entry at that offset
// or 0; doff[0] = ncols - 1.
template <class T>
__global__ __launch_bounds__(PB) void k_pack_dia(int32_t nrows, int32_t ncols, int64_t mul,
                                                 const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                 const double *__restrict__ v,
                                                 const int32_t *__restrict__ sptr, int32_t *__restrict__ doff,
                                                 T *__restrict__ val) {
  const int64_t t = (int64_t)blockIdx.x * PB + threadIdx.x;
  const int32_t s = (int32_t)(t >> 6), lane = (int32_t)(t & 63);
  if (s >= (nrows + SELL_C - 1) / SELL_C) return;
  const int32_t r = s * SELL_C + lane;
  const int32_t base = diag_base(r, mul);
  int32_t k = 0, end = 0;
  if (r < nrows) {
    k = rp[r];
    end = rp[r + 1];
  }
  const int32_t p0 = sptr[s], p1 = sptr[s + 1];
  int32_t j = 0;
  while (true) {
    const int32_t cur = k < end ? ci[k] - base : INT32_MAX;
    int32_t m = cur;
    for (int off = 32; off > 0; off >>= 1) m = min(m, __shfl_xor(m, off, 64));
    const int64_t d = (int64_t)p0 + (int64_t)j * SELL_C + lane;
    if (m == INT32_MAX || d >= p1) break;  // the second test never fires for a slice counted in full
    const bool has = cur == m;
    val[d] = has ? (T)v[k] : T(0);
    if (lane == 0) doff[1 + p0 / SELL_C + j] = m;
    if (has) ++k;
    ++j;
  }
  if (s == 0 && lane == 0) doff[0] = ncols - 1;
}

// *bad = 1 when a column lies outside [-32768, 32767] of its row's base (integer atomic only)
__global__ __launch_bounds__(PB) void k_fits16(int32_t nrows, const int32_t *__restrict__ rp,
                                               const int32_t *__restrict__ ci, int64_t mul, int32_t *bad) {
  const int32_t r = blockIdx.x * PB + threadIdx.x;
  if (r >= nrows) return;
  const int32_t base = diag_base(r, mul);
  for (int32_t k = rp[r]; k < rp[r + 1]; ++k) {
    const int64_t d = (int64_t)ci[k] - base;
    if (d < -32768 || d > 32767) {
      atomicOr(bad, 1);
      return;
    }
  }
}

// SELL-64: one thread per (slice, lane) slot, rows past the end included, so the padding is written too
template <class T>
__global__ __launch_bounds__(PB) void k_pack_sell(int32_t nrows, int32_t nslices, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                  const int32_t *__restrict__ sptr, int64_t mul, int32_t narrow,
                                                  int16_t *__restrict__ col16, int32_t *__restrict__ col,
                                                  T *__restrict__ val) {
  const int64_t slot = (int64_t)blockIdx.x * PB + threadIdx.x;
  if (slot >= (int64_t)nslices * SELL_C) return;
  const int32_t r = (int32_t)slot;
  const int32_t s = r / SELL_C, lane = r % SELL_C;
  const int32_t width = (sptr[s + 1] - sptr[s]) / SELL_C;
  const int32_t len = r < nrows ? rp[r + 1] - rp[r] : 0;
  const int32_t beg = r < nrows ? rp[r] : 0;
  const int32_t base = diag_base(r, mul);
  for (int32_t k = 0; k < width; ++k) {
    const int64_t d = (int64_t)sptr[s] + (int64_t)k * SELL_C + lane;
    const bool has = k < len;
    const int32_t c = has ? ci[beg + k] : -1;
    val[d] = has ? (T)v[beg + k] : T(0);
    if (narrow)
      col16[d] = has ? (int16_t)(c - base) : (int16_t)0;
    else
      col[d] = has ? c : 0;
  }
}

// Unit-row layout (device.hpp, UnitRows), one thread per row: an explicit row of rank l in slice s writes
// entry k (or padding: value 0, offset 0 or column 0) at ptr[s] + k * meta[2 s + 1] + l for k < the slice's
// width; a C point's row writes nothing
template <class T>
__global__ __launch_bounds__(PB) void k_pack_unit(int32_t nrows, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                  const int32_t *__restrict__ sptr, const uint64_t *__restrict__ mask,
                                                  const int32_t *__restrict__ meta, int64_t mul, int32_t narrow,
                                                  int16_t *__restrict__ col16, int32_t *__restrict__ col,
                                                  T *__restrict__ val) {
  const int32_t r = blockIdx.x * PB + threadIdx.x;
  if (r >= nrows) return;
  const int32_t s = r / SELL_C, lane = r % SELL_C;
  const uint64_t mk = mask[s];
  if ((mk >> lane) & 1) return;
  const int32_t l = lane - __popcll(mk & ((uint64_t(1) << lane) - 1));
  const int32_t m = meta[2 * s + 1];
  const int32_t width = (sptr[s + 1] - sptr[s]) / m;
  const int32_t len = rp[r + 1] - rp[r], beg = rp[r];
  const int32_t base = diag_base(r, mul);
  for (int32_t k = 0; k < width; ++k) {
    const int64_t d = (int64_t)sptr[s] + (int64_t)k * m + l;
    const bool has = k < len;
    val[d] = has ? (T)v[beg + k] : T(0);
    if (narrow)
      col16[d] = has ? (int16_t)(ci[beg + k] - base) : (int16_t)0;
    else
      col[d] = has ? ci[beg + k] : 0;
  }
}

// CSR with lane groups: the CSR arrays themselves, columns as offsets when narrow, values cast to T
template <class T>
__global__ __launch_bounds__(PB) void k_pack_csr(int32_t nrows, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                 int64_t mul, int32_t narrow, int16_t *__restrict__ col16,
                                                 int32_t *__restrict__ col, T *__restrict__ val) {
  const int32_t r = blockIdx.x * PB + threadIdx.x;
  if (r >= nrows) return;
  const int32_t base = diag_base(r, mul);
  for (int32_t k = rp[r]; k < rp[r + 1]; ++k) {
    val[k] = (T)v[k];
    if (narrow)
      col16[k] = (int16_t)(ci[k] - base);
    else
      col[k] = ci[k];
  }
}

// entries below / above the diagonal per row
__global__ __launch_bounds__(PB) void k_strict_count(int32_t n, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci, int32_t *__restrict__ nlo,
                                                     int32_t *__restrict__ nup) {
  const int32_t i = blockIdx.x * PB + threadIdx.x;
  if (i >= n) return;
  int32_t lo = 0, up = 0;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
    lo += ci[k] < i;
    up += ci[k] > i;
  }
  nlo[i] = lo;
  nup[i] = up;
}

// D^{-1}L and D^{-1}U (a_ij / a_ii in FP64), 1 / a_ii and 1 / sum_j |a_ij| (the sum in row order), as T
template <class T>
__global__ __launch_bounds__(PB) void k_smoother_data(int32_t n, const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                      const int32_t *__restrict__ lrp, const int32_t *__restrict__ urp,
                                                      int32_t *__restrict__ lci, double *__restrict__ lv,
                                                      int32_t *__restrict__ uci, double *__restrict__ uv,
                                                      T *__restrict__ dinv, T *__restrict__ dl1inv) {
  const int32_t i = blockIdx.x * PB + threadIdx.x;
  if (i >= n) return;
  double d = 0.0;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
    if (ci[k] == i) d = v[k];
  double l1 = 0.0;
  int32_t ql = lrp[i], qu = urp[i];
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
    const int32_t j = ci[k];
    l1 += fabs(v[k]);
    if (j < i) {
      lci[ql] = j;
      lv[ql++] = v[k] / d;
    } else if (j > i) {
      uci[qu] = j;
      uv[qu++] = v[k] / d;
    }
  }
  dinv[i] = (T)(1.0 / d);
  dl1inv[i] = (T)(1.0 / l1);
}

void check(const char *what) { hip_check(hipGetLastError(), what); }

// exclusive prefix sum of counts[0..n) into a host vector of n + 1 entries (32-bit, checked)
std::vector<int32_t> host_offsets(const std::vector<int32_t> &counts) {
  std::vector<int32_t> off(counts.size() + 1, 0);
  int64_t acc = 0;
  for (size_t q = 0; q < counts.size(); ++q) {
    acc += counts[q];
    if (acc > INT32_MAX) throw SetupError{NAMG_E_INVALID, "layout exceeds 2^31 entries"};
    off[q + 1] = (int32_t)acc;
  }
  return off;
}

}  // namespace

bool device_packing_enabled() { return std::getenv("NAMG_HOST_PACK") == nullptr; }

// The unit-row layout u of the prolongation D into M, as DMat::build_unit packs it (u computed on the host
// from the host copy of P and the level's C/F splitting).
template <class T>
void pack_unit_device(DMat<T> &M, const DCsr &D, const UnitRows &u, MemCounter *mc) {
  const int32_t nslices = (int32_t)u.mask.size();
  const std::vector<int32_t> meta = unit_meta(u);
  M.unit = true;
  M.group = 1;
  M.stored = u.stored;
  M.explicit_nnz = M.nnz;
  for (uint64_t mk : u.mask) M.explicit_nnz -= __builtin_popcountll(mk);
  M.explicit_rows = 0;
  for (int32_t c : u.count) M.explicit_rows += c;
  M.unit_pairs = unit_pairs_for(M.nrows, M.explicit_rows);
  M.ptr.alloc(u.ptr.size(), mc);
  M.ptr.upload(u.ptr.data(), u.ptr.size());
  M.umask.alloc(std::max<size_t>(u.mask.size(), 1), mc);
  M.umask.upload(u.mask.data(), u.mask.size());
  M.smeta.alloc(meta.size(), mc);
  M.smeta.upload(meta.data(), meta.size());
  if (M.narrow)
    M.col16.alloc((size_t)M.stored, mc);
  else
    M.col.alloc((size_t)M.stored, mc);
  M.val.alloc((size_t)M.stored, mc);
  if (nslices > 0) {
    hipLaunchKernelGGL(k_pack_unit<T>, dim3(pgrid(M.nrows)), dim3(PB), 0, 0, M.nrows, D.rp.get(), D.ci.get(),
                       D.v.get(), M.ptr.get(), M.umask.get(), M.smeta.get(), M.mul, (int32_t)M.narrow, M.col16.get(),
                       M.col.get(), M.val.get());
    check("k_pack_unit");
  }
}

template <class T>
void pack_device(DMat<T> &M, const DCsr &D, MemCounter *mc, int force_group, const UnitRows *unit, bool allow_dia) {
  M.unit = false;
  M.unit_pairs = false;
  M.dia = false;
  M.pairs_ok = dia_pairs_enabled();
  M.nrows = D.nr;
  M.ncols = D.nc;
  M.nnz = D.nnz;
  M.mul = diag_mul(M.nrows, M.ncols);
  DevBuf<int32_t> bad(1, &setup_mem());
  hip_check(hipMemset(bad.get(), 0, 4), "hipMemset");
  if (M.nrows > 0) {
    hipLaunchKernelGGL(k_fits16, dim3(pgrid(M.nrows)), dim3(PB), 0, 0, M.nrows, D.rp.get(), D.ci.get(), M.mul,
                       bad.get());
    check("k_fits16");
  }
  int32_t hbad = 0;
  hip_check(hipMemcpy(&hbad, bad.get(), 4, hipMemcpyDeviceToHost), "hipMemcpy D2H");
  M.narrow = hbad == 0;
  M.group = force_group > 0 ? force_group : choose_group(M.nrows, M.nnz);
  M.unroll = choose_unroll(M.group, M.nrows, M.nnz);
  if (unit && unit->ok && M.group == 1) {
    pack_unit_device(M, D, *unit, mc);
  } else if (M.group > 1) {
    M.stored = M.nnz;
    M.ptr.alloc((size_t)M.nrows + 1, mc);
    hip_check(hipMemcpy(M.ptr.get(), D.rp.get(), ((size_t)M.nrows + 1) * 4, hipMemcpyDeviceToDevice), "hipMemcpy D2D");
    if (M.narrow)
      M.col16.alloc((size_t)M.stored, mc);
    else
      M.col.alloc((size_t)M.stored, mc);
    M.val.alloc((size_t)M.stored, mc);
    if (M.nrows > 0) {
      hipLaunchKernelGGL(k_pack_csr<T>, dim3(pgrid(M.nrows)), dim3(PB), 0, 0, M.nrows, D.rp.get(), D.ci.get(),
                         D.v.get(), M.mul, (int32_t)M.narrow, M.col16.get(), M.col.get(), M.val.get());
      check("k_pack_csr");
    }
  } else {
    const int32_t nslices = (M.nrows + SELL_C - 1) / SELL_C;
    std::vector<int32_t> w(std::max(nslices, 1), 0);
    if (nslices > 0) {
      DevBuf<int32_t> dw((size_t)nslices, &setup_mem());
      hipLaunchKernelGGL(k_slice_width, dim3(pgrid(nslices)), dim3(PB), 0, 0, M.nrows, D.rp.get(), dw.get());
      check("k_slice_width");
      hip_check(hipMemcpy(w.data(), dw.get(), (size_t)nslices * 4, hipMemcpyDeviceToHost), "hipMemcpy D2H");
    }
    w.resize(nslices);
    if (allow_dia && nslices > 0 && layout_tuning().dia) {
      // the slice-diagonal choice, by the rule LayoutCount applies on the host
      std::vector<int32_t> uw(nslices, 0);
      int32_t unsorted = 0;
      {
        DevBuf<int32_t> duw((size_t)nslices, &setup_mem()), dflag(1, &setup_mem());
        hip_check(hipMemset(dflag.get(), 0, 4), "hipMemset");
        hipLaunchKernelGGL(k_dia_width, dim3(pgrid((int64_t)nslices * SELL_C)), dim3(PB), 0, 0, M.nrows, D.rp.get(),
                           D.ci.get(), M.mul, duw.get(), dflag.get());
        check("k_dia_width");
        hip_check(hipMemcpy(uw.data(), duw.get(), (size_t)nslices * 4, hipMemcpyDeviceToHost), "hipMemcpy D2H");
        hip_check(hipMemcpy(&unsorted, dflag.get(), 4, hipMemcpyDeviceToHost), "hipMemcpy D2H");
      }
      bool ok = unsorted == 0;
      int64_t sell_stored = 0, dia_stored = 0;
      for (int32_t q = 0; q < nslices; ++q) {
        ok = ok && uw[q] <= dia_cap(w[q] / SELL_C);
        sell_stored += w[q];
        dia_stored += (int64_t)uw[q] * SELL_C;
      }
      if (ok && dia_wins(sell_stored, dia_stored, M.narrow, sizeof(T))) {
        for (int32_t &q : uw) q *= SELL_C;
        const std::vector<int32_t> sptr = host_offsets(uw);
        M.dia = true;
        M.stored = sptr[nslices];
        M.unroll = 4;  // not used by the slice-diagonal kernels
        M.ptr.alloc(sptr.size(), mc);
        M.ptr.upload(sptr.data(), sptr.size());
        M.doff.alloc((size_t)(M.stored / SELL_C + 1), mc);
        M.val.alloc((size_t)M.stored, mc);
        hipLaunchKernelGGL(k_pack_dia<T>, dim3(pgrid((int64_t)nslices * SELL_C)), dim3(PB), 0, 0, M.nrows, M.ncols,
                           M.mul, D.rp.get(), D.ci.get(), D.v.get(), M.ptr.get(), M.doff.get(), M.val.get());
        check("k_pack_dia");
        hip_check(hipStreamSynchronize(nullptr), "hipStreamSynchronize");
        return;
      }
    }
    const std::vector<int32_t> sptr = host_offsets(w);
    M.stored = sptr[nslices];
    M.ptr.alloc(sptr.size(), mc);
    M.ptr.upload(sptr.data(), sptr.size());
    if (M.narrow)
      M.col16.alloc((size_t)M.stored, mc);
    else
      M.col.alloc((size_t)M.stored, mc);
    M.val.alloc((size_t)M.stored, mc);
    if (nslices > 0) {
      hipLaunchKernelGGL(k_pack_sell<T>, dim3(pgrid((int64_t)nslices * SELL_C)), dim3(PB), 0, 0, M.nrows, nslices,
                         D.rp.get(), D.ci.get(), D.v.get(), M.ptr.get(), M.mul, (int32_t)M.narrow, M.col16.get(),
                         M.col.get(), M.val.get());
      check("k_pack_sell");
    }
  }
  // the caller may release D (its blocks return to the cache) right after: wait for this null-stream work
  // only (the solves and setups of other requests run on streams of their own)
  hip_check(hipStreamSynchronize(nullptr), "hipStreamSynchronize");
}

template <class T>
void smoother_data_device(const DCsr &A, DCsr &lo, DCsr &up, DevBuf<T> &dinv, DevBuf<T> &dl1inv, MemCounter *mc) {
  const int32_t n = A.nr;
  DevBuf<int32_t> nlo((size_t)std::max(n, 1), &setup_mem()), nup((size_t)std::max(n, 1), &setup_mem());
  if (n > 0) {
    hipLaunchKernelGGL(k_strict_count, dim3(pgrid(n)), dim3(PB), 0, 0, n, A.rp.get(), A.ci.get(), nlo.get(),
                       nup.get());
    check("k_strict_count");
  }
  std::vector<int32_t> cl(n), cu(n);
  if (n > 0) {
    hip_check(hipMemcpy(cl.data(), nlo.get(), (size_t)n * 4, hipMemcpyDeviceToHost), "hipMemcpy D2H");
    hip_check(hipMemcpy(cu.data(), nup.get(), (size_t)n * 4, hipMemcpyDeviceToHost), "hipMemcpy D2H");
  }
  const std::vector<int32_t> lrp = host_offsets(cl), urp = host_offsets(cu);
  for (DCsr *tri : {&lo, &up}) {
    tri->nr = n;
    tri->nc = A.nc;
  }
  lo.nnz = lrp[n];
  up.nnz = urp[n];
  lo.rp.alloc(lrp.size(), &setup_mem());
  lo.rp.upload(lrp.data(), lrp.size());
  up.rp.alloc(urp.size(), &setup_mem());
  up.rp.upload(urp.data(), urp.size());
  lo.ci.alloc((size_t)std::max<int64_t>(lo.nnz, 1), &setup_mem());
  lo.v.alloc((size_t)std::max<int64_t>(lo.nnz, 1), &setup_mem());
  up.ci.alloc((size_t)std::max<int64_t>(up.nnz, 1), &setup_mem());
  up.v.alloc((size_t)std::max<int64_t>(up.nnz, 1), &setup_mem());
  dinv.alloc((size_t)std::max(n, 1), mc);
  dl1inv.alloc((size_t)std::max(n, 1), mc);
  if (n > 0) {
    hipLaunchKernelGGL(k_smoother_data<T>, dim3(pgrid(n)), dim3(PB), 0, 0, n, A.rp.get(), A.ci.get(), A.v.get(),
                       lo.rp.get(), up.rp.get(), lo.ci.get(), lo.v.get(), up.ci.get(), up.v.get(), dinv.get(),
                       dl1inv.get());
    check("k_smoother_data");
  }
  hip_check(hipStreamSynchronize(nullptr), "hipStreamSynchronize");
}

template void pack_device<float>(DMat<float> &, const DCsr &, MemCounter *, int, const UnitRows *, bool);
template void pack_device<double>(DMat<double> &, const DCsr &, MemCounter *, int, const UnitRows *, bool);
template void smoother_data_device<float>(const DCsr &, DCsr &, DCsr &, DevBuf<float> &, DevBuf<float> &,
                                          MemCounter *);
template void smoother_data_device<double>(const DCsr &, DCsr &, DCsr &, DevBuf<double> &, DevBuf<double> &,
                                           MemCounter *);

}  // namespace namg

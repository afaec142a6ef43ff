// Device construction of the AMG hierarchy with PMIS coarsening and BAMG direct interpolation (Section 5.1
// of arXiv 2112.14681), level by level on one GPU:
//   strength flags per entry of A (|a_ij| >= theta max_{k != i} |a_ik|) and the transposed strength
//   graph; PMIS in rounds (weights |S^T_i| + u_i, u_i a SplitMix64 draw); BAMG direct interpolation
//   P; R = P^T with rows sorted by fine index; A P and R (A P) by row-wise sparse products.
// Every result equals the CPU reference bit for bit: decisions are integer or comparisons of identical
// doubles; each PMIS round reads only the previous round's state, so thread order does not matter; each
// product entry is a running sum in the canonical order (row i of X in stored order, then row j of Y in
// stored order, the first product starting the sum), taken by one thread per output row.
// Each level's operators are copied to the host, where the smoother data, the coarse inverse and the
// device layouts of the solve phase are built as for the host setup.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <condition_variable>
#include <memory>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/namg.h"
#include "device.hpp"
#include "gpu_setup.hpp"
#include "pack.hpp"
#include "setup_host.hpp"

// Every product and sum of the setup is rounded on its own (no fused multiply-add), as in the oracle, so
// that P and the Galerkin operators match it bit for bit.
#pragma clang fp contract(off)

namespace namg {
namespace {

constexpr int TB = 256;
inline unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>((n + TB - 1) / TB, 1); }

enum : int8_t { PT_U = 0, PT_C = 1, PT_F = 2 };

// SplitMix64 (Steele, Lea and Flood 2014): output k >= 1 of the stream seeded with s is
// mix(s + k * 0x9E3779B97F4A7C15); point i draws output i + 1, top 53 bits scaled to [0, 1).
__device__ __forceinline__ double uniform01(uint64_t seed, int64_t i) {
  uint64_t z = seed + ((uint64_t)i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1.0p-53;
}

// Row i: flag[k] = 1 when column ci[k] != i strongly influences i; stcount[j] += 1 per row depending on j.
__global__ __launch_bounds__(TB) void k_strength(int32_t n, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                 double theta, uint8_t *__restrict__ flag, int32_t *stcount) {
  const int32_t i = blockIdx.x * TB + threadIdx.x;
  if (i >= n) return;
  const int32_t a = rp[i], b = rp[i + 1];
  double m = 0.0;
  for (int32_t k = a; k < b; ++k)
    if (ci[k] != i) m = fmax(m, fabs(v[k]));
  const double thr = theta * m;
  for (int32_t k = a; k < b; ++k) {
    const bool s = m != 0.0 && ci[k] != i && fabs(v[k]) >= thr;
    flag[k] = s ? 1 : 0;
    if (s) atomicAdd(&stcount[ci[k]], 1);
  }
}

// Transposed strength graph: row j lists the rows i that strongly depend on j (in no particular order).
__global__ __launch_bounds__(TB) void k_st_fill(int32_t n, const int32_t *__restrict__ rp,
                                                const int32_t *__restrict__ ci, const uint8_t *__restrict__ flag,
                                                const int32_t *__restrict__ st_rp, int32_t *cursor,
                                                int32_t *__restrict__ st_ci) {
  const int32_t i = blockIdx.x * TB + threadIdx.x;
  if (i >= n) return;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
    if (flag[k]) {
      const int32_t j = ci[k];
      st_ci[st_rp[j] + atomicAdd(&cursor[j], 1)] = i;
    }
}

__global__ __launch_bounds__(TB) void k_pmis_init(int32_t n, const int32_t *__restrict__ stcount, uint64_t seed,
                                                  double *__restrict__ w, int8_t *__restrict__ state) {
  const int32_t i = blockIdx.x * TB + threadIdx.x;
  if (i >= n) return;
  w[i] = (double)stcount[i] + uniform01(seed, i);
  state[i] = stcount[i] == 0 ? PT_F : PT_U;
}

__device__ __forceinline__ bool beats(double wi, int32_t i, double wj, int32_t j) {
  return wi > wj || (wi == wj && i < j);
}

// One PMIS round, first half: an undecided point that beats every undecided strong neighbour (either
// direction) is selected.
__global__ __launch_bounds__(TB) void k_pmis_select(int32_t n, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ ci, const uint8_t *__restrict__ flag,
                                                    const int32_t *__restrict__ st_rp,
                                                    const int32_t *__restrict__ st_ci, const double *__restrict__ w,
                                                    const int8_t *__restrict__ state, uint8_t *__restrict__ newc) {
  const int32_t i = blockIdx.x * TB + threadIdx.x;
  if (i >= n) return;
  if (state[i] != PT_U) {
    newc[i] = 0;
    return;
  }
  const double wi = w[i];
  bool best = true;
  for (int32_t k = rp[i]; k < rp[i + 1] && best; ++k) {
    const int32_t j = ci[k];
    if (flag[k] && state[j] == PT_U && !beats(wi, i, w[j], j)) best = false;
  }
  for (int32_t q = st_rp[i]; q < st_rp[i + 1] && best; ++q) {
    const int32_t j = st_ci[q];
    if (state[j] == PT_U && !beats(wi, i, w[j], j)) best = false;
  }
  newc[i] = best ? 1 : 0;
}

// Second half: selected points become C, undecided points strongly depending on one of them become F;
// the rest stay undecided and are counted.
__global__ __launch_bounds__(TB) void k_pmis_apply(int32_t n, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci, const uint8_t *__restrict__ flag,
                                                   const uint8_t *__restrict__ newc, int8_t *__restrict__ state,
                                                   int32_t *remaining) {
  const int32_t i = blockIdx.x * TB + threadIdx.x;
  if (i >= n || state[i] != PT_U) return;
  if (newc[i]) {
    state[i] = PT_C;
    return;
  }
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
    if (flag[k] && newc[ci[k]]) {
      state[i] = PT_F;
      return;
    }
  atomicAdd(remaining, 1);
}

// out[i] = 1 for C points (i < n), out[n] = 0: scanned into the coarse numbering.
__global__ __launch_bounds__(TB) void k_is_c(int32_t n, const int8_t *__restrict__ state, int32_t *__restrict__ out) {
  const int32_t i = blockIdx.x * TB + threadIdx.x;
  if (i < n) out[i] = state[i] == PT_C ? 1 : 0;
  if (i == n) out[n] = 0;
}

// Entries per row of P: 1 for a C point, the number of strong C neighbours for an F point; cnt[n] = 0.
__global__ __launch_bounds__(TB) void k_interp_count(int32_t n, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci, const uint8_t *__restrict__ flag,
                                                     const int8_t *__restrict__ state, int32_t *__restrict__ cnt) {
  const int32_t i = blockIdx.x * TB + threadIdx.x;
  if (i == n) cnt[n] = 0;
  if (i >= n) return;
  if (state[i] == PT_C) {
    cnt[i] = 1;
    return;
  }
  int32_t c = 0;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
    if (flag[k] && state[ci[k]] == PT_C) ++c;
  cnt[i] = c;
}

// BAMG direct interpolation: w_ij = -(a_ij + beta_i / n_i) / (a_ii + sum of the weak a_ik), beta_i the
// sum over strong F neighbours, both sums in stored (ascending column) order.
__global__ __launch_bounds__(TB) void k_interp_fill(int32_t n, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                    const uint8_t *__restrict__ flag, const int8_t *__restrict__ state,
                                                    const int32_t *__restrict__ cidx, const int32_t *__restrict__ prp,
                                                    int32_t *__restrict__ pci, double *__restrict__ pv) {
  const int32_t i = blockIdx.x * TB + threadIdx.x;
  if (i >= n) return;
  int32_t out = prp[i];
  if (state[i] == PT_C) {
    pci[out] = cidx[i];
    pv[out] = 1.0;
    return;
  }
  const int32_t ni = prp[i + 1] - out;
  if (ni == 0) return;
  const int32_t a = rp[i], b = rp[i + 1];
  double dd = 0.0;
  for (int32_t k = a; k < b; ++k)
    if (ci[k] == i) dd = v[k];
  double beta = 0.0;
  for (int32_t k = a; k < b; ++k) {
    const int32_t j = ci[k];
    if (j == i) continue;
    if (!flag[k])
      dd += v[k];
    else if (state[j] != PT_C)
      beta += v[k];
  }
  for (int32_t k = a; k < b; ++k) {
    const int32_t j = ci[k];
    if (j != i && flag[k] && state[j] == PT_C) {
      pci[out] = cidx[j];
      pv[out] = -(v[k] + beta / ni) / dd;
      ++out;
    }
  }
}

// Column counts of P (entries per row of R = P^T); cnt[nc] stays 0.
__global__ __launch_bounds__(TB) void k_col_count(int64_t nnz, const int32_t *__restrict__ pci, int32_t *cnt) {
  const int64_t e = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (e < nnz) atomicAdd(&cnt[pci[e]], 1);
}

__global__ __launch_bounds__(TB) void k_transpose_fill(int32_t n, const int32_t *__restrict__ prp,
                                                       const int32_t *__restrict__ pci, const double *__restrict__ pv,
                                                       const int32_t *__restrict__ rrp, int32_t *cursor,
                                                       int32_t *__restrict__ rci, double *__restrict__ rv) {
  const int32_t i = blockIdx.x * TB + threadIdx.x;
  if (i >= n) return;
  for (int32_t e = prp[i]; e < prp[i + 1]; ++e) {
    const int32_t J = pci[e];
    const int32_t pos = rrp[J] + atomicAdd(&cursor[J], 1);
    rci[pos] = i;
    rv[pos] = pv[e];
  }
}

// Sort each row's (column, value) pairs by column (insertion sort; columns within a row are distinct).
__global__ __launch_bounds__(TB) void k_sort_rows(int32_t nrows, const int32_t *__restrict__ rp,
                                                  int32_t *__restrict__ col, double *__restrict__ val) {
  const int32_t r = blockIdx.x * TB + threadIdx.x;
  if (r >= nrows) return;
  const int32_t a = rp[r], b = rp[r + 1];
  for (int32_t k = a + 1; k < b; ++k) {
    const int32_t c = col[k];
    const double x = val[k];
    int32_t q = k - 1;
    while (q >= a && col[q] > c) {
      col[q + 1] = col[q];
      val[q + 1] = val[q];
      --q;
    }
    col[q + 1] = c;
    val[q + 1] = x;
  }
}

// Hash-table size per output row of X Y: 0 for an empty product, else the power of two >= 2 * (number of
// products), so a table is at most half full; tsize[nrows] = 0.
__global__ __launch_bounds__(TB) void k_spgemm_size(int32_t nrows, const int32_t *__restrict__ xrp,
                                                    const int32_t *__restrict__ xci, const int32_t *__restrict__ yrp,
                                                    int64_t *__restrict__ tsize) {
  const int32_t i = blockIdx.x * TB + threadIdx.x;
  if (i == nrows) tsize[nrows] = 0;
  if (i >= nrows) return;
  int64_t bound = 0;
  for (int32_t k = xrp[i]; k < xrp[i + 1]; ++k) bound += yrp[xci[k] + 1] - yrp[xci[k]];
  int64_t ts = 0;
  if (bound > 0) {
    ts = 16;
    while (ts < 2 * bound) ts <<= 1;
  }
  tsize[i] = ts;
}

// Short rows of X Y, one wavefront per row: a row whose X row has at most WAVE entries and at most WAVE
// products. Lane k < len(X row) holds X's entry k and the length of Y's row x_ci[k]; an inclusive scan of
// the lengths places every product, so lane l computes product l of the canonical order (X's entries in
// order, each Y row in order). A bitonic sort of the keys (column << 6 | l) across the wavefront brings each
// column's products together in that order, and the first lane of each run sums the run left to right,
// starting from its first product: the running sums of the canonical order, bit for bit. The distinct
// columns, sorted, go to the row's table region with order[base + q] = q and cnt[i] = their number. All
// lanes of a wavefront stay active through the shuffles; the early returns are uniform per wavefront.
constexpr int WAVE = 64;
constexpr int WROWS = 4;  // wavefronts (rows) per block

__device__ __forceinline__ bool wave_product_row(int32_t i, const int32_t *__restrict__ xrp,
                                                 const int32_t *__restrict__ xci, const int32_t *__restrict__ yrp) {
  const int32_t a = xrp[i], lx = xrp[i + 1] - a;
  if (lx > WAVE) return false;
  int64_t bound = 0;
  for (int32_t k = a; k < a + lx; ++k) bound += yrp[xci[k] + 1] - yrp[xci[k]];
  return bound <= WAVE;
}

__global__ __launch_bounds__(WAVE * WROWS) void k_spgemm_wave(int32_t nrows, const int32_t *__restrict__ xrp,
                                                            const int32_t *__restrict__ xci,
                                                            const double *__restrict__ xv,
                                                            const int32_t *__restrict__ yrp,
                                                            const int32_t *__restrict__ yci,
                                                            const double *__restrict__ yv,
                                                            const int64_t *__restrict__ toff, int32_t *__restrict__ tkey,
                                                            double *__restrict__ tval, int32_t *__restrict__ order,
                                                            int32_t *__restrict__ cnt) {
  const int lane = (int)(threadIdx.x % WAVE);
  const int32_t i = (int32_t)(blockIdx.x * WROWS + threadIdx.x / WAVE);
  if (i >= nrows) return;
  const int32_t xb = xrp[i], lx = xrp[i + 1] - xb;
  if (lx > WAVE) return;
  int32_t ylen = 0, ystart = 0;
  double x = 0.0;
  if (lane < lx) {
    const int32_t j = xci[xb + lane];
    x = xv[xb + lane];
    ystart = yrp[j];
    ylen = yrp[j + 1] - ystart;
  }
  int32_t incl = ylen;
  for (int d = 1; d < WAVE; d <<= 1) {
    const int32_t t = __shfl_up(incl, d);
    if (lane >= d) incl += t;
  }
  const int32_t bound = __shfl(incl, WAVE - 1);
  if (bound > WAVE) return;  // the per-row table kernel takes this row
  if (bound == 0) {
    if (lane == 0) cnt[i] = 0;
    return;
  }
  // product `lane`: the X entry kk it belongs to, then its place in Y's row
  int32_t kk = 0;
  for (int32_t k = 0; k < lx; ++k) kk += (__shfl(incl, k) <= lane) ? 1 : 0;
  kk = kk < WAVE ? kk : WAVE - 1;
  const int32_t excl_k = __shfl(incl - ylen, kk);
  const int32_t ystart_k = __shfl(ystart, kk);
  const double x_k = __shfl(x, kk);
  unsigned long long key = ~0ull;
  double val = 0.0;
  if (lane < bound) {
    const int32_t q = ystart_k + (lane - excl_k);
    key = ((unsigned long long)(uint32_t)yci[q] << 6) | (unsigned long long)lane;
    val = x_k * yv[q];
  }
  for (int size = 2; size <= WAVE; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const unsigned long long ok = __shfl_xor(key, stride);
      const double ov = __shfl_xor(val, stride);
      const bool up = (lane & size) == 0, lower = (lane & stride) == 0;
      const bool take = lower ? (up ? ok < key : ok > key) : (up ? ok > key : ok < key);
      if (take) {
        key = ok;
        val = ov;
      }
    }
  const unsigned long long prev = __shfl_up(key, 1);
  const bool head = lane < bound && (lane == 0 || (prev >> 6) != (key >> 6));
  double sum = val;
  bool run = head;
  for (int32_t m = 1; m < lx; ++m) {
    const int src = lane + m < WAVE ? lane + m : WAVE - 1;
    const unsigned long long km = __shfl(key, src);
    const double vm = __shfl(val, src);
    if (run && lane + m < bound && (km >> 6) == (key >> 6))
      sum += vm;
    else
      run = false;
  }
  const unsigned long long heads = __ballot(head);
  const int64_t base = toff[i];
  if (head) {
    const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (WAVE - lane));
    const int32_t rank = (int32_t)__popcll(heads & below);
    tkey[base + rank] = (int32_t)(key >> 6);
    tval[base + rank] = sum;
    order[base + rank] = rank;
  }
  if (lane == 0) cnt[i] = (int32_t)__popcll(heads);
}

// Row i of X Y accumulated into its own open-addressing table [toff[i], toff[i+1]) (keys cleared to -1
// beforehand); the slot of each new column is appended to order[toff[i] + c], so the row's entries can be
// read back without scanning the table; cnt[i] = distinct columns, cnt[nrows] = 0.
__global__ __launch_bounds__(TB) void k_spgemm_accumulate(int32_t nrows, const int32_t *__restrict__ xrp,
                                                          const int32_t *__restrict__ xci,
                                                          const double *__restrict__ xv,
                                                          const int32_t *__restrict__ yrp,
                                                          const int32_t *__restrict__ yci,
                                                          const double *__restrict__ yv,
                                                          const int64_t *__restrict__ toff, int32_t *__restrict__ tkey,
                                                          double *__restrict__ tval, int32_t *__restrict__ order,
                                                          int32_t *__restrict__ cnt) {
  const int32_t i = blockIdx.x * TB + threadIdx.x;
  if (i == nrows) cnt[nrows] = 0;
  if (i >= nrows) return;
  if (wave_product_row(i, xrp, xci, yrp)) return;  // k_spgemm_wave's row
  const int64_t base = toff[i];
  const int64_t ts = toff[i + 1] - base;
  if (ts == 0) {
    cnt[i] = 0;
    return;
  }
  int32_t *key = tkey + base;
  double *acc = tval + base;
  int32_t *ord = order + base;
  const uint32_t mask = (uint32_t)(ts - 1);
  int32_t c = 0;
  for (int32_t k = xrp[i]; k < xrp[i + 1]; ++k) {
    const int32_t j = xci[k];
    const double x = xv[k];
    for (int32_t q = yrp[j]; q < yrp[j + 1]; ++q) {
      const int32_t J = yci[q];
      const double prod = x * yv[q];
      uint32_t h = ((uint32_t)J * 2654435761u) & mask;
      while (key[h] != J && key[h] != -1) h = (h + 1) & mask;
      if (key[h] == -1) {
        key[h] = J;
        acc[h] = prod;
        ord[c] = (int32_t)h;
        ++c;
      } else {
        acc[h] += prod;
      }
    }
  }
  cnt[i] = c;
}

// Row i of the product sorted by column. Rows of at most EMIT_CAP entries are sorted in LDS: each thread
// owns one column of the block's arrays (entry q of lane l at q * EMIT_TB + l, so a wavefront's accesses
// fall in distinct banks); it gathers its row's (column, slot) pairs, sorts them by insertion, then writes
// the columns and reads the values in sorted order. Longer rows are copied out in insertion order and
// sorted in place in global memory. Columns within a row are distinct, so both give the same result.
constexpr int EMIT_TB = 64;
constexpr int EMIT_CAP = 64;

__global__ __launch_bounds__(EMIT_TB) void k_spgemm_emit(int32_t nrows, const int64_t *__restrict__ toff,
                                                         const int32_t *__restrict__ tkey,
                                                         const double *__restrict__ tval,
                                                         const int32_t *__restrict__ order,
                                                         const int32_t *__restrict__ crp, int32_t *__restrict__ cci,
                                                         double *__restrict__ cv) {
  __shared__ int32_t skey[EMIT_CAP * EMIT_TB];
  __shared__ int32_t sslot[EMIT_CAP * EMIT_TB];
  const int32_t i = blockIdx.x * EMIT_TB + threadIdx.x;
  if (i >= nrows) return;
  const int64_t base = toff[i];
  const int32_t a = crp[i], b = crp[i + 1];
  const int32_t c = b - a;
  if (c <= EMIT_CAP) {
    int32_t *K = skey + threadIdx.x, *S = sslot + threadIdx.x;
#pragma unroll 4
    for (int32_t q = 0; q < c; ++q) {
      const int32_t slot = order[base + q];
      S[q * EMIT_TB] = slot;
      K[q * EMIT_TB] = tkey[base + slot];
    }
    for (int32_t q = 1; q < c; ++q) {
      const int32_t key = K[q * EMIT_TB], slot = S[q * EMIT_TB];
      int32_t j = q;
      while (j > 0 && K[(j - 1) * EMIT_TB] > key) {
        K[j * EMIT_TB] = K[(j - 1) * EMIT_TB];
        S[j * EMIT_TB] = S[(j - 1) * EMIT_TB];
        --j;
      }
      K[j * EMIT_TB] = key;
      S[j * EMIT_TB] = slot;
    }
#pragma unroll 4
    for (int32_t q = 0; q < c; ++q) {
      cci[a + q] = K[q * EMIT_TB];
      cv[a + q] = tval[base + S[q * EMIT_TB]];
    }
    return;
  }
  int32_t out = a;
  for (int32_t q = 0; q < c; ++q) {
    const int64_t h = base + order[base + q];
    cci[out] = tkey[h];
    cv[out] = tval[h];
    ++out;
  }
  for (int32_t k = a + 1; k < out; ++k) {
    const int32_t col = cci[k];
    const double x = cv[k];
    int32_t q = k - 1;
    while (q >= a && cci[q] > col) {
      cci[q + 1] = cci[q];
      cv[q + 1] = cv[q];
      --q;
    }
    cci[q + 1] = col;
    cv[q + 1] = x;
  }
}

struct Guard {
  int prev = -1;
  explicit Guard(int dev) {
    hip_check(hipGetDevice(&prev), "hipGetDevice");
    if (prev != dev) hip_check(hipSetDevice(dev), "hipSetDevice");
  }
  ~Guard() {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
  }
};

struct Stream {
  hipStream_t s = nullptr;
  Stream() { hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreateWithFlags"); }
  ~Stream() {
    if (s) (void)hipStreamDestroy(s);
  }
};


class Builder {
 public:
  explicit Builder(hipStream_t s) : s_(s) {}

  void check(const char *what) { hip_check(hipGetLastError(), what); }

  // copies through pinned staging; synchronises the stream
  template <class T>
  void to_host(std::vector<T> &h, const DevBuf<T> &d, size_t n) {
    h.resize(n);
    copy_to_host(h.data(), d.get(), n * sizeof(T), s_);
  }
  void sync() { hip_check(hipStreamSynchronize(s_), "hipStreamSynchronize"); }

  // exclusive scan of in[0..count) into out[0..count)
  template <class T>
  void scan(const T *in, T *out, int64_t count) {
    size_t bytes = 0;
    hip_check(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, (int)count, s_), "scan size");
    // a null temp pointer would turn the second call into another size query
    if (bytes > temp_.size() || temp_.get() == nullptr) temp_.alloc(std::max<size_t>(bytes, 1), &setup_mem());
    hip_check(hipcub::DeviceScan::ExclusiveSum(temp_.get(), bytes, in, out, (int)count, s_), "scan");
  }

  template <class T>
  T read_at(const T *p) {
    T h{};
    hip_check(hipMemcpyAsync(&h, p, sizeof(T), hipMemcpyDeviceToHost, s_), "D2H scalar");
    sync();
    return h;
  }

  void upload(DCsr &D, const HostCsr &A) {
    D.nr = A.nr;
    D.nc = A.nc;
    D.nnz = A.nnz();
    D.rp.alloc(A.rp.size(), &setup_mem());
    D.ci.alloc(A.ci.size(), &setup_mem());
    D.v.alloc(A.v.size(), &setup_mem());
    D.rp.upload(A.rp.data(), A.rp.size());
    D.ci.upload(A.ci.data(), A.ci.size());
    D.v.upload(A.v.data(), A.v.size());
  }

  void download(HostCsr &H, const DCsr &D) {
    H.nr = D.nr;
    H.nc = D.nc;
    to_host(H.rp, D.rp, (size_t)D.nr + 1);
    to_host(H.ci, D.ci, (size_t)D.nnz);
    to_host(H.v, D.v, (size_t)D.nnz);
    sync();
  }

  // C = X Y (X.nc == Y.nr), rows of C sorted by column
  void spgemm(const DCsr &X, const DCsr &Y, DCsr &C) {
    const int32_t nr = X.nr;
    DevBuf<int64_t> tsize((size_t)nr + 1, &setup_mem()), toff((size_t)nr + 1, &setup_mem());
    hipLaunchKernelGGL(k_spgemm_size, dim3(grid_for((int64_t)nr + 1)), dim3(TB), 0, s_, nr, X.rp.get(), X.ci.get(),
                       Y.rp.get(), tsize.get());
    check("k_spgemm_size");
    scan(tsize.get(), toff.get(), (int64_t)nr + 1);
    const int64_t total = read_at(toff.get() + nr);
    // every table is at least twice its row's entry count, so total / 2 bounds the product's entries,
    // whose row pointers are 32-bit
    if (total / 2 >= (int64_t)INT32_MAX) throw SetupError{NAMG_E_INVALID, "sparse product exceeds 2^31 entries"};
    DevBuf<int32_t> tkey((size_t)std::max<int64_t>(total, 1), &setup_mem());
    DevBuf<double> tval((size_t)std::max<int64_t>(total, 1), &setup_mem());
    DevBuf<int32_t> order((size_t)std::max<int64_t>(total, 1), &setup_mem());
    DevBuf<int32_t> cnt((size_t)nr + 1, &setup_mem());
    // every key to -1 (all bytes 0xFF) in one coalesced pass
    hip_check(hipMemsetAsync(tkey.get(), 0xFF, (size_t)std::max<int64_t>(total, 1) * 4, s_), "memset");
    if (nr > 0) {
      hipLaunchKernelGGL(k_spgemm_wave, dim3((unsigned)(((int64_t)nr + WROWS - 1) / WROWS)), dim3(WAVE * WROWS), 0, s_,
                         nr, X.rp.get(), X.ci.get(), X.v.get(), Y.rp.get(), Y.ci.get(), Y.v.get(), toff.get(),
                         tkey.get(), tval.get(), order.get(), cnt.get());
      check("k_spgemm_wave");
    }
    hipLaunchKernelGGL(k_spgemm_accumulate, dim3(grid_for((int64_t)nr + 1)), dim3(TB), 0, s_, nr, X.rp.get(),
                       X.ci.get(), X.v.get(), Y.rp.get(), Y.ci.get(), Y.v.get(), toff.get(), tkey.get(), tval.get(),
                       order.get(), cnt.get());
    check("k_spgemm_accumulate");
    C.nr = nr;
    C.nc = Y.nc;
    C.rp.alloc((size_t)nr + 1, &setup_mem());
    scan(cnt.get(), C.rp.get(), (int64_t)nr + 1);
    C.nnz = read_at(C.rp.get() + nr);
    C.ci.alloc((size_t)std::max<int64_t>(C.nnz, 1), &setup_mem());
    C.v.alloc((size_t)std::max<int64_t>(C.nnz, 1), &setup_mem());
    const unsigned emit_grid = (unsigned)std::max<int64_t>(((int64_t)nr + EMIT_TB - 1) / EMIT_TB, 1);
    hipLaunchKernelGGL(k_spgemm_emit, dim3(emit_grid), dim3(EMIT_TB), 0, s_, nr, toff.get(), tkey.get(), tval.get(),
                       order.get(), C.rp.get(), C.ci.get(), C.v.get());
    check("k_spgemm_emit");
    sync();
  }

  // R = P^T with each row's entries in ascending fine index
  void transpose(const DCsr &P, DCsr &R) {
    R.nr = P.nc;
    R.nc = P.nr;
    R.nnz = P.nnz;
    DevBuf<int32_t> cnt((size_t)P.nc + 1, &setup_mem()), cursor((size_t)std::max(P.nc, 1), &setup_mem());
    hip_check(hipMemsetAsync(cnt.get(), 0, ((size_t)P.nc + 1) * 4, s_), "memset");
    hip_check(hipMemsetAsync(cursor.get(), 0, (size_t)std::max(P.nc, 1) * 4, s_), "memset");
    if (P.nnz) {
      hipLaunchKernelGGL(k_col_count, dim3(grid_for(P.nnz)), dim3(TB), 0, s_, P.nnz, P.ci.get(), cnt.get());
      check("k_col_count");
    }
    R.rp.alloc((size_t)P.nc + 1, &setup_mem());
    scan(cnt.get(), R.rp.get(), (int64_t)P.nc + 1);
    R.ci.alloc((size_t)std::max<int64_t>(P.nnz, 1), &setup_mem());
    R.v.alloc((size_t)std::max<int64_t>(P.nnz, 1), &setup_mem());
    hipLaunchKernelGGL(k_transpose_fill, dim3(grid_for(P.nr)), dim3(TB), 0, s_, P.nr, P.rp.get(), P.ci.get(),
                       P.v.get(), R.rp.get(), cursor.get(), R.ci.get(), R.v.get());
    check("k_transpose_fill");
    hipLaunchKernelGGL(k_sort_rows, dim3(grid_for(R.nr)), dim3(TB), 0, s_, R.nr, R.rp.get(), R.ci.get(), R.v.get());
    check("k_sort_rows");
    sync();
  }

  // PMIS + BAMG direct interpolation of A; returns false when the level should not be coarsened (no C
  // point, or every point C). cf: 1 = C, 0 = F.
  bool coarsen(const DCsr &A, double theta, uint64_t seed, std::vector<int8_t> &cf, DCsr &P) {
    const int32_t n = A.nr;
    DevBuf<uint8_t> flag((size_t)std::max<int64_t>(A.nnz, 1), &setup_mem());
    DevBuf<int32_t> stcount((size_t)n + 1, &setup_mem()), st_rp((size_t)n + 1, &setup_mem()), cursor((size_t)n, &setup_mem());
    hip_check(hipMemsetAsync(stcount.get(), 0, ((size_t)n + 1) * 4, s_), "memset");
    hip_check(hipMemsetAsync(cursor.get(), 0, (size_t)n * 4, s_), "memset");
    hipLaunchKernelGGL(k_strength, dim3(grid_for(n)), dim3(TB), 0, s_, n, A.rp.get(), A.ci.get(), A.v.get(), theta,
                       flag.get(), stcount.get());
    check("k_strength");
    scan(stcount.get(), st_rp.get(), (int64_t)n + 1);
    const int32_t nst = read_at(st_rp.get() + n);
    DevBuf<int32_t> st_ci((size_t)std::max(nst, 1), &setup_mem());
    hipLaunchKernelGGL(k_st_fill, dim3(grid_for(n)), dim3(TB), 0, s_, n, A.rp.get(), A.ci.get(), flag.get(),
                       st_rp.get(), cursor.get(), st_ci.get());
    check("k_st_fill");
    DevBuf<double> w((size_t)n, &setup_mem());
    DevBuf<int8_t> state((size_t)n, &setup_mem());
    DevBuf<uint8_t> newc((size_t)n, &setup_mem());
    DevBuf<int32_t> remaining(1, &setup_mem());
    hipLaunchKernelGGL(k_pmis_init, dim3(grid_for(n)), dim3(TB), 0, s_, n, stcount.get(), seed, w.get(), state.get());
    check("k_pmis_init");
    // every round makes the heaviest undecided point C, so n rounds always suffice
    for (int64_t round = 0;; ++round) {
      if (round > n) throw SetupError{NAMG_E_INVALID, "PMIS did not terminate"};
      hip_check(hipMemsetAsync(remaining.get(), 0, 4, s_), "memset");
      hipLaunchKernelGGL(k_pmis_select, dim3(grid_for(n)), dim3(TB), 0, s_, n, A.rp.get(), A.ci.get(), flag.get(),
                         st_rp.get(), st_ci.get(), w.get(), state.get(), newc.get());
      check("k_pmis_select");
      hipLaunchKernelGGL(k_pmis_apply, dim3(grid_for(n)), dim3(TB), 0, s_, n, A.rp.get(), A.ci.get(), flag.get(),
                         newc.get(), state.get(), remaining.get());
      check("k_pmis_apply");
      if (read_at(remaining.get()) == 0) break;
    }
    DevBuf<int32_t> isc((size_t)n + 1, &setup_mem()), cidx((size_t)n + 1, &setup_mem());
    hipLaunchKernelGGL(k_is_c, dim3(grid_for((int64_t)n + 1)), dim3(TB), 0, s_, n, state.get(), isc.get());
    check("k_is_c");
    scan(isc.get(), cidx.get(), (int64_t)n + 1);
    const int32_t nc = read_at(cidx.get() + n);
    std::vector<int8_t> st;
    to_host(st, state, (size_t)n);
    sync();
    cf.resize(n);
    for (int32_t i = 0; i < n; ++i) cf[i] = st[i] == PT_C ? 1 : 0;
    if (nc == 0 || nc == n) return false;
    DevBuf<int32_t> cnt((size_t)n + 1, &setup_mem());
    hipLaunchKernelGGL(k_interp_count, dim3(grid_for((int64_t)n + 1)), dim3(TB), 0, s_, n, A.rp.get(), A.ci.get(),
                       flag.get(), state.get(), cnt.get());
    check("k_interp_count");
    P.nr = n;
    P.nc = nc;
    P.rp.alloc((size_t)n + 1, &setup_mem());
    scan(cnt.get(), P.rp.get(), (int64_t)n + 1);
    P.nnz = read_at(P.rp.get() + n);
    P.ci.alloc((size_t)std::max<int64_t>(P.nnz, 1), &setup_mem());
    P.v.alloc((size_t)std::max<int64_t>(P.nnz, 1), &setup_mem());
    hipLaunchKernelGGL(k_interp_fill, dim3(grid_for(n)), dim3(TB), 0, s_, n, A.rp.get(), A.ci.get(), A.v.get(),
                       flag.get(), state.get(), cidx.get(), P.rp.get(), P.ci.get(), P.v.get());
    check("k_interp_fill");
    sync();
    return true;
  }

 private:
  hipStream_t s_;
  DevBuf<uint8_t> temp_;
};

// At most MAX_DEVICE_SETUPS device phases run at once per process (each holds a few GB of scratch at
// 10^6-10^7 rows, outside any serving budget); the host part that follows is not limited.
constexpr int MAX_DEVICE_SETUPS = 8;

class SetupSlots {
 public:
  void acquire() {
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return busy_ < MAX_DEVICE_SETUPS; });
    ++busy_;
  }
  void release() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      --busy_;
    }
    cv_.notify_one();
  }

 private:
  std::mutex mu_;
  std::condition_variable cv_;
  int busy_ = 0;
};

struct SlotHold {
  SetupSlots &s;
  explicit SlotHold(SetupSlots &slots) : s(slots) { s.acquire(); }
  ~SlotHold() { s.release(); }
};

// The levels of H (whose level 0 holds A_0) built on the device, on a stream of their own.
void device_levels(HostHierarchy &H, const namg_setup_params &p) {
  static SetupSlots slots;
  const bool trace = std::getenv("NAMG_SETUP_TRACE") != nullptr;
  auto now = [] { return std::chrono::steady_clock::now(); };
  auto ms = [](auto a, auto b) { return std::chrono::duration<double, std::milli>(b - a).count(); };
  const auto t_wait = now();
  SlotHold hold(slots);
  const auto t_start = now();
  Guard g(p.device);
  Stream st;
  Builder B(st.s);
  auto keep = std::make_shared<DeviceLevels>();
  DCsr A;
  B.upload(A, H.lv[0].A);
  if (trace) std::fprintf(stderr, "[namg device setup] slot wait %.1f ms, upload %.1f ms\n", ms(t_wait, t_start),
                          ms(t_start, now()));
  while (true) {
    HostLevel &L = H.lv.back();
    const int32_t n = L.A.nr;
    if (n <= p.max_coarse || (int)H.lv.size() >= p.max_levels) break;
    std::vector<int8_t> cf;
    DCsr P;
    const auto t0 = now();
    if (!B.coarsen(A, p.theta, p.seed + (uint64_t)(H.lv.size() - 1), cf, P)) break;
    const auto t1 = now();
    DCsr R, AP, Ac;
    B.transpose(P, R);
    B.spgemm(A, P, AP);
    const auto t2 = now();
    B.spgemm(R, AP, Ac);
    const auto t3 = now();
    L.cf = std::move(cf);
    B.download(L.P, P);
    // the solver packs R from the device level; a host copy only serves the host packing
    L.host_restriction = !H.pack_on_device;
    if (L.host_restriction) B.download(L.R, R);
    HostLevel next;
    B.download(next.A, Ac);
    if (trace)
      std::fprintf(stderr,
                   "[namg device setup]   level %d n %d nnz %lld: strength+pmis+interp %.2f, R and AP %.2f, R(AP) "
                   "%.2f, download %.2f ms (nnz P %lld AP %lld Ac %lld)\n",
                   (int)H.lv.size() - 1, n, (long long)A.nnz, ms(t0, t1), ms(t1, t2), ms(t2, t3), ms(t3, now()),
                   (long long)P.nnz, (long long)AP.nnz, (long long)Ac.nnz);
    // rows are sorted by column: the diagonal by binary search
    for (int32_t i = 0; i < next.A.nr; ++i) {
      const int32_t *b = next.A.ci.data() + next.A.rp[i], *e = next.A.ci.data() + next.A.rp[i + 1];
      const int32_t *q = std::lower_bound(b, e, i);
      if (q == e || *q != i || next.A.v[q - next.A.ci.data()] == 0.0)
        throw SetupError{NAMG_E_ZERO_PIVOT, "zero diagonal in a coarse operator"};
    }
    H.lv.push_back(std::move(next));
    keep->A.push_back(std::move(A));
    keep->P.push_back(std::move(P));
    keep->R.push_back(std::move(R));
    A = std::move(Ac);
  }
  keep->A.push_back(std::move(A));
  // the levels stay on the device for the solve-phase layouts (packed there, see pack.hip)
  H.device_levels = keep;
}

}  // namespace

HostHierarchy build_hierarchy_pmis_device(HostCsr &&A0, const namg_setup_params &p) {
  validate_hierarchy_params(p);
  if (p.device < 0) throw SetupError{NAMG_E_INVALID, "PMIS setup runs on a device (device >= 0)"};
  if (p.agg_levels > 0) throw SetupError{NAMG_E_INVALID, "aggressive coarsening needs coarsen = NAMG_COARSEN_RS"};
  HostHierarchy H;
  H.anorm_inf = inf_norm(A0);
  H.lv.emplace_back();
  H.lv.back().A = std::move(A0);
  H.pack_on_device = device_packing_enabled();
  const auto t0 = std::chrono::steady_clock::now();
  device_levels(H, p);
  const auto t1 = std::chrono::steady_clock::now();
  // the solver packs the polynomial-GS data from the device levels: the host copy is not built
  finish_hierarchy(H, p, !H.pack_on_device);
  H.t_levels = std::chrono::duration<double>(t1 - t0).count();
  H.t_finish = std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
  return H;
}

}  // namespace namg

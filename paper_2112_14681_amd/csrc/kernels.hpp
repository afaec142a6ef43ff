// HIP kernels of the namg solve phase for gfx950 (CDNA4, 64-wide wavefronts).
//
// Every hot kernel is a streaming sparse or vector operation (arithmetic intensity <= 0.25 flop/byte),
// so the HBM roofline bounds them; none is a dense contraction, and MFMA is not used. Sparse operators
// use SELL-64 (one lane per row, contiguous wavefront loads) or CSR with a lane group per row (long
// coarse-level rows). Reductions are deterministic: a fixed xor-butterfly inside the wavefront, a fixed
// order across wavefronts and blocks, no floating-point atomics.
//
// Each kernel is a __device__ body taking its block index within one problem. Two kinds of launch use
// the same bodies: the single-problem kernels (k_*), and the batched kernels (kb_*). A batched kernel
// serves every in-flight solve of the serving scheduler in one launch: a task table lists one problem
// per entry, and a prefix table of block offsets maps each block to its task. Because the per-row
// arithmetic and the reduction partitions are the same, a solve gives bit-identical results either way.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"

namespace namg {

constexpr int BLK = 256;
constexpr int WAVES = BLK / 64;
constexpr int MAX_BATCH = 256;  // tasks per batched launch

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + BLK - 1) / BLK); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block sum of one double; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *lds) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < WAVES; ++q) t += lds[q];
  __syncthreads();
  return t;
}

// acc + v x with one rounding. The row kernels add every product this way, so that the rounding of a row sum
// does not depend on whether the compiler keeps a product and its sum in one basic block (it fuses them only
// then): every layout gives the same bits for the same row.
__device__ __forceinline__ double mul_add(double v, double x, double acc) { return __builtin_fma(v, x, acc); }
__device__ __forceinline__ float mul_add(float v, float x, float acc) { return __builtin_fmaf(v, x, acc); }

// This thread's share of sum(p[0..n)): p[tid] + p[tid + BLK] + ..., added in that order. Loads go in
// groups of eight so that a long sum waits on one memory latency per group, not per element.
__device__ __forceinline__ double strided_sum(const double *__restrict__ p, int32_t n) {
  double t = 0.0;
  int32_t k = threadIdx.x;
  for (; k + 7 * BLK < n; k += 8 * BLK) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[k + u * BLK];
#pragma unroll
    for (int u = 0; u < 8; ++u) t += v[u];
  }
  for (; k < n; k += BLK) t += p[k];
  return t;
}

// Row `row` of a sparse matrix times x, reduced over the G lanes of the row's group (every lane of the
// group returns the full sum). G == 1: SELL-64, one lane per row. G > 1: CSR, lane `sub` takes entries
// sub, sub + G, ...; groups are aligned inside the wavefront, so the butterfly never leaves the group.
// Entries go in chunks of U (4; 8 for SELL matrices whose rows are long, see DMat::unroll): the chunk's
// index and value loads are all issued, then all its gathers, then the multiply-adds in entry order. A short row thus waits on two dependent memory latencies per
// chunk rather than two per entry. Slots past the row's end reload the chunk's first entry (in bounds)
// and are not added, so the sum is the plain in-order one. NARROW: columns are 16-bit offsets from the
// row's scaled diagonal (the matrix-wide choice is a uniform branch in row_dot).
template <int G, bool NARROW, int U, class Acc, class TM, class TX>
__device__ __forceinline__ Acc row_dot_impl(const MatView<TM> &A, const TX *__restrict__ x, int32_t row, int sub) {
  constexpr int32_t STEP = G == 1 ? SELL_C : G;
  int32_t k, end;
  if constexpr (G == 1) {
    const int32_t s = row >> 6;
    k = A.ptr[s] + (row & 63);
    end = A.ptr[s + 1];
  } else {
    k = A.ptr[row] + sub;
    end = A.ptr[row + 1];
  }
  const int32_t base = NARROW ? diag_base(row, A.mul) : 0;
  Acc acc = Acc(0);
  for (; k < end; k += U * STEP) {
    int32_t c[U];
    TM v[U];
    TX xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t kk = k + u * STEP < end ? k + u * STEP : k;
      if constexpr (NARROW)
        c[u] = base + (int32_t)A.col16[kk];
      else
        c[u] = A.col[kk];
      v[u] = A.val[kk];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k + u * STEP < end) acc = mul_add((Acc)v[u], (Acc)xv[u], acc);
  }
  if constexpr (G > 1) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  }
  return acc;
}

// K slots j .. j + K - 1 of one slice-diagonal row (all of them exist): the K offsets (wave-uniform, one
// merged scalar load), then K value loads and K gathers, none waiting on another, then the K products in
// slot order. A slot's column is the row's scaled diagonal `base` (the row itself in a square matrix) plus the
// slot's offset. A padding slot (value 0) adds 0 times an in-range element of x: the sum is the row's
// CSR-order sum whenever x is finite (a -0 sum may come out +0).
template <int K, class Acc, class TM, class TX>
__device__ __forceinline__ void dia_slots(const TM *__restrict__ vp, const int32_t *__restrict__ off,
                                          const TX *__restrict__ x, int32_t base, int32_t cmax, int32_t j, Acc &acc) {
  int32_t o[K];
  TM v[K];
  TX xv[K];
#pragma unroll
  for (int u = 0; u < K; ++u) o[u] = off[j + u];
#pragma unroll
  for (int u = 0; u < K; ++u) {
    v[u] = vp[(int64_t)(j + u) * SELL_C];
    xv[u] = x[min(max(base + o[u], 0), cmax)];
  }
  // every product is added, padding slots included (value 0 times an element of x, which is finite in any
  // solve that has not already failed its non-finite check): with no condition, no gather can be sunk
  // behind a wait
#pragma unroll
  for (int u = 0; u < K; ++u) acc = mul_add((Acc)v[u], (Acc)xv[u], acc);
}

// Slots j .. w - 1 of one row: chunks of eight, then one chunk of exactly the rest (a wave-uniform switch), so
// no slot past the slice's end is loaded and a row of w slots waits on ceil(w / 8) rounds of loads.
template <class Acc, class TM, class TX>
__device__ __forceinline__ void dia_row_from(const TM *__restrict__ vp, const int32_t *__restrict__ off,
                                             const TX *__restrict__ x, int32_t base, int32_t cmax, int32_t j, int32_t w,
                                             Acc &acc) {
  for (; j + 8 <= w; j += 8) dia_slots<8>(vp, off, x, base, cmax, j, acc);
  switch (w - j) {
    case 7: dia_slots<7>(vp, off, x, base, cmax, j, acc); break;
    case 6: dia_slots<6>(vp, off, x, base, cmax, j, acc); break;
    case 5: dia_slots<5>(vp, off, x, base, cmax, j, acc); break;
    case 4: dia_slots<4>(vp, off, x, base, cmax, j, acc); break;
    case 3: dia_slots<3>(vp, off, x, base, cmax, j, acc); break;
    case 2: dia_slots<2>(vp, off, x, base, cmax, j, acc); break;
    case 1: dia_slots<1>(vp, off, x, base, cmax, j, acc); break;
    default: break;
  }
}

// Row `row` of a slice-diagonal matrix (device.hpp) times x, one lane per row and a wavefront per slice: the
// slice's pointers and slot offsets are wave-uniform and come through the scalar unit.
template <class Acc, class TM, class TX>
__device__ __forceinline__ Acc dia_dot(const MatView<TM> &A, const TX *__restrict__ x, int32_t row) {
  const int32_t s = __builtin_amdgcn_readfirstlane(row >> 6), lane = row & 63;
  const int32_t p0 = A.ptr[s], p1 = A.ptr[s + 1];
  Acc acc = Acc(0);
  dia_row_from(A.val + p0 + lane, A.dia + 1 + (p0 >> 6), x, diag_base(row, A.mul), A.dia[0], 0, (p1 - p0) >> 6,
               acc);
  return acc;
}

template <int G, class Acc, int U = 4, class TM, class TX>
__device__ __forceinline__ Acc row_dot(const MatView<TM> &A, const TX *__restrict__ x, int32_t row, int sub) {
  if constexpr (G == 1) {
    if (A.dia) return dia_dot<Acc>(A, x, row);
  }
  if (A.col16) return row_dot_impl<G, true, U, Acc>(A, x, row, sub);
  return row_dot_impl<G, false, U, Acc>(A, x, row, sub);
}

// The row one thread of a row kernel computes: SELL-64 (G == 1), one row per lane; CSR lane groups (G > 1),
// lane `sub` of the group of one row. (Two rows per lane, the same lane of two adjacent slices, measured
// slower once the slice-diagonal form and SELL-64 for the 175 K-row level were in place: 4.62-4.68 against
// 4.55-4.56 ms per FP32 C2 solve, 4.47 with SELL-64 from 2^17 rows.) R is kept as the bodies' row count.
template <int G, class TM>
struct ThreadRows {
  static constexpr int R = 1;
  int32_t row[R];
  bool ok[R];
  int sub;
  __device__ __forceinline__ ThreadRows(uint32_t lb, int32_t nrows) {
    const int64_t g = (int64_t)lb * BLK + threadIdx.x;
    row[0] = (int32_t)(g / G);
    sub = (int)(g % G);
    ok[0] = row[0] < nrows;
  }
};

// Blocks of a row kernel over nrows rows with `group` lanes per row.
inline unsigned row_blocks(int64_t nrows, int group) { return blocks_for(nrows * group); }

// The row sums of this thread's rows (every lane of a CSR group gets its row's full sum).
template <int G, class Acc, int U = 4, class TM, class TX>
__device__ __forceinline__ void row_dots(const MatView<TM> &A, const TX *__restrict__ x, const ThreadRows<G, TM> &t,
                                         Acc (&out)[ThreadRows<G, TM>::R]) {
  out[0] = row_dot<G, Acc, U>(A, x, t.row[0], t.sub);
}

// ---------------------------------------------------------------------------------------- row bodies

// y = A x  (restriction R r, the GMRES product w = A z with z promoted on load, the coarse inverse),
// optionally f = d .* y as well: the restriction also produces the first term f = D^{-1} b of the
// coarse level's polynomial Gauss-Seidel sweep (same product as the residual pass with x = 0).
template <int G, class Acc, int U = 4, class TM, class TX, class TY>
__device__ __forceinline__ void spmv_body(uint32_t lb, const MatView<TM> &A, const TX *__restrict__ x,
                                          TY *__restrict__ y, const TY *__restrict__ d, TY *__restrict__ f) {
  constexpr int R = ThreadRows<G, TM>::R;
  const ThreadRows<G, TM> t(lb, A.nrows);
  if (!t.ok[0]) return;
  TY dv[R];
#pragma unroll
  for (int q = 0; q < R; ++q) dv[q] = (f && t.ok[q]) ? d[t.row[q]] : TY(0);
  Acc v[R];
  row_dots<G, Acc, U>(A, x, t, v);
  if (t.sub != 0) return;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    if (!t.ok[q]) continue;
    const TY yv = (TY)v[q];
    y[t.row[q]] = yv;
    if (f) f[t.row[q]] = dv[q] * yv;
  }
}

// r = b - A x (x == nullptr means x = 0), optionally f = d .* r. One pass: SpMV, subtract, scale.
template <int G, class T, int U = 4>
__device__ __forceinline__ void residual_body(uint32_t lb, const MatView<T> &A, const T *__restrict__ b,
                                              const T *__restrict__ x, const T *__restrict__ d, T *__restrict__ r,
                                              T *__restrict__ f) {
  constexpr int R = ThreadRows<G, T>::R;
  const ThreadRows<G, T> t(lb, A.nrows);
  if (!t.ok[0]) return;
  T bv[R], dv[R], acc[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    bv[q] = t.ok[q] ? b[t.row[q]] : T(0);
    dv[q] = (f && t.ok[q]) ? d[t.row[q]] : T(0);
    acc[q] = T(0);
  }
  if (x) row_dots<G, T, U>(A, x, t, acc);
  if (t.sub != 0) return;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    if (!t.ok[q]) continue;
    const T rr = bv[q] - acc[q];
    if (r) r[t.row[q]] = rr;
    if (f) f[t.row[q]] = dv[q] * rr;
  }
}

// One Neumann / Jacobi inner term on a pre-scaled strict triangle S:
//   out = [acc +] [scale .*] (f - S in)
// Polynomial GS: S = D^{-1}L (or D^{-1}U), f = D^{-1} r; ILU: S = L_s with f = r, or S = U_s with
// f = D_U^{-1} y. `acc` may alias `out` (x += ...); `in` never aliases `out`.
template <int G, class T, int U = 4>
__device__ __forceinline__ void neumann_body(uint32_t lb, const MatView<T> &S, const T *__restrict__ f,
                                             const T *__restrict__ in, const T *__restrict__ scale, const T *acc,
                                             T *out) {
  constexpr int R = ThreadRows<G, T>::R;
  const ThreadRows<G, T> t(lb, S.nrows);
  if (!t.ok[0]) return;
  T fv[R], sc[R], av[R], sv[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int32_t row = t.ok[q] ? t.row[q] : t.row[0];
    fv[q] = f[row];
    sc[q] = scale ? scale[row] : T(1);
    av[q] = acc ? acc[row] : T(0);
  }
  row_dots<G, T, U>(S, in, t, sv);
  if (t.sub != 0) return;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    if (!t.ok[q]) continue;
    T v = fv[q] - sv[q];
    if (scale) v *= sc[q];
    if (acc) v += av[q];
    out[t.row[q]] = v;
  }
}

// x += P e for P in the unit-row SELL layout (device.hpp, UnitRows), on the rows of ThreadRows<1, T> (one
// row per lane). A C point's row adds e[c], c = the C points before it,
// as a virtual first entry of value 1 (0 + 1 * e[c] is e[c] exactly); an F row of rank l among its slice's m
// F rows sums the slots ptr[s] + l, ptr[s] + l + m, ... (padding: value 0 at a valid column) in order. Both
// go through one loop: entries in chunks of U, every index and value load of a chunk issued before its
// gathers, as in row_dot; a slot past its row's end loads an in-bounds entry, gathers a valid column and is
// not added.
template <bool NARROW, int U, class T>
__device__ __forceinline__ void prolong_unit_rows(const MatView<T> &P, const T *__restrict__ e, T *x,
                                                  const ThreadRows<1, T> &t) {
  constexpr int R = ThreadRows<1, T>::R;
  int32_t k[R], lim[R], end[R], m[R], cu[R], base[R];
  bool virt[R];
  T xv[R], acc[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int32_t row = t.ok[q] ? t.row[q] : t.row[0];
    // a wavefront's rows q are one slice (ThreadRows): the slice's mask, counts and pointers are loaded
    // once per wavefront through the scalar unit
    const int32_t s = __builtin_amdgcn_readfirstlane(row >> 6), lane = row & 63;
    const uint64_t um = P.umask[s];
    const int32_t before = P.smeta[2 * s], mm = P.smeta[2 * s + 1];
    const int32_t p0 = P.ptr[s], p1 = P.ptr[s + 1];
    xv[q] = x[row];
    const int32_t below = __popcll(um & ((uint64_t(1) << lane) - 1));
    const bool unit = (um >> lane) & 1;
    virt[q] = t.ok[q] && unit;
    // the load cursor: an F row's own slots; a C point's lane follows the F row of rank `below` (its
    // neighbour), so that every lane of a wavefront loads from the same cache lines
    k[q] = p0 + (unit ? (mm > 0 ? min(below, mm - 1) : 0) : lane - below);
    lim[q] = p1;
    end[q] = (unit || !t.ok[q]) ? p0 : p1;  // the slots whose entries this row adds
    m[q] = mm > 0 ? mm : 1;
    cu[q] = before + below;
    base[q] = NARROW ? diag_base(row, P.mul) : 0;
    acc[q] = T(0);
  }
  while (true) {
    bool more = false;
#pragma unroll
    for (int q = 0; q < R; ++q) more = more || virt[q] || k[q] < end[q];
    if (!more) break;
    bool ok[R][U];
    int32_t c[R][U];
    T v[R][U], ev[R][U];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      // an in-bounds slot for loads past the slice's end (the buffers hold at least one)
      const int32_t kb = k[q] < lim[q] ? k[q] : (lim[q] > 0 ? lim[q] - 1 : 0);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t kk = k[q] + u * m[q] < lim[q] ? k[q] + u * m[q] : kb;
        ok[q][u] = k[q] + u * m[q] < end[q];
        // every loaded index is used, so the loads are issued unconditionally, as one batch; a slot that is
        // not this row's decodes another row's offset, so columns are clamped into [0, ncols)
        const int32_t col = NARROW ? base[q] + (int32_t)P.col16[kk] : P.col[kk];
        c[q][u] = min(max(col, 0), P.ncols - 1);
        v[q][u] = P.val[kk];
      }
      if (virt[q]) {  // the unit row's virtual entry takes slot 0 (its row has no stored slots)
        ok[q][0] = true;
        c[q][0] = cu[q];
        v[q][0] = T(1);
      }
    }
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
      for (int u = 0; u < U; ++u) ev[q][u] = e[c[q][u]];
#pragma unroll
    for (int q = 0; q < R; ++q) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ok[q][u]) acc[q] = mul_add(v[q][u], ev[q][u], acc[q]);
      virt[q] = false;
      k[q] += U * m[q];
    }
  }
#pragma unroll
  for (int q = 0; q < R; ++q)
    if (t.ok[q]) x[t.row[q]] = xv[q] + acc[q];
}

// Rows of a block of the pair form of the unit-row prolongation kernel: a wavefront per pair of 64-row slices.
constexpr int UNIT_PAIR_ROWS = 2 * SELL_C;
constexpr int UNIT_BLOCK_ROWS = WAVES * UNIT_PAIR_ROWS;


// x += P e for P in the unit-row SELL layout (device.hpp, UnitRows). Wavefront w of block lb takes slices
// s = 2 (4 lb + w) and s + 1. Its lanes first take the pair's F rows (those of slice s, then of slice s + 1,
// each in rank order), 64 at a time, then its C points' rows the same way, so every lane of a pass has a row
// of the kind the pass computes (a red-black splitting puts about 32 of each kind in a slice: one lane per
// row left half the lanes of the F loop idle). The position of a lane's row comes from a table in LDS that
// the wavefront builds from the two slices' masks.
//   F row of rank l in slice q: entries k at ptr[s_q] + k m_q + l, in chunks of U (every index, value and
//   gather of a chunk issued before its products); a slot past the row's end loads a stored slot of the
//   pair and adds 0 times a gathered element (its column clamped into [0, ncols)), which leaves the sum as
//   it is: acc starts at +0 and so is never -0, and e is finite.
//   C point of rank l in slice q: its coarse index is the C points before slice q plus l, and its row adds
//   0 + 1 e[c] (that is e[c], +0 for -0), as the virtual first entry of the layout's definition.
// Each row's sum is its entries' in-order sum, so the result is the plain layout's, bit for bit.
template <bool NARROW, int U, class T>
__device__ __forceinline__ void prolong_unit_pairs(uint32_t lb, const MatView<T> &P, const T *__restrict__ e, T *x) {
  __shared__ int16_t tab[WAVES][2][UNIT_PAIR_ROWS];  // per wavefront: [F or C][rank in the pair] = row in the pair
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int32_t nslices = (P.nrows + SELL_C - 1) / SELL_C;
  const int32_t s0 = ((int32_t)lb * WAVES + wave) * 2;
  uint64_t um[2] = {0, 0};
  int32_t before[2] = {0, 0}, m[2] = {0, 0}, p[2] = {0, 0}, w[2] = {0, 0}, nc[2] = {0, 0}, nr[2] = {0, 0};
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int32_t s = s0 + q;
    if (s < nslices) {  // uniform
      um[q] = P.umask[s];
      before[q] = P.smeta[2 * s];
      m[q] = P.smeta[2 * s + 1];
      p[q] = P.ptr[s];
      w[q] = m[q] > 0 ? (P.ptr[s + 1] - p[q]) / m[q] : 0;
      nr[q] = min(SELL_C, P.nrows - s * SELL_C);
      nc[q] = __popcll(um[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    if (lane < nr[q]) {
      const uint64_t below = (uint64_t(1) << lane) - 1;
      if ((um[q] >> lane) & 1)
        tab[wave][1][q * nc[0] + __popcll(um[q] & below)] = (int16_t)(q * SELL_C + lane);
      else
        tab[wave][0][q * m[0] + __popcll(~um[q] & below)] = (int16_t)(q * SELL_C + lane);
    }
  }
  __syncthreads();
  const int32_t row0 = s0 * SELL_C;
  // C points' rows (at most two passes of 64: a pair has at most 128): their loads go out first, ahead of the
  // F rows' chains (a C row's x and e are no F row's, so the order of their loads and the F rows' stores does
  // not matter); their stores come last
  const int32_t ncp = nc[0] + nc[1];
  int32_t crow[2];
  T cev[2], cxv[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int32_t c = r * SELL_C + lane;
    crow[r] = -1;
    if (c < ncp) {
      const int32_t col = c >= nc[0] ? before[1] + (c - nc[0]) : before[0] + c;
      crow[r] = row0 + (int32_t)tab[wave][1][c];
      cev[r] = e[col];
      cxv[r] = x[crow[r]];
    }
  }
  // F rows
  const int32_t nf = m[0] + m[1];
  const int32_t wmax = max(m[0] > 0 ? w[0] : 0, m[1] > 0 ? w[1] : 0);
  const int32_t safe = (m[0] > 0 && w[0] > 0) ? p[0] : p[1];  // a stored slot of the pair (used when wmax > 0)
  for (int32_t f0 = 0; f0 < nf; f0 += SELL_C) {
    const int32_t f = f0 + lane;
    const bool act = f < nf;
    const bool second = f >= m[0];
    const int32_t rank = second ? f - m[0] : f;
    const int32_t mq = second ? m[1] : m[0], pq = second ? p[1] : p[0];
    const int32_t wl = act ? (second ? w[1] : w[0]) : 0;
    const int32_t row = row0 + (act ? (int32_t)tab[wave][0][f] : 0);
    const T xv = act ? x[row] : T(0);
    const int32_t base = NARROW ? diag_base(row, P.mul) : 0;
    T acc = T(0);
    for (int32_t k = 0; k < wmax; k += U) {
      int32_t c[U];
      T v[U], ev[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = k + u < wl;
        const int32_t kk = ok ? pq + (k + u) * mq + rank : safe;
        const int32_t col = NARROW ? base + (int32_t)P.col16[kk] : P.col[kk];
        const T vv = P.val[kk];  // loaded unconditionally (kk is a stored slot), then selected
        c[u] = min(max(col, 0), P.ncols - 1);
        v[u] = ok ? vv : T(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) ev[u] = e[c[u]];
#pragma unroll
      for (int u = 0; u < U; ++u) acc = mul_add(v[u], ev[u], acc);
    }
    if (act) x[row] = xv + acc;
  }
#pragma unroll
  for (int r = 0; r < 2; ++r)
    if (crow[r] >= 0) x[crow[r]] = cxv[r] + mul_add(T(1), cev[r], T(0));
}

// x += P e  (prolongation and correction in one pass)
template <int G, class T>
__device__ __forceinline__ void prolong_body(uint32_t lb, const MatView<T> &P, const T *__restrict__ e, T *x) {
  if constexpr (G == 1) {
    if (P.umask) {
      // chunks of eight when the F rows average more than four entries (one dependent round instead of two
      // for the six-entry rows of a stencil's P); UNIT_PAIRS: the kernel of a wavefront per pair of slices
      // (DMat::unit_pairs), whose every thread reaches the kernel's barrier
      const int chunk = P.unroll & ~UNIT_PAIRS;
      if (P.unroll & UNIT_PAIRS) {
        if (chunk == 8) {
          if (P.col16)
            prolong_unit_pairs<true, 8>(lb, P, e, x);
          else
            prolong_unit_pairs<false, 8>(lb, P, e, x);
        } else {
          if (P.col16)
            prolong_unit_pairs<true, 4>(lb, P, e, x);
          else
            prolong_unit_pairs<false, 4>(lb, P, e, x);
        }
        return;
      }
      const ThreadRows<1, T> t(lb, P.nrows);
      if (!t.ok[0]) return;
      if (chunk == 8) {
        if (P.col16)
          prolong_unit_rows<true, 8>(P, e, x, t);
        else
          prolong_unit_rows<false, 8>(P, e, x, t);
      } else {
        if (P.col16)
          prolong_unit_rows<true, 4>(P, e, x, t);
        else
          prolong_unit_rows<false, 4>(P, e, x, t);
      }
      return;
    }
  }
  constexpr int R = ThreadRows<G, T>::R;
  const ThreadRows<G, T> t(lb, P.nrows);
  if (!t.ok[0]) return;
  T xv[R], v[R];
#pragma unroll
  for (int q = 0; q < R; ++q) xv[q] = x[t.ok[q] ? t.row[q] : t.row[0]];
  row_dots<G, T>(P, e, t, v);
  if (t.sub != 0) return;
#pragma unroll
  for (int q = 0; q < R; ++q)
    if (t.ok[q]) x[t.row[q]] = xv[q] + v[q];
}

// out = [acc +] [scale .*] f
template <class T>
__device__ __forceinline__ void axpy_body(uint32_t lb, const T *__restrict__ f, const T *__restrict__ scale,
                                          const T *acc, T *out, int32_t n) {
  const int32_t row = (int32_t)lb * BLK + threadIdx.x;
  if (row >= n) return;
  T v = f[row];
  if (scale) v *= scale[row];
  if (acc) v += acc[row];
  out[row] = v;
}

// --------------------------------------------------------------------------- single-problem kernels
//
// The single-problem kernels take a sparse operator as plain fields: row/slice pointers, one index array
// (int32 columns or 16-bit offsets, `narrow` says which), values, row count; then the operands the body
// loads first; then the rest. The build preloads the first 56 bytes of kernel arguments into scalar
// registers (kernarg preloading on gfx950), so the first loads of a launch do not wait for a
// kernel-argument load. The bodies get the MatView rebuilt in registers.
#define NAMG_MAT_HEAD(T) \
  const int32_t *__restrict__ m_ptr, const void *__restrict__ m_idx, const T *__restrict__ m_val, int32_t m_nrows, \
      int32_t m_form

// form: 0 = 32-bit columns, 1 = 16-bit offsets, 2 = slice-diagonal (idx = the slot offsets)
template <class T>
__device__ __forceinline__ MatView<T> make_view(const int32_t *ptr, const void *idx, const T *val, int32_t nrows,
                                                int32_t form, int64_t mul) {
  MatView<T> v;
  v.ptr = ptr;
  v.col = form == 0 ? static_cast<const int32_t *>(idx) : nullptr;
  v.col16 = form == 1 ? static_cast<const int16_t *>(idx) : nullptr;
  v.dia = form == 2 ? static_cast<const int32_t *>(idx) : nullptr;
  v.val = val;
  v.mul = mul;
  v.nrows = nrows;
  return v;
}
#define NAMG_MAT_VIEW(T) make_view<T>(m_ptr, m_idx, m_val, m_nrows, m_form, m_mul)

template <int G, class Acc, class TM, class TX, class TY, int U = 4>
__global__ __launch_bounds__(BLK) void k_spmv(NAMG_MAT_HEAD(TM), const TX *__restrict__ x, const TY *__restrict__ d,
                                              TY *__restrict__ y, TY *__restrict__ f, int64_t m_mul) {
  spmv_body<G, Acc, U>(blockIdx.x, NAMG_MAT_VIEW(TM), x, y, d, f);
}

template <int G, class T, int U = 4>
__global__ __launch_bounds__(BLK) void k_residual(NAMG_MAT_HEAD(T), const T *__restrict__ b, const T *__restrict__ d,
                                                  const T *__restrict__ x, T *__restrict__ r, T *__restrict__ f,
                                                  int64_t m_mul) {
  residual_body<G, T, U>(blockIdx.x, NAMG_MAT_VIEW(T), b, x, d, r, f);
}

template <int G, class T, int U = 4>
__global__ __launch_bounds__(BLK) void k_neumann(NAMG_MAT_HEAD(T), const T *__restrict__ f, const T *__restrict__ scale,
                                                 const T *acc, const T *__restrict__ in, T *out, int64_t m_mul) {
  neumann_body<G, T, U>(blockIdx.x, NAMG_MAT_VIEW(T), f, in, scale, acc, out);
}

// ------------------------------------------------- one Neumann term, FP32 slice-diagonal, two rows per lane

// In a slice-diagonal matrix rows 2h and 2h + 1 of a slice keep their values side by side in every slot
// (ptr[s] + 64 k + 2h and + 1). K slots j .. j + K - 1 of that pair: the offsets o (one merged scalar load
// per slice; the lane takes its half-wavefront's slice), one 8-byte value load, and the two gathers
// x[r + o] and x[r + 1 + o] as one 8-byte load at the pair's first column clamped into [0, cmax - 1], from
// which the select below gives in[clamp(r + o)] and in[clamp(r + 1 + o)] exactly (clamp to [0, cmax]).
template <int K>
__device__ __forceinline__ void dia_pair_slots(const float *__restrict__ vp, const int32_t *__restrict__ offA,
                                               const int32_t *__restrict__ offB, bool second,
                                               const float *__restrict__ x, int32_t r, int32_t cmax, int32_t j,
                                               float &acc0, float &acc1) {
  typedef float pair_u __attribute__((ext_vector_type(2), aligned(4)));
  int32_t oa[K], ob[K];
  float2 v[K];
  pair_u g[K];
  int32_t c[K];
#pragma unroll
  for (int u = 0; u < K; ++u) {
    oa[u] = offA[j + u];
    ob[u] = offB[j + u];
  }
#pragma unroll
  for (int u = 0; u < K; ++u) {
    c[u] = r + (second ? ob[u] : oa[u]);
    v[u] = *reinterpret_cast<const float2 *>(vp + (int64_t)(j + u) * SELL_C);
    g[u] = *reinterpret_cast<const pair_u *>(x + min(max(c[u], 0), cmax - 1));
  }
#pragma unroll
  for (int u = 0; u < K; ++u) {
    acc0 = mul_add(v[u].x, c[u] >= cmax ? g[u].y : g[u].x, acc0);
    acc1 = mul_add(v[u].y, c[u] < 0 ? g[u].x : g[u].y, acc1);
  }
}

// One Neumann term out = [acc +] [scale .*] (f - S in), as k_neumann, on a square slice-diagonal FP32
// triangle with at least two columns: a wavefront takes slices 2w and 2w + 1 (lanes 0-31 and 32-63) and lane
// h of a half takes rows 2h and 2h + 1 of its slice, so values and the row vectors move as 8-byte pairs: with
// 4-byte values one row per lane moves half the bytes per load of the FP64 kernel, and this term is bound by
// its loads in flight, not by HBM. Each row still sums its own slice's slots in slot order, padding included,
// with the same operations as the one-row kernel, so every output has the same bits. Wavefronts whose two
// slices differ in width, or that reach the matrix's last (possibly partial) slice, take the rows one at a
// time with the lane's own slice data.
__global__ __launch_bounds__(BLK) void k_neumann_pairs(NAMG_MAT_HEAD(float), const float *__restrict__ f,
                                                       const float *__restrict__ scale, const float *acc,
                                                       const float *__restrict__ in, float *out) {
  const int32_t nrows = m_nrows;
  const int32_t *__restrict__ dia = static_cast<const int32_t *>(m_idx);
  const int32_t nslices = (nrows + SELL_C - 1) / SELL_C;
  // wave-uniform (readfirstlane), so the slices' pointers and offsets come through the scalar unit
  const int32_t sA = __builtin_amdgcn_readfirstlane(2 * (int32_t)(blockIdx.x * WAVES + (threadIdx.x >> 6)));
  if (sA >= nslices) return;
  const int32_t lane = threadIdx.x & 63;
  const bool second = lane >= 32;
  const int32_t r = (sA + (second ? 1 : 0)) * SELL_C + 2 * (lane & 31);
  const int32_t cmax = dia[0];
  const bool full = (sA + 2) * SELL_C <= nrows;  // both slices exist and hold 64 rows each
  if (full) {
    const int32_t pA = m_ptr[sA], pB = m_ptr[sA + 1], pE = m_ptr[sA + 2];
    const int32_t w = (pB - pA) >> 6;
    if (w == (pE - pB) >> 6) {
      const int32_t p = second ? pB : pA;
      const float2 fv = *reinterpret_cast<const float2 *>(f + r);
      const float2 sc = scale ? *reinterpret_cast<const float2 *>(scale + r) : make_float2(1.f, 1.f);
      const float2 av = acc ? *reinterpret_cast<const float2 *>(acc + r) : make_float2(0.f, 0.f);
      const float *vp = m_val + p + 2 * (lane & 31);
      const int32_t *offA = dia + 1 + (pA >> 6), *offB = dia + 1 + (pB >> 6);
      float s0 = 0.f, s1 = 0.f;
      int32_t j = 0;
      for (; j + 8 <= w; j += 8) dia_pair_slots<8>(vp, offA, offB, second, in, r, cmax, j, s0, s1);
      switch (w - j) {
        case 7: dia_pair_slots<7>(vp, offA, offB, second, in, r, cmax, j, s0, s1); break;
        case 6: dia_pair_slots<6>(vp, offA, offB, second, in, r, cmax, j, s0, s1); break;
        case 5: dia_pair_slots<5>(vp, offA, offB, second, in, r, cmax, j, s0, s1); break;
        case 4: dia_pair_slots<4>(vp, offA, offB, second, in, r, cmax, j, s0, s1); break;
        case 3: dia_pair_slots<3>(vp, offA, offB, second, in, r, cmax, j, s0, s1); break;
        case 2: dia_pair_slots<2>(vp, offA, offB, second, in, r, cmax, j, s0, s1); break;
        case 1: dia_pair_slots<1>(vp, offA, offB, second, in, r, cmax, j, s0, s1); break;
        default: break;
      }
      float v0 = fv.x - s0, v1 = fv.y - s1;
      if (scale) {
        v0 *= sc.x;
        v1 *= sc.y;
      }
      if (acc) {
        v0 += av.x;
        v1 += av.y;
      }
      *reinterpret_cast<float2 *>(out + r) = make_float2(v0, v1);
      return;
    }
  }
  // the rows one at a time, each with its own slice's pointers and offsets
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int32_t row = r + q;
    if (row >= nrows) continue;
    const int32_t s = row >> 6;
    const int32_t p0 = m_ptr[s], w = (m_ptr[s + 1] - p0) >> 6;
    const float *vp = m_val + p0 + (row & 63);
    const int32_t *off = dia + 1 + (p0 >> 6);
    float sv = 0.f;
    for (int32_t k = 0; k < w; ++k) sv = mul_add(vp[(int64_t)k * SELL_C], in[min(max(row + off[k], 0), cmax)], sv);
    float v = f[row] - sv;
    if (scale) v *= scale[row];
    if (acc) v += acc[row];
    out[row] = v;
  }
}

// Blocks of k_neumann_pairs for nrows rows: two 64-row slices per wavefront.
inline unsigned neumann_pairs_blocks(int32_t nrows) {
  const int64_t nslices = ((int64_t)nrows + SELL_C - 1) / SELL_C;
  return (unsigned)((nslices + 2 * WAVES - 1) / (2 * WAVES));
}

// A prolongation may be packed in the unit-row layout: its per-slice masks and counts (null for the plain
// layout) complete the view, and prolong_body dispatches on them. The other row kernels never receive a
// unit-row matrix (the host refuses to launch them on one).
template <int G, class T>
__global__ __launch_bounds__(BLK) void k_prolong(NAMG_MAT_HEAD(T), T *x, const T *__restrict__ e, int64_t m_mul,
                                                 const uint64_t *__restrict__ m_umask,
                                                 const int32_t *__restrict__ m_smeta, int32_t m_ncols,
                                                 int32_t m_unroll) {
  MatView<T> P = NAMG_MAT_VIEW(T);
  P.umask = m_umask;
  P.smeta = m_smeta;
  P.ncols = m_ncols;
  P.unroll = m_unroll;
  prolong_body<G>(blockIdx.x, P, e, x);
}

template <class T>
__global__ __launch_bounds__(BLK) void k_axpy(const T *__restrict__ f, const T *__restrict__ scale, const T *acc, T *out,
                                              int32_t n) {
  axpy_body(blockIdx.x, f, scale, acc, out, n);
}

// One dependency level of a direct triangular solve g = (I + S)^{-1} f: rows of the level only read g of
// earlier levels. Position q = beg + thread holds row order[q]; rp / ci / val store the rows in schedule
// order, so the row index and the entry range load together, and a row's entries are loaded in chunks
// of four before their gathers. The subtraction order is the row's entry order.
template <class T>
__global__ __launch_bounds__(BLK) void k_tri_level(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                   const T *__restrict__ val, const int32_t *__restrict__ order,
                                                   int32_t beg, int32_t cnt, const T *__restrict__ f, T *g) {
  constexpr int U = 4;
  const int32_t t = blockIdx.x * BLK + threadIdx.x;
  if (t >= cnt) return;
  const int32_t q = beg + t;
  const int32_t i = order[q];
  int32_t k = rp[q];
  const int32_t end = rp[q + 1];
  T acc = f[i];
  for (; k < end; k += U) {
    int32_t c[U];
    T v[U], x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t kk = k + u < end ? k + u : k;
      c[u] = ci[kk];
      v[u] = val[kk];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = g[c[u]];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k + u < end) acc -= v[u] * x[u];
  }
  g[i] = acc;
}

template <class TI, class TO>
__global__ __launch_bounds__(BLK) void k_cast(const TI *__restrict__ in, TO *__restrict__ out, int32_t n) {
  const int32_t row = blockIdx.x * BLK + threadIdx.x;
  if (row < n) out[row] = (TO)in[row];
}

template <class T>
__global__ __launch_bounds__(BLK) void k_fill(T *__restrict__ out, T v, int32_t n) {
  const int32_t row = blockIdx.x * BLK + threadIdx.x;
  if (row < n) out[row] = v;
}

// ------------------------------------------------------------------------------ FP64 Krylov bodies

// r = b - A x in FP64 (true residual), optional low-precision copy of r, per-block partial of |r|^2.
template <class TL>
__device__ __forceinline__ void residual64_body(uint32_t lb, const MatView<double> &A, const double *__restrict__ b,
                                                const double *__restrict__ x, double *__restrict__ r,
                                                TL *__restrict__ rlow, double *__restrict__ partial) {
  __shared__ double lds[WAVES];
  const int32_t row = (int32_t)lb * BLK + threadIdx.x;
  double rr = 0.0;
  if (row < A.nrows) {
    rr = b[row] - row_dot<1, double>(A, x, row, 0);
    r[row] = rr;
    if (rlow) rlow[row] = (TL)rr;
  }
  const double t = block_sum(rr * rr, lds);
  if (threadIdx.x == 0) partial[lb] = t;
}

// partial[lb] = sum over block lb's rows of x^2
__device__ __forceinline__ void sumsq_body(uint32_t lb, const double *__restrict__ x, int32_t n,
                                           double *__restrict__ partial) {
  __shared__ double lds[WAVES];
  const int32_t row = (int32_t)lb * BLK + threadIdx.x;
  const double v = row < n ? x[row] : 0.0;
  const double t = block_sum(v * v, lds);
  if (threadIdx.x == 0) partial[lb] = t;
}

// out[0] = sum of partial[0..n) in a fixed order (one block); out may be host-mapped memory.
__device__ __forceinline__ void reduce_body(const double *__restrict__ partial, int32_t n, double *out) {
  __shared__ double lds[WAVES];
  const double t = block_sum(strided_sum(partial, n), lds);
  if (threadIdx.x == 0) out[0] = t;
}

// Block lb: out[lb] = sum over b < nblk of partial[lb * nblk + b], in a fixed order.
__device__ __forceinline__ void colreduce_body(uint32_t lb, const double *__restrict__ partial, int32_t nblk,
                                               double *__restrict__ out) {
  __shared__ double lds[WAVES];
  const double t = block_sum(strided_sum(partial + (int64_t)lb * nblk, nblk), lds);
  if (threadIdx.x == 0) out[lb] = t;
}

// The single fused reduction of an Arnoldi step (Algorithm 1, the global synchronisation):
// c = V_{i+1}^T v_{i+1} and d = V_{i+1}^T w in one pass over V. Block lb owns the contiguous row range
// [lb * rows_per_blk, (lb + 1) * rows_per_blk) (rows_per_blk even); each thread takes row pairs with
// 16-byte loads, so every wavefront load moves 1 KiB, and PAIRS row pairs per iteration with all their
// loads issued before the multiply-adds (the sums stay in row order). Columns go in chunks of CH (slots past
// ncols repeat the last column and are discarded). Partial sums are written value-major:
// partial[v * nblk + lb], v < ncols for c, ncols + v for d.
template <int CH, int PAIRS = 1>
__device__ __forceinline__ void multidot_body(uint32_t lb, const double *__restrict__ V, int64_t ldv, int32_t ncols,
                                              const double *__restrict__ w, int32_t n, int32_t rows_per_blk,
                                              double *__restrict__ partial, int32_t nblk) {
  __shared__ double lds[2 * CH][WAVES];
  const int32_t r0 = (int32_t)lb * rows_per_blk;
  const int32_t r1 = min(n, r0 + rows_per_blk);
  const double *v = V + (int64_t)(ncols - 1) * ldv;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int32_t j0 = 0; j0 < ncols; j0 += CH) {
    double ac[CH], ad[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) ac[c] = ad[c] = 0.0;
    // every slot loads a valid column (slots past ncols repeat the last one and are discarded below), so
    // there is no branch between the loads and all of them are in flight together
    const double *cols[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) cols[c] = V + (int64_t)min(j0 + c, ncols - 1) * ldv;
    int32_t r = r0 + 2 * (int32_t)threadIdx.x;
    for (; r + 2 * BLK * (PAIRS - 1) + 1 < r1; r += 2 * BLK * PAIRS) {
      double2 vr[PAIRS], wr[PAIRS], vj[PAIRS][CH];
#pragma unroll
      for (int p = 0; p < PAIRS; ++p) {
        const int32_t rr = r + 2 * BLK * p;
        vr[p] = *reinterpret_cast<const double2 *>(v + rr);
        wr[p] = w ? *reinterpret_cast<const double2 *>(w + rr) : make_double2(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < CH; ++c) vj[p][c] = *reinterpret_cast<const double2 *>(cols[c] + rr);
      }
#pragma unroll
      for (int p = 0; p < PAIRS; ++p)
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          ac[c] += vj[p][c].x * vr[p].x;
          ac[c] += vj[p][c].y * vr[p].y;
          ad[c] += vj[p][c].x * wr[p].x;
          ad[c] += vj[p][c].y * wr[p].y;
        }
    }
    for (; r < r1; r += 2 * BLK) {
      if (r + 1 < r1) {
        const double2 vr = *reinterpret_cast<const double2 *>(v + r);
        const double2 wr = w ? *reinterpret_cast<const double2 *>(w + r) : make_double2(0.0, 0.0);
        double2 vj[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) vj[c] = *reinterpret_cast<const double2 *>(cols[c] + r);
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          ac[c] += vj[c].x * vr.x;
          ac[c] += vj[c].y * vr.y;
          ad[c] += vj[c].x * wr.x;
          ad[c] += vj[c].y * wr.y;
        }
      } else {
        const double vr = v[r];
        const double wr = w ? w[r] : 0.0;
        double vj[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) vj[c] = cols[c][r];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          ac[c] += vj[c] * vr;
          ad[c] += vj[c] * wr;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (j0 + c >= ncols) break;  // uniform: the discarded slots are not reduced
      ac[c] = wave_sum(ac[c]);
      ad[c] = wave_sum(ad[c]);
      if (lane == 0) {
        lds[c][wave] = ac[c];
        lds[CH + c][wave] = ad[c];
      }
    }
    __syncthreads();
    if (threadIdx.x < 2 * CH) {
      const int c = threadIdx.x % CH;
      const bool isd = threadIdx.x >= CH;
      const int32_t col = j0 + c;
      if (col < ncols && (!isd || w)) {
        double t = 0.0;
        for (int q = 0; q < WAVES; ++q) t += lds[threadIdx.x][q];
        partial[(int64_t)((isd ? ncols : 0) + col) * nblk + lb] = t;
      }
    }
    __syncthreads();
  }
}

// Partition of the fused reduction over n rows: at most 512 blocks (two per compute unit) of an even
// number of rows (at least 512), so that a thread takes several row pairs and the block-level reduction of
// the 2 (i + 1) sums is paid once per 512 rows or more.
inline int32_t dot_rows_per_block(int64_t n) {
  const int64_t nb = std::min<int64_t>(512, std::max<int64_t>(1, (n + 511) / 512));
  const int64_t rows = (n + nb - 1) / nb;
  return (int32_t)std::max<int64_t>(2, (rows + 1) / 2 * 2);
}
inline int32_t dot_blocks(int64_t n) {
  return (int32_t)std::max<int64_t>(1, (n + dot_rows_per_block(n) - 1) / dot_rows_per_block(n));
}

// Column completion (Algorithm 1, lagged normalisation), one workgroup. c = the sum of partial[0..nblk)
// is ||v_{i+1}||^2, reduced in the pass that wrote v_{i+1} (the true residual for i = 0, the projection
// otherwise), so the column is finished without waiting for the next step's fused reduction.
// rho = sqrt(c); i == 0: g_0 = rho. i >= 1: Hessenberg column i-1 = [s of step i-1; rho] gets the
// previous Givens rotations and a new one, giving the residual estimate |g_i| / ||b|| (beta = ||b||).
// The stop flag is raised on |g_i| / denom <= tol (denom = ||b||, or ||b|| + ||A||_inf ||x_0|| for the
// backward-error rule of Section 3), on the last column of the cycle, or on breakdown (rho == 0),
// and set to -1 on a non-finite value; (est, flag) also go to host_out, host-mapped memory the host reads
// after the stream synchronises.
__device__ __forceinline__ void finish_body(KState *__restrict__ st, const double *__restrict__ partial, int32_t nblk,
                                            int32_t i, int32_t last, double tol, double beta, double denom,
                                            double *host_out) {
  __shared__ double lds[WAVES];
  const double t = block_sum(strided_sum(partial, nblk), lds);
  if (threadIdx.x != 0) return;
  const double rho = sqrt(t);
  int flag = 0;
  st->rho = rho;
  st->rho_inv = rho > 0.0 ? 1.0 / rho : 0.0;
  st->zs[i] = st->rho_inv;
  if (i == 0) {
    st->g[0] = rho;
    st->est = rho / beta;
  } else {
    double *h = st->H + (int64_t)(i - 1) * KS_LD;
    for (int j = 0; j < i; ++j) h[j] = st->s[j];
    h[i] = rho;
    for (int j = 0; j < i - 1; ++j) {
      const double a = h[j], b = h[j + 1];
      h[j] = st->cs[j] * a + st->sn[j] * b;
      h[j + 1] = -st->sn[j] * a + st->cs[j] * b;
    }
    double cj = 1.0, sj = 0.0;
    if (h[i] != 0.0) {
      const double den = hypot(h[i - 1], h[i]);
      cj = h[i - 1] / den;
      sj = h[i] / den;
    }
    st->cs[i - 1] = cj;
    st->sn[i - 1] = sj;
    h[i - 1] = cj * h[i - 1] + sj * h[i];
    h[i] = 0.0;
    const double gi = st->g[i - 1];
    st->g[i] = -sj * gi;
    st->g[i - 1] = cj * gi;
    st->est = fabs(st->g[i]) / beta;
    if (fabs(st->g[i]) / denom <= tol || last || rho == 0.0) flag = 1;
  }
  if (!isfinite(rho) || !isfinite(st->est)) flag = -1;
  st->flag = flag;
  host_out[0] = st->est;
  host_out[1] = (double)flag;
}

// Small dense part of Arnoldi step i (0-based: columns 0..i of V are V_{i+1}), one workgroup, after the
// column completion has set rho = ||v_{i+1}||. cd holds the fused reduction's inner products
// c_j = cd[j] (j < i) and d_j = cd[i + 1 + j] (j <= i). New row of L: c_j / rho; q: d_j / rho, the last
// one d_i / rho^2; s = T q. t_mode 0: T = (I + L)^{-1} by forward substitution; t_mode p >= 1:
// T = sum_{j=0..p} (-L)^j, the Neumann series truncated at degree p (Section 1), by Horner (s <- q, then
// p times s <- q - L s); p = 1 is T = I - L.
__device__ __forceinline__ void step_body(KState *__restrict__ st, const double *__restrict__ cd, int32_t i,
                                          int32_t t_mode) {
  __shared__ double c[KS_LD], q[KS_LD], s[KS_LD], u[KS_LD];
  const double ri = 1.0 / st->rho;
  for (int j = threadIdx.x; j <= i; j += BLK) {
    const double dj = cd[i + 1 + j];
    if (j < i) {
      c[j] = cd[j];
      st->L[(int64_t)i * KS_LD + j] = c[j] * ri;
      q[j] = dj * ri;
    } else {
      q[j] = dj * ri * ri;
    }
  }
  __syncthreads();
  if (t_mode > 0) {
    // Horner steps s <- q - L s from s = q (row i of L is read from c: it is being written)
    for (int deg = 0; deg < t_mode; ++deg) {
      const double *prev = deg == 0 ? q : u;
      for (int j = threadIdx.x; j <= i; j += BLK) {
        double a = q[j];
        for (int l = 0; l < j; ++l) {
          const double Ljl = (j == i) ? c[l] * ri : st->L[(int64_t)j * KS_LD + l];
          a -= Ljl * prev[l];
        }
        s[j] = a;
      }
      __syncthreads();
      if (deg + 1 < t_mode) {
        for (int j = threadIdx.x; j <= i; j += BLK) u[j] = s[j];
        __syncthreads();
      }
    }
  } else {
    // (I + L) s = q by column-oriented forward substitution
    for (int j = 0; j <= i; ++j) {
      const double sj = q[j];
      __syncthreads();
      if (threadIdx.x == 0) s[j] = sj;
      for (int l = j + 1 + threadIdx.x; l <= i; l += BLK) {
        const double Llj = (l == i) ? c[j] * ri : st->L[(int64_t)l * KS_LD + j];
        q[l] -= Llj * sj;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j <= i; j += BLK) st->s[j] = s[j];
}

// Lagged normalisation and projection (Algorithm 1): v_{i+1} <- v_{i+1} / rho and
// v_{i+2} = w / rho - V_{i+1} s, with an optional low-precision copy of v_{i+2} for the next V-cycle,
// and the block's partial sum of |v_{i+2}|^2 for the next column completion.
template <class TL>
__device__ __forceinline__ void project_body(uint32_t lb, double *__restrict__ V, int64_t ldv, int32_t i,
                                             const double *__restrict__ w, const KState *__restrict__ st, int32_t n,
                                             TL *__restrict__ vlow, double *__restrict__ partial) {
  __shared__ double s[KS_LD];
  __shared__ double ri;
  __shared__ double lds[WAVES];
  for (int j = threadIdx.x; j <= i; j += BLK) s[j] = st->s[j];
  if (threadIdx.x == 0) ri = st->rho_inv;
  __syncthreads();
  const int32_t row = (int32_t)lb * BLK + threadIdx.x;
  double acc = 0.0;
  if (row < n) {
    const double vi = V[(int64_t)i * ldv + row] * ri;
    V[(int64_t)i * ldv + row] = vi;
    acc = w[row] * ri;
    for (int j = 0; j < i; ++j) acc -= s[j] * V[(int64_t)j * ldv + row];
    acc -= s[i] * vi;
    V[(int64_t)(i + 1) * ldv + row] = acc;
    if (vlow) vlow[row] = (TL)acc;
  }
  const double t = block_sum(acc * acc, lds);
  if (threadIdx.x == 0) partial[lb] = t;
}

// y from the rotated k x k triangle (Algorithm 1, least squares), then y_j *= zs_j.
__device__ __forceinline__ void backsolve_body(KState *__restrict__ st, int32_t k) {
  if (threadIdx.x != 0) return;
  double *y = st->y;
  for (int j = k - 1; j >= 0; --j) {
    double acc = st->g[j];
    for (int l = j + 1; l < k; ++l) acc -= st->H[(int64_t)l * KS_LD + j] * y[l];
    y[j] = acc / st->H[(int64_t)j * KS_LD + j];
  }
  for (int j = 0; j < k; ++j) y[j] *= st->zs[j];
}

// x += Z_k y  (Algorithm 1, solution update; flexible GMRES uses the stored Z)
template <class TZ>
__device__ __forceinline__ void update_x_body(uint32_t lb, const TZ *__restrict__ Z, int64_t ldz, int32_t k,
                                              const KState *__restrict__ st, double *__restrict__ x, int32_t n) {
  __shared__ double y[KS_LD];
  for (int j = threadIdx.x; j < k; j += BLK) y[j] = st->y[j];
  __syncthreads();
  const int32_t row = (int32_t)lb * BLK + threadIdx.x;
  if (row >= n) return;
  double acc = 0.0;
  for (int j = 0; j < k; ++j) acc += (double)Z[(int64_t)j * ldz + row] * y[j];
  x[row] += acc;
}

// ------------------------------------------------------------------ single-problem Krylov kernels

template <class TL>
__global__ __launch_bounds__(BLK) void k_residual64(NAMG_MAT_HEAD(double), const double *__restrict__ b,
                                                    const double *__restrict__ x, double *__restrict__ r,
                                                    TL *__restrict__ rlow, double *__restrict__ partial, int64_t m_mul) {
  residual64_body(blockIdx.x, NAMG_MAT_VIEW(double), b, x, r, rlow, partial);
}

__global__ __launch_bounds__(BLK) void k_sumsq(const double *__restrict__ x, int32_t n, double *__restrict__ partial) {
  sumsq_body(blockIdx.x, x, n, partial);
}

__global__ __launch_bounds__(BLK) void k_reduce(const double *__restrict__ partial, int32_t n, double *out) {
  reduce_body(partial, n, out);
}

__global__ __launch_bounds__(BLK) void k_colreduce(const double *__restrict__ partial, int32_t nblk,
                                                   double *__restrict__ out) {
  colreduce_body(blockIdx.x, partial, nblk, out);
}

template <int CH, int PAIRS = 1>
__global__ __launch_bounds__(BLK) void k_multidot(const double *__restrict__ V, int64_t ldv, int32_t ncols,
                                                  const double *__restrict__ w, int32_t n, int32_t rows_per_blk,
                                                  double *__restrict__ partial, int32_t nblk) {
  multidot_body<CH, PAIRS>(blockIdx.x, V, ldv, ncols, w, n, rows_per_blk, partial, nblk);
}

// The fused reduction's kernel for ncols columns: one chunk of exactly ncols columns up to eight (two row
// pairs per iteration up to four columns, where registers allow), else chunks of eight.
using MultidotKernel = void (*)(const double *, int64_t, int32_t, const double *, int32_t, int32_t, double *, int32_t);
inline MultidotKernel multidot_kernel(int32_t ncols) {
  switch (ncols) {
    case 1: return &k_multidot<1, 2>;
    case 2: return &k_multidot<2, 2>;
    case 3: return &k_multidot<3, 2>;
    case 4: return &k_multidot<4, 2>;
    case 5: return &k_multidot<5>;
    case 6: return &k_multidot<6>;
    case 7: return &k_multidot<7>;
    default: return &k_multidot<8>;
  }
}

__global__ __launch_bounds__(BLK) void k_finish(KState *__restrict__ st, const double *__restrict__ partial, int32_t nblk,
                                                int32_t i, int32_t last, double tol, double beta, double denom,
                                                double *host_out) {
  finish_body(st, partial, nblk, i, last, tol, beta, denom, host_out);
}

__global__ __launch_bounds__(BLK) void k_step(KState *__restrict__ st, const double *__restrict__ cd, int32_t i,
                                              int32_t t_mode) {
  step_body(st, cd, i, t_mode);
}

template <class TL>
__global__ __launch_bounds__(BLK) void k_project(double *__restrict__ V, int64_t ldv, int32_t i,
                                                 const double *__restrict__ w, const KState *__restrict__ st,
                                                 int32_t n, TL *__restrict__ vlow, double *__restrict__ partial) {
  project_body(blockIdx.x, V, ldv, i, w, st, n, vlow, partial);
}

__global__ __launch_bounds__(BLK) void k_backsolve(KState *__restrict__ st, int32_t k) { backsolve_body(st, k); }

template <class TZ>
__global__ __launch_bounds__(BLK) void k_update_x(const TZ *__restrict__ Z, int64_t ldz, int32_t k,
                                                  const KState *__restrict__ st, double *__restrict__ x, int32_t n) {
  update_x_body(blockIdx.x, Z, ldz, k, st, x, n);
}

// ------------------------------------------------------------------------------ batched kernels

// The task of this block: the largest k with off[k] <= blockIdx.x (off has ntasks + 1 entries). The
// offsets are staged in LDS once per block and searched there.
__device__ __forceinline__ int find_task(const uint32_t *__restrict__ off, int ntasks, uint32_t &local_block) {
  __shared__ uint32_t s_off[MAX_BATCH + 1];
  for (int k = threadIdx.x; k <= ntasks; k += BLK) s_off[k] = off[k];
  __syncthreads();
  int lo = 0, hi = ntasks - 1;
  const uint32_t b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_off[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  local_block = b - s_off[lo];
  return lo;
}

// One row operation on one level of one solve. Operand meaning per operation:
//   ROP_RESIDUAL: a = b, b = x (may be null), c = D^{-1} (null unless o1 is set), o0 = r, o1 = f
//   ROP_NEUMANN:  a = f, b = in, c = scale, d = acc, o0 = out
//   ROP_SPMV:     b = x, o0 = y, optionally c = d and o1 = f = d .* y
//   ROP_PROLONG:  b = e, o0 = x
//   ROP_AXPY:     a = f, c = scale, d = acc, o0 = out, n rows
//   ROP_FILL:     o0 = 0, n rows
enum { ROP_RESIDUAL = 0, ROP_NEUMANN = 1, ROP_SPMV = 2, ROP_PROLONG = 3, ROP_AXPY = 4, ROP_FILL = 5 };

template <class T>
struct RowTask {
  MatView<T> M;
  const T *a, *b, *c, *d;
  T *o0, *o1;
  int32_t n, pad;
};

template <int OP, int G, class T, int U = 4>
__global__ __launch_bounds__(BLK) void kb_rows(const RowTask<T> *__restrict__ tasks, const uint32_t *__restrict__ off,
                                               int ntasks) {
  uint32_t lb;
  const RowTask<T> &t = tasks[find_task(off, ntasks, lb)];
  if constexpr (OP == ROP_RESIDUAL) residual_body<G, T, U>(lb, t.M, t.a, t.b, t.c, t.o0, t.o1);
  if constexpr (OP == ROP_NEUMANN) neumann_body<G, T, U>(lb, t.M, t.a, t.b, t.c, t.d, t.o0);
  if constexpr (OP == ROP_SPMV) spmv_body<G, T, U>(lb, t.M, t.b, t.o0, t.c, t.o1);
  if constexpr (OP == ROP_PROLONG) prolong_body<G>(lb, t.M, t.b, t.o0);
  if constexpr (OP == ROP_AXPY) axpy_body(lb, t.a, t.c, t.d, t.o0, t.n);
  if constexpr (OP == ROP_FILL) {
    const int32_t row = (int32_t)lb * BLK + threadIdx.x;
    if (row < t.n) t.o0[row] = T(0);
  }
}

// One Krylov operation of one solve (fields used per operation are listed at the launch site).
enum {
  KOP_RESIDUAL64 = 0, KOP_SPMV64 = 1, KOP_MULTIDOT = 2, KOP_COLREDUCE = 3, KOP_STEP = 4, KOP_PROJECT = 5,
  KOP_BACKSOLVE = 6, KOP_UPDATE = 7, KOP_REDUCE = 8, KOP_SUMSQ = 9, KOP_FINISH = 10
};

template <class T>
struct KTask {
  MatView<double> A;
  const double *b;
  double *x, *V, *w, *partial, *cd, *host_out;
  T *Z, *vlow;
  const T *zin;
  KState *ks;
  int64_t ldv, ldz;
  int32_t n, i, ncols, has_w, last, k, nblk, rows_per_blk;
  int32_t t_mode, pad;  // the solve's correction T (see step_body)
  double beta, denom, tol;
};

template <int OP, class T>
__global__ __launch_bounds__(BLK) void kb_krylov(const KTask<T> *__restrict__ tasks, const uint32_t *__restrict__ off,
                                                 int ntasks) {
  uint32_t lb;
  const KTask<T> &t = tasks[find_task(off, ntasks, lb)];
  if constexpr (OP == KOP_RESIDUAL64) residual64_body(lb, t.A, t.b, t.x, t.V, t.vlow, t.partial);
  if constexpr (OP == KOP_SPMV64)
    spmv_body<1, double>(lb, t.A, t.zin, t.w, (const double *)nullptr, (double *)nullptr);
  if constexpr (OP == KOP_MULTIDOT)
    multidot_body<8>(lb, t.V, t.ldv, t.ncols, t.has_w ? t.w : (const double *)nullptr, t.n, t.rows_per_blk, t.partial,
                     t.nblk);
  if constexpr (OP == KOP_COLREDUCE) colreduce_body(lb, t.partial, t.nblk, t.cd);
  if constexpr (OP == KOP_STEP) step_body(t.ks, t.cd, t.i, t.t_mode);
  if constexpr (OP == KOP_PROJECT) project_body(lb, t.V, t.ldv, t.i, t.w, t.ks, t.n, t.vlow, t.partial);
  if constexpr (OP == KOP_FINISH) finish_body(t.ks, t.partial, t.nblk, t.i, t.last, t.tol, t.beta, t.denom, t.host_out);
  if constexpr (OP == KOP_BACKSOLVE) backsolve_body(t.ks, t.k);
  if constexpr (OP == KOP_UPDATE) update_x_body(lb, (const T *)t.Z, t.ldz, t.k, t.ks, t.x, t.n);
  if constexpr (OP == KOP_REDUCE) reduce_body(t.partial, t.nblk, t.host_out);
  if constexpr (OP == KOP_SUMSQ) sumsq_body(lb, t.x, t.n, t.partial);
}

}  // namespace namg

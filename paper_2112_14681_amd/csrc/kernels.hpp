// HIP kernels of the namg solve phase for gfx950 (CDNA4, 64-wide wavefronts).
//
// Every hot kernel is a streaming sparse or vector operation (arithmetic intensity <= 0.25 flop/byte),
// so the HBM roofline bounds them; none is a dense contraction, and MFMA is not used. Sparse operators
// use the SELL-64 layout (one wavefront per slice of 64 rows, one row per lane): the value and column
// loads of a wavefront are 512 B / 256 B contiguous, and the x-gathers of a 3-D stencil hit the same or
// neighbouring cache lines. Reductions are deterministic: a fixed xor-butterfly inside the wavefront,
// a fixed order across wavefronts and blocks, no floating-point atomics.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"

namespace namg {

constexpr int BLK = 256;
constexpr int WAVES = BLK / 64;

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + BLK - 1) / BLK); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Row `row` of a sparse matrix times x, reduced over the G lanes of the row's group (every lane of the
// group returns the full sum). G == 1: SELL-64, one lane per row. G > 1: CSR, lane `sub` takes entries
// sub, sub + G, ...; groups are aligned inside the wavefront, so the butterfly never leaves the group.
template <int G, class Acc, class TM, class TX>
__device__ __forceinline__ Acc row_dot(const MatView<TM> &A, const TX *__restrict__ x, int32_t row, int sub) {
  Acc acc = Acc(0);
  const bool nt = (A.flags & KF_NT_LOADS) != 0;
  if constexpr (G == 1) {
    const int32_t s = row >> 6;
    const int32_t end = A.ptr[s + 1];
    if (nt) {
#pragma unroll 4
      for (int32_t k = A.ptr[s] + (row & 63); k < end; k += SELL_C)
        acc += (Acc)__builtin_nontemporal_load(A.val + k) * (Acc)x[__builtin_nontemporal_load(A.col + k)];
    } else {
#pragma unroll 4
      for (int32_t k = A.ptr[s] + (row & 63); k < end; k += SELL_C) acc += (Acc)A.val[k] * (Acc)x[A.col[k]];
    }
  } else {
    const int32_t end = A.ptr[row + 1];
    if (nt) {
#pragma unroll 2
      for (int32_t k = A.ptr[row] + sub; k < end; k += G)
        acc += (Acc)__builtin_nontemporal_load(A.val + k) * (Acc)x[__builtin_nontemporal_load(A.col + k)];
    } else {
#pragma unroll 2
      for (int32_t k = A.ptr[row] + sub; k < end; k += G) acc += (Acc)A.val[k] * (Acc)x[A.col[k]];
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  }
  return acc;
}

// Logical block index: with KF_XCD_REMAP, XCD x (which receives blocks x, x+8, x+16, ...) is given the
// contiguous logical range [x*q + min(x, r), ...) of the nb = 8q + r blocks.
__device__ __forceinline__ uint32_t logical_block(uint32_t flags) {
  const uint32_t b = blockIdx.x;
  if (!(flags & KF_XCD_REMAP)) return b;
  const uint32_t nb = gridDim.x, q = nb >> 3, r = nb & 7u, x = b & 7u;
  return x * q + min(x, r) + (b >> 3);
}

#define NAMG_ROW_PROLOGUE(G, M)                                                  \
  const int64_t gtid_ = (int64_t)logical_block((M).flags) * BLK + threadIdx.x;   \
  const int32_t row = (int32_t)(gtid_ / (G));                                     \
  const int sub = (int)(gtid_ % (G));                                             \
  if (row >= (M).nrows) return;

// y = A x  (restriction R r, the GMRES product w = A z with z promoted on load, the coarse inverse)
template <int G, class Acc, class TM, class TX, class TY>
__global__ __launch_bounds__(BLK) void k_spmv(MatView<TM> A, const TX *__restrict__ x, TY *__restrict__ y) {
  NAMG_ROW_PROLOGUE(G, A)
  const Acc v = row_dot<G, Acc>(A, x, row, sub);
  if (sub == 0) y[row] = (TY)v;
}

// r = b - A x (x == nullptr means x = 0), optionally f = d .* r. One pass: SpMV, subtract, scale.
template <int G, class T>
__global__ __launch_bounds__(BLK) void k_residual(MatView<T> A, const T *__restrict__ b, const T *__restrict__ x,
                                                  const T *__restrict__ d, T *__restrict__ r, T *__restrict__ f) {
  NAMG_ROW_PROLOGUE(G, A)
  const T acc = x ? row_dot<G, T>(A, x, row, sub) : T(0);
  if (sub != 0) return;
  const T rr = b[row] - acc;
  if (r) r[row] = rr;
  if (f) f[row] = d[row] * rr;
}

// One Neumann / Jacobi inner term on a pre-scaled strict triangle S:
//   out = [acc +] [scale .*] (f - S in)
// Polynomial GS: S = D^{-1}L (or D^{-1}U), f = D^{-1} r; ILU: S = L_s with f = r, or S = U_s with
// f = D_U^{-1} y. `acc` may alias `out` (x += ...); `in` never aliases `out`.
template <int G, class T>
__global__ __launch_bounds__(BLK) void k_neumann(MatView<T> S, const T *__restrict__ f, const T *__restrict__ in,
                                                 const T *__restrict__ scale, const T *acc, T *out) {
  NAMG_ROW_PROLOGUE(G, S)
  const T sv = row_dot<G, T>(S, in, row, sub);
  if (sub != 0) return;
  T v = f[row] - sv;
  if (scale) v *= scale[row];
  if (acc) v += acc[row];
  out[row] = v;
}

// x += P e  (prolongation and correction in one pass)
template <int G, class T>
__global__ __launch_bounds__(BLK) void k_prolong(MatView<T> P, const T *__restrict__ e, T *x) {
  NAMG_ROW_PROLOGUE(G, P)
  const T v = row_dot<G, T>(P, e, row, sub);
  if (sub == 0) x[row] += v;
}

// out = [acc +] [scale .*] f
template <class T>
__global__ __launch_bounds__(BLK) void k_axpy(const T *__restrict__ f, const T *__restrict__ scale, const T *acc, T *out,
                                              int32_t n) {
  const int32_t row = blockIdx.x * BLK + threadIdx.x;
  if (row >= n) return;
  T v = f[row];
  if (scale) v *= scale[row];
  if (acc) v += acc[row];
  out[row] = v;
}

// One dependency level of a direct triangular solve g = (I + S)^{-1} f: rows of the level only read
// g of earlier levels.
template <class T>
__global__ __launch_bounds__(BLK) void k_tri_level(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                   const T *__restrict__ val, const int32_t *__restrict__ order,
                                                   int32_t beg, int32_t cnt, const T *__restrict__ f, T *g) {
  const int32_t q = blockIdx.x * BLK + threadIdx.x;
  if (q >= cnt) return;
  const int32_t i = order[beg + q];
  T acc = f[i];
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) acc -= val[k] * g[ci[k]];
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

// ------------------------------------------------------------------------------------------------
// FP64 Krylov kernels.

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

// r = b - A x in FP64 (true residual), optional low-precision copy of r, per-block partial of |r|^2.
template <class TL>
__global__ __launch_bounds__(BLK) void k_residual64(MatView<double> A, const double *__restrict__ b,
                                                    const double *__restrict__ x, double *__restrict__ r,
                                                    TL *__restrict__ rlow, double *__restrict__ partial) {
  __shared__ double lds[WAVES];
  const int32_t row = blockIdx.x * BLK + threadIdx.x;
  double rr = 0.0;
  if (row < A.nrows) {
    rr = b[row] - row_dot<1, double>(A, x, row, 0);
    r[row] = rr;
    if (rlow) rlow[row] = (TL)rr;
  }
  const double t = block_sum(rr * rr, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// partial[b] = sum over block b's rows of x^2
__global__ __launch_bounds__(BLK) void k_sumsq(const double *__restrict__ x, int32_t n, double *__restrict__ partial) {
  __shared__ double lds[WAVES];
  const int32_t row = blockIdx.x * BLK + threadIdx.x;
  const double v = row < n ? x[row] : 0.0;
  const double t = block_sum(v * v, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// out[0] = sum of partial[0..n) in a fixed order (one block); out may be host-mapped memory.
__global__ __launch_bounds__(BLK) void k_reduce(const double *__restrict__ partial, int32_t n, double *out) {
  __shared__ double lds[WAVES];
  double t = 0.0;
  for (int32_t k = threadIdx.x; k < n; k += BLK) t += partial[k];
  t = block_sum(t, lds);
  if (threadIdx.x == 0) out[0] = t;
}

// Block v: out[v] = sum over b < nblk of partial[v * nblk + b], in a fixed order.
__global__ __launch_bounds__(BLK) void k_colreduce(const double *__restrict__ partial, int32_t nblk,
                                                   double *__restrict__ out) {
  __shared__ double lds[WAVES];
  const double *p = partial + (int64_t)blockIdx.x * nblk;
  double t = 0.0;
  for (int32_t k = threadIdx.x; k < nblk; k += BLK) t += p[k];
  t = block_sum(t, lds);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// The single fused reduction of an Arnoldi step (Algorithm 1, the global synchronisation):
// c = V_{i+1}^T v_{i+1} and d = V_{i+1}^T w in one pass over V. Block b owns a contiguous row range and
// writes its partial sums value-major: partial[v * nblk + b], v < ncols for c, ncols + v for d.
template <int CH>
__global__ __launch_bounds__(BLK) void k_multidot(const double *__restrict__ V, int64_t ldv, int32_t ncols,
                                                  const double *__restrict__ w, int32_t n, int32_t rows_per_blk,
                                                  double *__restrict__ partial, int32_t nblk) {
  __shared__ double lds[2 * CH][WAVES];
  const int32_t r0 = blockIdx.x * rows_per_blk;
  const int32_t r1 = min(n, r0 + rows_per_blk);
  const double *v = V + (int64_t)(ncols - 1) * ldv;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int32_t j0 = 0; j0 < ncols; j0 += CH) {
    double ac[CH], ad[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) ac[c] = ad[c] = 0.0;
    for (int32_t r = r0 + threadIdx.x; r < r1; r += BLK) {
      const double vr = v[r];
      const double wr = w ? w[r] : 0.0;
#pragma unroll
      for (int c = 0; c < CH; ++c)
        if (j0 + c < ncols) {
          const double vj = V[(int64_t)(j0 + c) * ldv + r];
          ac[c] += vj * vr;
          ad[c] += vj * wr;
        }
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
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
        partial[(int64_t)((isd ? ncols : 0) + col) * nblk + blockIdx.x] = t;
      }
    }
    __syncthreads();
  }
}

// Small dense part of Arnoldi step i (0-based: columns 0..i of V are V_{i+1}), one workgroup; beta = ||b||.
// cd holds the reduced inner products: c_j = cd[j], d_j = cd[i + 1 + j], j <= i.
// rho = sqrt(c_i) is the lagged norm of v_{i+1}; Hessenberg column i-1 = [previous s; rho] gets the
// Givens rotations and yields the residual estimate |g_i| / ||b||; then the new row of L (c_j / rho),
// q (d_j / rho, the last one d_i / rho^2) and s = T q with T = I - L (Neumann) or T = (I + L)^{-1}
// (forward substitution). Writes s, 1/rho and the stop flag to the state, and (est, flag) to host_out,
// host-mapped memory the host reads after the stream synchronises.
__global__ __launch_bounds__(BLK) void k_arnoldi_step(KState *__restrict__ st, const double *__restrict__ cd, int32_t i,
                                                      int32_t has_w, int32_t t_direct, int32_t last, double tol,
                                                      double beta, double *host_out) {
  __shared__ double c[KS_LD], d[KS_LD], q[KS_LD], s[KS_LD];
  __shared__ double rho_sh;
  __shared__ int stop_sh;
  for (int j = threadIdx.x; j <= i; j += BLK) {
    c[j] = cd[j];
    d[j] = has_w ? cd[i + 1 + j] : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double rho = sqrt(c[i]);
    int flag = 0;
    st->rho_inv = rho > 0.0 ? 1.0 / rho : 0.0;
    st->zs[i] = st->rho_inv;
    if (i == 0) {
      st->g[0] = rho;
      st->est = rho / beta;
    } else {
      double *h = st->H + (int64_t)(i - 1) * KS_LD;
      for (int j = 0; j < i; ++j) h[j] = st->rprev[j];
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
      if (st->est <= tol || last || rho == 0.0) flag = 1;
    }
    if (!isfinite(rho) || !isfinite(st->est)) flag = -1;
    st->flag = flag;
    host_out[0] = st->est;
    host_out[1] = (double)flag;
    rho_sh = rho;
    stop_sh = flag;
  }
  __syncthreads();
  if (!has_w || stop_sh != 0) return;
  const double ri = 1.0 / rho_sh;
  for (int j = threadIdx.x; j <= i; j += BLK) {
    if (j < i) {
      st->L[(int64_t)i * KS_LD + j] = c[j] * ri;
      q[j] = d[j] * ri;
    } else {
      q[j] = d[j] * ri * ri;
    }
  }
  __syncthreads();
  if (!t_direct) {
    // s = (I - L) q: one matrix-vector product
    for (int j = threadIdx.x; j <= i; j += BLK) {
      double a = q[j];
      for (int l = 0; l < j; ++l) {
        const double Ljl = (j == i) ? c[l] * ri : st->L[(int64_t)j * KS_LD + l];
        a -= Ljl * q[l];
      }
      s[j] = a;
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
  for (int j = threadIdx.x; j <= i; j += BLK) {
    st->s[j] = s[j];
    st->rprev[j] = s[j];
  }
}

// Lagged normalisation and projection (Algorithm 1): v_{i+1} <- v_{i+1} / rho and
// v_{i+2} = w / rho - V_{i+1} s, with an optional low-precision copy of v_{i+2} for the next V-cycle.
template <class TL>
__global__ __launch_bounds__(BLK) void k_project(double *__restrict__ V, int64_t ldv, int32_t i,
                                                 const double *__restrict__ w, const KState *__restrict__ st,
                                                 int32_t n, TL *__restrict__ vlow) {
  __shared__ double s[KS_LD];
  __shared__ double ri;
  for (int j = threadIdx.x; j <= i; j += BLK) s[j] = st->s[j];
  if (threadIdx.x == 0) ri = st->rho_inv;
  __syncthreads();
  const int32_t row = blockIdx.x * BLK + threadIdx.x;
  if (row >= n) return;
  const double vi = V[(int64_t)i * ldv + row] * ri;
  V[(int64_t)i * ldv + row] = vi;
  double acc = w[row] * ri;
  for (int j = 0; j < i; ++j) acc -= s[j] * V[(int64_t)j * ldv + row];
  acc -= s[i] * vi;
  V[(int64_t)(i + 1) * ldv + row] = acc;
  if (vlow) vlow[row] = (TL)acc;
}

// y from the rotated k x k triangle (Algorithm 1, least squares), then y_j *= zs_j.
__global__ void k_backsolve(KState *__restrict__ st, int32_t k) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
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
__global__ __launch_bounds__(BLK) void k_update_x(const TZ *__restrict__ Z, int64_t ldz, int32_t k,
                                                  const KState *__restrict__ st, double *__restrict__ x, int32_t n) {
  __shared__ double y[KS_LD];
  for (int j = threadIdx.x; j < k; j += BLK) y[j] = st->y[j];
  __syncthreads();
  const int32_t row = blockIdx.x * BLK + threadIdx.x;
  if (row >= n) return;
  double acc = 0.0;
  for (int j = 0; j < k; ++j) acc += (double)Z[(int64_t)j * ldz + row] * y[j];
  x[row] += acc;
}

}  // namespace namg

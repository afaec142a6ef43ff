// Device-side containers of the namg library: owned device buffers, the two sparse layouts used by the
// streaming kernels, CSR views for the level-scheduled direct comparators and the Krylov state.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <iterator>
#include <map>
#include <mutex>
#include <type_traits>
#include <string>
#include <utility>
#include <vector>

#include "../../include/namg.h"
#include "setup_host.hpp"

namespace namg {

struct HipError {
  int code;
  std::string msg;
};

inline void hip_check(hipError_t e, const char *what) {
  if (e == hipSuccess) return;
  if (e == hipErrorOutOfMemory) throw HipError{NAMG_E_NOMEM, std::string(what) + ": out of device memory"};
  throw HipError{NAMG_E_HIP, std::string(what) + ": " + hipGetErrorString(e)};
}

// Counts the device bytes a set of DevBufs holds (one hierarchy, or every device setup of the process):
// the size class each one allocated (see BlockCache), not the bytes it asked for; peak is the high-water
// mark. Safe to share between threads.
struct MemCounter {
  std::atomic<int64_t> bytes{0}, peak{0};
  void add(int64_t b) {
    const int64_t now = bytes.fetch_add(b) + b;
    int64_t p = peak.load();
    while (now > p && !peak.compare_exchange_weak(p, now)) {
    }
  }
  void sub(int64_t b) { bytes.fetch_sub(b); }
};

// Device memory of the device setup (uploaded A_0, scratch of coarsening and sparse products, the levels
// kept for the solve-phase layouts, the temporaries of device packing): outside any solver's footprint.
// The part of a server's default device budget left to it (peak_setup_device_bytes reports the measured need).
constexpr int64_t SETUP_DEVICE_RESERVE = int64_t(32) << 30;
inline MemCounter &setup_mem() {
  static MemCounter m;
  return m;
}

// Host<->device copies of pageable memory go through a pool of pinned staging buffers (64 MiB chunks):
// the runtime's own pageable path shares one staging route among all threads, and many setup threads copy
// at once. The pool holds as many buffers as copies ever ran at the same time, for the life of the
// process.
class PinnedPool {
 public:
  static constexpr size_t CHUNK = size_t(64) << 20;
  static PinnedPool &instance() {
    static PinnedPool p;
    return p;
  }
  char *acquire() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (!free_.empty()) {
        char *b = free_.back();
        free_.pop_back();
        return b;
      }
    }
    void *b = nullptr;
    hip_check(hipHostMalloc(&b, CHUNK, hipHostMallocDefault), "hipHostMalloc");
    return static_cast<char *>(b);
  }
  void release(char *b) {
    std::lock_guard<std::mutex> lk(mu_);
    free_.push_back(b);
  }

 private:
  std::mutex mu_;
  std::vector<char *> free_;
};

// Synchronous copies through one pinned staging buffer, split into SLOTS slices that form a pipeline: the
// DMA of one slice overlaps the host memcpy of another, and an event per slice says when it is reusable.
constexpr int STAGE_SLOTS = 8;

// Declared after the StageBuffer it guards: on every exit, errors included, it waits for the copies it has
// recorded before the buffer goes back to the pool.
struct StageEvents {
  hipEvent_t e[STAGE_SLOTS] = {};
  StageEvents() {
    for (auto &x : e) hip_check(hipEventCreateWithFlags(&x, hipEventDisableTiming), "hipEventCreateWithFlags");
  }
  ~StageEvents() {
    for (auto &x : e)
      if (x) {
        (void)hipEventSynchronize(x);
        (void)hipEventDestroy(x);
      }
  }
};

struct StageBuffer {
  PinnedPool &pool = PinnedPool::instance();
  char *b = pool.acquire();
  ~StageBuffer() { pool.release(b); }
};

// Copies of pageable memory on stream s (the null stream by default); return when the copy is complete.
inline void copy_to_device(void *dst, const void *src, size_t bytes, hipStream_t s = nullptr) {
  if (bytes == 0) return;
  constexpr size_t SL = PinnedPool::CHUNK / STAGE_SLOTS;
  StageBuffer stage;
  StageEvents ev;
  const size_t n = (bytes + SL - 1) / SL;
  for (size_t k = 0; k < n; ++k) {
    const int j = (int)(k % STAGE_SLOTS);
    const size_t off = k * SL, c = std::min(SL, bytes - off);
    if (k >= (size_t)STAGE_SLOTS) hip_check(hipEventSynchronize(ev.e[j]), "hipEventSynchronize");
    std::memcpy(stage.b + j * SL, static_cast<const char *>(src) + off, c);
    hip_check(hipMemcpyAsync(static_cast<char *>(dst) + off, stage.b + j * SL, c, hipMemcpyHostToDevice, s), "H2D");
    hip_check(hipEventRecord(ev.e[j], s), "hipEventRecord");
  }
  for (size_t k = (n > (size_t)STAGE_SLOTS ? n - STAGE_SLOTS : 0); k < n; ++k)
    hip_check(hipEventSynchronize(ev.e[k % STAGE_SLOTS]), "hipEventSynchronize");
}

inline void copy_to_host(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  constexpr size_t SL = PinnedPool::CHUNK / STAGE_SLOTS;
  StageBuffer stage;
  StageEvents ev;
  const size_t n = (bytes + SL - 1) / SL;
  auto issue = [&](size_t k) {
    const int j = (int)(k % STAGE_SLOTS);
    const size_t off = k * SL, c = std::min(SL, bytes - off);
    hip_check(hipMemcpyAsync(stage.b + j * SL, static_cast<const char *>(src) + off, c, hipMemcpyDeviceToHost, s),
              "D2H");
    hip_check(hipEventRecord(ev.e[j], s), "hipEventRecord");
  };
  for (size_t k = 0; k < std::min(n, (size_t)STAGE_SLOTS); ++k) issue(k);
  for (size_t k = 0; k < n; ++k) {
    const int j = (int)(k % STAGE_SLOTS);
    const size_t off = k * SL, c = std::min(SL, bytes - off);
    hip_check(hipEventSynchronize(ev.e[j]), "hipEventSynchronize");
    std::memcpy(static_cast<char *>(dst) + off, stage.b + j * SL, c);
    if (k + STAGE_SLOTS < n) issue(k + STAGE_SLOTS);  // slice j has been copied out
  }
}

// Device memory blocks are recycled instead of freed: a released block is kept per (device, size class)
// and handed to the next allocation of that class, so a process that keeps setting up and solving
// systems (a server) reaches a steady state without hipMalloc or hipFree; a free can wait for work on
// every stream of the device. Size classes are 1/8-octave steps above 4 KiB (at most 12.5 % rounding);
// at most CACHE_CAP bytes stay cached per device, beyond that blocks are freed. Cached blocks live until
// the process ends.
class BlockCache {
 public:
  static constexpr size_t CACHE_CAP = size_t(32) << 30;
  static BlockCache &instance() {
    static BlockCache c;
    return c;
  }
  static size_t size_class(size_t bytes) {
    if (bytes <= 4096) return 4096;
    int k = 63 - __builtin_clzll((unsigned long long)bytes);
    const size_t step = size_t(1) << (k - 3);
    return (bytes + step - 1) / step * step;
  }
  void *take(int dev, size_t cls) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = free_.find({dev, cls});
    if (it == free_.end() || it->second.empty()) return nullptr;
    void *p = it->second.back();
    it->second.pop_back();
    cached_[dev] -= cls;
    return p;
  }
  // Frees every cached block of device dev (current device must be dev); returns the bytes released.
  size_t trim(int dev) {
    std::lock_guard<std::mutex> lk(mu_);
    size_t freed = 0;
    for (auto it = free_.begin(); it != free_.end();) {
      if (it->first.first != dev) {
        ++it;
        continue;
      }
      for (void *p : it->second) {
        (void)hipFree(p);
        freed += it->first.second;
      }
      it = free_.erase(it);
    }
    cached_[dev] = 0;
    return freed;
  }
  // true when the block was kept; false: the caller frees it
  bool put(int dev, size_t cls, void *p) {
    std::lock_guard<std::mutex> lk(mu_);
    if (cached_[dev] + cls > CACHE_CAP) return false;
    free_[{dev, cls}].push_back(p);
    cached_[dev] += cls;
    return true;
  }

 private:
  std::mutex mu_;
  std::map<std::pair<int, size_t>, std::vector<void *>> free_;
  std::map<int, size_t> cached_;
};

// Device bytes that DevBuf::alloc(n) of elem-byte elements takes (its size class).
inline int64_t alloc_bytes(int64_t n, int64_t elem) {
  return (int64_t)BlockCache::size_class((size_t)std::max<int64_t>(n, 1) * (size_t)elem);
}

// One device allocation, returned to the block cache by the destructor (so a failed setup leaks nothing).
template <class T>
class DevBuf {
 public:
  DevBuf() = default;
  DevBuf(size_t n, MemCounter *mc) { alloc(n, mc); }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept { *this = std::move(o); }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) {
      release();
      p_ = o.p_;
      n_ = o.n_;
      mc_ = o.mc_;
      dev_ = o.dev_;
      cls_ = o.cls_;
      o.p_ = nullptr;
      o.n_ = 0;
      o.mc_ = nullptr;
    }
    return *this;
  }
  void alloc(size_t n, MemCounter *mc) {
    release();
    if (n == 0) n = 1;
    hip_check(hipGetDevice(&dev_), "hipGetDevice");
    cls_ = BlockCache::size_class(n * sizeof(T));
    p_ = static_cast<T *>(BlockCache::instance().take(dev_, cls_));
    if (!p_) {
      void *q = nullptr;
      hipError_t e = hipMalloc(&q, cls_);
      if (e == hipErrorOutOfMemory && BlockCache::instance().trim(dev_) > 0) {
        (void)hipGetLastError();  // clear the failed allocation's error, then retry with the cache emptied
        e = hipMalloc(&q, cls_);
      }
      hip_check(e, "hipMalloc");
      p_ = static_cast<T *>(q);
    }
    n_ = n;
    mc_ = mc;
    if (mc_) mc_->add((int64_t)cls_);
  }
  void upload(const T *h, size_t n) { copy_to_device(p_, h, n * sizeof(T)); }
  void release() {
    if (p_) {
      // Released while an exception unwinds the stack (a failed setup, upload or solve): work queued before
      // the error may still use the block, so the device drains before the block can be handed out again.
      const bool unwinding = std::uncaught_exceptions() > 0;
      const bool cached = !unwinding && BlockCache::instance().put(dev_, cls_, p_);
      if (!cached) {
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (cur != dev_) (void)hipSetDevice(dev_);
        if (unwinding) {
          (void)hipDeviceSynchronize();
          (void)hipGetLastError();
        }
        if (!unwinding || !BlockCache::instance().put(dev_, cls_, p_)) (void)hipFree(p_);
        if (cur != dev_ && cur >= 0) (void)hipSetDevice(cur);
      }
      if (mc_) mc_->sub((int64_t)cls_);
    }
    p_ = nullptr;
    n_ = 0;
  }
  T *get() const { return p_; }
  size_t size() const { return n_; }

 private:
  T *p_ = nullptr;
  size_t n_ = 0;
  MemCounter *mc_ = nullptr;
  int dev_ = 0;
  size_t cls_ = 0;
};

// A CSR matrix on the device with FP64 values.
struct DCsr {
  int32_t nr = 0, nc = 0;
  int64_t nnz = 0;
  DevBuf<int32_t> rp, ci;
  DevBuf<double> v;
};

// The operators of a hierarchy built on the device, kept there for its solve-phase layouts: A for every
// level, P and R for every level but the coarsest.
struct DeviceLevels {
  std::vector<DCsr> A, P, R;
};

// Sparse operators on the device come in one of two layouts, chosen per matrix at setup from its row
// lengths so that every row kernel keeps enough independent loads in flight:
//  * group == 1: SELL-64. Rows are cut into slices of 64 consecutive rows (one wavefront); slice s
//    stores entry k of each of its rows at val[ptr[s] + 64*k + lane], padded with value 0 up to the
//    slice's longest row. One lane per row; the loads of a wavefront are contiguous.
//  * group == G in {2, 4, ..., 64}: CSR, G lanes per row. Lane j of a row's group takes entries
//    j, j+G, ...; the G partial sums are combined by a fixed xor-butterfly. Used for the long rows of
//    the Galerkin operators on coarse levels, where one lane per row would walk 30-100 dependent
//    entries.
//  * slice-diagonal SELL-64: a SELL-64 matrix whose rows within each slice share a few column offsets
//    from their scaled diagonal base(r) below (stencil operators in natural order, their red-black
//    coarsenings and the restrictions between them) stores no per-entry column at all. Slot k of slice s
//    holds, for all 64 rows, the entries at column base(r) + d(s, k) (value 0 where a row has no entry
//    there); the slots of a slice are the union of its rows' offsets in increasing order, so each row's
//    entries keep their CSR order. One int32 offset per slot (64 entries) replaces the 2- or 4-byte column of every entry, and
//    a slot's gathers are 64 consecutive elements of x. Chosen per matrix, see LayoutCount.
// Column indices are stored in one of two widths, also chosen per matrix: as 16-bit offsets from the
// row's scaled diagonal, base(r) = (r * mul) >> 20 with mul = (ncols << 20) / nrows, when every column
// of the matrix lies within [-32768, 32767] of its row's base (stencil operators and their Galerkin
// coarsenings up to about 180^2 unknowns per plane), else as plain 32-bit columns. The narrow form cuts
// a pass over an FP64 matrix from 12 to 10 bytes per entry, and from 8 to 6 in FP32. Padding entries
// carry offset 0 (column base(r)) or column 0.
// Row order and the order of entries within a row are those of the CSR input.
constexpr int SELL_C = 64;
constexpr int SELL_C_UNIT = SELL_C;
constexpr int COL_SHIFT = 20;

__host__ __device__ inline int32_t diag_base(int32_t row, int64_t mul) {
  return (int32_t)(((int64_t)row * mul) >> COL_SHIFT);
}

inline int64_t diag_mul(int64_t nrows, int64_t ncols) { return nrows > 0 ? (ncols << COL_SHIFT) / nrows : 0; }

// True when every column of A fits the 16-bit offset form.
inline bool fits_col16(const HostCsr &A) {
  const int64_t mul = diag_mul(A.nr, A.nc);
  for (int32_t r = 0; r < A.nr; ++r) {
    const int32_t base = diag_base(r, mul);
    for (int32_t k = A.rp[r]; k < A.rp[r + 1]; ++k) {
      const int64_t d = (int64_t)A.ci[k] - base;
      if (d < -32768 || d > 32767) return false;
    }
  }
  return true;
}

template <class T>
struct MatView {
  const int32_t *ptr = nullptr;    // SELL slice pointers (group 1) or CSR row pointers (group > 1)
  const int32_t *col = nullptr;    // 32-bit columns, or null when col16 is used
  const int16_t *col16 = nullptr;  // 16-bit offsets from diag_base(row, mul), or null
  const int32_t *dia = nullptr;    // slice-diagonal form: [ncols - 1, then one offset per stored slot], or null
  const T *val = nullptr;
  const uint64_t *umask = nullptr;  // unit-row SELL (prolongations): per slice, bit l = row 64 s + l is a unit row
  const int32_t *smeta = nullptr;   // unit-row SELL: per slice, unit rows before it and explicit rows in it
  int64_t mul = 0;
  int32_t nrows = 0;
  int32_t ncols = 0;   // set by DMat::view (and for the prolongation kernels)
  int32_t unroll = 4;  // unit-row layout: entries per chunk of the prolongation loop (4 or 8)
  bool pairs = false;  // the host launches this matrix's Neumann terms as k_neumann_pairs (set by DMat::view)
};

// Unit rows of a prolongation. The row of a C point is the unit vector of its coarse index (one entry of
// value exactly 1), and coarse indices number the C points in fine order. The unit-row SELL layout stores no
// entries for those rows: within slice s, the l-th explicit row (rank l among the slice's F rows) keeps entry
// k at ptr[s] + k * m_s + l (m_s explicit rows, padded to the slice's longest explicit row), and the column
// of a unit row is the number of C points before it. Built from P and its level's C/F splitting cf; it
// applies when there is a C point and every C row has that form (always, for P of a C/F splitting), else
// the matrix keeps the plain SELL-64 layout.
struct UnitRows {
  bool ok = false;
  std::vector<uint64_t> mask;   // per slice: bit l set when row 64 s + l is a C point
  std::vector<int32_t> width;   // per slice: longest explicit row
  std::vector<int32_t> count;   // per slice: explicit rows
  std::vector<int32_t> before;  // per slice: C points before it
  std::vector<int32_t> ptr;     // per slice: first stored slot (nslices + 1 entries)
  int64_t stored = 0;           // sum over slices of width * count
};

inline UnitRows unit_rows_of(const HostCsr &P, const std::vector<int8_t> &cf) {
  UnitRows u;
  if ((int64_t)cf.size() != (int64_t)P.nr) return u;
  const int32_t nslices = (P.nr + SELL_C_UNIT - 1) / SELL_C_UNIT;
  u.mask.assign(nslices, 0);
  u.width.assign(nslices, 0);
  u.count.assign(nslices, 0);
  u.before.assign(nslices, 0);
  u.ptr.assign(nslices + 1, 0);
  int64_t units = 0;
  for (int32_t s = 0; s < nslices; ++s) {
    u.before[s] = (int32_t)units;
    for (int32_t r = s * SELL_C_UNIT; r < std::min(P.nr, (s + 1) * SELL_C_UNIT); ++r) {
      const int32_t len = P.rp[r + 1] - P.rp[r];
      if (cf[r] == 1) {
        if (len != 1 || P.v[P.rp[r]] != 1.0 || P.ci[P.rp[r]] != units) return UnitRows{};
        u.mask[s] |= uint64_t(1) << (r - s * SELL_C_UNIT);
        ++units;
      } else {
        u.width[s] = std::max(u.width[s], len);
        u.count[s]++;
      }
    }
    u.stored += (int64_t)u.width[s] * u.count[s];
    if (u.stored > INT32_MAX) return UnitRows{};
    u.ptr[s + 1] = (int32_t)u.stored;
  }
  u.ok = units > 0;
  return u;
}

// Layout tuning, read once from the environment (defaults in parentheses):
//   NAMG_LANE_ENTRIES (8): CSR lane groups are sized so that a lane takes about this many entries;
//   NAMG_LANE_ENTRIES_SMALL, NAMG_SMALL_ROWS (as NAMG_LANE_ENTRIES, 65536): the same for matrices of fewer
//   rows, whose kernels are latency-bound (shorter chains per lane);
//   NAMG_SELL_MIN_ROWS (131072): a matrix with at least this many rows uses SELL-64 whatever its row
//   length (one lane per row already fills the device);
//   NAMG_WIDE_ROWS (off): SELL-64 matrices whose rows average more entries load them in chunks of eight;
//   NAMG_UNIT_UNROLL (by row length): 4 or 8 entries per chunk for prolongations in the unit-row layout;
//   NAMG_DIA (1): 0 keeps every matrix out of the slice-diagonal form.
struct LayoutTuning {
  int lane_entries = 8;
  int lane_entries_small = 8;            // the same for matrices of fewer than small_rows rows
  int64_t small_rows = int64_t(1) << 16;
  int64_t sell_min_rows = int64_t(1) << 17;
  double wide_rows = 1e9;
  int unit_unroll = 0;  // 0: by the F rows' average length
  bool dia = true;
  // two rows per lane (DMat::pairs_ok) for triangles of at most this many slots per slice on average: at C2
  // in FP32 the level-0 triangles (3 slots) gain 11.6 -> 10.5 us per term; the level-1 triangles (about 10)
  // lose, and with them the solve reads 4.66-4.67 ms against 4.51-4.54 with one row per lane and 4.44-4.47
  // with this bound
  double dia_pairs_maxw = 4.0;
};

inline const LayoutTuning &layout_tuning() {
  static const LayoutTuning t = [] {
    LayoutTuning v;
    if (const char *e = std::getenv("NAMG_LANE_ENTRIES")) v.lane_entries = v.lane_entries_small = std::max(1, std::atoi(e));
    if (const char *e = std::getenv("NAMG_LANE_ENTRIES_SMALL")) v.lane_entries_small = std::max(1, std::atoi(e));
    if (const char *e = std::getenv("NAMG_SMALL_ROWS")) v.small_rows = std::max<int64_t>(1, std::atoll(e));
    if (const char *e = std::getenv("NAMG_SELL_MIN_ROWS")) v.sell_min_rows = std::max<int64_t>(1, std::atoll(e));
    if (const char *e = std::getenv("NAMG_WIDE_ROWS")) v.wide_rows = std::atof(e);
    if (const char *e = std::getenv("NAMG_UNIT_UNROLL")) v.unit_unroll = std::atoi(e) == 8 ? 8 : 4;
    if (const char *e = std::getenv("NAMG_DIA")) v.dia = std::atoi(e) != 0;
    if (const char *e = std::getenv("NAMG_DIA_PAIRS_MAXW")) v.dia_pairs_maxw = std::atof(e);
    return v;
  }();
  return t;
}

// FP32 Neumann terms on square slice-diagonal triangles with two rows per lane (k_neumann_pairs): on unless
// NAMG_DIA_PAIRS=0, read each time a matrix is laid out, so that one process can hold both forms.
inline bool dia_pairs_enabled() {
  const char *e = std::getenv("NAMG_DIA_PAIRS");
  return !e || std::atoi(e) != 0;
}

// Entries per chunk of the row kernels for a matrix in the given layout: 8 for a SELL-64 matrix whose rows
// average more than NAMG_WIDE_ROWS entries (fewer dependent load rounds per row), else 4.
inline int choose_unroll(int group, int64_t nrows, int64_t nnz) {
  return group == 1 && nrows > 0 && (double)nnz > layout_tuning().wide_rows * (double)nrows ? 8 : 4;
}

// Lanes per row for a matrix with the given shape: one lane when rows are short or the matrix is large enough
// to fill the device with one lane per row (NAMG_SELL_MIN_ROWS rows: at C2 one row per lane of the 175 K-row,
// 34-entry level 2 measured 0.25 ms per FP64 solve and 0.1 ms per FP32 solve faster than lane groups; from
// 16 K rows down it was slower); otherwise a power of two up to 64 that gives each lane about
// NAMG_LANE_ENTRIES entries.
inline int choose_group(int64_t nrows, int64_t nnz) {
  const LayoutTuning &t = layout_tuning();
  const double avg = nrows > 0 ? (double)nnz / (double)nrows : 0.0;
  if (avg <= 10.0 || nrows >= t.sell_min_rows) return 1;
  const int per_lane = nrows < t.small_rows ? t.lane_entries_small : t.lane_entries;
  int g = 2;
  while (g < 64 && g * per_lane < avg) g <<= 1;
  return g;
}

// The slice-diagonal form (see the layout notes above) is taken by a matrix of group 1 that is not a unit-row
// prolongation when
//   * every row's columns strictly increase (so the slots' offset order is each row's entry order),
//   * no slice's union of offsets exceeds dia_cap(its longest row), and
//   * it stores fewer bytes than SELL-64: slots x 64 x value bytes + 4 per slot, against SELL-64's
//     entries x (value bytes + column bytes).
// DMat::build, pack_device and the serving footprint all decide through LayoutCount or these functions.
__host__ __device__ inline int64_t dia_cap(int64_t longest_row) { return 2 * longest_row + 8; }
inline bool dia_wins(int64_t sell_stored, int64_t dia_stored, bool narrow, int64_t val_bytes) {
  if (!layout_tuning().dia) return false;
  const int64_t sell = sell_stored * (val_bytes + (narrow ? 2 : 4));
  const int64_t dia = dia_stored * val_bytes + 4 * (dia_stored / SELL_C + 1);
  return dia < sell;
}

// Sizes of one DMat layout, counted row by row in increasing row order (each row's col() calls, in its
// entry order, then row()): the entries, the SELL-64 storage (each slice as wide as its longest row),
// whether every column fits the 16-bit offset form, and the slice-diagonal storage (each slice as wide as
// the union of its rows' offsets) with whether that form is allowed.
struct LayoutCount {
  int64_t nnz = 0, sell_stored = 0, dia_stored = 0;
  int32_t slice_w = 0;
  bool narrow = true;
  bool dia_ok = true;  // rows strictly increasing and every completed slice within its cap
  std::vector<int32_t> row_off, prev_off, uni, merged;  // prev_off: the slice's last row that was merged

  void col(int64_t offset) {
    if (offset < -32768 || offset > 32767) narrow = false;
    if (!dia_ok) return;
    if (!row_off.empty() && offset <= row_off.back()) {
      dia_ok = false;
      return;
    }
    row_off.push_back((int32_t)offset);
  }
  void row(int32_t r, int32_t len) {
    nnz += len;
    slice_w = std::max(slice_w, len);
    // a row with the offsets of the slice's previous row adds nothing to the union (the stencil case)
    if (dia_ok && !row_off.empty() && row_off != prev_off) {
      merged.clear();
      std::set_union(uni.begin(), uni.end(), row_off.begin(), row_off.end(), std::back_inserter(merged));
      uni.swap(merged);
      prev_off.swap(row_off);
    }
    row_off.clear();
    if ((r + 1) % SELL_C == 0) {
      sell_stored += (int64_t)slice_w * SELL_C;
      if (dia_ok) {
        if ((int64_t)uni.size() > dia_cap(slice_w))
          dia_ok = false;
        else
          dia_stored += (int64_t)uni.size() * SELL_C;
      }
      uni.clear();
      prev_off.clear();
      slice_w = 0;
    }
  }
  // A whole row at once, for a count that does not consider the slice-diagonal form (dia_ok false): len
  // entries whose column offsets lie in [mn, mx]. The same sizes as col() for each entry, then row().
  void row_span(int32_t r, int32_t len, int64_t mn, int64_t mx) {
    if (len > 0 && (mn < -32768 || mx > 32767)) narrow = false;
    nnz += len;
    slice_w = std::max(slice_w, len);
    if ((r + 1) % SELL_C == 0) {
      sell_stored += (int64_t)slice_w * SELL_C;
      slice_w = 0;
    }
  }
  // the storage with the last, partial slice (nr rows counted)
  int64_t sell_total() const { return sell_stored + (int64_t)slice_w * SELL_C; }
  int64_t dia_total() const { return dia_stored + (int64_t)uni.size() * SELL_C; }
  // the slice-diagonal choice for a DMat<T> of group `group`
  template <class T>
  bool use_dia(int group) const {
    return group == 1 && dia_ok && (int64_t)uni.size() <= dia_cap(slice_w) &&
           dia_wins(sell_total(), dia_total(), narrow, sizeof(T));
  }
  // device bytes of the DMat<T> of nr rows: DMat::build's layout choice, and the size class each of its
  // buffers (pointers, column indices or slot offsets, values) allocates
  template <class T>
  int64_t bytes(int32_t nr, int force_group = 0) const {
    const int group = force_group > 0 ? force_group : choose_group(nr, nnz);
    const int64_t ib = narrow ? 2 : 4;
    if (group > 1) return alloc_bytes((int64_t)nr + 1, 4) + alloc_bytes(nnz, ib) + alloc_bytes(nnz, sizeof(T));
    const int64_t nslices = ((int64_t)nr + SELL_C - 1) / SELL_C;
    if (use_dia<T>(group)) {
      const int64_t st = dia_total();
      return alloc_bytes(nslices + 1, 4) + alloc_bytes(st / SELL_C + 1, 4) + alloc_bytes(st, sizeof(T));
    }
    const int64_t stored = sell_total();
    return alloc_bytes(nslices + 1, 4) + alloc_bytes(stored, ib) + alloc_bytes(stored, sizeof(T));
  }
};

// LayoutCount of every entry of A (allow_dia false: the slice-diagonal form is not considered, nor counted,
// and each row is counted from the range of its offsets in one tight pass).
inline LayoutCount layout_count(const HostCsr &A, bool allow_dia = true) {
  LayoutCount c;
  c.dia_ok = allow_dia;
  const int64_t mul = diag_mul(A.nr, A.nc);
  for (int32_t r = 0; r < A.nr; ++r) {
    const int32_t base = diag_base(r, mul);
    if (!allow_dia) {
      int64_t mn = INT64_MAX, mx = INT64_MIN;
      for (int32_t k = A.rp[r]; k < A.rp[r + 1]; ++k) {
        const int64_t d = (int64_t)A.ci[k] - base;
        mn = std::min(mn, d);
        mx = std::max(mx, d);
      }
      c.row_span(r, A.rp[r + 1] - A.rp[r], mn, mx);
      continue;
    }
    for (int32_t k = A.rp[r]; k < A.rp[r + 1]; ++k) c.col((int64_t)A.ci[k] - base);
    c.row(r, A.rp[r + 1] - A.rp[r]);
  }
  return c;
}

// Flag in MatView::unroll of a unit-row prolongation whose kernel takes a pair of slices per wavefront, its
// lanes first on the pair's F rows, then on its C points' rows (prolong_unit_pairs), instead of one lane per
// row (prolong_unit_rows).
constexpr int UNIT_PAIRS = 16;

// The pair form pays where a slice's F rows are about half its rows (a red-black splitting: with one lane per
// row half the lanes of the F loop idle) and the matrix fills the device; with more F rows a pair takes two
// passes of 64 lanes, and on small levels half as many wavefronts run (measured at 128^3: level 0, 50 % F
// rows, 30.4 -> 22.7 us; level 1, 83 % F rows, 14.0 -> 15.7 us; levels 2-4 2-3 us slower each).
inline bool unit_pairs_for(int64_t nrows, int64_t explicit_rows) {
  return nrows >= (int64_t(1) << 19) && 32 * explicit_rows <= 17 * nrows;
}

// Per-slice (C points before the slice, explicit rows in it) pairs of the unit-row layout.
inline std::vector<int32_t> unit_meta(const UnitRows &u) {
  std::vector<int32_t> m(2 * std::max<size_t>(u.mask.size(), 1), 0);
  for (size_t s = 0; s < u.mask.size(); ++s) {
    m[2 * s] = u.before[s];
    m[2 * s + 1] = u.count[s];
  }
  return m;
}

template <class T>
struct DMat {
  int32_t nrows = 0, ncols = 0, group = 1;
  int64_t nnz = 0, stored = 0, mul = 0;
  int64_t explicit_nnz = 0, explicit_rows = 0;  // unit-row layout: the entries and count of the explicit rows
  bool narrow = false;
  bool unit = false;  // the unit-row SELL layout (prolongations, see UnitRows)
  bool unit_pairs = false;  // its kernel in the pair form (unit_pairs_for)
  bool dia = false;   // the slice-diagonal SELL layout (see LayoutCount)
  bool pairs_ok = false;  // dia_pairs_enabled() when the matrix was laid out
  int unroll = 4;     // entries per chunk of the row kernels (choose_unroll; unit-row layout: see view())
  DevBuf<int32_t> ptr, col;
  DevBuf<int16_t> col16;
  DevBuf<T> val;
  DevBuf<uint64_t> umask;
  DevBuf<int32_t> smeta;
  DevBuf<int32_t> doff;  // slice-diagonal form: ncols - 1, then the offset of every stored slot
  MatView<T> view() const {
    MatView<T> v;
    v.ptr = ptr.get();
    v.col = (narrow || dia) ? nullptr : col.get();
    v.col16 = (narrow && !dia) ? col16.get() : nullptr;
    v.dia = dia ? doff.get() : nullptr;
    v.val = val.get();
    v.umask = unit ? umask.get() : nullptr;
    v.smeta = unit ? smeta.get() : nullptr;
    v.mul = mul;
    v.nrows = nrows;
    v.ncols = ncols;
    v.unroll = unit ? (layout_tuning().unit_unroll ? layout_tuning().unit_unroll
                                                   : (explicit_nnz > 4 * explicit_rows ? 8 : 4)) |
                          (unit_pairs ? UNIT_PAIRS : 0)
                    : unroll;
    // two rows per lane for FP32 square slice-diagonal matrices (k_neumann_pairs)
    const int64_t nslices = ((int64_t)nrows + SELL_C - 1) / SELL_C;
    v.pairs = dia && std::is_same<T, float>::value && nrows == ncols && ncols >= 2 && pairs_ok &&
              (double)stored <= layout_tuning().dia_pairs_maxw * SELL_C * (double)nslices;
    return v;
  }
  // algorithmic bytes of one pass over the matrix (entries once, row/slice pointers once; in the unit-row
  // layout the explicit rows' entries and the per-slice mask and counts, unit rows carry no entries)
  double bytes() const {
    const double nslices = (double)((nrows + SELL_C - 1) / SELL_C);
    if (unit) return (double)explicit_nnz * (sizeof(T) + (narrow ? 2.0 : 4.0)) + 4.0 * (nslices + 1.0) + 16.0 * nslices;
    if (dia) return (double)stored * sizeof(T) + 4.0 * ((double)stored / SELL_C + 1.0) + 4.0 * (nslices + 1.0);
    const double nptr = group > 1 ? (double)nrows + 1.0 : nslices + 1.0;
    return (double)nnz * (sizeof(T) + (narrow ? 2.0 : 4.0)) + 4.0 * nptr;
  }

  // unit_cf: A is a prolongation and unit_cf its level's C/F splitting; packed in the unit-row layout when
  // it applies (see UnitRows). allow_dia false: the slice-diagonal form is not considered.
  void build(const HostCsr &A, MemCounter *mc, int force_group = 0, const std::vector<int8_t> *unit_cf = nullptr,
             bool allow_dia = true) {
    nrows = A.nr;
    ncols = A.nc;
    nnz = A.nnz();
    mul = diag_mul(nrows, ncols);
    narrow = fits_col16(A);
    group = force_group > 0 ? force_group : choose_group(nrows, nnz);
    unroll = choose_unroll(group, nrows, nnz);
    unit = false;
    unit_pairs = false;
    dia = false;
    pairs_ok = dia_pairs_enabled();
    if (unit_cf && group == 1) {
      const UnitRows u = unit_rows_of(A, *unit_cf);
      if (u.ok) {
        build_unit(A, u, mc);
        return;
      }
    }
    if (allow_dia && group == 1 && layout_count(A).use_dia<T>(group)) {
      build_dia(A, mc);
      return;
    }
    std::vector<int32_t> hptr;
    std::vector<int32_t> hcol;  // wide columns (padding: column 0)
    std::vector<int16_t> h16;   // narrow offsets from the owning row's base (padding: offset 0)
    std::vector<T> hval;
    if (group > 1) {
      stored = nnz;
      hptr = A.rp;
      hval.assign(A.v.begin(), A.v.end());
      if (narrow) {
        h16.resize(nnz);
        for (int32_t r = 0; r < nrows; ++r) {
          const int32_t base = diag_base(r, mul);
          for (int32_t k = A.rp[r]; k < A.rp[r + 1]; ++k) h16[k] = (int16_t)(A.ci[k] - base);
        }
      } else {
        hcol = A.ci;
      }
    } else {
      const int32_t nslices = (nrows + SELL_C - 1) / SELL_C;
      hptr.assign(nslices + 1, 0);
      for (int32_t s = 0; s < nslices; ++s) {
        int32_t w = 0;
        for (int32_t r = s * SELL_C; r < std::min(nrows, (s + 1) * SELL_C); ++r)
          w = std::max(w, A.rp[r + 1] - A.rp[r]);
        hptr[s + 1] = hptr[s] + w * SELL_C;
      }
      stored = hptr[nslices];
      hval.resize(stored);
      if (narrow)
        h16.resize(stored);
      else
        hcol.resize(stored);
      // one pass in storage order (entry k of every row of the slice, lane by lane), so the writes stream
      // and the reads come from 64 row cursors
      for (int32_t s = 0; s < nslices; ++s) {
        const int32_t r0 = s * SELL_C;
        const int32_t width = (hptr[s + 1] - hptr[s]) / SELL_C;
        int64_t d = hptr[s];
        for (int32_t k = 0; k < width; ++k) {
          for (int32_t lane = 0; lane < SELL_C; ++lane, ++d) {
            const int32_t r = r0 + lane;
            const bool has = r < nrows && k < A.rp[r + 1] - A.rp[r];
            const int32_t c = has ? A.ci[A.rp[r] + k] : -1;
            hval[d] = has ? (T)A.v[A.rp[r] + k] : T(0);
            if (narrow)
              h16[d] = has ? (int16_t)(c - diag_base(r, mul)) : (int16_t)0;
            else
              hcol[d] = has ? c : 0;
          }
        }
      }
    }
    ptr.alloc(hptr.size(), mc);
    ptr.upload(hptr.data(), hptr.size());
    if (narrow) {
      col16.alloc(h16.size(), mc);
      col16.upload(h16.data(), h16.size());
    } else {
      col.alloc(hcol.size(), mc);
      col.upload(hcol.data(), hcol.size());
    }
    val.alloc(hval.size(), mc);
    val.upload(hval.data(), hval.size());
  }

  // The slice-diagonal layout of A (LayoutCount::use_dia holds): slice s stores its union
  // of offsets in increasing order, slot k at ptr[s] + 64 k (entries) and doff[1 + ptr[s] / 64 + k] (offset);
  void build_dia(const HostCsr &A, MemCounter *mc) {
    dia = true;
    group = 1;
    unroll = 4;  // not used by the slice-diagonal kernels (they chunk by the slice's width)
    const int32_t nslices = (nrows + SELL_C - 1) / SELL_C;
    std::vector<int32_t> hptr(nslices + 1, 0);
    std::vector<int32_t> hoff(1, ncols - 1);
    std::vector<int32_t> uni, merged, ro;
    for (int32_t s = 0; s < nslices; ++s) {
      uni.clear();
      for (int32_t r = s * SELL_C; r < std::min(nrows, (s + 1) * SELL_C); ++r) {
        merged.clear();
        ro.clear();
        const int32_t base = diag_base(r, mul);
        for (int32_t k = A.rp[r]; k < A.rp[r + 1]; ++k) ro.push_back(A.ci[k] - base);
        std::set_union(uni.begin(), uni.end(), ro.begin(), ro.end(), std::back_inserter(merged));
        uni.swap(merged);
      }
      hptr[s + 1] = hptr[s] + (int32_t)uni.size() * SELL_C;
      hoff.insert(hoff.end(), uni.begin(), uni.end());
    }
    stored = hptr[nslices];
    std::vector<T> hval(stored, T(0));
    for (int32_t s = 0; s < nslices; ++s) {
      const int32_t *o = hoff.data() + 1 + hptr[s] / SELL_C;
      const int32_t w = (hptr[s + 1] - hptr[s]) / SELL_C;
      for (int32_t r = s * SELL_C; r < std::min(nrows, (s + 1) * SELL_C); ++r) {
        int32_t j = 0;
        for (int32_t k = A.rp[r]; k < A.rp[r + 1]; ++k) {
          while (j < w && o[j] != A.ci[k] - diag_base(r, mul)) ++j;
          hval[(int64_t)hptr[s] + (int64_t)j * SELL_C + (r - s * SELL_C)] = (T)A.v[k];
        }
      }
    }
    ptr.alloc(hptr.size(), mc);
    ptr.upload(hptr.data(), hptr.size());
    doff.alloc(hoff.size(), mc);
    doff.upload(hoff.data(), hoff.size());
    val.alloc(hval.size(), mc);
    val.upload(hval.data(), hval.size());
  }

  // The unit-row SELL layout of A (u = unit_rows_of(A), u.ok): per slice the explicit rows' entries, entry k
  // of the l-th explicit row at ptr[s] + k * count_s + l; padding value 0 with offset 0 or column 0.
  void build_unit(const HostCsr &A, const UnitRows &u, MemCounter *mc) {
    unit = true;
    group = 1;
    const int32_t nslices = (int32_t)u.mask.size();
    const std::vector<int32_t> &hptr = u.ptr;
    const std::vector<int32_t> hmeta = unit_meta(u);
    stored = u.stored;
    explicit_nnz = 0;
    explicit_rows = 0;
    for (int32_t c : u.count) explicit_rows += c;
    unit_pairs = unit_pairs_for(nrows, explicit_rows);
    std::vector<T> hval(stored);
    std::vector<int32_t> hcol;
    std::vector<int16_t> h16;
    if (narrow)
      h16.assign(stored, 0);
    else
      hcol.assign(stored, 0);
    for (int32_t s = 0; s < nslices; ++s) {
      int32_t l = 0;
      for (int32_t r = s * SELL_C; r < std::min(nrows, (s + 1) * SELL_C); ++r) {
        if ((u.mask[s] >> (r - s * SELL_C)) & 1) continue;
        const int32_t len = A.rp[r + 1] - A.rp[r];
        const int32_t base = diag_base(r, mul);
        explicit_nnz += len;
        for (int32_t k = 0; k < u.width[s]; ++k) {
          const int64_t d = (int64_t)hptr[s] + (int64_t)k * u.count[s] + l;
          const bool has = k < len;
          hval[d] = has ? (T)A.v[A.rp[r] + k] : T(0);
          if (narrow)
            h16[d] = has ? (int16_t)(A.ci[A.rp[r] + k] - base) : (int16_t)0;
          else
            hcol[d] = has ? A.ci[A.rp[r] + k] : 0;
        }
        ++l;
      }
    }
    ptr.alloc(hptr.size(), mc);
    ptr.upload(hptr.data(), hptr.size());
    umask.alloc(std::max<size_t>(u.mask.size(), 1), mc);
    umask.upload(u.mask.data(), u.mask.size());
    smeta.alloc(hmeta.size(), mc);
    smeta.upload(hmeta.data(), hmeta.size());
    if (narrow) {
      col16.alloc(h16.size(), mc);
      col16.upload(h16.data(), h16.size());
    } else {
      col.alloc(hcol.size(), mc);
      col.upload(hcol.data(), hcol.size());
    }
    val.alloc(hval.size(), mc);
    val.upload(hval.data(), hval.size());
  }
};

// CSR rows grouped by dependency level, for the level-scheduled direct triangular solves. The rows are
// stored in schedule order (position q holds row order[q] with its entries in their CSR order), so a
// thread finds its row's entries from its position alone and the row index and the entry range load
// in parallel.
template <class T>
struct DTri {
  int32_t n = 0;
  DevBuf<int32_t> rp, ci, order;  // rp, ci, val: rows in schedule order
  DevBuf<T> val;
  std::vector<int32_t> lev_ptr;  // host copy: positions lev_ptr[k] .. lev_ptr[k+1] form level k
  int64_t nnz = 0;

  void build(const HostCsr &S, const LevelSchedule &sch, MemCounter *mc) {
    n = S.nr;
    nnz = S.nnz();
    std::vector<int32_t> hrp(n + 1, 0), hci;
    std::vector<T> hv;
    hci.reserve(S.ci.size());
    hv.reserve(S.v.size());
    for (int32_t q = 0; q < n; ++q) {
      const int32_t i = sch.order[q];
      for (int32_t k = S.rp[i]; k < S.rp[i + 1]; ++k) {
        hci.push_back(S.ci[k]);
        hv.push_back((T)S.v[k]);
      }
      hrp[q + 1] = (int32_t)hci.size();
    }
    rp.alloc(hrp.size(), mc);
    rp.upload(hrp.data(), hrp.size());
    ci.alloc(hci.size(), mc);
    ci.upload(hci.data(), hci.size());
    val.alloc(hv.size(), mc);
    val.upload(hv.data(), hv.size());
    order.alloc(sch.order.size(), mc);
    order.upload(sch.order.data(), sch.order.size());
    lev_ptr = sch.ptr;
  }
};

// Low-synchronization GMRES state kept on the device (FP64), written by the single-workgroup step
// kernel and read by the projection and update kernels.
constexpr int KS_MAXR = NAMG_MAX_RESTART;
constexpr int KS_LD = KS_MAXR + 2;

struct KState {
  double est;      // |g_{i+1}| / ||b|| after the latest column
  double rho;      // ||v_{i+1}||, the lagged norm of the current step
  double rho_inv;  // 1 / rho (0 on breakdown)
  int32_t flag;    // 0 continue, 1 stop (converged / last column / breakdown), -1 non-finite
  int32_t pad;
  double s[KS_LD];      // projection coefficients of the latest step (top of the pending H column)
  double g[KS_LD];      // rotated right-hand side
  double cs[KS_LD], sn[KS_LD];
  double zs[KS_LD];     // lagged normalisation factors of z_j, folded into y
  double y[KS_LD];      // y_j * zs_j after the back-substitution
  double H[KS_LD * KS_LD];  // rotated Hessenberg, column j at H[j * KS_LD + row]
  double L[KS_LD * KS_LD];  // strictly lower L, row r at L[r * KS_LD + col]
};

}  // namespace namg

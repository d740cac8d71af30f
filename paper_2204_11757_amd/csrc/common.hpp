// Internal declarations of the gfx950 coarsening library: device helpers
// for 64-lane wavefronts, the context, the workspace arena and the
// host-side launch plumbing.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "spc.h"

namespace spc {

constexpr int WAVE = 64;
constexpr uint64_t KEY_INF = ~0ull;

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  return (1ull << lane_id()) - 1ull;
}

// Wave-aggregated append: every active lane with pred gets a distinct slot
// in [*counter, *counter + popcount) with one atomic per wave.
__device__ __forceinline__ int64_t wave_append(unsigned long long* counter, bool pred) {
  uint64_t mask = __ballot(pred);
  if (mask == 0) return -1;
  int leader = __ffsll((long long)mask) - 1;
  unsigned long long base = 0;
  if (lane_id() == leader) base = atomicAdd(counter, (unsigned long long)__popcll(mask));
  base = __shfl(base, leader);
  return pred ? (int64_t)(base + __popcll(mask & lanemask_lt())) : -1;
}

template <typename T>
__device__ __forceinline__ T wave_incl_sum(T v) {
  int l = lane_id();
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    T t = __shfl_up(v, o);
    if (l >= o) v += t;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_incl_max(T v) {
  int l = lane_id();
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    T t = __shfl_up(v, o);
    if (l >= o) v = (t > v) ? t : v;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    T t = __shfl_xor(v, o);
    v = (t > v) ? t : v;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    T t = __shfl_xor(v, o);
    v = (t < v) ? t : v;
  }
  return v;
}

// Block-wide inclusive scan (sum or max) for BS threads; tmp: LDS T[BS/64].
// Returns the inclusive value; *total receives the block total.
template <typename T, int BS, bool MAX>
__device__ __forceinline__ T block_incl_scan(T v, T* tmp, T* total) {
  constexpr int NW = BS / WAVE;
  int w = threadIdx.x / WAVE, l = lane_id();
  T x = MAX ? wave_incl_max(v) : wave_incl_sum(v);
  if (l == WAVE - 1) tmp[w] = x;
  __syncthreads();
  if (w == 0) {
    T y;
    if (MAX) {
      y = (l < NW) ? tmp[l] : tmp[0];
      y = wave_incl_max(y);
    } else {
      y = (l < NW) ? tmp[l] : (T)0;
      y = wave_incl_sum(y);
    }
    if (l < NW) tmp[l] = y;
  }
  __syncthreads();
  T pre = (w > 0) ? tmp[w - 1] : (T)0;
  T res;
  if (MAX) res = (w > 0 && pre > x) ? pre : x;
  else res = x + pre;
  if (total) *total = tmp[NW - 1];
  __syncthreads();
  return res;
}

// Largest r in [0, nrows) with ptr[r] <= x, for a nondecreasing ptr with
// ptr[0] <= x.  Executed by one full wave (64 lanes active); every lane
// returns the result.  A 64-ary search: ~log64(nrows) rounds of loads.
__device__ __forceinline__ int64_t wave_upper_search(const int64_t* __restrict__ ptr, int64_t nrows,
                                                     int64_t x) {
  int64_t lo = 0, hi = nrows - 1;
  int l = lane_id();
  while (hi - lo >= WAVE) {
    int64_t step = (hi - lo + WAVE - 1) / WAVE;
    int64_t pos = lo + (int64_t)l * step;
    if (pos > hi) pos = hi;
    bool pred = (l == 0) || (ptr[pos] <= x);
    uint64_t mask = __ballot(pred);
    int k = __popcll(mask) - 1;  // pred is monotone in l
    int64_t nlo = lo + (int64_t)k * step;
    if (nlo > hi) nlo = hi;
    int64_t nhi = (k == WAVE - 1) ? hi : lo + (int64_t)(k + 1) * step - 1;
    if (nhi > hi) nhi = hi;
    lo = nlo;
    hi = nhi;
  }
  int64_t pos = lo + l;
  bool pred = (pos <= hi) && ((l == 0) || ptr[pos] <= x);
  uint64_t mask = __ballot(pred);
  return lo + __popcll(mask) - 1;
}

// atomicMax on a value many blocks raise: a block whose candidate does not
// exceed the value already visible skips the atomic (a stale read only costs
// an unneeded atomic)
__device__ __forceinline__ void atomic_max_lazy(unsigned long long* p, unsigned long long v) {
  if (v > __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(p, v);
}

__device__ __forceinline__ void atomic_min_lazy(unsigned long long* p, unsigned long long v) {
  if (v < __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(p, v);
}

// LDS layout of a tile's row map: thread t owns positions [t*PER, t*PER+PER)
// during the scan; one pad word per PER positions keeps those reads free of
// bank conflicts.
template <int T, int BS>
struct Lbs {
  static constexpr int PER = T / BS;
  static constexpr int SIZE = T + BS;
  __device__ __forceinline__ static int at(int k) { return k + k / PER; }
};

// Workgroups are dispatched round-robin over the chip's 8 XCDs, each with its
// own L2.  xcd_tile renumbers block b of G so that every XCD takes one
// contiguous run of tiles: neighbouring tiles, which read and write the same
// cache lines (mirror entries, neighbouring rows), then share an L2.  It is
// a bijection on [0, G) for any G.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t G) {
  int64_t x = b & 7, i = b >> 3, q = G >> 3, r = G & 7;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Load-balanced mapping of a tile of T consecutive positions
// [p0, p0 + T) of a CSR-like prefix array ptr[0..nrows] onto rows:
// srow[Lbs<T,BS>::at(k)] = row containing position p0 + k (srow holds
// Lbs<T,BS>::SIZE words).  Called by all BS threads.  lbs_fill is given the
// rows r0 <= r1 that hold the tile's first and last positions (r1 may be
// any later row: rows starting at or past the tile's end are skipped);
// lbs_tile finds them by searching ptr.
template <int T, int BS>
__device__ __forceinline__ void lbs_fill(const int64_t* __restrict__ ptr, int64_t r0, int64_t r1, int64_t p0,
                                         int32_t* srow, int32_t* scan_tmp) {
  using L = Lbs<T, BS>;
  int tid = threadIdx.x;
  for (int k = tid; k < T; k += BS) srow[L::at(k)] = (int32_t)r0;
  __syncthreads();
  for (int64_t r = r0 + 1 + tid; r <= r1; r += BS) {
    int64_t p = ptr[r] - p0;
    if (p > 0 && p < T) atomicMax(&srow[L::at((int)p)], (int32_t)r);
  }
  __syncthreads();
  // inclusive max-scan over srow
  constexpr int PER = L::PER;
  static_assert(T % BS == 0, "tile must be a multiple of the block");
  int32_t loc[PER];
  int32_t run = INT32_MIN;
#pragma unroll
  for (int i = 0; i < PER; i++) {
    int32_t v = srow[L::at(tid * PER + i)];
    run = v > run ? v : run;
    loc[i] = run;
  }
  int32_t tot;
  int32_t inc = block_incl_scan<int32_t, BS, true>(run, scan_tmp, &tot);
  // exclusive prefix-max for this thread = max over earlier threads
  int32_t prev = __shfl_up(inc, 1);
  int w = tid / WAVE;
  if (lane_id() == 0) prev = (w > 0) ? scan_tmp[w - 1] : INT32_MIN;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; i++) {
    int32_t v = loc[i] > prev ? loc[i] : prev;
    srow[L::at(tid * PER + i)] = v;
  }
  __syncthreads();
}

template <int T, int BS>
__device__ __forceinline__ void lbs_tile(const int64_t* __restrict__ ptr, int64_t nrows, int64_t p0,
                                         int32_t* srow, int64_t* sh, int32_t* scan_tmp) {
  static_assert(BS >= 2 * WAVE, "the tile's first and last rows are searched by two wavefronts");
  int tid = threadIdx.x;
  if (tid < WAVE) {
    int64_t r0 = wave_upper_search(ptr, nrows, p0);
    if (tid == 0) sh[0] = r0;
  } else if (tid < 2 * WAVE) {
    int64_t total = ptr[nrows];
    int64_t last = p0 + T - 1;
    if (last > total - 1) last = total - 1;
    int64_t r1 = wave_upper_search(ptr, nrows, last);
    if (tid == WAVE) sh[1] = r1;
  }
  __syncthreads();
  lbs_fill<T, BS>(ptr, sh[0], sh[1], p0, srow, scan_tmp);
}

// ---------------------------------------------------------------------------
// union-find with hooking of the larger root under the smaller one, so the
// root of every tree is its smallest member
// ---------------------------------------------------------------------------
// The root of x given p, a value of parent[x] already read (parent
// pointers only ever move towards the root, so any earlier value will do).
__device__ __forceinline__ int32_t uf_find_from(int32_t* parent, int32_t x, int32_t p) {
  while (p != x) {
    int32_t gp = __hip_atomic_load(&parent[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (gp != p) {
      // path halving: parent pointers only ever move towards the root
      __hip_atomic_store(&parent[x], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    x = p;
    p = gp;
  }
  return x;
}

__device__ __forceinline__ int32_t uf_find(int32_t* parent, int32_t x) {
  int32_t p = __hip_atomic_load(&parent[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  while (p != x) {
    int32_t gp = __hip_atomic_load(&parent[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (gp != p) {
      // path halving: parent pointers only ever move towards the root
      __hip_atomic_store(&parent[x], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    x = p;
    p = gp;
  }
  return x;
}

__device__ __forceinline__ void uf_union(int32_t* parent, int32_t a, int32_t b) {
  while (true) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a > b) {
      int32_t t = a;
      a = b;
      b = t;
    }
    int32_t old = atomicCAS(&parent[b], b, a);
    if (old == b) return;
  }
}

__host__ __device__ __forceinline__ int bitlen64(uint64_t x) {
  return x ? 64 - __builtin_clzll(x) : 0;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct Arena {
  char* base = nullptr;
  size_t cap = 0, off = 0;
  bool counting = false;
  template <typename T>
  T* take(size_t count) {
    size_t a = (off + 255) & ~(size_t)255;
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = sizeof(T);
    off = a + bytes;
    if (counting || base == nullptr) return nullptr;
    if (off > cap) return nullptr;
    return reinterpret_cast<T*>(base + a);
  }
};

}  // namespace spc

// Launch settings that results never depend on (spc_autotune picks them per
// size class of the input; 0 = the built-in rule).
struct spc_tune {
  int lane_max = 32;      // contraction rows of 17..lane_max records: one thread each (16 or 32)
  int wave_max = 512;     // rows up to wave_max records: one wavefront each; larger: one block
  int small_rpt = 0;      // rows per thread of the small-row contraction (1, 2, 4)
  int huge_tile = 0;      // records per tile of the dense huge-row accumulation (1024, 4096)
  int sel_blocks = 0;     // blocks of the radix select (at most 128)
  int64_t bv_short = 0;   // live lists up to this length: 4 items per thread in the hooking pass
};

struct spc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  void* (*alloc_fn)(size_t, void*) = nullptr;
  void (*free_fn)(void*, void*) = nullptr;
  void* alloc_user = nullptr;
  void* ws = nullptr;
  size_t ws_cap = 0;
  int64_t* h_pinned = nullptr;  // pinned readback area (host-coherent)
  int64_t rb_token = 0;         // last token a readback published in h_pinned
  int err_code = 0;
  std::string err;
  int num_cus = 256;
  uint64_t* scan_state = nullptr;  // look-back words of the single-pass scan
  int64_t scan_cap = 0;            // words
  uint32_t scan_epoch = 0;
  uint32_t lb_epoch = 0;       // last look-back epoch handed out
  int64_t lb_words = 0;        // size of the current level's look-back array
  unsigned long long sel_epoch = 0;   // radix-select barrier epochs handed out this level
  int forest_batch = 2;        // forest rounds issued before the first wait (from the last level)
  int forest_batch_cls[64] = {};   // the same per input size class (bit length of nnz; 0: none yet)
  // knobs
  int force_rank_mode = 0;   // use the sorted-rank order even when a packed key fits
  int force_full_filter = 0; // run the spanning-forest phase over every edge
  int seg_full_band = 0;     // a batch's level redone over every edge (a band fell short)
  int seg_band_shrink = 0;   // test option: batch bands aim at a quarter of the merges
  int force_huge_sort = 0;   // contract huge rows by sorting even when dense accumulators fit
  int force_redo_rank = 0;   // flag every packed-key level as inexact (redone with rank keys)
  int force_bad_guess = 0;   // give the cutoff selection key bounds that some keys lie outside
  int force_scan_flag = 0;   // the next level finds the scan chain's error flag raised (once)
  // launch settings in effect, and the tuned ones per size class (key:
  // bit length of the input's nnz, plus 64 for batches)
  spc_tune tune;
  std::vector<std::pair<int, spc_tune>> tuned;
  spc_tune tune_set{0, 0, 0, 0, 0, 0};   // settings fixed by spc_set_option (0: not fixed)
  int tune_forced = 0;       // spc_autotune's trials: keep ctx->tune as set
  // the entry point that allocates nothing: this device's scratch array
  // (resolved once per device at creation; null if that failed) and, during
  // such a call, 1 so that nothing on the level path allocates
  void* scratch = nullptr;
  int no_alloc = 0;
  int contract_wait = 0;     // 0: as the last level suggests, 1: the host reads the row-class counts
                             // before the class kernels, 2: never (when the huge rows fit)
  int contract_dev = 0;      // the last level's row classes suited the contraction without that wait
  int contract_classes_seen = 7;  // row classes (1: 32-entry, 2: wavefront, 4: block) the last level had
  int spec_ok = 0;           // the last level's forest was complete after its first batch, in one band
  int speculate = 0;         // 0: as spec_ok says, 1: never, 2: always, with a one-round first batch
  // per-kernel timing: events recorded around launches on the context stream
  int timing = 0;
  std::vector<hipEvent_t> ev_pool;
  struct Mark {
    const char* name;
    hipEvent_t a, b;
    double units;
  };
  std::vector<Mark> marks;
};

namespace spc {

inline hipEvent_t ev_get(spc_ctx* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records an event pair around the launches in its scope when timing is on.
// `units` is the work the launch covers (edges, nodes, ...) for reports.
struct TimedScope {
  spc_ctx* ctx;
  const char* name;
  double units;
  hipEvent_t a = nullptr;
  TimedScope(spc_ctx* c, const char* nm, double u = 0.0) : ctx(c), name(nm), units(u) {
    if (ctx->timing) {
      a = ev_get(ctx);
      if (a) (void)hipEventRecord(a, ctx->stream);
    }
  }
  ~TimedScope() {
    if (!a) return;
    hipEvent_t b = ev_get(ctx);
    if (!b) return;
    (void)hipEventRecord(b, ctx->stream);
    ctx->marks.push_back({name, a, b, units});
  }
};

}  // namespace spc

namespace spc {

int set_error(spc_ctx* ctx, int code, const char* fmt, ...);
int hip_error(spc_ctx* ctx, hipError_t e, const char* where);
void* dev_alloc(spc_ctx* ctx, size_t bytes);
void dev_free(spc_ctx* ctx, void* p);
int ensure_workspace(spc_ctx* ctx, size_t bytes);
int readback(spc_ctx* ctx, const void* dev, size_t bytes, void* host);

#define SPC_HIP(ctx, call)                                   \
  do {                                                       \
    hipError_t e__ = (call);                                 \
    if (e__ != hipSuccess) return ::spc::hip_error(ctx, e__, #call); \
  } while (0)

#define SPC_LAUNCH_CHECK(ctx, name)                          \
  do {                                                       \
    hipError_t e__ = hipGetLastError();                      \
    if (e__ != hipSuccess) return ::spc::hip_error(ctx, e__, name); \
  } while (0)

inline int grid_for(int64_t items, int per_block, int cap = 1 << 30) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace spc

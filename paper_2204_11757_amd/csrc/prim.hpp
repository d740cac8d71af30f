// Device-wide primitives: exclusive scan, radix select of the k-th smallest
// 64-bit key, and a merge sort with an arbitrary strict-weak comparator.
#pragma once

#include "common.hpp"

namespace spc {

// Stream compaction without a hot counter.  A single global counter that
// every block bumps serialises all blocks of a launch on one address; a
// decoupled look-back (Merrill and Garland, single-pass prefix scan with
// decoupled look-back, 2016) lets tile b find the sum of the counts of
// tiles 0..b-1 from its predecessors' published words instead.
//
// A state word is (epoch << 42) | (flag << 40) | value: flag 1 = the tile's
// own count, 2 = the inclusive prefix through the tile.  Words of an older
// epoch count as unpublished, so the array is zeroed once per level and
// every launch takes a fresh epoch.  A tile waits only on lower tiles, which
// the hardware dispatched before it and which publish before they wait, so
// every wait ends; a bound on the polling turns a broken invariant into an
// error flag instead of a hang.
constexpr uint64_t LB_VMASK = (1ull << 40) - 1;
constexpr uint32_t LB_MAX_EPOCH = (1u << 22) - 1;
constexpr uint32_t LB_SPIN_LIMIT = 1u << 20;

struct TileScan {
  uint64_t* state;            // [tiles] words of this chain
  uint32_t epoch;             // 1 .. LB_MAX_EPOCH, distinct per launch
  unsigned long long* err;    // set to 1 when a wait gives up
};

__device__ __forceinline__ void lb_publish(uint64_t* p, uint32_t epoch, uint64_t flag, uint64_t v) {
  __hip_atomic_store(p, ((uint64_t)epoch << 42) | (flag << 40) | (v & LB_VMASK), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of the counts of tiles 0..tile-1, computed by one whole wavefront:
// each probe reads the words of the 64 preceding tiles at once and stops at
// the nearest inclusive prefix (positions before tile 0 read as an
// inclusive prefix of 0).  Every lane returns the sum.
__device__ __forceinline__ uint64_t lb_exclusive_wave(const TileScan& ts, int64_t tile, uint64_t count) {
  int lane = lane_id();
  if (tile == 0) {
    if (lane == 0) lb_publish(&ts.state[0], ts.epoch, 2, count);
    return 0;
  }
  if (lane == 0) lb_publish(&ts.state[tile], ts.epoch, 1, count);
  uint64_t excl = 0;
  int64_t p0 = tile - 1;
  uint32_t spins = 0;
  while (true) {
    int64_t p = p0 - lane;
    uint64_t s = p >= 0 ? __hip_atomic_load(&ts.state[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                        : (((uint64_t)ts.epoch << 42) | (2ull << 40));
    bool pub = (uint32_t)(s >> 42) == ts.epoch;
    bool incl = pub && ((s >> 40) & 3) == 2;
    uint64_t incl_mask = __ballot(incl);
    uint64_t unpub_mask = __ballot(!pub);
    int first = incl_mask ? __ffsll((long long)incl_mask) - 1 : WAVE;
    uint64_t need = (first >= WAVE - 1) ? ~0ull : ((2ull << first) - 1);
    if (unpub_mask & need) {
      if (++spins > LB_SPIN_LIMIT) {
        if (lane == 0) atomicOr(ts.err, 1ull);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    excl += wave_sum<uint64_t>(lane <= first ? (s & LB_VMASK) : 0ull);
    if (first < WAVE) break;
    p0 -= WAVE;
  }
  if (lane == 0) lb_publish(&ts.state[tile], ts.epoch, 2, excl + count);
  return excl;
}

// Single-thread form for callers that run one chain per lane.
__device__ __forceinline__ uint64_t lb_exclusive(const TileScan& ts, int64_t tile, uint64_t count) {
  if (tile == 0) {
    lb_publish(&ts.state[0], ts.epoch, 2, count);
    return 0;
  }
  lb_publish(&ts.state[tile], ts.epoch, 1, count);
  uint64_t excl = 0;
  int64_t p = tile - 1;
  uint32_t spins = 0;
  while (true) {
    uint64_t s = __hip_atomic_load(&ts.state[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((uint32_t)(s >> 42) != ts.epoch) {
      if (++spins > LB_SPIN_LIMIT) {
        atomicOr(ts.err, 1ull);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    excl += s & LB_VMASK;
    if (((s >> 40) & 3) == 2) break;
    p--;
  }
  lb_publish(&ts.state[tile], ts.epoch, 2, excl + count);
  return excl;
}

// Block-wide reservation of `my` consecutive slots per thread, positions in
// tile order.  base_in (nullable) is added to every position: it is read
// before the tile publishes, so it may be the same counter as total_out,
// which the last tile sets to base_in + the sum of all counts.  All BS
// threads must call it.  tmp: LDS int[BS/64]; sh_base: LDS scalar.
template <int BS>
__device__ __forceinline__ int64_t block_reserve_lb(const TileScan& ts, int64_t tile, bool last_tile,
                                                    int my, const unsigned long long* base_in,
                                                    unsigned long long* total_out,
                                                    unsigned long long* sh_base, int* tmp) {
  int total;
  int incl = block_incl_scan<int, BS, false>(my, tmp, &total);
  if (threadIdx.x < WAVE) {
    uint64_t b0 = 0;
    if (base_in) {
      b0 = __hip_atomic_load(base_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();   // the read completes before this tile publishes
    }
    uint64_t ex = b0 + lb_exclusive_wave(ts, tile, (uint64_t)total);
    if (threadIdx.x == 0) {
      *sh_base = ex;
      if (last_tile) *total_out = ex + (uint64_t)total;
    }
  }
  __syncthreads();
  int64_t base = (int64_t)*sh_base + (incl - my);
  __syncthreads();
  return base;
}

// ===========================================================================
// exclusive scan: out[i] = sum in[0..i), out[n] = total (out has n+1 slots).
// One pass over tiles of SCAN_TILE items chained by the decoupled look-back
// of the compaction (level.hpp): sums travel in the 40-bit value field, so
// the inputs must be non-negative with a total below 2^40 (every scan here
// counts entries or adds integer weights, all below 2^31); a larger total
// sets the error flag.
// ===========================================================================
constexpr int SCAN_BS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BS * SCAN_ITEMS;
constexpr int SCAN_MAXB = 1024;   // size of the callers' legacy scratch (unused)

// With rb.out set, the last tile also copies to host-visible memory what the
// host reads after the scan: rb.ninfo words of rb.info, then the total, *rb.x1
// (or 0) and the chain's error word, at rb.out[0..ninfo+3); then, after a
// system-scope fence, rb.token (when nonzero) at rb.out[ninfo+3], which the
// host polls instead of waiting for the stream.
struct ScanReadback {
  const unsigned long long* info;
  int ninfo;
  const int32_t* x1;
  int64_t* out;
  int64_t token;
};

template <typename T>
__global__ void __launch_bounds__(SCAN_BS)
    k_scan_lb(const T* in, T* out, int64_t n, TileScan ts, ScanReadback rb) {
  __shared__ T buf[SCAN_TILE];
  __shared__ T tmp[SCAN_BS / WAVE];
  __shared__ T sh_excl;
  int tid = threadIdx.x;
  int64_t tile = blockIdx.x;
  int64_t base = tile * SCAN_TILE;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) {
    int64_t g = base + i * SCAN_BS + tid;
    buf[i * SCAN_BS + tid] = g < n ? in[g] : (T)0;
  }
  __syncthreads();
  T loc[SCAN_ITEMS];
  T run = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) {
    loc[i] = run;
    run += buf[tid * SCAN_ITEMS + i];
  }
  T tot;
  T inc = block_incl_scan<T, SCAN_BS, false>(run, tmp, &tot);
  if (tid < WAVE) {
    uint64_t ex = lb_exclusive_wave(ts, tile, (uint64_t)tot);
    if (tid == 0) {
      if ((uint64_t)tot > LB_VMASK || ex + (uint64_t)tot > LB_VMASK) atomicOr(ts.err, 1ull);
      sh_excl = (T)ex;
      if (tile == gridDim.x - 1) {
        out[n] = (T)(ex + (uint64_t)tot);
        if (rb.out) {
          for (int i = 0; i < rb.ninfo; i++) rb.out[i] = (int64_t)rb.info[i];
          rb.out[rb.ninfo] = (int64_t)(ex + (uint64_t)tot);
          rb.out[rb.ninfo + 1] = rb.x1 ? (int64_t)*rb.x1 : 0;
          rb.out[rb.ninfo + 2] =
              (int64_t)__hip_atomic_load(ts.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __threadfence_system();
          if (rb.token)
            __hip_atomic_store(&rb.out[rb.ninfo + 3], rb.token, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
      }
    }
  }
  __syncthreads();
  T pre = sh_excl + inc - run;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) buf[tid * SCAN_ITEMS + i] = pre + loc[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) {
    int64_t g = base + i * SCAN_BS + tid;
    if (g < n) out[g] = buf[i * SCAN_BS + tid];
  }
}

// Two exclusive scans of the same length in one launch (each tile scans
// both arrays; wavefront 0 runs the first chain's look-back, wavefront 1 the
// second's, side by side).
template <typename T1, typename T2>
__global__ void __launch_bounds__(SCAN_BS)
    k_scan2_lb(const T1* in1, T1* out1, const T2* in2, T2* out2, int64_t n, TileScan ts1, TileScan ts2) {
  static_assert(SCAN_BS >= 2 * WAVE, "two wavefronts run the chains");
  __shared__ T1 buf1[SCAN_TILE];
  __shared__ T2 buf2[SCAN_TILE];
  __shared__ T1 tmp1[SCAN_BS / WAVE];
  __shared__ T2 tmp2[SCAN_BS / WAVE];
  __shared__ T1 sh1;
  __shared__ T2 sh2;
  int tid = threadIdx.x;
  int64_t tile = blockIdx.x;
  int64_t base = tile * SCAN_TILE;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) {
    int64_t g = base + i * SCAN_BS + tid;
    buf1[i * SCAN_BS + tid] = g < n ? in1[g] : (T1)0;
    buf2[i * SCAN_BS + tid] = g < n ? in2[g] : (T2)0;
  }
  __syncthreads();
  T1 loc1[SCAN_ITEMS];
  T2 loc2[SCAN_ITEMS];
  T1 run1 = 0;
  T2 run2 = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) {
    loc1[i] = run1;
    loc2[i] = run2;
    run1 += buf1[tid * SCAN_ITEMS + i];
    run2 += buf2[tid * SCAN_ITEMS + i];
  }
  T1 tot1;
  T2 tot2;
  T1 inc1 = block_incl_scan<T1, SCAN_BS, false>(run1, tmp1, &tot1);
  T2 inc2 = block_incl_scan<T2, SCAN_BS, false>(run2, tmp2, &tot2);
  if (tid < WAVE) {
    uint64_t ex = lb_exclusive_wave(ts1, tile, (uint64_t)tot1);
    if (tid == 0) {
      if ((uint64_t)tot1 > LB_VMASK || ex + (uint64_t)tot1 > LB_VMASK) atomicOr(ts1.err, 1ull);
      sh1 = (T1)ex;
      if (tile == gridDim.x - 1) out1[n] = (T1)(ex + (uint64_t)tot1);
    }
  } else if (tid < 2 * WAVE) {
    uint64_t ex = lb_exclusive_wave(ts2, tile, (uint64_t)tot2);
    if (tid == WAVE) {
      if ((uint64_t)tot2 > LB_VMASK || ex + (uint64_t)tot2 > LB_VMASK) atomicOr(ts2.err, 1ull);
      sh2 = (T2)ex;
      if (tile == gridDim.x - 1) out2[n] = (T2)(ex + (uint64_t)tot2);
    }
  }
  __syncthreads();
  T1 pre1 = sh1 + inc1 - run1;
  T2 pre2 = sh2 + inc2 - run2;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) {
    buf1[tid * SCAN_ITEMS + i] = pre1 + loc1[i];
    buf2[tid * SCAN_ITEMS + i] = pre2 + loc2[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) {
    int64_t g = base + i * SCAN_BS + tid;
    if (g < n) {
      out1[g] = buf1[i * SCAN_BS + tid];
      out2[g] = buf2[i * SCAN_BS + tid];
    }
  }
}

// Makes room for `words` look-back words in the context (zeroed) and
// returns a fresh epoch; 0 on allocation failure.
uint32_t scan_state_reserve(spc_ctx* ctx, int64_t words);

// Zeroes `bytes` (a multiple of 4) at device address p with a kernel on the
// context's stream rather than a memset, so that a caller who captures the
// library's launches into a graph gets kernel nodes only.
void launch_zero(spc_ctx* ctx, void* p, size_t bytes);

// Host wrapper.  `partial` is unused (kept for callers' scratch layout).
// in may equal out (each tile reads all of its items before writing).
template <typename T>
int exclusive_scan(spc_ctx* ctx, const T* in, T* out, int64_t n, T* partial,
                   ScanReadback rb = ScanReadback{nullptr, 0, nullptr, nullptr, 0}) {
  (void)partial;
  if (n <= 0) {
    launch_zero(ctx, out, sizeof(T));
    SPC_LAUNCH_CHECK(ctx, "exclusive_scan (empty)");
    return SPC_OK;
  }
  int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  uint32_t epoch = scan_state_reserve(ctx, tiles);
  if (!epoch) return ctx->err_code ? ctx->err_code : SPC_ENOMEM;
  TileScan ts{ctx->scan_state, epoch, (unsigned long long*)(ctx->scan_state + ctx->scan_cap - 1)};
  hipLaunchKernelGGL(k_scan_lb<T>, dim3((unsigned)tiles), dim3(SCAN_BS), 0, ctx->stream, in, out, n, ts, rb);
  SPC_LAUNCH_CHECK(ctx, "exclusive_scan");
  return SPC_OK;
}

// Both exclusive scans (out[n] = total each) in one launch.
template <typename T1, typename T2>
int exclusive_scan2(spc_ctx* ctx, const T1* in1, T1* out1, const T2* in2, T2* out2, int64_t n) {
  if (n <= 0) {
    launch_zero(ctx, out1, sizeof(T1));
    launch_zero(ctx, out2, sizeof(T2));
    SPC_LAUNCH_CHECK(ctx, "exclusive_scan2 (empty)");
    return SPC_OK;
  }
  int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  uint32_t epoch = scan_state_reserve(ctx, 2 * tiles);
  if (!epoch) return ctx->err_code ? ctx->err_code : SPC_ENOMEM;
  unsigned long long* err = (unsigned long long*)(ctx->scan_state + ctx->scan_cap - 1);
  TileScan ts1{ctx->scan_state, epoch, err}, ts2{ctx->scan_state + tiles, epoch, err};
  hipLaunchKernelGGL((k_scan2_lb<T1, T2>), dim3((unsigned)tiles), dim3(SCAN_BS), 0, ctx->stream, in1, out1, in2,
                     out2, n, ts1, ts2);
  SPC_LAUNCH_CHECK(ctx, "exclusive_scan2");
  return SPC_OK;
}

// ===========================================================================
// radix select: the k-th smallest (0-based) of cnt 64-bit keys below 2^bits,
// in one launch of at most min(SEL_MAXB, CUs) blocks that meet at grid
// barriers (one block per CU at most is needed, so all are resident).  Each
// pass histograms one 11-bit digit of the keys that match the digits chosen
// so far; every block stores its histogram and its 32 group sums (64 bins
// each), meets the others at one barrier, then finds the group holding the
// k-th key from the stored group sums and the bin inside it from that
// group's stored bins, so all blocks pick the same bucket without atomics
// across the chip.  Each pass also finds the smallest and largest matching
// key: when every matching key lands in one bucket, the bits those two share
// are decided at once (a run of equal scores costs one pass, not one per
// digit).  Once at most SEL_SMALL keys match, each block copies its
// matches to an offset known from the stored histograms and one block
// finishes in LDS.  cnt and k may be read from device memory; the result is
// left in st->prefix.
// ===========================================================================
constexpr int SEL_DIGIT = 11;
constexpr int SEL_BINS = 1 << SEL_DIGIT;
constexpr int SEL_GBINS = 64;                     // bins per group
constexpr int SEL_NGRP = SEL_BINS / SEL_GBINS;    // 32 groups
constexpr int SEL_SMALL = 16384;   // keys one block finishes in LDS (128 KB)
constexpr int SEG_SMALL = 4096;    // the same for the per-graph selects of batches
constexpr int SEL_MAXB = 128;    // blocks of one select
constexpr int SEL_FLAG = 8;      // flag stride (one 64-byte line per block)

struct SelState {
  unsigned long long prefix, mask;
  unsigned long long ext[2];   // smallest and largest key (written by the one-block path)
  unsigned long long guess[2];  // likely bounds of a later selection's result (band selections)
  unsigned long long bmn[2][SEL_MAXB], bmx[2][SEL_MAXB];   // extreme matching keys per block
  unsigned long long bbelow[SEL_MAXB];                     // keys below the guessed range, per block
  unsigned int gsum[2][SEL_MAXB][SEL_NGRP];          // per-block group sums, pass p in [p % 2]
  unsigned int bhist[2][SEL_MAXB][SEL_BINS];         // per-block histograms
  uint64_t buf[SEL_SMALL];                           // gathered keys
};

// After the call st->prefix holds the selected key (device memory); a grid
// barrier that waited too long, or k >= cnt, sets *err (the result is then
// undefined).  flags: SEL_MAXB * SEL_FLAG words, zeroed when ctx->sel_epoch
// was last reset to 0; every select of that period uses epochs above the
// previous one's.  thr (nullable): also derive a band threshold from the
// selected key, in the same launch.  guess_lo / guess_hi (nullable, device
// words): likely bounds of the k-th key; the bits they share are taken as
// decided for the first pass, which also counts the keys below them and
// starts over without the guess when the k-th key is not among the keys
// that share those bits.
struct ThrSpec;
int radix_select(spc_ctx* ctx, const uint64_t* keys, const unsigned long long* cnt_dev,
                 int64_t cnt_bound, const unsigned long long* k_dev, unsigned long long k_host,
                 int bits, SelState* st, unsigned long long* flags, unsigned long long* err,
                 const ThrSpec* thr = nullptr, const unsigned long long* guess_lo = nullptr,
                 const unsigned long long* guess_hi = nullptr);

// Small launches that replace the runtime's fill and copy blits on the
// level path (each blit costs the host far more than a plain launch).
// k_clear zeroes a[0, na), b[0, nb), c[0, nc), the info slots whose bit is set in
// `slots` and *word; k_readback copies the info block (I_NINFO words, when info is not
// null) and up to three scalars (null: 0) into host-visible pinned memory
// at out[0..I_NINFO) and out[I_NINFO..I_NINFO+3), then the token (when
// nonzero) at out[I_NINFO + 3]; k_copy_u64 copies one word.
__global__ void k_clear(int32_t* a, int64_t na, uint64_t* b, int64_t nb, uint64_t* c, int64_t nc,
                        unsigned long long* info, uint32_t slots, unsigned long long* word);
__global__ void k_readback(const unsigned long long* info, int ninfo, const int64_t* x0,
                           const int32_t* x1, const uint64_t* x2, int64_t* out, int64_t token);
// Host waits.  The pinned copy is host-coherent: a kernel that fills it then
// writes a new token at out[I_NINFO + 3] after a system-scope fence, and the
// host polls that word instead of synchronising the stream (whose status it
// checks every few thousand polls, so a failed kernel still ends the wait).
// readback_wait launches k_readback with a new token and waits for it.
int wait_token(spc_ctx* ctx, int64_t token);
int readback_wait(spc_ctx* ctx, const unsigned long long* info, int ninfo, const int64_t* x0 = nullptr,
                  const int32_t* x1 = nullptr, const uint64_t* x2 = nullptr);
__global__ void k_copy_u64(unsigned long long* dst, const unsigned long long* src);
__global__ void k_fill_u64(uint64_t* __restrict__ a, int64_t n, uint64_t v);
// `word` (nullable) is one more word to zero (the scan chain's error flag).
void launch_clear(spc_ctx* ctx, int32_t* a, int64_t na, uint64_t* b, int64_t nb, unsigned long long* info,
                  uint32_t slots, uint64_t* c = nullptr, int64_t nc = 0, unsigned long long* word = nullptr);


// ===========================================================================
// merge sort of n elements of type E under a strict order `less` (a
// functor with `bool operator()(const E&, const E&) const`).  Tiles of 1024
// are sorted in LDS by a bitonic network, then merged pairwise with a
// per-thread merge-path split.  The order of elements that compare equal
// is unspecified; every use here has either unique keys or an
// order-insensitive consumer.
// ===========================================================================
constexpr int MS_BS = 256;
constexpr int MS_TILE = 1024;
constexpr int MS_ITEMS = 8;

template <typename E, typename Less>
__global__ void __launch_bounds__(MS_BS) k_block_sort(E* data, int64_t n, Less less) {
  __shared__ E s[MS_TILE];
  __shared__ unsigned char pad[MS_TILE];
  int64_t base = (int64_t)blockIdx.x * MS_TILE;
  int tid = threadIdx.x;
  for (int i = tid; i < MS_TILE; i += MS_BS) {
    int64_t g = base + i;
    pad[i] = g >= n;
    if (g < n) s[i] = data[g];
  }
  __syncthreads();
  for (int k = 2; k <= MS_TILE; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int p = tid; p < MS_TILE / 2; p += MS_BS) {
        int i = 2 * j * (p / j) + (p % j);
        int l = i + j;
        bool asc = (i & k) == 0;
        // lt(x, y): x strictly before y, padding last
        bool li = pad[l] ? false : (pad[i] ? true : less(s[l], s[i]));  // s[l] < s[i]
        bool il = pad[i] ? false : (pad[l] ? true : less(s[i], s[l]));  // s[i] < s[l]
        bool sw = asc ? li : il;
        if (sw) {
          E t = s[i];
          s[i] = s[l];
          s[l] = t;
          unsigned char q = pad[i];
          pad[i] = pad[l];
          pad[l] = q;
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < MS_TILE; i += MS_BS) {
    int64_t g = base + i;
    if (g < n) data[g] = s[i];
  }
}

template <typename E, typename Less>
__global__ void __launch_bounds__(MS_BS)
    k_merge_pass(const E* __restrict__ src, E* __restrict__ dst, int64_t n, int64_t w, Less less) {
  int64_t i = ((int64_t)blockIdx.x * MS_BS + threadIdx.x) * MS_ITEMS;
  if (i >= n) return;
  int64_t base = (i / (2 * w)) * (2 * w);
  int64_t a0 = base;
  int64_t a_len = (n - base) < w ? (n - base) : w;
  int64_t b0 = base + a_len;
  int64_t b_len = (n - b0) < w ? (n - b0) : w;
  if (b_len < 0) b_len = 0;
  int64_t diag = i - base;
  int64_t lo = diag - b_len > 0 ? diag - b_len : 0;
  int64_t hi = diag < a_len ? diag : a_len;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    // A[mid] goes before B[diag - mid - 1] unless B is strictly smaller
    if (!less(src[b0 + diag - mid - 1], src[a0 + mid])) lo = mid + 1;
    else hi = mid;
  }
  int64_t ia = a0 + lo, ib = b0 + diag - lo;
  int64_t ae = a0 + a_len, be = b0 + b_len;
  int64_t end = base + a_len + b_len;
  for (int k = 0; k < MS_ITEMS && i + k < end; k++) {
    bool takeA;
    if (ib >= be) takeA = true;
    else if (ia >= ae) takeA = false;
    else takeA = !less(src[ib], src[ia]);
    dst[i + k] = takeA ? src[ia++] : src[ib++];
  }
}

// Sorts a[0..n) using b as scratch; *out points at whichever holds the result.
template <typename E, typename Less>
int merge_sort(spc_ctx* ctx, E* a, E* b, int64_t n, Less less, E** out) {
  *out = a;
  if (n <= 1) return SPC_OK;
  hipLaunchKernelGGL((k_block_sort<E, Less>), dim3(grid_for(n, MS_TILE)), dim3(MS_BS), 0,
                     ctx->stream, a, n, less);
  E* cur = a;
  E* oth = b;
  for (int64_t w = MS_TILE; w < n; w <<= 1) {
    int64_t threads = (n + MS_ITEMS - 1) / MS_ITEMS;
    hipLaunchKernelGGL((k_merge_pass<E, Less>), dim3(grid_for(threads, MS_BS)), dim3(MS_BS), 0,
                       ctx->stream, cur, oth, n, w, less);
    E* t = cur;
    cur = oth;
    oth = t;
  }
  SPC_LAUNCH_CHECK(ctx, "merge_sort");
  *out = cur;
  return SPC_OK;
}

}  // namespace spc

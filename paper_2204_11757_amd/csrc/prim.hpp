// Device-wide primitives: exclusive scan, radix select of the k-th smallest
// 64-bit key, and a merge sort with an arbitrary strict-weak comparator.
#pragma once

#include "common.hpp"

namespace spc {

// ===========================================================================
// exclusive scan: out[i] = sum in[0..i), out[n] = total (out has n+1 slots).
// reduce-then-scan over <= SCAN_MAXB contiguous chunks.
// ===========================================================================
constexpr int SCAN_BS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BS * SCAN_ITEMS;
constexpr int SCAN_MAXB = 1024;

template <typename T>
__global__ void __launch_bounds__(SCAN_BS)
    k_scan_reduce(const T* __restrict__ in, int64_t n, int64_t chunk, T* __restrict__ partial) {
  __shared__ T tmp[SCAN_BS / WAVE];
  int64_t s = (int64_t)blockIdx.x * chunk;
  int64_t e = s + chunk < n ? s + chunk : n;
  T acc = 0;
  for (int64_t i = s + threadIdx.x; i < e; i += SCAN_BS) acc += in[i];
  acc = wave_sum(acc);
  if (lane_id() == 0) tmp[threadIdx.x / WAVE] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T t = 0;
    for (int w = 0; w < SCAN_BS / WAVE; w++) t += tmp[w];
    partial[blockIdx.x] = t;
  }
}

template <typename T>
__global__ void __launch_bounds__(1024) k_scan_partials(T* partial, int nb) {
  __shared__ T tmp[1024 / WAVE];
  int t = threadIdx.x;
  T v = t < nb ? partial[t] : (T)0;
  T tot;
  T inc = block_incl_scan<T, 1024, false>(v, tmp, &tot);
  if (t < nb) partial[t] = inc - v;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_BS)
    k_scan_apply(const T* in, T* out, int64_t n, int64_t chunk,
                 const T* __restrict__ partial, int nb) {
  __shared__ T buf[SCAN_TILE];
  __shared__ T tmp[SCAN_BS / WAVE];
  int64_t s = (int64_t)blockIdx.x * chunk;
  int64_t e = s + chunk < n ? s + chunk : n;
  T carry = partial[blockIdx.x];
  int tid = threadIdx.x;
  for (int64_t base = s; base < e; base += SCAN_TILE) {
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
      int64_t g = base + i * SCAN_BS + tid;
      buf[i * SCAN_BS + tid] = g < e ? in[g] : (T)0;
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
    T pre = carry + inc - run;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) buf[tid * SCAN_ITEMS + i] = pre + loc[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
      int64_t g = base + i * SCAN_BS + tid;
      if (g < e) out[g] = buf[i * SCAN_BS + tid];
    }
    carry += tot;
    __syncthreads();
  }
  if (blockIdx.x == nb - 1 && tid == 0) out[n] = carry;
}

// Host wrapper.  partial: device scratch of SCAN_MAXB elements.  in may
// equal out (the in-place case reads each tile before writing it).
template <typename T>
int exclusive_scan(spc_ctx* ctx, const T* in, T* out, int64_t n, T* partial) {
  if (n <= 0) {
    SPC_HIP(ctx, hipMemsetAsync(out, 0, sizeof(T), ctx->stream));
    return SPC_OK;
  }
  int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  int nb = (int)(tiles < SCAN_MAXB ? tiles : SCAN_MAXB);
  int64_t chunk = ((tiles + nb - 1) / nb) * SCAN_TILE;
  nb = (int)((n + chunk - 1) / chunk);
  hipLaunchKernelGGL(k_scan_reduce<T>, dim3(nb), dim3(SCAN_BS), 0, ctx->stream, in, n, chunk, partial);
  hipLaunchKernelGGL(k_scan_partials<T>, dim3(1), dim3(1024), 0, ctx->stream, partial, nb);
  hipLaunchKernelGGL(k_scan_apply<T>, dim3(nb), dim3(SCAN_BS), 0, ctx->stream, in, out, n, chunk,
                     partial, nb);
  SPC_LAUNCH_CHECK(ctx, "exclusive_scan");
  return SPC_OK;
}

// ===========================================================================
// radix select: the k-th smallest (0-based) of cnt 64-bit keys, using
// 11-bit digits from the most significant of `bits` bits down.  Runs fully
// on the device; cnt may be read from device memory.
// ===========================================================================
constexpr int SEL_DIGIT = 11;
constexpr int SEL_BINS = 1 << SEL_DIGIT;

struct SelState {
  unsigned long long prefix, mask, k, pad;
  unsigned int hist[SEL_BINS];
};

__global__ void k_sel_init(SelState* st, const unsigned long long* k_dev, unsigned long long k_host);
__global__ void k_sel_hist(const uint64_t* __restrict__ keys, const unsigned long long* cnt_dev,
                           int64_t cnt_host, SelState* st, int shift, int width);
__global__ void k_sel_pick(SelState* st, int shift, int width);

// After the call st->prefix holds the selected key (device memory).
int radix_select(spc_ctx* ctx, const uint64_t* keys, const unsigned long long* cnt_dev,
                 int64_t cnt_bound, const unsigned long long* k_dev, unsigned long long k_host,
                 int bits, SelState* st);

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

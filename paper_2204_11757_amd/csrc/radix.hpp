// Block-level pieces of the radix selects: LDS histograms, LDS list
// reservation, block min/max, and the one-block selection among keys held
// in LDS.  Shared by the whole-graph select and the per-graph select of
// batches.
#pragma once

#include "level.hpp"

namespace spc {

constexpr int SEL_BS = 256;
constexpr int SEL_UNROLL = 16;
constexpr long SEL_SPIN = 1l << 24;          // barrier polls before giving up (about a second)

// LDS histogram increment of bin `bin` for the lanes with `m` set: when all
// such lanes of the wave share one bin (skewed digits, ties), one lane adds
// their count, so equal keys do not serialise on one LDS address.
__device__ __forceinline__ void hist_add(unsigned int* h, bool m, uint32_t bin) {
  unsigned long long act = __ballot(m);
  if (!act) return;
  int leader = __ffsll((long long)act) - 1;
  uint32_t lb = (uint32_t)__shfl((int)bin, leader);
  unsigned long long same = __ballot(m && bin == lb);
  if (same == act) {
    if (lane_id() == leader) atomicAdd(&h[lb], (unsigned int)__popcll(act));
  } else if (m) {
    atomicAdd(&h[bin], 1u);
  }
}

// Slot in an LDS list for the lanes with `m` set: one LDS atomic per wave.
__device__ __forceinline__ unsigned int wave_reserve(unsigned int* counter, bool m) {
  unsigned long long act = __ballot(m);
  if (!act) return 0;
  int leader = __ffsll((long long)act) - 1;
  unsigned int base = 0;
  if (lane_id() == leader) base = atomicAdd(counter, (unsigned int)__popcll(act));
  base = (unsigned int)__shfl((int)base, leader);
  unsigned long long below = act & ((1ull << lane_id()) - 1);
  return base + (unsigned int)__popcll(below);
}

// Block-wide smallest and largest of the values the threads hold.
__device__ __forceinline__ void block_minmax(uint64_t& mn, uint64_t& mx, unsigned long long* red) {
  mn = wave_min(mn);
  mx = wave_max(mx);
  int w = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    red[w] = mn;
    red[SEL_BS / WAVE + w] = mx;
  }
  __syncthreads();
  mn = ~0ull;
  mx = 0;
  for (int i = 0; i < SEL_BS / WAVE; i++) {
    mn = red[i] < mn ? red[i] : mn;
    mx = red[SEL_BS / WAVE + i] > mx ? red[SEL_BS / WAVE + i] : mx;
  }
  __syncthreads();
}

// The k-th smallest of the c <= SEL_SMALL keys in s (LDS), by one block with
// 8-bit digits below the highest bit in which the keys differ.
__device__ __forceinline__ uint64_t lds_select(const uint64_t* s, int c, unsigned long long k, unsigned int* h,
                               unsigned long long* tmp, unsigned long long* red, unsigned long long* spick,
                               unsigned long long* err) {
  int t = threadIdx.x;
  if (k >= (unsigned long long)c) {
    if (t == 0) __hip_atomic_store(err, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return ~0ull;
  }
  uint64_t mn = ~0ull, mx = 0;
  for (int i = t; i < c; i += SEL_BS) {
    mn = s[i] < mn ? s[i] : mn;
    mx = s[i] > mx ? s[i] : mx;
  }
  block_minmax(mn, mx, red);
  uint64_t x = mn ^ mx;
  if (x == 0) return mn;
  int hi = 64 - __clzll((long long)x);
  uint64_t mask = hi == 64 ? 0ull : ~((1ull << hi) - 1);
  uint64_t prefix = mn & mask;
  while (hi > 0) {
    int lo = hi - 8 > 0 ? hi - 8 : 0;
    int nb = 1 << (hi - lo);
    uint64_t dm = (uint64_t)(nb - 1);
    h[t] = 0;
    __syncthreads();
    for (int i0 = 0; i0 < c; i0 += SEL_BS) {
      int i = i0 + t;
      uint64_t x = i < c ? s[i] : 0;
      hist_add(h, i < c && (x & mask) == prefix, (uint32_t)((x >> lo) & dm));
    }
    __syncthreads();
    unsigned long long cnt = t < nb ? h[t] : 0;
    unsigned long long tot;
    unsigned long long before = block_incl_scan<unsigned long long, SEL_BS, false>(cnt, tmp, &tot) - cnt;
    if (k >= before && k < before + cnt) {
      spick[0] = (unsigned long long)t;
      spick[1] = before;
      spick[2] = cnt;
    }
    __syncthreads();
    prefix |= spick[0] << lo;
    mask |= dm << lo;
    k -= spick[1];
    hi = lo;
    bool one = spick[2] == 1;
    __syncthreads();
    if (one && hi > 0) {
      // a single key is left in the bucket: find it
      for (int i = t; i < c; i += SEL_BS)
        if ((s[i] & mask) == prefix) spick[0] = s[i];
      __syncthreads();
      uint64_t r = spick[0];
      __syncthreads();
      return r;
    }
  }
  return prefix;
}

}  // namespace spc

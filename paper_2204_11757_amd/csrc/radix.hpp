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
// their count, so equal keys do not serialise on one LDS address.  Inside
// the branch the active lanes are exactly those with `m`, so the first one's
// bin is a scalar read (no cross-lane LDS traffic).
__device__ __forceinline__ void hist_add(unsigned int* h, bool m, uint32_t bin) {
  if (m) {
    uint32_t lb = __builtin_amdgcn_readfirstlane(bin);
    unsigned long long act = __ballot(1);
    unsigned long long same = __ballot(bin == lb);
    if (same == act) {
      if (lane_id() == __ffsll((long long)act) - 1) atomicAdd(&h[lb], (unsigned int)__popcll(act));
    } else {
      atomicAdd(&h[bin], 1u);
    }
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

// The k-th smallest of the c keys in s (LDS), by one block.
// It first finds the smallest and largest key and decides the bits they
// share (so a run of equal scores costs nothing); each round then
// histograms the next 11 bits of the keys still in play (8 bins per thread)
// and keeps the bucket of the k-th key.  Once that bucket holds at most
// LDS_SMALL2 keys they are copied to s2 and later rounds read only those;
// every copy or rescan also finds the bucket's smallest and largest key, so
// bits they share are skipped again.  h needs SEL_BS * 8 counters, s2
// LDS_SMALL2 keys.  ext (nullable): thread 0 stores the smallest and largest
// key there.
constexpr int LDS_SMALL2 = 1024;

__device__ __forceinline__ uint64_t lds_select(const uint64_t* s, int c, unsigned long long k, unsigned int* h,
                                               unsigned long long* tmp, unsigned long long* red,
                                               unsigned long long* spick, unsigned long long* err,
                                               uint64_t* s2, unsigned int* scount,
                                               unsigned long long* ext = nullptr) {
  constexpr int PER = 8;
  constexpr int DIG = 11;
  constexpr int U = 8;   // keys per thread whose LDS loads are issued together
  int t = threadIdx.x;
  if (k >= (unsigned long long)c) {
    if (t == 0) __hip_atomic_store(err, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return ~0ull;
  }
  uint64_t prefix = 0, mask = 0;
  const uint64_t* cur = s;
  int cc = c;
  // extremes of the keys matching (prefix, mask) in cur
  auto extremes = [&](uint64_t& mn, uint64_t& mx) {
    mn = ~0ull;
    mx = 0;
    for (int i0 = 0; i0 < cc; i0 += SEL_BS * U) {
      uint64_t v[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        int i = i0 + u * SEL_BS + t;
        v[u] = i < cc ? cur[i] : 0;
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        int i = i0 + u * SEL_BS + t;
        if (i < cc && (v[u] & mask) == prefix) {
          mn = v[u] < mn ? v[u] : mn;
          mx = v[u] > mx ? v[u] : mx;
        }
      }
    }
    block_minmax(mn, mx, red);
  };
  uint64_t mn, mx;
  extremes(mn, mx);
  if (ext && t == 0) {
    ext[0] = mn;
    ext[1] = mx;
  }
  while (true) {
    uint64_t x = mn ^ mx;
    if (x == 0) return mn;   // every key in play is equal
    int d = 63 - __clzll((long long)x);   // highest differing bit
    uint64_t low = d == 63 ? ~0ull : (2ull << d) - 1;
    prefix = mn & ~low;
    mask = ~low;
    int hi = d + 1;
    int lo = hi - DIG > 0 ? hi - DIG : 0;
    int nb = 1 << (hi - lo);
    uint64_t dm = (uint64_t)(nb - 1);
    for (int q = 0; q < PER; q++) h[PER * t + q] = 0;
    __syncthreads();
    for (int i0 = 0; i0 < cc; i0 += SEL_BS * U) {
      uint64_t v[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        int i = i0 + u * SEL_BS + t;
        v[u] = i < cc ? cur[i] : 0;
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        int i = i0 + u * SEL_BS + t;
        hist_add(h, i < cc && (v[u] & mask) == prefix, (uint32_t)((v[u] >> lo) & dm));
      }
    }
    __syncthreads();
    unsigned int cq[PER];
    unsigned long long cnt = 0;
    for (int q = 0; q < PER; q++) {
      int b = PER * t + q;
      cq[q] = b < nb ? h[b] : 0u;
      cnt += cq[q];
    }
    unsigned long long tot;
    unsigned long long before = block_incl_scan<unsigned long long, SEL_BS, false>(cnt, tmp, &tot) - cnt;
    if (k >= before && k < before + cnt) {
      unsigned long long acc = before;
      for (int q = 0; q < PER; q++) {
        if (k >= acc && k < acc + cq[q]) {
          spick[0] = (unsigned long long)(PER * t + q);
          spick[1] = acc;
          spick[2] = cq[q];
        }
        acc += cq[q];
      }
    }
    __syncthreads();
    prefix |= spick[0] << lo;
    mask |= dm << lo;
    k -= spick[1];
    unsigned long long cb = spick[2];
    __syncthreads();
    if (lo == 0) return prefix;
    if (cur == s && cb <= (unsigned long long)LDS_SMALL2) {
      // copy the bucket's keys (in any order) and take their extremes
      if (t == 0) *scount = 0;
      __syncthreads();
      mn = ~0ull;
      mx = 0;
      for (int i0 = 0; i0 < cc; i0 += SEL_BS * U) {
        uint64_t v[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
          int i = i0 + u * SEL_BS + t;
          v[u] = i < cc ? cur[i] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
          int i = i0 + u * SEL_BS + t;
          bool m = i < cc && (v[u] & mask) == prefix;
          unsigned int q = wave_reserve(scount, m);
          if (m) {
            if (q < (unsigned)LDS_SMALL2) s2[q] = v[u];
            mn = v[u] < mn ? v[u] : mn;
            mx = v[u] > mx ? v[u] : mx;
          }
        }
      }
      block_minmax(mn, mx, red);   // its barriers also publish s2 and *scount
      cur = s2;
      cc = (int)cb;
    } else {
      extremes(mn, mx);
    }
  }
}

}  // namespace spc

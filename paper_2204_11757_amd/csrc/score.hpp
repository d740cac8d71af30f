// Exact integer merge score of one edge (A2), shared by the score kernels
// and the kernels that re-evaluate single edges (Theorem 2's epsilon, the
// batched cutoff).
#pragma once

#include "level.hpp"

namespace spc {

// ---------------------------------------------------------------------------
// A2: exact fitness N / D of one edge (u, v) with weight wuv.
// D = d_u d_v and N = 2 D - 2 sum_{x in S(u) cap S(v)} min(a_ux d_v, a_vx d_u),
// where S(x) is the support of row x including its diagonal.  The common
// support is the intersection of the two CSR rows plus the diagonal
// positions x = u (if self_w[u] > 0) and x = v (if self_w[v] > 0).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

__device__ __forceinline__ uint64_t common_min_sum(const int32_t* __restrict__ col,
                                                   const int32_t* __restrict__ w, int64_t as,
                                                   int64_t ae, uint64_t fa, int64_t bs, int64_t be,
                                                   uint64_t fb) {
  // sum over x in both rows of min(w_a[x] * fa, w_b[x] * fb); rows ascending.
  uint64_t M = 0;
  int64_t la = ae - as, lb = be - bs;
  if (la > 4 * lb && la > 32) {
    // walk the short row b, galloping search in the long row a
    int64_t lo = as;
    for (int64_t j = bs; j < be && lo < ae; j++) {
      int32_t x = col[j];
      int64_t hi = ae;
      while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (col[mid] < x) lo = mid + 1;
        else hi = mid;
      }
      if (lo < ae && col[lo] == x) {
        M += umin64((uint64_t)w[lo] * fa, (uint64_t)w[j] * fb);
        lo++;
      }
    }
    return M;
  }
  if (lb > 4 * la && lb > 32) {
    int64_t lo = bs;
    for (int64_t i = as; i < ae && lo < be; i++) {
      int32_t x = col[i];
      int64_t hi = be;
      while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (col[mid] < x) lo = mid + 1;
        else hi = mid;
      }
      if (lo < be && col[lo] == x) {
        M += umin64((uint64_t)w[i] * fa, (uint64_t)w[lo] * fb);
        lo++;
      }
    }
    return M;
  }
  int64_t i = as, j = bs;
  if (i < ae && j < be) {
    int32_t x = col[i], y = col[j];
    while (true) {
      if (x < y) {
        if (++i >= ae) break;
        x = col[i];
      } else if (x > y) {
        if (++j >= be) break;
        y = col[j];
      } else {
        M += umin64((uint64_t)w[i] * fa, (uint64_t)w[j] * fb);
        if (++i >= ae || ++j >= be) break;
        x = col[i];
        y = col[j];
      }
    }
  }
  return M;
}

// position of u in row v (u < v, so it lies among v's lower entries)
__device__ __forceinline__ int64_t mirror_pos(const LevelIn& g, const int32_t* __restrict__ lc,
                                              int32_t v, int32_t u) {
  int64_t lo = g.rp[v], hi = g.rp[v] + lc[v];
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (g.col[mid] < u) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Rows of at most RC entries are read into registers with all loads issued
// at once (the common-support walk over global memory would chain one
// dependent load per step); longer rows take the walk.
constexpr int RC = 8;

// Also returns jm, the CSR position of the mirror entry (v -> u).
__device__ __forceinline__ void edge_score(const LevelIn& g, const uint64_t* __restrict__ deg,
                                           const int32_t* __restrict__ lc, int32_t u, int32_t v,
                                           int32_t wuv, uint64_t& N, uint64_t& D, int64_t& jm) {
  int64_t au = g.rp[u], bu = g.rp[u + 1], av = g.rp[v], bv = g.rp[v + 1];
  uint64_t du = deg[u], dv = deg[v];
  uint64_t su = g.self ? (uint64_t)g.self[u] : 0, sv = g.self ? (uint64_t)g.self[v] : 0;
  int64_t lu = bu - au, lv = bv - av;
  D = du * dv;
  uint64_t M = 0;
  if (lu <= RC && lv <= RC) {
    int32_t cu[RC], cv[RC];
    uint32_t wu[RC], wv[RC];
#pragma unroll
    for (int k = 0; k < RC; k++) {
      bool pu = k < lu, pv = k < lv;
      cu[k] = pu ? g.col[au + k] : -1;   // distinct sentinels never match
      wu[k] = pu ? (uint32_t)g.w[au + k] : 0u;
      cv[k] = pv ? g.col[av + k] : -2;
      wv[k] = pv ? (uint32_t)g.w[av + k] : 0u;
    }
    int below = 0;
#pragma unroll
    for (int k = 0; k < RC; k++) below += (k < lv && cv[k] < u) ? 1 : 0;
    jm = av + below;
#pragma unroll
    for (int i = 0; i < RC; i++) {
      uint32_t mw = 0;   // weight of cu[i] in row v (0: absent)
#pragma unroll
      for (int k = 0; k < RC; k++) mw = (cu[i] == cv[k]) ? wv[k] : mw;
      if (mw) M += umin64((uint64_t)wu[i] * dv, (uint64_t)mw * du);
    }
  } else {
    M = common_min_sum(g.col, g.w, au, bu, dv, av, bv, du);
    jm = mirror_pos(g, lc, v, u);
  }
  if (su) M += umin64(su * dv, (uint64_t)wuv * du);   // x = u
  if (sv) M += umin64((uint64_t)wuv * dv, sv * du);   // x = v
  N = 2 * D - 2 * M;
}

// floor(N * 2^b / D) for N < 2^63, D < 2^62, b <= 61 (the result is below 2^62).
__device__ __forceinline__ uint64_t fixed_key(uint64_t N, uint64_t D, int b) {
  if ((N >> (63 - b)) == 0) {
    uint64_t num = N << b;
    if (num < (1ull << 53) && D < (1ull << 53)) {
      // the correctly rounded quotient is at most one above the floor
      uint64_t q = (uint64_t)((double)num / (double)D);
      if (q * D > num) q--;
      return q;
    }
    return num / D;
  }
  unsigned __int128 num = (unsigned __int128)N << b;
  return (uint64_t)(num / D);
}

}  // namespace spc

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

// Rows are read into registers in chunks of RC entries with all loads of a
// chunk issued at once: a walk over global memory one entry at a time would
// chain one dependent load per step.
constexpr int RC = 8;

__device__ __forceinline__ int32_t chunk_last(const int32_t (&c)[RC], int64_t left) {
  // largest valid column of a chunk (rows ascending, so its last)
  int32_t m = INT32_MIN;
#pragma unroll
  for (int k = 0; k < RC; k++) m = (k < left && c[k] > m) ? c[k] : m;
  return m;
}

// Common-support sum of rows a = [as, ae) and b = [bs, be), a merge over
// chunks: after comparing the current chunks pair by pair, the chunk with
// the smaller last column advances (both on a tie), so every pair of chunks
// that can share a column meets exactly once and each step costs one round
// of independent loads.  Returns sum min(w_a[x] fa, w_b[x] fb); below counts
// b's columns smaller than lim, complete says whether that count is final.
__device__ __forceinline__ uint64_t chunk_merge_sum(const int32_t* __restrict__ col,
                                                    const int32_t* __restrict__ w, int64_t as,
                                                    int64_t ae, uint64_t fa, int64_t bs, int64_t be,
                                                    uint64_t fb, int32_t lim, int64_t& below,
                                                    bool& complete) {
  int32_t ca[RC], cb[RC];
  uint32_t wa[RC], wb[RC];
  uint64_t M = 0;
  bool seen = false;
  below = 0;
#pragma unroll
  for (int k = 0; k < RC; k++) {
    bool pa = as + k < ae, pb = bs + k < be;
    ca[k] = pa ? col[as + k] : -1;   // distinct sentinels never match
    wa[k] = pa ? (uint32_t)w[as + k] : 0u;
    cb[k] = pb ? col[bs + k] : -2;
    wb[k] = pb ? (uint32_t)w[bs + k] : 0u;
  }
#pragma unroll
  for (int k = 0; k < RC; k++) {
    below += (cb[k] >= 0 && cb[k] < lim) ? 1 : 0;
    seen |= cb[k] >= lim;
  }
  int64_t i = as, j = bs;
  while (i < ae && j < be) {
#pragma unroll
    for (int p = 0; p < RC; p++) {
      uint32_t mw = 0;
#pragma unroll
      for (int q = 0; q < RC; q++) mw = (ca[p] == cb[q]) ? wb[q] : mw;
      if (mw) M += umin64((uint64_t)wa[p] * fa, (uint64_t)mw * fb);
    }
    int32_t la = chunk_last(ca, ae - i), lb = chunk_last(cb, be - j);
    if (la <= lb) {
      i += RC;
#pragma unroll
      for (int k = 0; k < RC; k++) {
        bool pa = i + k < ae;
        ca[k] = pa ? col[i + k] : -1;
        wa[k] = pa ? (uint32_t)w[i + k] : 0u;
      }
    }
    if (lb <= la) {
      j += RC;
#pragma unroll
      for (int k = 0; k < RC; k++) {
        bool pb = j + k < be;
        cb[k] = pb ? col[j + k] : -2;
        wb[k] = pb ? (uint32_t)w[j + k] : 0u;
      }
#pragma unroll
      for (int k = 0; k < RC; k++) {
        below += (cb[k] >= 0 && cb[k] < lim) ? 1 : 0;
        seen |= cb[k] >= lim;
      }
    }
  }
  complete = seen || j >= be;
  return M;
}

constexpr int RS = 4;   // narrower than RC: each search keeps four values per column

// Common-support sum when row t = [ts, te) is much longer than row p =
// [ps, pe): p is read in chunks of RS and each column of a chunk is located in t by
// a branchless binary search (the largest position whose column is <= x),
// all searches of a chunk in step.  Returns sum min(w_p[x] fp, w_t[x] ft) and
// the number of p's columns smaller than lim.
__device__ __forceinline__ uint64_t chunk_search_sum(const int32_t* __restrict__ col,
                                                     const int32_t* __restrict__ w, int64_t ps,
                                                     int64_t pe, uint64_t fp, int64_t ts, int64_t te,
                                                     uint64_t ft, int32_t lim, int64_t& below) {
  uint64_t M = 0;
  below = 0;
  int32_t lt = (int32_t)(te - ts);
  int32_t t0 = col[ts];
  for (int64_t c = ps; c < pe; c += RS) {
    int32_t x[RS], base[RS], val[RS];
    uint32_t wx[RS];
#pragma unroll
    for (int k = 0; k < RS; k++) {
      bool in = c + k < pe;
      x[k] = in ? col[c + k] : -1;
      wx[k] = in ? (uint32_t)w[c + k] : 0u;
      base[k] = 0;
      val[k] = t0;
      below += (in && x[k] < lim) ? 1 : 0;
    }
    for (int32_t n = lt; n > 1;) {
      int32_t half = n >> 1;
#pragma unroll
      for (int k = 0; k < RS; k++) {
        int32_t y = col[ts + base[k] + half];
        if (y <= x[k]) {
          base[k] += half;
          val[k] = y;
        }
      }
      n -= half;
    }
#pragma unroll
    for (int k = 0; k < RS; k++)
      if (x[k] >= 0 && val[k] == x[k])
        M += umin64((uint64_t)wx[k] * fp, (uint64_t)(uint32_t)w[ts + base[k]] * ft);
  }
  return M;
}

__device__ __forceinline__ int ceil_log2(int64_t x) { return x <= 1 ? 0 : 64 - __clzll(x - 1); }

// Common-support sum when row T has a dense position map tmap (column ->
// position in T, stale entries allowed): row P is read in chunks of RC with
// every load of a chunk independent, and each column is looked up in the
// map and confirmed against T.  Returns the sum of min(w_P[x] fp, w_T[x] ft)
// and, in below, the number of P's columns smaller than lim.
__device__ __forceinline__ uint64_t mapped_min_sum(const int32_t* __restrict__ col,
                                                   const int32_t* __restrict__ w, int64_t ps,
                                                   int64_t pe, uint64_t fp, int64_t ts, int64_t te,
                                                   uint64_t ft, const int32_t* __restrict__ tmap,
                                                   int32_t lim, int64_t& below) {
  uint64_t M = 0;
  uint32_t lt = (uint32_t)(te - ts);
  below = 0;
  for (int64_t c = ps; c < pe; c += RC) {
    int32_t x[RC], p[RC];
    uint32_t wp[RC];
#pragma unroll
    for (int k = 0; k < RC; k++) {
      bool in = c + k < pe;
      x[k] = in ? col[c + k] : -1;
      wp[k] = in ? (uint32_t)w[c + k] : 0u;
    }
#pragma unroll
    for (int k = 0; k < RC; k++) {
      p[k] = x[k] >= 0 ? tmap[x[k]] : -1;
      below += (x[k] >= 0 && x[k] < lim) ? 1 : 0;
    }
#pragma unroll
    for (int k = 0; k < RC; k++) {
      if ((uint32_t)p[k] < lt) {
        int32_t y = col[ts + p[k]];
        uint32_t wt = (uint32_t)w[ts + p[k]];
        if (y == x[k]) M += umin64((uint64_t)wp[k] * fp, (uint64_t)wt * ft);
      }
    }
  }
  return M;
}

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
    // rounds of loads: the chunk merge reads both rows once; the search
    // reads the short row once and log2(long) entries per chunk of it
    int64_t ls = lu < lv ? lu : lv, ll = lu < lv ? lv : lu;
    int64_t c_merge = (lu + RC - 1) / RC + (lv + RC - 1) / RC;
    int64_t c_search = (ls + RS - 1) / RS * (ceil_log2(ll) + 2);
    int64_t below;
    if (c_search < c_merge && lv <= lu) {
      M = chunk_search_sum(g.col, g.w, av, bv, du, au, bu, dv, u, below);
      jm = av + below;
    } else if (c_search < c_merge) {
      M = chunk_search_sum(g.col, g.w, au, bu, dv, av, bv, du, INT32_MIN, below);
      jm = mirror_pos(g, lc, v, u);
    } else {
      bool complete;
      M = chunk_merge_sum(g.col, g.w, au, bu, dv, av, bv, du, u, below, complete);
      jm = complete ? av + below : mirror_pos(g, lc, v, u);
    }
  }
  if (su) M += umin64(su * dv, (uint64_t)wuv * du);   // x = u
  if (sv) M += umin64((uint64_t)wuv * dv, sv * du);   // x = v
  N = 2 * D - 2 * M;
}

// Products of a weight (or self-loop weight) and a degree.  Every weight
// of a row is at most its node's degree, so when the largest degree is
// below 2^24 all operands fit 24 bits and the full product takes the two
// full-rate 24-bit multiplies.
template <bool NARROW>
__device__ __forceinline__ uint64_t wmul(uint64_t a, uint64_t b) {
  if constexpr (NARROW) return (uint64_t)((uint32_t)a & 0xFFFFFFu) * (uint64_t)((uint32_t)b & 0xFFFFFFu);
  else return a * b;
}

// Common-support sum min(w_u[x] dv, w_v[x] du) of an edge whose rows
// [au, au + lu) and [av, av + lv) both hold between 1 and RC entries, in
// arrays of nnz >= RC entries.  Each row is read as the RC entries from its
// start, or the array's last RC entries when it ends within them, so every
// load is an immediate offset from one base and none waits on a branch;
// entries outside the row turn into sentinel columns above every node id
// (u's and v's differ, so they never match).  below: v's columns smaller
// than u.
template <bool NARROW>
__device__ __forceinline__ uint64_t short_rows_sum(const int32_t* __restrict__ col,
                                                   const int32_t* __restrict__ w, int64_t nnz, int64_t au,
                                                   int32_t lu, uint64_t du, int64_t av, int32_t lv, uint64_t dv,
                                                   uint32_t u, int32_t& below) {
  int64_t bu = au + RC <= nnz ? au : nnz - RC, bv = av + RC <= nnz ? av : nnz - RC;
  int32_t hu = (int32_t)(au - bu), hv = (int32_t)(av - bv);   // the row's first entry in the window
  const int32_t *cpu = col + bu, *wpu = w + bu, *cpv = col + bv, *wpv = w + bv;
  uint32_t cu[RC], cv[RC], wu[RC], wv[RC];
#pragma unroll
  for (int k = 0; k < RC; k++) {
    cu[k] = (uint32_t)cpu[k];
    wu[k] = (uint32_t)wpu[k];
    cv[k] = (uint32_t)cpv[k];
    wv[k] = (uint32_t)wpv[k];
  }
  below = 0;
#pragma unroll
  for (int k = 0; k < RC; k++) {
    cu[k] = (uint32_t)(k - hu) < (uint32_t)lu ? cu[k] : 0xFFFFFFFFu;
    cv[k] = (uint32_t)(k - hv) < (uint32_t)lv ? cv[k] : 0xFFFFFFFEu;
    below += cv[k] < u ? 1 : 0;
  }
  uint64_t M = 0;
#pragma unroll
  for (int p = 0; p < RC; p++) {
    uint32_t mw = 0;   // weight of cu[p] in row v (0: absent)
#pragma unroll
    for (int q = 0; q < RC; q++) mw = cu[p] == cv[q] ? wv[q] : mw;
    M += umin64(wmul<NARROW>(wu[p], dv), wmul<NARROW>(mw, du));
  }
  return M;
}

// floor(N * 2^b / D) for N < 2^63, D < 2^62, b <= 61 (the result is below 2^62);
// exact says whether the division left no remainder (then two edges with the
// same K have exactly the same score).
__device__ __forceinline__ uint64_t fixed_key(uint64_t N, uint64_t D, int b, bool& exact) {
  if ((N >> (63 - b)) == 0) {
    uint64_t num = N << b;
    uint64_t q;
    if (num < (1ull << 53) && D < (1ull << 53)) {
      // the correctly rounded quotient is at most one above the floor
      q = (uint64_t)((double)num / (double)D);
      if (q * D > num) q--;
    } else {
      q = num / D;
    }
    exact = q * D == num;
    return q;
  }
  unsigned __int128 num = (unsigned __int128)N << b;
  uint64_t q = (uint64_t)(num / D);
  exact = (unsigned __int128)q * D == num;
  return q;
}

// The same for b <= 50: the quotient is below 2^51, so its double-precision
// estimate (three correctly rounded steps, relative error under 2^-51) is
// within one of the floor, and one exact step on the remainder
// N 2^b - q D (in (-D, 2D), so exact modulo 2^64) corrects it.
__device__ __forceinline__ uint64_t fixed_key_fast(uint64_t N, uint64_t D, int b, bool& exact) {
  double x = (double)N / (double)D * (double)(1ull << b);
  uint64_t q = (uint64_t)x;
  int64_t r = (int64_t)((N << b) - q * D);
  if (r < 0) {
    q--;
    r += (int64_t)D;
  } else if (r >= (int64_t)D) {
    q++;
    r -= (int64_t)D;
  }
  exact = r == 0;
  return q;
}

__device__ __forceinline__ uint64_t fixed_key(uint64_t N, uint64_t D, int b) {
  bool exact;
  return fixed_key(N, D, b, exact);
}


}  // namespace spc

// Batched coarsening: many independent graphs coarsened as one block-diagonal
// graph, each to its own target.  Algorithm 1's merge loop runs per graph;
// since the graphs share no edge, the union's minimum spanning forest is the
// union of the graphs' forests, and graph i's merges are the components of
// its k[i] lightest forest edges.  The kernels below pick those per graph:
// forest edges are sorted by (graph, key) and the first k[i] of each graph's
// run are joined.  Edge ids, and so the tie-break, keep each graph's own
// (u, v) order because graph i's node ids are a contiguous, increasing range.
#include "score.hpp"

namespace spc {

struct KeyGK {
  uint64_t g, key, i;
};

struct LessGK {
  __device__ __forceinline__ bool operator()(const KeyGK& a, const KeyGK& b) const {
    return a.g < b.g || (a.g == b.g && a.key < b.key);
  }
};

// graph of node x: the last i with off[i] <= x
__device__ __forceinline__ int64_t graph_of(const int64_t* __restrict__ off, int64_t G, int64_t x) {
  int64_t lo = 0, hi = G - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// first position p in s[0..n) with s[p].g >= gid
__device__ __forceinline__ int64_t seg_lower(const KeyGK* __restrict__ s, int64_t n, uint64_t gid) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (s[mid].g < gid) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ void k_seg_records(const uint64_t* __restrict__ msfP, const uint64_t* __restrict__ msfO, int64_t n,
                              const int64_t* __restrict__ off, int64_t G, KeyGK* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t u = (int64_t)(uint32_t)msfO[i];
  out[i] = KeyGK{(uint64_t)graph_of(off, G, u), msfP[i], (uint64_t)i};
}

__device__ __forceinline__ void atomic_max_double(unsigned long long* p, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

// Joins each graph's first k lightest forest edges; the last accepted edge of
// each graph contributes its exact score to epsilon; with guarded keys, a
// forest edge of the cutoff's K bucket whose exact score differs from the
// cutoff's flags the level (the packed order inside that bucket may then be
// inexact).
__global__ void k_seg_accept(const KeyGK* __restrict__ s, int64_t n, const int64_t* __restrict__ kseg,
                             const uint64_t* __restrict__ msfO, int32_t* parent, LevelIn g,
                             const uint64_t* __restrict__ deg, const int32_t* __restrict__ lc,
                             const KeyND* __restrict__ exact, int ebits, unsigned long long* info) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  uint64_t gid = s[p].g;
  int64_t start = seg_lower(s, n, gid);
  int64_t k = kseg[gid];
  int64_t r = p - start;
  if (k <= 0) return;
  int64_t c = start + k - 1;              // the graph's cutoff position
  uint64_t uv = msfO[s[p].i];
  int32_t u = (int32_t)(uint32_t)uv, v = (int32_t)(uv >> 32);
  if (r < k) uf_union(parent, u, v);
  if (r == k - 1) {
    int64_t lo = g.rp[u], hi = g.rp[u + 1];
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (g.col[mid] < v) lo = mid + 1;
      else hi = mid;
    }
    uint64_t N, D;
    int64_t jm;
    edge_score(g, deg, lc, u, v, g.w[lo], N, D, jm);
    atomic_max_double(&info[I_EPS], (double)N / (double)D);
  }
  if (exact && info[I_GUARD] && c < n && s[c].g == gid && p != c) {
    uint64_t kp = s[p].key, kc = s[c].key;
    if ((kp >> ebits) == (kc >> ebits)) {
      uint64_t emask = (1ull << ebits) - 1;
      KeyND x = exact[kp & emask], y = exact[kc & emask];
      if ((unsigned __int128)x.N * y.D != (unsigned __int128)y.N * x.D) atomicOr(&info[I_VIOL], 1ull);
    }
  }
}

// a graph whose forest has fewer than k edges cannot reach its target
__global__ void k_seg_reach(const KeyGK* __restrict__ s, int64_t n, const int64_t* __restrict__ kseg, int64_t G,
                            unsigned long long* info) {
  int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= G) return;
  int64_t cnt = seg_lower(s, n, (uint64_t)gid + 1) - seg_lower(s, n, (uint64_t)gid);
  if (cnt < kseg[gid]) atomicOr(&info[I_SEG_SHORT], 1ull);
}

int seg_cutoff_union(spc_ctx* ctx, const LevelIn& g, LevelWork& W, const LevelResult& R, const Segments& seg,
                     int ebits, bool rank) {
  hipStream_t st = ctx->stream;
  int64_t n = R.msf;
  // the gather buffers of the contraction are free during selection and
  // hold 16 nnz + 64 bytes >= 24 bytes per forest edge; keysA keeps the
  // exact score records for the guarded checks
  KeyGK* A = (KeyGK*)W.gkeyA;
  KeyGK* B = (KeyGK*)W.gkeyB;
  KeyGK* sorted = A;
  if (n > 0) {
    hipLaunchKernelGGL(k_seg_records, dim3(grid_for(n, 256)), dim3(256), 0, st, W.msfP, W.msfO, n, seg.off,
                       seg.G, A);
    int rc = merge_sort<KeyGK, LessGK>(ctx, A, B, n, LessGK(), &sorted);
    if (rc) return rc;
    // packed keys: exact records (keysA) for the guarded check, consulted
    // only when the level's keys are guarded (info[I_GUARD])
    const KeyND* exact = rank ? nullptr : W.keysA;
    hipLaunchKernelGGL(k_seg_accept, dim3(grid_for(n, 256)), dim3(256), 0, st, sorted, n, seg.k, W.msfO,
                       W.parent, g, W.deg, W.lc, exact, ebits, W.info);
  }
  hipLaunchKernelGGL(k_seg_reach, dim3(grid_for(seg.G, 256)), dim3(256), 0, st, sorted, n, seg.k, seg.G, W.info);
  SPC_LAUNCH_CHECK(ctx, "batched cutoff");
  return SPC_OK;
}

}  // namespace spc

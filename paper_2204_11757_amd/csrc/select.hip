// Steps of one coarsening level up to the merge selection:
//   A1 degrees d_x (row sums of w_x, notation after Theorem 1),
//   A2 the fitness of every edge, || w_u/d_u - w_v/d_v ||_1 (Theorem 1,
//      Algorithm 1's fitness loop), evaluated exactly as N / D,
//   A3 a strict total order on edges (score, then smaller endpoint, then
//      larger endpoint) encoded as one unique 64-bit key per edge,
//   A4 the merge loop of Algorithm 1, computed as the components of the
//      lightest n - t edges of the minimum spanning forest under that order.
#include "level.hpp"

namespace spc {

// ---------------------------------------------------------------------------
// workspace plan
// ---------------------------------------------------------------------------
void plan_level(Arena& A, int64_t n, int64_t nnz, LevelWork& W) {
  int64_t m = nnz / 2;
  W.info = A.take<unsigned long long>(I_NINFO);
  W.deg = A.take<uint64_t>(n);
  W.lc = A.take<int32_t>(n);
  W.uptr = A.take<int64_t>(n + 1);
  W.longrows = A.take<int32_t>(n);
  W.P = A.take<uint64_t>(m);
  W.samples = A.take<uint64_t>(m / 64 + 2);
  W.bestA = A.take<uint64_t>(n);
  W.bestB = A.take<uint64_t>(n);
  W.parent = A.take<int32_t>(n);
  for (int i = 0; i < 2; i++) {
    W.lr[i] = A.take<uint64_t>(m);
    W.lp[i] = A.take<uint64_t>(m);
    W.lo[i] = A.take<uint64_t>(m);
  }
  W.msfP = A.take<uint64_t>(n);
  W.msfO = A.take<uint64_t>(n);
  W.root = A.take<int32_t>(n);
  W.flag = A.take<int32_t>(n + 1);
  W.sel = A.take<SelState>(1);
  W.sel2 = A.take<SelState>(1);
  W.scan_partial = A.take<int64_t>(SCAN_MAXB);
  W.keysA = A.take<KeyND>(m);
  W.keysB = A.take<KeyND>(m);
  W.mcount = A.take<int32_t>(n + 1);
  W.mptr = A.take<int32_t>(n + 1);
  W.members = A.take<int32_t>(n);
  W.gptr = A.take<int64_t>(n + 1);
  W.temp = A.take<uint64_t>(nnz);
  W.cnt = A.take<int64_t>(n + 1);
  W.midlist = A.take<int32_t>(n);
  W.hugelist = A.take<int32_t>(n);
  W.hmoff = A.take<int64_t>(n + 1);
  W.hmrow = A.take<int32_t>(n);
  W.hmnode = A.take<int32_t>(n);
  W.hpos = A.take<int64_t>(n + 1);
  W.gkeyA = A.take<uint64_t>(2 * nnz);
  W.gkeyB = A.take<uint64_t>(2 * nnz);
}

// ---------------------------------------------------------------------------
// A1: degrees, upper-entry counts, and per-level initialisation
// ---------------------------------------------------------------------------
constexpr int DEG_BS = 256;
constexpr int DEG_SHORT = 64;

__global__ void __launch_bounds__(DEG_BS)
    k_degree(LevelIn g, uint64_t* __restrict__ deg, int32_t* __restrict__ lc,
             int64_t* __restrict__ ucnt, uint64_t* __restrict__ bestA,
             uint64_t* __restrict__ bestB, int32_t* __restrict__ parent,
             int32_t* __restrict__ longrows, unsigned long long* info) {
  int64_t u = (int64_t)blockIdx.x * DEG_BS + threadIdx.x;
  uint64_t d = 0;
  bool isLong = false;
  if (u < g.n) {
    int64_t s = g.rp[u], e = g.rp[u + 1];
    // entries with col < u: binary search in the ascending row
    int64_t lo = s, hi = e;
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (g.col[mid] < u) lo = mid + 1;
      else hi = mid;
    }
    lc[u] = (int32_t)(lo - s);
    ucnt[u] = e - lo;
    if (e - s <= DEG_SHORT) {
      d = g.self ? (uint64_t)g.self[u] : 0;
      for (int64_t j = s; j < e; j++) d += (uint64_t)g.w[j];
      deg[u] = d;
    } else {
      isLong = true;
    }
    bestA[u] = KEY_INF;
    bestB[u] = KEY_INF;
    parent[u] = (int32_t)u;
  }
  int64_t slot = wave_append(&info[I_LONG], isLong);
  if (isLong) longrows[slot] = (int32_t)u;
  uint64_t mx = wave_max(d);
  uint64_t sm = wave_sum(d);
  if (lane_id() == 0) {
    if (mx) atomicMax(&info[I_DMAX], (unsigned long long)mx);
    if (sm) atomicAdd(&info[I_TOTAL], (unsigned long long)sm);
  }
}

__global__ void __launch_bounds__(DEG_BS)
    k_degree_long(LevelIn g, const int32_t* __restrict__ longrows, uint64_t* __restrict__ deg,
                  unsigned long long* info) {
  __shared__ uint64_t tmp[DEG_BS / WAVE];
  int64_t u = longrows[blockIdx.x];
  int64_t s = g.rp[u], e = g.rp[u + 1];
  uint64_t d = 0;
  for (int64_t j = s + threadIdx.x; j < e; j += DEG_BS) d += (uint64_t)g.w[j];
  d = wave_sum(d);
  if (lane_id() == 0) tmp[threadIdx.x / WAVE] = d;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = g.self ? (uint64_t)g.self[u] : 0;
    for (int i = 0; i < DEG_BS / WAVE; i++) t += tmp[i];
    deg[u] = t;
    atomicMax(&info[I_DMAX], (unsigned long long)t);
    atomicAdd(&info[I_TOTAL], (unsigned long long)t);
  }
}

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

__device__ __forceinline__ void edge_score(const LevelIn& g, const uint64_t* __restrict__ deg,
                                           int32_t u, int32_t v, int32_t wuv, uint64_t& N,
                                           uint64_t& D) {
  uint64_t du = deg[u], dv = deg[v];
  D = du * dv;
  uint64_t M = 0;
  if (g.self) {
    uint64_t su = (uint64_t)g.self[u], sv = (uint64_t)g.self[v];
    if (su) M += umin64(su * dv, (uint64_t)wuv * du);   // x = u
    if (sv) M += umin64((uint64_t)wuv * dv, sv * du);   // x = v
  }
  M += common_min_sum(g.col, g.w, g.rp[u], g.rp[u + 1], dv, g.rp[v], g.rp[v + 1], du);
  N = 2 * D - 2 * M;
}

// floor(N * 2^b / D) for N < 2^63, D < 2^62 and a result below 2^62.
__device__ __forceinline__ uint64_t fixed_key(uint64_t N, uint64_t D, int b) {
  if (b < 63 && (N >> (63 - b)) == 0) {
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

// ---------------------------------------------------------------------------
// A2 + A3 (packed key) and the first spanning-forest round, fused:
// one thread per edge (u < v), tiles of 256 consecutive edge ids mapped to
// rows by a load-balanced search over the upper-entry prefix uptr.
// ---------------------------------------------------------------------------
constexpr int TILE_E = 256;

struct EdgeTile {
  int32_t srow[TILE_E];
  int64_t sh[2];
  int32_t stmp[TILE_E / WAVE];
};

template <int MODE>  // 0: packed key, 1: write (N, D, e) for the rank sort
__global__ void __launch_bounds__(TILE_E)
    k_score(LevelIn g, const uint64_t* __restrict__ deg, const int32_t* __restrict__ lc,
            const int64_t* __restrict__ uptr, int64_t m, int b, int ebits,
            uint64_t* __restrict__ P, uint64_t* __restrict__ bestA,
            uint64_t* __restrict__ samples, KeyND* __restrict__ keys) {
  __shared__ EdgeTile T;
  int64_t e0 = (int64_t)blockIdx.x * TILE_E;
  lbs_tile<TILE_E, TILE_E>(uptr, g.n, e0, T.srow, T.sh, T.stmp);
  int tid = threadIdx.x;
  int64_t e = e0 + tid;
  if (e >= m) return;
  int32_t u = T.srow[tid];
  int64_t j = g.rp[u] + lc[u] + (e - uptr[u]);
  int32_t v = g.col[j];
  int32_t wuv = g.w[j];
  uint64_t N, D;
  edge_score(g, deg, u, v, wuv, N, D);
  if (MODE == 0) {
    uint64_t K = fixed_key(N, D, b);
    uint64_t key = (K << ebits) | (uint64_t)e;
    P[e] = key;
    atomicMin((unsigned long long*)&bestA[u], (unsigned long long)key);
    atomicMin((unsigned long long*)&bestA[v], (unsigned long long)key);
    if ((e & 63) == 0) samples[e >> 6] = key;
  } else {
    keys[e] = KeyND{N, D, (uint64_t)e};
  }
}

// Generic edge pass with the same tile mapping.  F(e, u, v, valid) is called
// by every thread of the block (valid is false beyond m).
template <typename F>
__global__ void __launch_bounds__(TILE_E)
    k_edge_pass(LevelIn g, const int32_t* __restrict__ lc, const int64_t* __restrict__ uptr,
                int64_t m, F f) {
  __shared__ EdgeTile T;
  int64_t e0 = (int64_t)blockIdx.x * TILE_E;
  lbs_tile<TILE_E, TILE_E>(uptr, g.n, e0, T.srow, T.sh, T.stmp);
  int tid = threadIdx.x;
  int64_t e = e0 + tid;
  bool valid = e < m;
  int32_t u = 0, v = 0;
  if (valid) {
    u = T.srow[tid];
    int64_t j = g.rp[u] + lc[u] + (e - uptr[u]);
    v = g.col[j];
  }
  f(e, u, v, valid);
}

// rank mode: P[e] = position of e in the sorted order
__global__ void k_rank_scatter(const KeyND* __restrict__ sorted, int64_t m, uint64_t* __restrict__ P) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < m) P[sorted[r].e] = (uint64_t)r;
}

struct BestFn {  // first spanning-forest round over every edge
  const uint64_t* P;
  uint64_t* best;
  __device__ void operator()(int64_t e, int32_t u, int32_t v, bool valid) const {
    if (!valid) return;
    uint64_t key = P[e];
    atomicMin((unsigned long long*)&best[u], (unsigned long long)key);
    atomicMin((unsigned long long*)&best[v], (unsigned long long)key);
  }
};

struct FilterFn {  // edges with key <= threshold form the live list
  const uint64_t* P;
  const unsigned long long* thr;
  uint64_t* lr;
  uint64_t* lp;
  uint64_t* lo;
  unsigned long long* cnt;
  __device__ void operator()(int64_t e, int32_t u, int32_t v, bool valid) const {
    uint64_t key = valid ? P[e] : KEY_INF;
    bool keep = valid && key <= *thr;
    int64_t s = wave_append(cnt, keep);
    if (keep) {
      uint64_t uv = (uint64_t)(uint32_t)u | ((uint64_t)(uint32_t)v << 32);
      lr[s] = uv;
      lp[s] = key;
      lo[s] = uv;
    }
  }
};

// ---------------------------------------------------------------------------
// A4: spanning-forest rounds (Boruvka) on the live list.
// ---------------------------------------------------------------------------
constexpr int BV_BS = 256;

// Every component adopts its lightest live edge; those edges are joined and
// recorded as forest edges.
__global__ void __launch_bounds__(BV_BS)
    k_bv_merge(const uint64_t* __restrict__ lr, const uint64_t* __restrict__ lp,
               const uint64_t* __restrict__ lo, const unsigned long long* cnt,
               const uint64_t* __restrict__ best, int32_t* parent, uint64_t* __restrict__ msfP,
               uint64_t* __restrict__ msfO, unsigned long long* msfcnt, int64_t msf_cap) {
  int64_t n = (int64_t)*cnt;
  int64_t stride = (int64_t)gridDim.x * BV_BS;
  for (int64_t base = (int64_t)blockIdx.x * BV_BS; base < n; base += stride) {
    int64_t i = base + threadIdx.x;
    bool chosen = false;
    uint64_t key = 0, uv = 0;
    if (i < n) {
      uv = lr[i];
      key = lp[i];
      int32_t a = (int32_t)(uint32_t)uv, b = (int32_t)(uv >> 32);
      chosen = (best[a] == key) || (best[b] == key);
      if (chosen) uf_union(parent, a, b);
    }
    int64_t s = wave_append(msfcnt, chosen);
    if (chosen && s < msf_cap) {  // a forest has fewer than n edges
      msfP[s] = key;
      msfO[s] = lo[i];
    }
  }
}

// Live edges between different components, with the endpoints replaced by
// their current roots, move to the next list; each component's lightest
// live edge is found with atomicMin on the key.  The other best array is
// reset at every root that still has a live edge.
__global__ void __launch_bounds__(BV_BS)
    k_bv_candidates(const uint64_t* __restrict__ lr_in, const uint64_t* __restrict__ lp_in,
                    const uint64_t* __restrict__ lo_in, const unsigned long long* cnt_in,
                    uint64_t* __restrict__ lr_out, uint64_t* __restrict__ lp_out,
                    uint64_t* __restrict__ lo_out, unsigned long long* cnt_out, uint64_t* cur,
                    uint64_t* nxt, int32_t* parent) {
  int64_t n = (int64_t)*cnt_in;
  int64_t stride = (int64_t)gridDim.x * BV_BS;
  for (int64_t base = (int64_t)blockIdx.x * BV_BS; base < n; base += stride) {
    int64_t i = base + threadIdx.x;
    bool keep = false;
    uint64_t key = 0, ruv = 0;
    if (i < n) {
      uint64_t uv = lr_in[i];
      key = lp_in[i];
      int32_t a = uf_find(parent, (int32_t)(uint32_t)uv);
      int32_t b = uf_find(parent, (int32_t)(uv >> 32));
      if (a != b) {
        keep = true;
        atomicMin((unsigned long long*)&cur[a], (unsigned long long)key);
        atomicMin((unsigned long long*)&cur[b], (unsigned long long)key);
        nxt[a] = KEY_INF;
        nxt[b] = KEY_INF;
        ruv = (uint64_t)(uint32_t)a | ((uint64_t)(uint32_t)b << 32);
      }
    }
    int64_t s = wave_append(cnt_out, keep);
    if (keep) {
      lr_out[s] = ruv;
      lp_out[s] = key;
      lo_out[s] = lo_in[i];
    }
  }
}

// ---------------------------------------------------------------------------
// components of the forest edges with key <= T, canonical numbering
// ---------------------------------------------------------------------------
__global__ void k_iota(int32_t* __restrict__ a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = (int32_t)i;
}

__global__ void k_cc_union(const uint64_t* __restrict__ msfP, const uint64_t* __restrict__ msfO,
                           const unsigned long long* cnt, const SelState* thr, int32_t* parent) {
  int64_t n = (int64_t)*cnt;
  uint64_t T = thr->prefix;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    if (msfP[i] <= T) {
      uint64_t uv = msfO[i];
      uf_union(parent, (int32_t)(uint32_t)uv, (int32_t)(uv >> 32));
    }
  }
}

__global__ void k_cc_flatten(int32_t* parent, int32_t* __restrict__ root, int32_t* __restrict__ flag,
                             int64_t n) {
  int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < n) {
    int32_t r = uf_find(parent, (int32_t)x);
    root[x] = r;
    flag[x] = (r == (int32_t)x) ? 1 : 0;
  }
}

__global__ void k_relabel(const int32_t* __restrict__ root, const int32_t* __restrict__ cid,
                          int32_t* __restrict__ cluster_of, int64_t n) {
  int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < n) cluster_of[x] = cid[root[x]];
}

// ---------------------------------------------------------------------------
// radix select (declared in prim.hpp)
// ---------------------------------------------------------------------------
__global__ void k_sel_init(SelState* st, const unsigned long long* k_dev, unsigned long long k_host) {
  int t = threadIdx.x;
  if (t == 0) {
    st->prefix = 0;
    st->mask = 0;
    st->k = k_dev ? *k_dev : k_host;
  }
  for (int b = t; b < SEL_BINS; b += blockDim.x) st->hist[b] = 0;
}

__global__ void __launch_bounds__(256)
    k_sel_hist(const uint64_t* __restrict__ keys, const unsigned long long* cnt_dev, int64_t cnt_host,
               SelState* st, int shift, int width) {
  __shared__ unsigned int h[SEL_BINS];
  int nb = 1 << width;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) h[b] = 0;
  __syncthreads();
  int64_t n = cnt_dev ? (int64_t)*cnt_dev : cnt_host;
  uint64_t prefix = st->prefix, mask = st->mask;
  uint64_t dm = (uint64_t)(nb - 1);
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    uint64_t k = keys[i];
    if ((k & mask) == prefix) atomicAdd(&h[(k >> shift) & dm], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
    if (h[b]) atomicAdd(&st->hist[b], h[b]);
}

__global__ void __launch_bounds__(1024) k_sel_pick(SelState* st, int shift, int width) {
  __shared__ unsigned long long tmp[1024 / WAVE];
  int t = threadIdx.x;
  int nb = 1 << width;
  // thread t owns bins 2t and 2t+1
  unsigned long long c0 = (2 * t < nb) ? st->hist[2 * t] : 0;
  unsigned long long c1 = (2 * t + 1 < nb) ? st->hist[2 * t + 1] : 0;
  unsigned long long tot;
  unsigned long long inc = block_incl_scan<unsigned long long, 1024, false>(c0 + c1, tmp, &tot);
  unsigned long long before = inc - c0 - c1;
  unsigned long long k = st->k;
  __syncthreads();
  int bucket = -1;
  unsigned long long sub = 0;
  if (k >= before && k < before + c0) {
    bucket = 2 * t;
    sub = before;
  } else if (k >= before + c0 && k < before + c0 + c1) {
    bucket = 2 * t + 1;
    sub = before + c0;
  }
  __syncthreads();
  if (bucket >= 0) {
    st->k = k - sub;
    st->prefix |= (unsigned long long)bucket << shift;
    st->mask |= (unsigned long long)(nb - 1) << shift;
  }
  __syncthreads();
  for (int b = t; b < SEL_BINS; b += blockDim.x) st->hist[b] = 0;
}

int radix_select(spc_ctx* ctx, const uint64_t* keys, const unsigned long long* cnt_dev,
                 int64_t cnt_bound, const unsigned long long* k_dev, unsigned long long k_host,
                 int bits, SelState* st) {
  hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, ctx->stream, st, k_dev, k_host);
  int grid = grid_for(cnt_bound, 256 * 16, 4096);
  for (int hi = bits; hi > 0;) {
    int lo = hi - SEL_DIGIT > 0 ? hi - SEL_DIGIT : 0;
    int width = hi - lo;
    hipLaunchKernelGGL(k_sel_hist, dim3(grid), dim3(256), 0, ctx->stream, keys, cnt_dev, cnt_bound,
                       st, lo, width);
    hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(1024), 0, ctx->stream, st, lo, width);
    hi = lo;
  }
  SPC_LAUNCH_CHECK(ctx, "radix_select");
  return SPC_OK;
}

// ---------------------------------------------------------------------------
// host orchestration of A1-A4
// ---------------------------------------------------------------------------
__global__ void k_set_u64(unsigned long long* p, unsigned long long v) { *p = v; }

__global__ void k_fill_u64(uint64_t* __restrict__ a, int64_t n, uint64_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// threshold of the live list: the selected sample key, or "everything"
__global__ void k_thr_from_sel(const SelState* st, unsigned long long* thr, int all) {
  *thr = all ? KEY_INF : st->prefix;
}

// Theorem 2's epsilon: the score of the heaviest accepted edge, which is
// the forest edge whose key equals the cutoff.
__global__ void k_eps(LevelIn g, const uint64_t* __restrict__ deg, const uint64_t* __restrict__ msfP,
                      const uint64_t* __restrict__ msfO, const unsigned long long* cnt,
                      const SelState* st, double* out) {
  int64_t n = (int64_t)*cnt;
  uint64_t T = st->prefix;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    if (msfP[i] != T) continue;
    uint64_t uv = msfO[i];
    int32_t u = (int32_t)(uint32_t)uv, v = (int32_t)(uv >> 32);
    int64_t lo = g.rp[u], hi = g.rp[u + 1];
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (g.col[mid] < v) lo = mid + 1;
      else hi = mid;
    }
    uint64_t N, D;
    edge_score(g, deg, u, v, g.w[lo], N, D);
    *out = (double)N / (double)D;
  }
}

static int spanning_forest(spc_ctx* ctx, LevelWork& W, int64_t n, int64_t& rounds,
                           int64_t& live0) {
  unsigned long long* info = W.info;
  int64_t* hinfo = ctx->h_pinned;
  // round 1 on the filtered list with bestA from the score pass
  SPC_HIP(ctx, hipMemcpyAsync(hinfo, info, sizeof(unsigned long long) * I_NINFO,
                              hipMemcpyDeviceToHost, ctx->stream));
  SPC_HIP(ctx, hipStreamSynchronize(ctx->stream));
  int64_t cnt = hinfo[I_LIVE0];
  live0 = cnt;
  rounds = 1;
  int maxgrid = ctx->num_cus * 8;
  hipLaunchKernelGGL(k_bv_merge, dim3(grid_for(cnt, BV_BS, maxgrid)), dim3(BV_BS), 0, ctx->stream,
                     W.lr[0], W.lp[0], W.lo[0], &info[I_LIVE0], W.bestA, W.parent, W.msfP, W.msfO,
                     &info[I_MSF], n);
  int in = 0;
  uint64_t* cur = W.bestB;
  uint64_t* nxt = W.bestA;
  while (cnt > 0) {
    // every round at least halves the components that still have live
    // edges, so more than 64 rounds means corrupted state
    if (rounds > 64) return set_error(ctx, SPC_EINVAL, "internal: spanning forest did not converge");
    int out = in ^ 1;
    int ci = in == 0 ? I_LIVE0 : I_LIVE1;
    int co = out == 0 ? I_LIVE0 : I_LIVE1;
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, ctx->stream, &info[co], 0ull);
    hipLaunchKernelGGL(k_bv_candidates, dim3(grid_for(cnt, BV_BS, maxgrid)), dim3(BV_BS), 0,
                       ctx->stream, W.lr[in], W.lp[in], W.lo[in], &info[ci], W.lr[out], W.lp[out],
                       W.lo[out], &info[co], cur, nxt, W.parent);
    SPC_LAUNCH_CHECK(ctx, "boruvka candidates");
    SPC_HIP(ctx, hipMemcpyAsync(&hinfo[co], &info[co], sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, ctx->stream));
    SPC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    cnt = hinfo[co];
    if (cnt == 0) break;
    rounds++;
    hipLaunchKernelGGL(k_bv_merge, dim3(grid_for(cnt, BV_BS, maxgrid)), dim3(BV_BS), 0,
                       ctx->stream, W.lr[out], W.lp[out], W.lo[out], &info[co], cur, W.parent,
                       W.msfP, W.msfO, &info[I_MSF], n);
    SPC_LAUNCH_CHECK(ctx, "boruvka merge");
    uint64_t* t = cur;
    cur = nxt;
    nxt = t;
    in = out;
  }
  return SPC_OK;
}

int select_level(spc_ctx* ctx, const LevelIn& g, int64_t t, int32_t* cluster_of, LevelWork& W,
                 LevelResult& R) {
  hipStream_t st = ctx->stream;
  int64_t n = g.n, m = g.nnz / 2;
  int64_t k = n - t;  // merges
  unsigned long long* info = W.info;
  int64_t* hinfo = ctx->h_pinned;
  SPC_HIP(ctx, hipMemsetAsync(info, 0, sizeof(unsigned long long) * I_NINFO, st));

  // A1
  hipLaunchKernelGGL(k_degree, dim3(grid_for(n, DEG_BS)), dim3(DEG_BS), 0, st, g, W.deg, W.lc, W.uptr,
                     W.bestA, W.bestB, W.parent, W.longrows, info);
  SPC_LAUNCH_CHECK(ctx, "degree");
  SPC_HIP(ctx, hipMemcpyAsync(hinfo, info, sizeof(unsigned long long) * I_NINFO,
                              hipMemcpyDeviceToHost, st));
  SPC_HIP(ctx, hipStreamSynchronize(st));
  int64_t nlong = hinfo[I_LONG];
  if (nlong > 0) {
    hipLaunchKernelGGL(k_degree_long, dim3((unsigned)nlong), dim3(DEG_BS), 0, st, g, W.longrows,
                       W.deg, info);
    SPC_LAUNCH_CHECK(ctx, "degree_long");
    SPC_HIP(ctx, hipMemcpyAsync(hinfo, info, sizeof(unsigned long long) * I_NINFO,
                                hipMemcpyDeviceToHost, st));
    SPC_HIP(ctx, hipStreamSynchronize(st));
  }
  uint64_t dmax = (uint64_t)hinfo[I_DMAX];
  uint64_t total = (uint64_t)hinfo[I_TOTAL];
  if (total > 2147483647ull)
    return set_error(ctx, SPC_EOVERFLOW, "total integer weight %llu exceeds 2^31-1",
                     (unsigned long long)total);
  {
    int rc = exclusive_scan<int64_t>(ctx, W.uptr, W.uptr, n, (int64_t*)W.scan_partial);
    if (rc) return rc;
  }
  if (k <= 0 || m == 0) {
    if (k > 0) return set_error(ctx, SPC_EUNREACHABLE, "graph has no edges");
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n, 256)), dim3(256), 0, st, cluster_of, n);
    R.n_c = n;
    R.eps = 0.0;
    return SPC_OK;
  }

  // A2 + A3
  int L = bitlen64(dmax > 0 ? dmax - 1 : 0);  // dmax <= 2^L
  int b = 4 * L;                               // 2^b >= (max D)^2
  int ebits = bitlen64((uint64_t)(m - 1));
  if (ebits < 1) ebits = 1;
  bool packed = (b + 2 + ebits <= 64) && !ctx->force_rank_mode;
  R.key_mode = packed ? 0 : 1;
  R.key_bits = packed ? b + 2 + ebits : bitlen64((uint64_t)(m - 1));
  int eg = grid_for(m, TILE_E);
  KeyND* sorted = nullptr;
  if (packed) {
    hipLaunchKernelGGL(k_score<0>, dim3(eg), dim3(TILE_E), 0, st, g, W.deg, W.lc, W.uptr, m, b,
                       ebits, W.P, W.bestA, W.samples, (KeyND*)nullptr);
    SPC_LAUNCH_CHECK(ctx, "score");
  } else {
    hipLaunchKernelGGL(k_score<1>, dim3(eg), dim3(TILE_E), 0, st, g, W.deg, W.lc, W.uptr, m, b,
                       ebits, (uint64_t*)nullptr, (uint64_t*)nullptr, (uint64_t*)nullptr, W.keysA);
    SPC_LAUNCH_CHECK(ctx, "score(rank)");
    int rc = merge_sort<KeyND, LessND>(ctx, W.keysA, W.keysB, m, LessND(), &sorted);
    if (rc) return rc;
    hipLaunchKernelGGL(k_rank_scatter, dim3(grid_for(m, 256)), dim3(256), 0, st, sorted, m, W.P);
    hipLaunchKernelGGL((k_edge_pass<BestFn>), dim3(eg), dim3(TILE_E), 0, st, g, W.lc, W.uptr, m,
                       BestFn{W.P, W.bestA});
    SPC_LAUNCH_CHECK(ctx, "rank best");
  }

  // A4: live list of the lightest edges, spanning forest, cutoff, components
  unsigned long long* thr = &info[I_BAD];  // reuse a slot for the live threshold
  int64_t target = k + k / 2 + 4096;
  bool all = ctx->force_full_filter || target >= m;
  for (int attempt = 0; attempt < 2; attempt++) {
    if (attempt == 1) {
      // not enough forest edges below the threshold: redo over every edge
      all = true;
      hipLaunchKernelGGL(k_iota, dim3(grid_for(n, 256)), dim3(256), 0, st, W.parent, n);
      hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, st, W.bestA, n, KEY_INF);
      hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, st, W.bestB, n, KEY_INF);
      hipLaunchKernelGGL((k_edge_pass<BestFn>), dim3(eg), dim3(TILE_E), 0, st, g, W.lc, W.uptr, m,
                         BestFn{W.P, W.bestA});
      hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, &info[I_MSF], 0ull);
    }
    if (all) {
      hipLaunchKernelGGL(k_thr_from_sel, dim3(1), dim3(1), 0, st, W.sel, thr, 1);
    } else if (packed) {
      int64_t ns = (m + 63) / 64;
      int64_t q = (int64_t)((double)target / 64.0 * 1.05) + 16;
      if (q >= ns) {
        hipLaunchKernelGGL(k_thr_from_sel, dim3(1), dim3(1), 0, st, W.sel, thr, 1);
      } else {
        int rc = radix_select(ctx, W.samples, nullptr, ns, nullptr, (unsigned long long)q,
                              b + 2 + ebits, W.sel);
        if (rc) return rc;
        hipLaunchKernelGGL(k_thr_from_sel, dim3(1), dim3(1), 0, st, W.sel, thr, 0);
      }
    } else {
      hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, thr, (unsigned long long)(target - 1));
    }
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, &info[I_LIVE0], 0ull);
    hipLaunchKernelGGL((k_edge_pass<FilterFn>), dim3(eg), dim3(TILE_E), 0, st, g, W.lc, W.uptr, m,
                       FilterFn{W.P, thr, W.lr[0], W.lp[0], W.lo[0], &info[I_LIVE0]});
    SPC_LAUNCH_CHECK(ctx, "filter");
    int64_t rounds = 0, live0 = 0;
    int rc = spanning_forest(ctx, W, n, rounds, live0);
    if (rc) return rc;
    SPC_HIP(ctx, hipMemcpyAsync(hinfo, info, sizeof(unsigned long long) * I_NINFO,
                                hipMemcpyDeviceToHost, st));
    SPC_HIP(ctx, hipStreamSynchronize(st));
    R.rounds = rounds;
    R.candidates = live0;
    R.msf = hinfo[I_MSF];
    if (R.msf >= k) break;
    if (all) return set_error(ctx, SPC_EUNREACHABLE,
                              "only %lld merges possible, %lld requested (graph has more than %lld components)",
                              (long long)R.msf, (long long)k, (long long)t);
  }

  // cutoff: the k-th lightest forest edge
  int bits = packed ? (b + 2 + ebits) : bitlen64((uint64_t)(m - 1));
  {
    int rc = radix_select(ctx, W.msfP, &info[I_MSF], n, nullptr, (unsigned long long)(k - 1), bits,
                          W.sel2);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_iota, dim3(grid_for(n, 256)), dim3(256), 0, st, W.parent, n);
  hipLaunchKernelGGL(k_cc_union, dim3(grid_for(R.msf, 256, ctx->num_cus * 8)), dim3(256), 0, st,
                     W.msfP, W.msfO, &info[I_MSF], W.sel2, W.parent);
  hipLaunchKernelGGL(k_cc_flatten, dim3(grid_for(n, 256)), dim3(256), 0, st, W.parent, W.root,
                     W.flag, n);
  SPC_LAUNCH_CHECK(ctx, "components");
  {
    int rc = exclusive_scan<int32_t>(ctx, W.flag, W.flag, n, (int32_t*)W.scan_partial);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_relabel, dim3(grid_for(n, 256)), dim3(256), 0, st, W.root, W.flag,
                     cluster_of, n);
  double* deps = (double*)&info[I_EPS];
  hipLaunchKernelGGL(k_eps, dim3(grid_for(R.msf, 256, ctx->num_cus * 4)), dim3(256), 0, st, g, W.deg,
                     W.msfP, W.msfO, &info[I_MSF], W.sel2, deps);
  SPC_LAUNCH_CHECK(ctx, "relabel");
  int32_t nc32 = 0;
  SPC_HIP(ctx, hipMemcpyAsync(&nc32, W.flag + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  SPC_HIP(ctx, hipMemcpyAsync(hinfo, info, sizeof(unsigned long long) * I_NINFO,
                              hipMemcpyDeviceToHost, st));
  SPC_HIP(ctx, hipStreamSynchronize(st));
  double eps;
  memcpy(&eps, &hinfo[I_EPS], sizeof(double));
  R.eps = eps;
  R.n_c = nc32;
  if (R.n_c != t)
    return set_error(ctx, SPC_EINVAL, "internal: %lld super-nodes produced, %lld expected",
                     (long long)R.n_c, (long long)t);
  return SPC_OK;
}

}  // namespace spc

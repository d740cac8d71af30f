// Batched coarsening: many independent graphs coarsened as one block-diagonal
// graph, each to its own target.  Algorithm 1's merge loop runs per graph;
// since the graphs share no edge, the union's minimum spanning forest is the
// union of the graphs' forests, and graph i's merges are the components of
// its k[i] lightest forest edges.  Every forest edge hooked exactly one
// component root, so keying the forest by hooked node puts graph i's forest
// edges in its own node range: one block per graph selects its k[i]-th key
// there and joins the edges up to it.  Edge ids, and so the tie-break, keep
// each graph's own (u, v) order because graph i's node ids are a contiguous,
// increasing range.
#include "radix.hpp"
#include "score.hpp"

namespace spc {

// fkey[x] = key of the forest edge that hooked node x, fidx[x] = its record
__global__ void k_forest_by_node(const uint64_t* __restrict__ msfP, const int32_t* __restrict__ msfC,
                                 const unsigned long long* cnt, uint64_t* __restrict__ fkey,
                                 uint64_t* __restrict__ fidx) {
  int64_t n = (int64_t)*cnt;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    int32_t x = msfC[i];
    fkey[x] = msfP[i];
    fidx[x] = (uint64_t)i;
  }
}

__device__ __forceinline__ void atomic_max_double(unsigned long long* p, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

// One block per graph: the (k-1)-th smallest forest key of the graph's node
// range (radix passes over the range with an LDS histogram, the extreme-key
// skip, and an LDS finish once at most SEG_SMALL keys remain), then the union
// of every forest edge up to it.  The cutoff edge's exact score goes into
// epsilon; with guarded keys, a forest edge of the cutoff's K bucket whose
// exact score differs from the cutoff's flags the level.  A graph with fewer
// than k forest edges sets info[I_SEG_SHORT].
__global__ void __launch_bounds__(SEL_BS)
    k_seg_select(const uint64_t* __restrict__ fkey, const uint64_t* __restrict__ fidx,
                 const int64_t* __restrict__ off, const int64_t* __restrict__ kseg,
                 const uint64_t* __restrict__ msfO, int32_t* parent, LevelIn g,
                 const uint64_t* __restrict__ deg, const int32_t* __restrict__ lc,
                 const KeyND* __restrict__ exact, const uint64_t* __restrict__ kexact, int ebits,
                 unsigned long long* info) {
  __shared__ unsigned int h[SEL_BINS];
  __shared__ uint64_t sbuf[SEG_SMALL];
  __shared__ uint64_t s2[LDS_SMALL2];
  __shared__ unsigned int s2cnt;
  __shared__ unsigned long long tmp[SEL_BS / WAVE];
  __shared__ unsigned long long red[2 * (SEL_BS / WAVE)];
  __shared__ unsigned long long spick[3];
  __shared__ unsigned int slocal;
  int t = threadIdx.x;
  int64_t gid = blockIdx.x;
  int64_t lo = off[gid], hi_n = off[gid + 1];
  int64_t kk = kseg[gid];
  if (kk <= 0) return;   // no merges in this graph
  unsigned long long k = (unsigned long long)(kk - 1);
  uint64_t prefix = 0, mask = 0;
  int hi = 64;
  int64_t cb = -1;   // keys matching (prefix, mask); unknown before the first pass
  bool first = true;
  while (hi > 0 && (cb < 0 || cb > SEG_SMALL)) {
    int lo_b = hi - SEL_DIGIT > 0 ? hi - SEL_DIGIT : 0;
    int nb = 1 << (hi - lo_b);
    uint64_t dm = (uint64_t)(nb - 1);
    for (int b = t; b < SEL_BINS; b += SEL_BS) h[b] = 0;
    __syncthreads();
    uint64_t mn = ~0ull, mx = 0;
    for (int64_t i0 = lo; i0 < hi_n; i0 += SEL_BS * SEL_UNROLL) {
      uint64_t x[SEL_UNROLL];
#pragma unroll
      for (int u = 0; u < SEL_UNROLL; u++) {
        int64_t i = i0 + u * SEL_BS + t;
        x[u] = i < hi_n ? fkey[i] : KEY_INF;
      }
#pragma unroll
      for (int u = 0; u < SEL_UNROLL; u++) {
        bool m = x[u] != KEY_INF && (x[u] & mask) == prefix;
        hist_add(h, m, (uint32_t)((x[u] >> lo_b) & dm));
        if (m) {
          mn = x[u] < mn ? x[u] : mn;
          mx = x[u] > mx ? x[u] : mx;
        }
      }
    }
    __syncthreads();
    block_minmax(mn, mx, red);
    unsigned long long cnt = 0;
    for (int q = 0; q < SEL_BINS / SEL_BS; q++) {
      int b = SEL_BINS / SEL_BS * t + q;
      cnt += b < nb ? h[b] : 0u;
    }
    unsigned long long total;
    unsigned long long before = block_incl_scan<unsigned long long, SEL_BS, false>(cnt, tmp, &total) - cnt;
    if (first && total <= k) {
      // fewer forest edges than merges: the target is out of reach
      if (t == 0) atomicOr(&info[I_SEG_SHORT], 1ull);
      return;
    }
    if (k >= before && k < before + cnt) {
      unsigned long long acc = before;
      for (int q = 0; q < SEL_BINS / SEL_BS; q++) {
        int b = SEL_BINS / SEL_BS * t + q;
        unsigned long long c = b < nb ? h[b] : 0u;
        if (k >= acc && k < acc + c) {
          spick[0] = (unsigned long long)b;
          spick[1] = acc;
          spick[2] = c;
        }
        acc += c;
      }
    }
    __syncthreads();
    bool all_one = (unsigned long long)spick[2] == total;
    prefix |= spick[0] << lo_b;
    mask |= dm << lo_b;
    k -= spick[1];
    cb = (int64_t)spick[2];
    hi = lo_b;
    first = false;
    __syncthreads();
    if (all_one) {
      // every matching key is in this bucket: the bits the extreme ones share
      uint64_t xx = mn ^ mx;
      if (xx == 0) {
        prefix = mn;
        mask = ~0ull;
        hi = 0;
      } else {
        int d = 63 - __clzll((long long)xx);
        if (d + 1 < hi) {
          uint64_t low = (2ull << d) - 1;
          prefix = mn & ~low;
          mask = ~low;
          hi = d + 1;
        }
      }
    }
  }
  uint64_t cut;
  if (hi == 0) {
    cut = prefix;
  } else {
    // at most SEG_SMALL keys match: gather them and finish in LDS
    if (t == 0) slocal = 0;
    __syncthreads();
    for (int64_t i0 = lo; i0 < hi_n; i0 += SEL_BS) {
      int64_t i = i0 + t;
      uint64_t x = i < hi_n ? fkey[i] : KEY_INF;
      bool m = x != KEY_INF && (x & mask) == prefix;
      unsigned int q = wave_reserve(&slocal, m);
      if (m && q < (unsigned)SEG_SMALL) sbuf[q] = x;
    }
    __syncthreads();
    unsigned int c = slocal < (unsigned)SEG_SMALL ? slocal : (unsigned)SEG_SMALL;
    cut = lds_select(sbuf, (int)c, k, h, tmp, red, spick, &info[I_LBERR], s2, &s2cnt);
  }
  // join the forest edges up to the cutoff; the cutoff edge gives epsilon.
  // SJ nodes per thread at a time: their keys, records and endpoints are
  // each loaded together before the joins
  bool guarded = exact && info[I_GUARD];
  uint64_t emask = (1ull << ebits) - 1;
  constexpr int SJ = 4;
  for (int64_t x0 = lo; x0 < hi_n; x0 += SEL_BS * SJ) {
    uint64_t ks[SJ], uvs[SJ];
    int64_t fs[SJ];
#pragma unroll
    for (int q = 0; q < SJ; q++) {
      int64_t x = x0 + q * SEL_BS + t;
      ks[q] = x < hi_n ? fkey[x] : KEY_INF;
    }
#pragma unroll
    for (int q = 0; q < SJ; q++) {
      int64_t x = x0 + q * SEL_BS + t;
      fs[q] = ks[q] <= cut ? (int64_t)fidx[x] : -1;
    }
#pragma unroll
    for (int q = 0; q < SJ; q++) uvs[q] = fs[q] >= 0 ? msfO[fs[q]] : 0;
    for (int q = 0; q < SJ; q++) {
      uint64_t key = ks[q];
      if (key == KEY_INF) continue;
      if (key <= cut) {
        uint64_t uv = uvs[q];
        int32_t u = (int32_t)(uint32_t)uv, v = (int32_t)(uv >> 32);
        uf_union(parent, u, v);
        if (key == cut) {
          int64_t a = g.rp[u], b = g.rp[u + 1];
          while (a < b) {
            int64_t mid = (a + b) >> 1;
            if (g.col[mid] < v) a = mid + 1;
            else b = mid;
          }
          uint64_t N, D;
          int64_t jm;
          edge_score(g, deg, lc, u, v, g.w[a], N, D, jm);
          atomic_max_double(&info[I_EPS], (double)N / (double)D);
        }
      }
      if (guarded && key != cut && (key >> ebits) == (cut >> ebits) &&
          !(key_exact(kexact, key & emask) && key_exact(kexact, cut & emask))) {
        KeyND p = exact[key & emask], r = exact[cut & emask];
        if ((unsigned __int128)p.N * r.D != (unsigned __int128)r.N * p.D) atomicOr(&info[I_VIOL], 1ull);
      }
    }
  }
}

// Each node's graph: one block per graph writes its node range.
__global__ void k_seg_gid(const int64_t* __restrict__ off, int32_t* __restrict__ gid) {
  int64_t lo = off[blockIdx.x], hi = off[blockIdx.x + 1];
  for (int64_t u = lo + threadIdx.x; u < hi; u += blockDim.x) gid[u] = (int32_t)blockIdx.x;
}

// One block per graph: its band threshold.  The graph's CSR entries hold
// each of its edges' keys twice (both directions), so SB_S entries taken at
// even spacing sample the key distribution of its edges; sorted in LDS, the
// sample at the band's share (plus 5 % and two samples) gives the threshold.
// The band aims at 2 k + 64 edges for k merges: on triangle meshes of unit
// weight a graph's k-th forest edge lies at up to about 1.7 k in key order
// (the first two halving levels; less later), and a band that falls short
// costs the level a second selection over every edge.
// Graphs without merges take no candidates; graphs whose band would hold
// all of their edges take all of them.  (shrink, a test option: bands aim at
// a quarter of the merges and are not extended over ties, so that they fall
// short.)
constexpr int SB_S = 2048;
constexpr int SB_BS = 256;

__global__ void __launch_bounds__(SB_BS)
    k_seg_band(const int64_t* __restrict__ off, const int64_t* __restrict__ kseg, LevelIn g,
               const int64_t* __restrict__ uptr, const uint64_t* __restrict__ Pc, const unsigned long long* info,
               int ebits, int shrink, uint64_t* __restrict__ thrg) {
  __shared__ uint64_t sb[SB_S];
  int t = threadIdx.x;
  int64_t gi = blockIdx.x;
  int64_t lo = off[gi], hi = off[gi + 1];
  int64_t kk = kseg[gi];
  int64_t a = g.rp[lo], b = g.rp[hi];
  int64_t nnz_g = b - a, m_g = nnz_g / 2;
  int64_t target = shrink ? kk / 4 : 2 * kk + 64;
  if (kk <= 0 || target >= m_g) {   // (uniform over the block)
    if (t == 0) thrg[gi] = kk <= 0 ? 0ull : KEY_INF;
    return;
  }
  int S = nnz_g < SB_S ? (int)nnz_g : SB_S;
  for (int i = t; i < SB_S; i += SB_BS) sb[i] = i < S ? Pc[a + (int64_t)i * nnz_g / S] : KEY_INF;
  __syncthreads();
  // ascending bitonic sort of the samples
  for (int k = 2; k <= SB_S; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int p = t; p < SB_S / 2; p += SB_BS) {
        int i = 2 * j * (p / j) + (p % j);
        int l = i + j;
        bool asc = (i & k) == 0;
        uint64_t x = sb[i], y = sb[l];
        if (asc ? (y < x) : (x < y)) {
          sb[i] = y;
          sb[l] = x;
        }
      }
      __syncthreads();
    }
  }
  if (t != 0) return;
  double share = (double)target / (double)m_g * 1.05;
  int q = (int)(share * (double)S) + 2;
  if (q >= S) {
    thrg[gi] = KEY_INF;
    return;
  }
  uint64_t emask = (1ull << ebits) - 1;
  uint64_t p = sb[q];
  uint64_t thr = p;
  if (info[I_GUARD]) {
    // guarded keys order one K bucket only approximately: all of it
    thr = p | emask;
  } else if (!shrink && q >= 16 && (sb[q - 16] >> ebits) == (p >> ebits)) {
    // inside a tied K bucket, read in edge order (consecutive rows): cover
    // about 1.1 k rows of the graph
    double rows = 1.1 * (double)kk * (double)m_g / (double)(hi - lo) + 64.0;
    int64_t span = rows >= (double)(m_g - 1) ? m_g - 1 : (int64_t)rows;
    uint64_t tie = (p & ~emask) | (uint64_t)(uptr[lo] + span);
    thr = tie > thr ? tie : thr;
  }
  thrg[gi] = thr;
}

int seg_bands(spc_ctx* ctx, const LevelIn& g, LevelWork& W, const Segments& seg, int ebits, bool shrink) {
  hipLaunchKernelGGL(k_seg_gid, dim3((unsigned)seg.G), dim3(256), 0, ctx->stream, seg.off, W.gid);
  hipLaunchKernelGGL(k_seg_band, dim3((unsigned)seg.G), dim3(SB_BS), 0, ctx->stream, seg.off, seg.k, g, W.uptr,
                     W.Pc, W.info, ebits, shrink ? 1 : 0, W.thrg);
  SPC_LAUNCH_CHECK(ctx, "batch bands");
  return SPC_OK;
}

int seg_cutoff_union(spc_ctx* ctx, const LevelIn& g, LevelWork& W, const LevelResult& R, const Segments& seg,
                     int ebits, bool rank) {
  hipStream_t st = ctx->stream;
  int64_t n = g.n;
  // the lightest-key arrays of the forest rounds are free now
  uint64_t* fkey = W.bestA;
  uint64_t* fidx = W.bestB;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, st, fkey, n, KEY_INF);
  if (R.msf > 0)
    hipLaunchKernelGGL(k_forest_by_node, dim3(grid_for(R.msf, 256, ctx->num_cus * 16)), dim3(256), 0, st,
                       W.msfP, W.msfC, &W.info[I_MSF], fkey, fidx);
  // packed keys: exact records (keysA) for the guarded check, consulted
  // only when the level's keys are guarded (info[I_GUARD])
  const KeyND* exact = rank ? nullptr : W.keysA;
  hipLaunchKernelGGL(k_seg_select, dim3((unsigned)seg.G), dim3(SEL_BS), 0, st, fkey, fidx, seg.off, seg.k,
                     W.msfO, W.root, g, W.deg, W.lc, exact, W.kexact, ebits, W.info);
  SPC_LAUNCH_CHECK(ctx, "batched cutoff");
  return SPC_OK;
}

}  // namespace spc

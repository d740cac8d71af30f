// A2 and A3 of a coarsening level: the exact score of every edge and its
// order key, the sorted-rank scatter of the fallback order, and Theorem 2's
// epsilon of the accepted merges.
#include "score.hpp"

namespace spc {



// The edges of the mapped rows: one thread per entry j of a mapped row h,
// the other endpoint x = col[j].  Row x is read in chunks and looked up in
// h's map (when x is mapped too and its row is longer, the roles swap; such
// an edge is scored by the smaller endpoint's row only).
constexpr int HS_BLOCKS = 256;   // about one entry per thread for the rows seen in practice

template <int MODE>
__device__ __forceinline__ void score_mapped_block(
    int bid, LevelIn g, const uint64_t* __restrict__ deg, const int32_t* __restrict__ lc,
    const int64_t* __restrict__ uptr, int c, int ebits, uint64_t* __restrict__ Pc,
    uint64_t* __restrict__ samples, KeyND* __restrict__ keys, int write_keys, unsigned long long* info,
    const int32_t* __restrict__ htab, const int32_t* __restrict__ hmap, int sshift, uint64_t* sred) {
  int s = bid / HS_BLOCKS;
  unsigned long long nh = info[I_LONGROW];
  int hc = nh < (unsigned long long)H_MAX ? (int)nh : H_MAX;
  if (s >= hc) return;   // uniform over the block
  if (MODE == 0 && write_keys < 0) {
    unsigned __int128 d2 = (unsigned __int128)info[I_DMAX] * info[I_DMAX];
    write_keys = (d2 >> 64) != 0 || d2 * d2 > ((unsigned __int128)1 << c) ? 1 : 0;
  }
  int32_t hrow[H_MAX];
#pragma unroll
  for (int q = 0; q < H_MAX; q++) hrow[q] = q < hc ? htab[q] : -1;
  int32_t h = hrow[s];
  int64_t ah = g.rp[h], bh = g.rp[h + 1];
  uint64_t dh = deg[h];
  uint64_t sh_ = g.self ? (uint64_t)g.self[h] : 0;
  uint64_t dmx = 0;
  for (int64_t j = ah + (int64_t)(bid % HS_BLOCKS) * BS + threadIdx.x; j < bh;
       j += (int64_t)HS_BLOCKS * BS) {
    int32_t x = g.col[j];
    int32_t wx = g.w[j];
    int xs = -1;
#pragma unroll
    for (int q = 0; q < H_MAX; q++) xs = hrow[q] == x ? q : xs;
    if (xs >= 0 && x < h) continue;   // the edge belongs to row x's threads
    int64_t ax = g.rp[x], bx = g.rp[x + 1];
    uint64_t dx = deg[x];
    uint64_t sx = g.self ? (uint64_t)g.self[x] : 0;
    int64_t below;
    uint64_t M;
    if (xs >= 0 && bx - ax > bh - ah) {
      // both rows mapped, x's longer: walk h's row in x's map
      M = mapped_min_sum(g.col, g.w, ah, bh, dx, ax, bx, dh, hmap + (int64_t)xs * g.n, INT32_MIN, below);
      below = hmap[(int64_t)xs * g.n + h];
    } else {
      M = mapped_min_sum(g.col, g.w, ax, bx, dh, ah, bh, dx, hmap + (int64_t)s * g.n, h, below);
    }
    if (sh_) M += umin64(sh_ * dx, (uint64_t)wx * dh);   // column h
    if (sx) M += umin64((uint64_t)wx * dx, sx * dh);     // column x
    uint64_t D = dh * dx;
    uint64_t N = 2 * D - 2 * M;
    dmx = D > dmx ? D : dmx;
    int64_t jm = ax + below;   // entry (x -> h)
    int64_t e = h < x ? uptr[h] + (j - ah - lc[h]) : uptr[x] + (below - lc[x]);
    if (MODE == 0) {
      uint64_t key = (fixed_key(N, D, c) << ebits) | (uint64_t)e;
      Pc[j] = key;
      Pc[jm] = key;
      if ((e & ((1ll << sshift) - 1)) == 0) samples[e >> sshift] = key;
    }
    if (MODE == 1 || write_keys) keys[e] = KeyND{N, D, (uint64_t)e};
  }
  dmx = wave_max(dmx);
  if (lane_id() == 0) sred[threadIdx.x / WAVE] = dmx;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t a = 0;
    for (int w = 0; w < BS / WAVE; w++) a = sred[w] > a ? sred[w] : a;
    atomic_max_lazy(&info[I_DMAXE], (unsigned long long)a);
  }
}

// ---------------------------------------------------------------------------
// A2 + A3: 3 edges (u < v) per thread; tiles of SCORE_TILE consecutive edge
// ids are mapped to rows by a load-balanced search over the upper-entry
// prefix uptr, starting from the tile's first row, which the degree pass
// recorded (trow).
// ---------------------------------------------------------------------------
constexpr int TILE_S = SCORE_TILE;
constexpr int EPT = TILE_S / BS;

// Writes edge e's key into both of its entries (and its sample and exact
// record); returns whether the packed key is exact.
template <int MODE>
__device__ __forceinline__ bool emit_key(int64_t e, int64_t j, int64_t jm, uint64_t N, uint64_t D, int c,
                                         int ebits, uint64_t* __restrict__ Pc, uint64_t* __restrict__ samples,
                                         KeyND* __restrict__ keys, int write_keys, int sshift) {
  bool ex = false;
  if (MODE == 0) {
    uint64_t K = c <= 50 ? fixed_key_fast(N, D, c, ex) : fixed_key(N, D, c, ex);
    uint64_t key = (K << ebits) | (uint64_t)e;
    Pc[j] = key;    // entry (u -> v)
    Pc[jm] = key;   // entry (v -> u)
    if ((e & ((1ll << sshift) - 1)) == 0) samples[e >> sshift] = key;
  }
  if (MODE == 1 || write_keys) keys[e] = KeyND{N, D, (uint64_t)e};
  return ex;
}

// The edge tile of k_score.  The loads come in rounds that each serve all of
// the thread's edges at once: u's row bounds, offsets and degree; the edge's
// entry (v and the weight); v's bounds and degree; then the two rows of each
// edge whose rows both hold at most RC entries (others take edge_score,
// after the short ones).  NARROW: every degree is below 2^24.
template <int MODE, bool NARROW>
__device__ __forceinline__ void score_tile(const LevelIn& g, const uint64_t* __restrict__ deg,
                                           const int32_t* __restrict__ lc, const int64_t* __restrict__ uptr,
                                           int64_t m, int c, int ebits, uint64_t* __restrict__ Pc,
                                           uint64_t* __restrict__ samples, KeyND* __restrict__ keys,
                                           int write_keys, uint64_t* __restrict__ kexact, int sshift,
                                           const int32_t* srow, int64_t e0, const int32_t (&hrow)[H_MAX],
                                           uint64_t& dmx, uint4* sdesc, int* sfb, unsigned long long* sbits) {
  using L = Lbs<TILE_S, BS>;
  int tid = threadIdx.x;
  int32_t eu[EPT], ev[EPT];
  uint32_t ew[EPT];
  int64_t ej[EPT], au[EPT], av[EPT];
  int32_t lu[EPT], lv[EPT];
  uint64_t du[EPT], dv[EPT], su[EPT], ms[EPT];
  bool live[EPT];
#pragma unroll
  for (int i = 0; i < EPT; i++) {
    int k = tid + i * BS;
    live[i] = e0 + k < m;
    eu[i] = live[i] ? srow[L::at(k)] : 0;
  }
  // first loads: row u
#pragma unroll
  for (int i = 0; i < EPT; i++) {
    int32_t u = eu[i];
    au[i] = g.rp[u];
    lu[i] = (int32_t)(g.rp[u + 1] - au[i]);
    ej[i] = au[i] + lc[u] + (e0 + tid + i * BS - uptr[u]);
    du[i] = deg[u];
    su[i] = g.self ? (uint64_t)g.self[u] : 0;
  }
  // second loads: the edge's entry
#pragma unroll
  for (int i = 0; i < EPT; i++) {
    ej[i] = live[i] ? ej[i] : 0;   // (entry 0 exists: the tile holds an edge)
    ev[i] = g.col[ej[i]];
    ew[i] = (uint32_t)g.w[ej[i]];
  }
  // third loads: row v, and the diagonal terms x = u and x = v of the sum
#pragma unroll
  for (int i = 0; i < EPT; i++) {
    int32_t v = ev[i];
    av[i] = g.rp[v];
    lv[i] = (int32_t)(g.rp[v + 1] - av[i]);
    dv[i] = deg[v];
    uint64_t sv = g.self ? (uint64_t)g.self[v] : 0;
    ms[i] = umin64(wmul<NARROW>(su[i], dv[i]), wmul<NARROW>(ew[i], du[i])) +
            umin64(wmul<NARROW>(ew[i], dv[i]), wmul<NARROW>(sv, du[i]));
  }
  uint32_t shrt = 0, exm = 0;
#pragma unroll
  for (int i = 0; i < EPT; i++) {
    bool mapped = false;
#pragma unroll
    for (int s = 0; s < H_MAX; s++) mapped |= hrow[s] == eu[i] || hrow[s] == ev[i];
    // edges of a mapped row are scored by the mapped rows' blocks (their bit stays clear)
    live[i] = live[i] && !mapped;
    // (a live edge's rows both hold it, so neither is empty)
    shrt |= (live[i] && lu[i] <= RC && lv[i] <= RC && g.nnz >= RC ? 1u : 0u) << i;
  }
  // then the rows of the short edges, one edge after the other
#pragma unroll
  for (int i = 0; i < EPT; i++) {
    if (shrt >> i & 1u) {
      int32_t below;
      uint64_t M = ms[i] + short_rows_sum<NARROW>(g.col, g.w, g.nnz, au[i], lu[i], du[i], av[i], lv[i],
                                                  dv[i], (uint32_t)eu[i], below);
      uint64_t D = wmul<NARROW>(du[i], dv[i]);
      dmx = D > dmx ? D : dmx;
      bool ex = emit_key<MODE>(e0 + tid + i * BS, ej[i], av[i] + below, 2 * D - 2 * M, D, c, ebits, Pc,
                               samples, keys, write_keys, sshift);
      exm |= (ex ? 1u : 0u) << i;
    }
  }
  if (MODE == 0) {
    // the short edges' exactness bits: word (wavefront, slot) of the tile's map
#pragma unroll
    for (int i = 0; i < EPT; i++) {
      uint64_t bits = __ballot(exm >> i & 1u);
      if (lane_id() == 0) sbits[tid / WAVE + i * (BS / WAVE)] = bits;
    }
  }
  // The block's other live edges (a row longer than RC) are compacted into
  // LDS (endpoints, weight, place in the tile) and then taken by all of its
  // threads in turn: a wavefront would otherwise run the long-row path once
  // per slot that holds one, with most of its lanes idle.
#pragma unroll
  for (int i = 0; i < EPT; i++) {
    bool take = live[i] && !(shrt >> i & 1u);
    uint64_t mask = __ballot(take);
    if (mask == 0) continue;   // (uniform over the wavefront)
    int lead = __ffsll((long long)mask) - 1;
    int base = 0;
    if (lane_id() == lead) base = atomicAdd(sfb, (int)__popcll(mask));
    base = __shfl(base, lead);
    if (take)
      sdesc[base + (int)__popcll(mask & ((1ull << lane_id()) - 1))] =
          make_uint4((uint32_t)eu[i], (uint32_t)ev[i], ew[i], (uint32_t)(tid + i * BS));
  }
  __syncthreads();
  int nf = *sfb;
  for (int k = tid; k < nf; k += BS) {
    uint4 d = sdesc[k];
    int32_t u = (int32_t)d.x, v = (int32_t)d.y;
    int64_t e = e0 + d.w;
    int64_t j = g.rp[u] + lc[u] + (e - uptr[u]);   // entry (u -> v)
    uint64_t N, D;
    int64_t jm;
    edge_score(g, deg, lc, u, v, (int32_t)d.z, N, D, jm);
    dmx = D > dmx ? D : dmx;
    bool ex = emit_key<MODE>(e, j, jm, N, D, c, ebits, Pc, samples, keys, write_keys, sshift);
    if (MODE == 0 && ex) atomicOr(&sbits[d.w / WAVE], 1ull << (d.w % WAVE));
  }
  __syncthreads();
  if (MODE == 0 && tid < TILE_S / WAVE) {
    // the exactness map: 64 consecutive edges make one word
    int64_t ew0 = e0 + (int64_t)tid * WAVE;
    if (ew0 < m) kexact[ew0 >> 6] = sbits[tid];
  }
}

// four waves per SIMD: the register budget that keeps the rounds of loads
// of three edges in flight free of spills
template <int MODE>  // 0: 64-bit key (+ optional exact records), 1: exact records only
__global__ void __launch_bounds__(BS, 4)
    k_score(LevelIn g, const uint64_t* __restrict__ deg, const int32_t* __restrict__ lc,
            const int64_t* __restrict__ uptr, int64_t m, int c, int ebits,
            uint64_t* __restrict__ Pc, uint64_t* __restrict__ samples, KeyND* __restrict__ keys,
            int write_keys, unsigned long long* info, const int32_t* __restrict__ htab,
            uint64_t* __restrict__ kexact, int sshift, int tiles, const int32_t* __restrict__ hmap,
            const int32_t* __restrict__ trow) {
  // write_keys < 0: exact records only when the packed key is not exact
  // for sure, i.e. when dmax^4 > 2^c
  uint64_t dmax = info[I_DMAX];
  if (MODE == 0 && write_keys < 0) {
    unsigned __int128 d2 = (unsigned __int128)dmax * dmax;
    write_keys = (d2 >> 64) != 0 || d2 * d2 > ((unsigned __int128)1 << c) ? 1 : 0;
    if (write_keys && blockIdx.x == 0 && threadIdx.x == 0) info[I_KEYS] = 1;
  }
  __shared__ int32_t srow[Lbs<TILE_S, BS>::SIZE];
  __shared__ int32_t stmp[BS / WAVE];
  __shared__ uint64_t sred[BS / WAVE];
  __shared__ uint4 sdesc[TILE_S];                      // the tile's long-row edges
  __shared__ unsigned long long sbits[TILE_S / WAVE];  // the tile's exactness map
  __shared__ int sfb;                                  // its long-row edges
  if ((int)blockIdx.x >= tiles) {
    // the blocks past the edge tiles score the mapped long rows' edges
    // (dispatched last, they fill the tail of the launch)
    score_mapped_block<MODE>((int)blockIdx.x - tiles, g, deg, lc, uptr, c, ebits, Pc, samples, keys,
                             write_keys, info, htab, hmap, sshift, sred);
    return;
  }
  int64_t t = xcd_tile(blockIdx.x, tiles);
  int64_t e0 = t * TILE_S;
  int64_t r1 = t + 1 < tiles ? trow[t + 1] : g.n - 1;
  if (threadIdx.x == 0) sfb = 0;   // (lbs_fill synchronises the block before it is used)
  lbs_fill<TILE_S, BS>(uptr, trow[t], r1, e0, srow, stmp);
  uint64_t dmx = 0;
  // rows with a position map (uniform over the block)
  unsigned long long nh = info[I_LONGROW];
  int hc = nh < (unsigned long long)H_MAX ? (int)nh : H_MAX;
  int32_t hrow[H_MAX];
#pragma unroll
  for (int s = 0; s < H_MAX; s++) hrow[s] = s < hc ? htab[s] : -1;
  if (dmax < (1ull << 24))
    score_tile<MODE, true>(g, deg, lc, uptr, m, c, ebits, Pc, samples, keys, write_keys, kexact, sshift, srow,
                           e0, hrow, dmx, sdesc, &sfb, sbits);
  else
    score_tile<MODE, false>(g, deg, lc, uptr, m, c, ebits, Pc, samples, keys, write_keys, kexact, sshift, srow,
                            e0, hrow, dmx, sdesc, &sfb, sbits);
  dmx = wave_max(dmx);
  if (lane_id() == 0) sred[threadIdx.x / WAVE] = dmx;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t a = 0;
    for (int w = 0; w < BS / WAVE; w++) a = sred[w] > a ? sred[w] : a;
    atomic_max_lazy(&info[I_DMAXE], (unsigned long long)a);
  }
}

// rank order: P[e] = position of e in the exact sorted order
__global__ void k_rank_scatter(const KeyND* __restrict__ sorted, int64_t m, uint64_t* __restrict__ P) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < m) P[sorted[r].e] = (uint64_t)r;
}

// ---------------------------------------------------------------------------
// edge passes over 4096-edge tiles (16 edges per thread)
// ---------------------------------------------------------------------------
constexpr int TILE_F = 4096;
constexpr int F_PER = TILE_F / BS;

// rank order: the rank of edge e into both of its CSR entries
__global__ void __launch_bounds__(BS)
    k_rank_mirror(LevelIn g, const int32_t* __restrict__ lc, const int64_t* __restrict__ uptr,
                  int64_t m, const uint64_t* __restrict__ P, uint64_t* __restrict__ Pc) {
  __shared__ int32_t srow[Lbs<TILE_F, BS>::SIZE];
  __shared__ int64_t sh[2];
  __shared__ int32_t stmp[BS / WAVE];
  int64_t e0 = (int64_t)blockIdx.x * TILE_F;
  lbs_tile<TILE_F, BS>(uptr, g.n, e0, srow, sh, stmp);
  for (int i = 0; i < F_PER; i++) {
    int k = threadIdx.x + i * BS;
    int64_t e = e0 + k;
    if (e >= m) break;
    int32_t u = srow[Lbs<TILE_F, BS>::at(k)];
    int64_t j = g.rp[u] + lc[u] + (e - uptr[u]);
    int32_t v = g.col[j];
    uint64_t key = P[e];
    Pc[j] = key;
    Pc[mirror_pos(g, lc, v, u)] = key;
  }
}

// Labels and Theorem 2's epsilon in one launch.  Labels: every node takes
// its component root's number, clamped to [0, t) (they are there by
// construction; the clamp keeps a later contraction in bounds should a check
// done at the host's next read of the info block fail).  Epsilon (with
// cnt non-null): the score of the heaviest accepted edge, which is the
// forest edge whose key equals the cutoff.
__global__ void k_relabel_eps(LevelIn g, const int32_t* __restrict__ root, const int32_t* __restrict__ cid,
                              int32_t* __restrict__ cluster_of, int64_t t,
                              const uint64_t* __restrict__ deg, const int32_t* __restrict__ lc,
                              const uint64_t* __restrict__ msfP, const uint64_t* __restrict__ msfO,
                              const unsigned long long* cnt, const SelState* st, double* out) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < g.n; x += stride) {
    int64_t c = cid[root[x]];
    cluster_of[x] = (int32_t)(c < 0 ? 0 : c >= t ? t - 1 : c);
  }
  if (!cnt) return;
  int64_t n = (int64_t)*cnt;
  uint64_t T = st->prefix;
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
    int64_t jm;
    edge_score(g, deg, lc, u, v, g.w[lo], N, D, jm);
    *out = (double)N / (double)D;
  }
}

void launch_score(spc_ctx* ctx, const LevelIn& g, const LevelWork& W, int64_t m, int c, int ebits,
                  int mode) {
  int tiles = grid_for(m, TILE_S);
  bool maps = g.nnz > HUGE_T;   // (their position maps come with the degree totals)
  // one launch: the edge tiles, then (when rows can be long) the mapped rows' blocks
  int grid = tiles + (maps ? H_MAX * HS_BLOCKS : 0);
  if (mode == 0) {
    TimedScope ts(ctx, "score", (double)m);
    hipLaunchKernelGGL(k_score<0>, dim3(grid), dim3(BS), 0, ctx->stream, g, W.deg, W.lc, W.uptr, m, c, ebits,
                       W.Pc, W.samples, W.keysA, -1, W.info, W.htab, W.kexact, sample_shift(m), tiles, W.hmap,
                       W.trow);
  } else {
    TimedScope ts(ctx, "score_rank", (double)m);
    hipLaunchKernelGGL(k_score<1>, dim3(grid), dim3(BS), 0, ctx->stream, g, W.deg, W.lc, W.uptr, m, c, ebits,
                       (uint64_t*)nullptr, (uint64_t*)nullptr, W.keysA, 1, W.info, W.htab, (uint64_t*)nullptr,
                       sample_shift(m), tiles, W.hmap, W.trow);
  }
}

void launch_rank_mirror(spc_ctx* ctx, const LevelIn& g, const LevelWork& W, int64_t m) {
  hipLaunchKernelGGL(k_rank_mirror, dim3(grid_for(m, TILE_F)), dim3(BS), 0, ctx->stream, g, W.lc, W.uptr,
                     m, W.P, W.Pc);
}

void launch_rank_scatter(spc_ctx* ctx, const LevelIn& g, const LevelWork& W, int64_t m,
                         const KeyND* sorted) {
  hipLaunchKernelGGL(k_rank_scatter, dim3(grid_for(m, 256)), dim3(256), 0, ctx->stream, sorted, m, W.P);
  launch_rank_mirror(ctx, g, W, m);
}

void launch_relabel_eps(spc_ctx* ctx, const LevelIn& g, const LevelWork& W, int32_t* cluster_of, int64_t t,
                        int64_t msf_bound, bool eps) {
  int64_t items = g.n > msf_bound ? g.n : msf_bound;
  hipLaunchKernelGGL(k_relabel_eps, dim3(grid_for(items, 256)), dim3(256), 0, ctx->stream, g, W.parent, W.flag,
                     cluster_of, t, W.deg, W.lc, W.msfP, W.msfO,
                     eps ? (const unsigned long long*)&W.info[I_MSF] : (const unsigned long long*)nullptr,
                     W.sel2, (double*)&W.info[I_EPS]);
}

}  // namespace spc

// Steps of one coarsening level up to the merge selection:
//   A1 degrees d_x (row sums of w_x, notation after Theorem 1),
//   A2 the fitness of every edge, || w_u/d_u - w_v/d_v ||_1 (Theorem 1,
//      Algorithm 1's fitness loop), evaluated exactly as N / D (kernels in
//      score.hip),
//   A3 a strict total order on edges (score, then smaller endpoint, then
//      larger endpoint) encoded as one 64-bit key per edge,
//   A4 the merge loop of Algorithm 1, computed as the components of the
//      lightest n - t edges of the minimum spanning forest under that order.
//
// The order key.  With e the edge's position in (u, v) order and
// K = floor(score * 2^c), c = 62 - bits(e), the key is P = (K << bits(e)) | e.
// Two different scores N1/D1 != N2/D2 differ by at least 1/(D1 D2), so K
// separates them whenever 2^c >= Dmax^2 ("exact" keys).  Otherwise the keys
// are "guarded": every decision that could hinge on two edges sharing one
// K bucket (a component's lightest edge, the rank cutoff) is re-checked
// with the exact cross-multiplied comparison, and a level whose check fails
// is redone with keys = ranks from an exact comparison sort.
#include "level.hpp"
#include "radix.hpp"

namespace spc {

// ---------------------------------------------------------------------------
// workspace plan
// ---------------------------------------------------------------------------
constexpr int DEG_PER = 4;
constexpr int DEG_ROWS = BS * DEG_PER;
constexpr int DEG_SHORT = 64;

void plan_level(Arena& A, int64_t n, int64_t nnz, LevelWork& W, bool fp) {
  int64_t m = nnz / 2;
  W.info = A.take<unsigned long long>(I_NINFO);
  W.lbstate = A.take<uint64_t>(lb_words(n, nnz));
  W.deg = A.take<uint64_t>(n);
  W.degpart = A.take<uint64_t>(n / DEG_ROWS + 2);
  W.lc = A.take<int32_t>(n);
  W.uptr = A.take<int64_t>(n + 1);
  W.trow = A.take<int32_t>(m / SCORE_TILE + 2);
  W.ptrow = A.take<int32_t>(nnz / ENTRY_TILE + 2);
  W.gid = A.take<int32_t>(n);
  W.thrg = A.take<uint64_t>(n);
  W.P = A.take<uint64_t>(m);
  W.Pc = A.take<uint64_t>(nnz);
  W.samples = A.take<uint64_t>(m / 64 + 2);
  W.kexact = A.take<uint64_t>(m / 64 + 2);
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
  W.msfC = A.take<int32_t>(n);
  W.root = A.take<int32_t>(n);
  W.flag = A.take<int32_t>(n + 1);
  W.sel = A.take<SelState>(1);
  W.sel2 = A.take<SelState>(1);
  W.selflag = A.take<uint64_t>(SEL_MAXB * SEL_FLAG);
  W.scan_partial = A.take<int64_t>(SCAN_MAXB);
  W.keysA = A.take<KeyND>(m);
  W.keysB = A.take<KeyND>(m);
  W.mcount = A.take<int32_t>(n + 1);
  W.mptr = A.take<int32_t>(n + 1);
  W.members = A.take<int32_t>(n);
  W.gptr = A.take<int64_t>(n + 1);
  W.temp = A.take<uint64_t>(nnz + n);
  W.cnt = A.take<int64_t>(n + 1);
  W.r32list = A.take<int32_t>(n);
  W.midlist = A.take<int32_t>(n);
  W.blocklist = A.take<int32_t>(n);
  W.hugelist = A.take<int32_t>(n);
  W.hmoff = A.take<int64_t>(n + 1);
  W.hmrow = A.take<int32_t>(n);
  W.hmnode = A.take<int32_t>(n);
  W.hpos = A.take<int64_t>(n + 1);
  W.hmrs = A.take<int64_t>(n);
  W.htab = A.take<int32_t>(H_MAX);
  W.hmap = A.take<int32_t>((int64_t)H_MAX * n);
  W.gkeyA = A.take<uint64_t>(2 * nnz + 8);
  W.gkeyB = A.take<uint64_t>(2 * nnz + 8);
  if (fp) {
    W.ones = A.take<int32_t>(nnz);
    W.wtmp = A.take<int32_t>(nnz);
    W.selftmp = A.take<int64_t>(n);
    W.acc = A.take<uint64_t>((int64_t)FP_LIMBS * nnz);
    W.selfacc = A.take<uint64_t>((int64_t)FP_LIMBS * n);
    W.emap = A.take<int32_t>(nnz);
  } else {
    W.ones = W.wtmp = W.emap = nullptr;
    W.selftmp = nullptr;
    W.acc = W.selfacc = nullptr;
  }
  W.fd_sorted = nullptr;
}

// ---------------------------------------------------------------------------
// A1: degrees, upper-entry counts, and per-level initialisation.
// A block covers 1024 consecutive rows, 4 per thread.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(BS)
    k_degree(LevelIn g, uint64_t* __restrict__ deg, int32_t* __restrict__ lc,
             int64_t* __restrict__ uptr, uint64_t* __restrict__ bestA,
             uint64_t* __restrict__ bestB, int32_t* __restrict__ parent, int32_t* __restrict__ cc,
             uint64_t* __restrict__ part, int32_t* __restrict__ htab, unsigned long long* info,
             TileScan ts, int32_t* __restrict__ trow, int32_t* __restrict__ ptrow) {
  __shared__ int stmp[BS / WAVE];
  __shared__ int64_t stmp64[BS / WAVE];
  __shared__ int64_t sbase;
  __shared__ uint64_t smx[BS / WAVE], ssm[BS / WAVE];
  __shared__ int32_t slong[DEG_ROWS];
  __shared__ int sdefer;
  int tid = threadIdx.x;
  int64_t base = (int64_t)blockIdx.x * DEG_ROWS;
  uint64_t mx = 0, sm = 0;
  uint32_t longmask = 0;
  int nlong = 0;
  int64_t ucnt[DEG_PER];   // upper entries of this thread's rows
  int64_t rs[DEG_PER], re[DEG_PER];   // their bounds, loaded together
#pragma unroll
  for (int i = 0; i < DEG_PER; i++) {
    ucnt[i] = 0;
    int64_t u = base + i * BS + tid;
    rs[i] = u < g.n ? g.rp[u] : 0;
    re[i] = u < g.n ? g.rp[u + 1] : 0;
  }
#pragma unroll
  for (int i = 0; i < DEG_PER; i++) {
    int64_t u = base + i * BS + tid;
    if (u >= g.n) break;
    int64_t s = rs[i], e = re[i];
    if (e - s <= DEG_SHORT) {
      // weights summed and lower entries counted in one sweep, the loads of
      // each chunk of 8 entries issued together
      uint64_t d = g.self ? (uint64_t)g.self[u] : 0;
      int32_t below = 0;
      for (int64_t j0 = s; j0 < e; j0 += 8) {
        int32_t cc[8];
        uint32_t ww[8];
#pragma unroll
        for (int q = 0; q < 8; q++) {
          bool in = j0 + q < e;
          cc[q] = in ? g.col[j0 + q] : INT32_MAX;
          ww[q] = in ? (uint32_t)g.w[j0 + q] : 0u;
        }
#pragma unroll
        for (int q = 0; q < 8; q++) {
          d += ww[q];
          below += cc[q] < u ? 1 : 0;
        }
      }
      lc[u] = below;
      ucnt[i] = (e - s) - below;
      deg[u] = d;
      mx = d > mx ? d : mx;
      sm += d;
    } else {
      int64_t lo = s, hi = e;   // entries with col < u
      while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (g.col[mid] < u) lo = mid + 1;
        else hi = mid;
      }
      lc[u] = (int32_t)(lo - s);
      ucnt[i] = e - lo;
      longmask |= 1u << i;
      nlong++;
    }
    bestA[u] = KEY_INF;
    bestB[u] = KEY_INF;
    parent[u] = (int32_t)u;   // the spanning forest's union-find
    cc[u] = (int32_t)u;       // the merge cutoff's components
  }
  // uptr: exclusive prefix of the upper-entry counts in row order (the
  // edge id of each row's first upper entry), block offsets chained by a
  // decoupled look-back; the last block also stores uptr[n] = m
  {
    int64_t run = 0, pre[DEG_PER];
#pragma unroll
    for (int i = 0; i < DEG_PER; i++) {
      int64_t tot;
      int64_t inc = block_incl_scan<int64_t, BS, false>(ucnt[i], stmp64, &tot);
      pre[i] = run + inc - ucnt[i];
      run += tot;
    }
    if (tid < WAVE) {
      uint64_t ex = lb_exclusive_wave(ts, blockIdx.x, (uint64_t)run);
      if (tid == 0) {
        sbase = (int64_t)ex;
        if (blockIdx.x == gridDim.x - 1) uptr[g.n] = (int64_t)ex + run;
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < DEG_PER; i++) {
      int64_t u = base + i * BS + tid;
      if (u < g.n) {
        int64_t e = sbase + pre[i];
        uptr[u] = e;
        // the score tiles whose first edge lies in this row (the row that a
        // search of uptr for that edge would find)
        for (int64_t t = (e + SCORE_TILE - 1) / SCORE_TILE; t * SCORE_TILE < e + ucnt[i]; t++)
          trow[t] = (int32_t)u;
        // and the entry tiles whose first entry lies in this row
        for (int64_t t = (rs[i] + ENTRY_TILE - 1) / ENTRY_TILE; t * ENTRY_TILE < re[i]; t++)
          ptrow[t] = (int32_t)u;
      }
    }
  }
  // rows longer than DEG_SHORT: up to HUGE_T entries one wavefront sums
  // each of them (the block's four wavefronts take turns over its list);
  // longer ones the whole block, except the first H_MAX rows longer than
  // HUGE_T, which get a position map for the scores and are summed by
  // k_sum_parts with a block of its own
  int total_long;
  int p = block_incl_scan<int, BS, false>(nlong, stmp, &total_long) - nlong;
  for (int i = 0; i < DEG_PER; i++)
    if (longmask >> i & 1u) slong[p++] = (int32_t)(base + i * BS + tid);
  __syncthreads();
  for (int r = tid / WAVE; r < total_long; r += BS / WAVE) {
    int64_t u = slong[r];
    int64_t s = g.rp[u], e = g.rp[u + 1];
    if (e - s > HUGE_T) continue;   // (uniform over the wavefront)
    uint64_t d = 0;
    for (int64_t j = s + lane_id(); j < e; j += WAVE) d += (uint64_t)g.w[j];
    d = wave_sum(d);
    if (lane_id() == 0) {
      uint64_t t = d + (g.self ? (uint64_t)g.self[u] : 0);
      deg[u] = t;
      mx = t > mx ? t : mx;
      sm += t;
    }
  }
  for (int r = 0; r < total_long; r++) {
    int64_t u = slong[r];
    int64_t s = g.rp[u], e = g.rp[u + 1];
    if (e - s <= HUGE_T) continue;   // (uniform over the block; summed above)
    {
      if (tid == 0) {
        // few rows are this long, so one atomic each stays cheap
        unsigned long long slot = atomicAdd(&info[I_LONGROW], 1ull);
        sdefer = slot < (unsigned long long)H_MAX ? 1 : 0;
        if (sdefer) htab[slot] = (int32_t)u;
      }
      __syncthreads();
      int defer = sdefer;
      __syncthreads();
      if (defer) continue;
    }
    uint64_t d = 0;
    for (int64_t j = s + tid; j < e; j += BS) d += (uint64_t)g.w[j];
    d = wave_sum(d);
    if (lane_id() == 0) smx[tid / WAVE] = d;
    __syncthreads();
    if (tid == 0) {
      uint64_t t = g.self ? (uint64_t)g.self[u] : 0;
      for (int w = 0; w < BS / WAVE; w++) t += smx[w];
      deg[u] = t;
      mx = t > mx ? t : mx;
      sm += t;
    }
    __syncthreads();
  }
  mx = wave_max(mx);
  sm = wave_sum(sm);
  if (lane_id() == 0) {
    smx[tid / WAVE] = mx;
    ssm[tid / WAVE] = sm;
  }
  __syncthreads();
  if (tid == 0) {
    uint64_t a = 0, b = 0;
    for (int w = 0; w < BS / WAVE; w++) {
      a = smx[w] > a ? smx[w] : a;
      b += ssm[w];
    }
    atomic_max_lazy(&info[I_DMAX], (unsigned long long)a);
    part[blockIdx.x] = b;
  }
}

// Degrees of the mapped long rows (at most H_MAX, registered by k_degree),
// each summed by the whole block with 8 loads per thread in flight; then the
// total weight from the per-block sums and those rows (saturating, so that
// an overflowing input still reads as too large).
constexpr int SP_BS = 1024;
constexpr int SP_UNROLL = 8;

__device__ __forceinline__ uint64_t sat_add(uint64_t a, uint64_t b) { return a + b < a ? ~0ull : a + b; }

// Blocks past the first (when the launch has them) write the mapped rows'
// position maps instead: for each of the first H_MAX registered rows,
// hmap[s * n + col[j]] = j - rp[row], SP_MAP blocks per row.  Entries of
// other columns keep stale values, which the lookups confirm against the row
// itself.
constexpr int SP_MAP = 8;

__global__ void __launch_bounds__(SP_BS)
    k_sum_parts(const uint64_t* __restrict__ part, int64_t np, LevelIn g, const int32_t* __restrict__ htab,
                uint64_t* __restrict__ deg, unsigned long long* info, int32_t* __restrict__ hmap) {
  __shared__ uint64_t tmp[SP_BS / WAVE];
  int tid = threadIdx.x;
  if (blockIdx.x > 0) {
    int sr = (blockIdx.x - 1) / SP_MAP;
    if ((unsigned long long)sr >= info[I_LONGROW]) return;
    int32_t u = htab[sr];
    int64_t a = g.rp[u], b = g.rp[u + 1];
    int32_t* map = hmap + (int64_t)sr * g.n;
    for (int64_t j = a + (int64_t)((blockIdx.x - 1) % SP_MAP) * SP_BS + tid; j < b; j += (int64_t)SP_MAP * SP_BS)
      map[g.col[j]] = (int32_t)(j - a);
    return;
  }
  unsigned long long nh = info[I_LONGROW];
  int hc = nh < (unsigned long long)H_MAX ? (int)nh : H_MAX;
  uint64_t extra = 0, dmx = 0;   // thread 0's
  for (int r = 0; r < hc; r++) {
    int32_t u = htab[r];
    int64_t a = g.rp[u], b = g.rp[u + 1];
    uint64_t d = 0;
    for (int64_t j0 = a + tid; j0 < b; j0 += (int64_t)SP_BS * SP_UNROLL) {
      uint32_t v[SP_UNROLL];
#pragma unroll
      for (int q = 0; q < SP_UNROLL; q++) {
        int64_t j = j0 + (int64_t)q * SP_BS;
        v[q] = j < b ? (uint32_t)g.w[j] : 0u;
      }
#pragma unroll
      for (int q = 0; q < SP_UNROLL; q++) d += v[q];
    }
    d = wave_sum(d);
    if (lane_id() == 0) tmp[tid / WAVE] = d;
    __syncthreads();
    if (tid == 0) {
      uint64_t t = g.self ? (uint64_t)g.self[u] : 0;
      for (int w = 0; w < SP_BS / WAVE; w++) t += tmp[w];
      deg[u] = t;
      dmx = t > dmx ? t : dmx;
      extra += t;
    }
    __syncthreads();
  }
  uint64_t s = 0;
  for (int64_t i = tid; i < np; i += SP_BS) s = sat_add(s, part[i]);
  for (int o = WAVE / 2; o > 0; o >>= 1) s = sat_add(s, __shfl_xor(s, o));
  if (lane_id() == 0) tmp[tid / WAVE] = s;
  __syncthreads();
  if (tid == 0) {
    uint64_t t = extra;
    for (int w = 0; w < SP_BS / WAVE; w++) t = sat_add(t, tmp[w]);
    info[I_TOTAL] = t;
    if (hc > 0) atomic_max_lazy(&info[I_DMAX], (unsigned long long)dmx);
  }
}

// Row pass over CSR entries, tiles of 2048 entries (8 consecutive entries
// per thread, keys staged in LDS):
//  - with do_best, every node's lightest incident key (the first
//    spanning-forest round), a segmented minimum per row; only row pieces
//    that straddle a thread's 16 entries combine with atomicMin, so best[]
//    must hold +inf on entry;
//  - upper entries (u < v) with lo < key <= hi form the live list (lo is
//    absent for the first band); its roots are still the original endpoints,
//    so the list's endpoint array is not written (readers take lr for it).
constexpr int TILE_R = ENTRY_TILE;
constexpr int R_PER = TILE_R / BS;

__global__ void __launch_bounds__(BS)
    k_rowpass(LevelIn g, const int32_t* __restrict__ lc, const uint64_t* __restrict__ Pc,
              const unsigned long long* thr_lo, const unsigned long long* thr_hi, int use_lo,
              int do_best, uint64_t* best, uint64_t* __restrict__ lr, uint64_t* __restrict__ lp,
              unsigned long long* cnt, unsigned long long* cnt_copy, TileScan ts,
              const int32_t* __restrict__ ptrow, const int32_t* __restrict__ gid,
              const uint64_t* __restrict__ thrg) {
  using L = Lbs<TILE_R, BS>;
  static_assert(R_PER == 8, "one 8-byte flag word per thread");
  __shared__ int32_t srow[L::SIZE];
  __shared__ uint64_t sp[L::SIZE];   // keys, then per-row minima at each row's first position
  __shared__ __align__(16) uint8_t sfl[TILE_R];   // bit 0: upper entry, bit 1: row head in tile
  __shared__ int64_t sh[2];
  __shared__ int32_t stmp[BS / WAVE];
  __shared__ unsigned long long sbase;
  __shared__ int stot;
  int64_t j0 = (int64_t)blockIdx.x * TILE_R;
  int64_t nnz = g.nnz;
  uint64_t tlo = use_lo ? *thr_lo : 0, thi = *thr_hi;   // issued early, used at the end
  int tid = threadIdx.x;
  // the tile's keys and columns, loaded before the row search (which does
  // not need them) so that their latency overlaps it
  uint64_t pk[R_PER];
  int32_t ck[R_PER];
#pragma unroll
  for (int i = 0; i < R_PER; i++) {
    int64_t j = j0 + tid + i * BS;
    pk[i] = j < nnz ? Pc[j] : KEY_INF;
    ck[i] = j < nnz ? g.col[j] : 0;
  }
  if (ptrow) {
    // the tile's first row from the degree pass (uniform over the block)
    int64_t t = blockIdx.x;
    int64_t r1 = t + 1 < (int64_t)gridDim.x ? ptrow[t + 1] : g.n - 1;
    lbs_fill<TILE_R, BS>(g.rp, ptrow[t], r1, j0, srow, stmp);
  } else {
    lbs_tile<TILE_R, BS>(g.rp, g.n, j0, srow, sh, stmp);
  }
  // the key, and from the column the upper / row-head flags
#pragma unroll
  for (int i = 0; i < R_PER; i++) {
    int k = tid + i * BS;
    int64_t j = j0 + k;
    uint32_t f = 0;
    if (j < nnz) {
      int32_t u = srow[L::at(k)];
      f = (ck[i] > u ? 1u : 0u) | ((k == 0 || srow[L::at(k - 1)] != u) ? 2u : 0u);
    }
    sp[L::at(k)] = pk[i];
    sfl[k] = (uint8_t)f;
  }
  __syncthreads();
  int kb = tid * R_PER;
  int64_t cb = j0 + kb;                    // this thread's entries [cb, cb + R_PER)
  uint64_t kp[R_PER];
  int32_t ku[R_PER];
  uint8_t fl[R_PER];
  {
    uint2 f2 = *(const uint2*)&sfl[kb];
    uint32_t fw[2] = {f2.x, f2.y};
#pragma unroll
    for (int i = 0; i < R_PER; i++) fl[i] = (uint8_t)(fw[i >> 2] >> (8 * (i & 3)));
  }
#pragma unroll
  for (int i = 0; i < R_PER; i++) {
    kp[i] = sp[L::at(kb + i)];
    ku[i] = srow[L::at(kb + i)];
  }
  __syncthreads();
  if (do_best) {
#pragma unroll
    for (int i = 0; i < R_PER; i++) sp[L::at(kb + i)] = KEY_INF;
    // a row continued from an earlier thread: its first position in the tile
    int first_slot = 0;
    if (cb < nnz && !(fl[0] & 2)) {
      int64_t rs = g.rp[ku[0]];
      first_slot = rs > j0 ? (int)(rs - j0) : 0;
    }
    __syncthreads();
    // row pieces of this thread: minimum into the slot at the row's first
    // position inside the tile
    int32_t cur = -1;
    uint64_t run = KEY_INF;
    int slot = 0;
#pragma unroll
    for (int i = 0; i < R_PER; i++) {
      if (cb + i >= nnz) break;
      bool head = fl[i] & 2;
      if (i == 0 || head) {
        if (cur >= 0) atomicMin((unsigned long long*)&sp[L::at(slot)], (unsigned long long)run);
        cur = ku[i];
        run = kp[i];
        slot = head ? kb + i : first_slot;
      } else {
        run = kp[i] < run ? kp[i] : run;
      }
    }
    if (cur >= 0) atomicMin((unsigned long long*)&sp[L::at(slot)], (unsigned long long)run);
    __syncthreads();
    // the thread holding a row's first position in the tile publishes it:
    // a plain store when the whole row lies inside the tile
    int32_t last_row = srow[L::at(TILE_R - 1)];
#pragma unroll
    for (int i = 0; i < R_PER; i++) {
      int64_t j = cb + i;
      if (j >= nnz) break;
      if (!(fl[i] & 2)) continue;
      int32_t u = ku[i];
      uint64_t v = sp[L::at(kb + i)];
      bool starts = kb + i > 0 || g.rp[u] == j0;
      bool ends = last_row != u && j0 + TILE_R <= nnz;
      if (starts && ends) best[u] = v;
      else atomicMin((unsigned long long*)&best[u], (unsigned long long)v);
    }
  }
  uint32_t keep = 0;
  int nk = 0;
#pragma unroll
  for (int i = 0; i < R_PER; i++) {
    int64_t j = cb + i;
    if (j >= nnz) break;
    uint64_t p = kp[i];
    // a batch's graphs each have their own band (thrg, by the row's graph)
    uint64_t th = thrg ? thrg[gid[ku[i]]] : thi;
    if ((fl[i] & 1) && p <= th && (!use_lo || p > tlo)) {
      keep |= 1u << i;
      nk++;
    }
  }
  int64_t pos = block_reserve_lb<BS>(ts, blockIdx.x, blockIdx.x == gridDim.x - 1, nk, nullptr, cnt,
                                    &sbase, stmp);
  if (tid == 0 && blockIdx.x == gridDim.x - 1) *cnt_copy = *cnt;   // this thread set *cnt
  // the block's records are staged in LDS (sp is free now) and written out
  // one word per lane, so every wave stores whole lines
  int64_t bbase = (int64_t)sbase;
  int loc = (int)(pos - bbase);
  if (tid == BS - 1) stot = loc + nk;
  int q = loc;
#pragma unroll
  for (int i = 0; i < R_PER; i++) {
    if (!(keep >> i & 1u)) continue;
    int32_t v = g.col[cb + i];
    sp[q++] = (uint64_t)(uint32_t)ku[i] | ((uint64_t)(uint32_t)v << 32);
  }
  __syncthreads();
  int tot = stot;
  for (int k = tid; k < tot; k += BS) lr[bbase + k] = sp[k];
  __syncthreads();
  q = loc;
#pragma unroll
  for (int i = 0; i < R_PER; i++)
    if (keep >> i & 1u) sp[q++] = kp[i];
  __syncthreads();
  for (int k = tid; k < tot; k += BS) lp[bbase + k] = sp[k];
}

// ---------------------------------------------------------------------------
// A4: spanning-forest rounds (Boruvka) on the live list.  A hooking pass
// takes 4096 items per block (16 per thread) on long lists and 1024 (4 per
// thread, their loads issued side by side) on short ones, where too few
// blocks would leave each thread a long chain of dependent loads; the root
// lookups take 1024 (an item's lookups are chains of dependent loads).
// ---------------------------------------------------------------------------
constexpr int BV_LONG = 16;
constexpr int BV_SHORT = 4;
constexpr int BV_BATCH = 4;   // items whose loads a thread issues together
constexpr int64_t BV_SHORT_MAX = 1000000;   // lists up to this many items use BV_SHORT
constexpr int BC_CHUNK = 1024;
constexpr int BC_PER = BC_CHUNK / BS;

// Guarded keys: the winner w of a component must not have a same-bucket
// rival x with an exactly smaller score.
// Two keys of one bucket whose K were both computed without remainder have
// equal scores, so their packed order (by edge id) is the exact one.
__device__ __forceinline__ void guard_check(const KeyND* __restrict__ keys, const uint64_t* __restrict__ kexact,
                                            int ebits, uint64_t key, uint64_t w, int* viol) {
  if (w == key || w == KEY_INF || (w >> ebits) != (key >> ebits)) return;
  uint64_t emask = (1ull << ebits) - 1;
  uint64_t ek = key & emask, ew = w & emask;
  if (key_exact(kexact, ek) && key_exact(kexact, ew)) return;
  if (exact_less(keys[ek], keys[ew])) *viol = 1;
}

// Every component adopts its lightest live edge; those edges are joined and
// recorded as forest edges.  PER items per thread.
template <int PER>
__global__ void __launch_bounds__(BS)
    k_bv_merge(const uint64_t* __restrict__ lr, const uint64_t* __restrict__ lp,
               const uint64_t* __restrict__ lo, const unsigned long long* cnt,
               const uint64_t* __restrict__ best, int32_t* parent, uint64_t* __restrict__ msfP,
               uint64_t* __restrict__ msfO, int32_t* __restrict__ msfC, unsigned long long* msfcnt,
               int64_t msf_cap,
               const KeyND* __restrict__ keys, const uint64_t* __restrict__ kexact,
               const unsigned long long* guard, int ebits, int* viol, TileScan ts,
               unsigned long long* rounds) {
  constexpr int CHUNK = PER * BS;
  // the items are taken HB at a time, all of a batch's loads of one kind
  // issued together (a thread's chain of dependent loads is PER / HB
  // batches long, not PER items)
  constexpr int HB = PER < BV_BATCH ? PER : BV_BATCH;
  static_assert(PER % HB == 0, "whole batches");
  __shared__ int stmp[BS / WAVE];
  __shared__ unsigned long long sbase;
  __shared__ uint64_t sst[CHUNK];
  __shared__ int stot;
  int64_t n = (int64_t)*cnt;
  int tid = threadIdx.x;
  int64_t base = (int64_t)blockIdx.x * CHUNK;
  if (base >= n) return;
  if (blockIdx.x == 0 && tid == 0) {   // rounds points at info[I_ROUNDS]
    atomicAdd(rounds, 1ull);
    atomicAdd(rounds + (I_MIN - I_ROUNDS), (unsigned long long)n);
  }
  if (keys && !*guard) keys = nullptr;
  uint32_t chosen = 0;
  int nc = 0;
  int32_t hooked[PER];
#pragma unroll
  for (int b0 = 0; b0 < PER; b0 += HB) {
    uint64_t suv[HB], skey[HB], swa[HB], swb[HB];
#pragma unroll
    for (int q = 0; q < HB; q++) {
      int64_t idx = base + tid + (b0 + q) * BS;
      suv[q] = idx < n ? lr[idx] : 0;
      skey[q] = idx < n ? lp[idx] : KEY_INF;
    }
#pragma unroll
    for (int q = 0; q < HB; q++) {
      int64_t idx = base + tid + (b0 + q) * BS;
      swa[q] = idx < n ? best[(int32_t)(uint32_t)suv[q]] : KEY_INF;
      swb[q] = idx < n ? best[(int32_t)(suv[q] >> 32)] : KEY_INF;
    }
#pragma unroll
    for (int q = 0; q < HB; q++) {
      int i = b0 + q;
      int64_t idx = base + tid + i * BS;
      hooked[i] = 0;
      if (idx >= n) continue;
      uint64_t uv = suv[q], key = skey[q], wa = swa[q], wb = swb[q];
      int32_t a = (int32_t)(uint32_t)uv, b = (int32_t)(uv >> 32);
      if (keys) {
        guard_check(keys, kexact, ebits, key, wa, viol);
        guard_check(keys, kexact, ebits, key, wb, viol);
      }
      bool ca = wa == key, cb = wb == key;
      if (ca || cb) {
        // a and b are roots at the start of this round and each root adopts
        // exactly one edge, so each root's parent is written at most once;
        // when both adopt this edge the smaller id stays the root
        int32_t child = (ca && cb) ? (a > b ? a : b) : (ca ? a : b);
        int32_t to = (ca && cb) ? (a > b ? b : a) : (ca ? b : a);
        __hip_atomic_store(&parent[child], to, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        hooked[i] = child;
        chosen |= 1u << i;
        nc++;
      }
    }
  }
  int64_t pos = block_reserve_lb<BS>(ts, blockIdx.x, base + CHUNK >= n, nc, msfcnt, msfcnt,
                                     &sbase, stmp);
  // the block's records are staged in LDS, one array at a time, and written
  // out one word per lane (a forest has fewer than n edges: positions at or
  // beyond msf_cap are dropped)
  int64_t bbase = (int64_t)sbase;
  int loc = (int)(pos - bbase);
  if (tid == BS - 1) stot = loc + nc;
  int q = loc;
  for (int i = 0; i < PER; i++)
    if (chosen >> i & 1u) sst[q++] = lp[base + tid + i * BS];
  __syncthreads();
  int tot = stot;
  for (int k = tid; k < tot; k += BS)
    if (bbase + k < msf_cap) msfP[bbase + k] = sst[k];
  __syncthreads();
  q = loc;
  for (int i = 0; i < PER; i++)
    if (chosen >> i & 1u) sst[q++] = lo[base + tid + i * BS];
  __syncthreads();
  for (int k = tid; k < tot; k += BS)
    if (bbase + k < msf_cap) msfO[bbase + k] = sst[k];
  __syncthreads();
  int32_t* sc = reinterpret_cast<int32_t*>(sst);
  q = loc;
  for (int i = 0; i < PER; i++)
    if (chosen >> i & 1u) sc[q++] = hooked[i];
  __syncthreads();
  for (int k = tid; k < tot; k += BS)
    if (bbase + k < msf_cap) msfC[bbase + k] = sc[k];
}

static void launch_bv_merge(spc_ctx* ctx, LevelWork& W, int64_t bound, const uint64_t* lr, const uint64_t* lp,
                            const uint64_t* lo, const unsigned long long* cnt, const uint64_t* best, int64_t n,
                            const KeyND* guard_keys, int ebits) {
  unsigned long long* info = W.info;
  if (bound <= (ctx->tune.bv_short > 0 ? ctx->tune.bv_short : (int64_t)BV_SHORT_MAX))
    hipLaunchKernelGGL(k_bv_merge<BV_SHORT>, dim3(grid_for(bound, BV_SHORT * BS)), dim3(BS), 0, ctx->stream,
                       lr, lp, lo, cnt, best, W.parent, W.msfP, W.msfO, W.msfC, &info[I_MSF], n, guard_keys,
                       W.kexact, &info[I_GUARD], ebits, (int*)&info[I_VIOL], next_scan(ctx, W),
                       &info[I_ROUNDS]);
  else
    hipLaunchKernelGGL(k_bv_merge<BV_LONG>, dim3(grid_for(bound, BV_LONG * BS)), dim3(BS), 0, ctx->stream,
                       lr, lp, lo, cnt, best, W.parent, W.msfP, W.msfO, W.msfC, &info[I_MSF], n, guard_keys,
                       W.kexact, &info[I_GUARD], ebits, (int*)&info[I_VIOL], next_scan(ctx, W),
                       &info[I_ROUNDS]);
}

// Pointer jumping after a merge round, over the roots that round hooked
// (forest records [*lo, *hi)): each follows its parent chain to the root,
// picking up the shortcuts the others write concurrently.  Every other node
// points at a root of the previous round, so its next lookup takes at most
// two steps.  Hooking in edge order can chain roots deeply (on a bipartite
// mesh every score ties and each node hooks to its lowest-numbered
// neighbour); without this the next round's lookups would walk those chains.
__global__ void k_shortcut(int32_t* parent, const int32_t* __restrict__ hooked,
                           const unsigned long long* lo, const unsigned long long* hi) {
  int64_t end = (int64_t)*hi;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)*lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < end; i += stride) {
    int32_t x = hooked[i];
    int32_t p = __hip_atomic_load(&parent[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (true) {
      int32_t gp = __hip_atomic_load(&parent[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (gp == p) break;
      p = gp;
      __hip_atomic_store(&parent[x], p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Live edges between different components, with the endpoints replaced by
// their current roots, move to the next list; each component's lightest
// live edge is found with atomicMin on the key.  The other best array is
// reset at every root that still has a live edge.
__global__ void __launch_bounds__(BS)
    k_bv_candidates(const uint64_t* __restrict__ lr_in, const uint64_t* __restrict__ lp_in,
                    const uint64_t* __restrict__ lo_in, const unsigned long long* cnt_in,
                    uint64_t* __restrict__ lr_out, uint64_t* __restrict__ lp_out,
                    uint64_t* __restrict__ lo_out, unsigned long long* cnt_out, uint64_t* cur,
                    uint64_t* nxt, int32_t* parent, TileScan ts, unsigned long long* stats,
                    const unsigned long long* msf_now, unsigned long long* msf_mark,
                    unsigned long long* cnt_copy) {
  __shared__ int stmp[BS / WAVE];
  __shared__ unsigned long long sbase;
  __shared__ uint64_t sst[BC_CHUNK];
  __shared__ int stot;
  int64_t n = (int64_t)*cnt_in;
  int tid = threadIdx.x;
  int64_t base = (int64_t)blockIdx.x * BC_CHUNK;
  if (base >= n) {
    if (n == 0 && blockIdx.x == 0 && tid == 0) {   // no tile runs: the empty list's count
      *cnt_out = 0;
      *msf_mark = *msf_now;
      if (cnt_copy) *cnt_copy = 0;
    }
    return;
  }
  uint32_t keep = 0;
  int nk = 0;
  uint64_t ruv[BC_PER];
  // the items' words, then their endpoints' first parent steps, are each
  // loaded together; the lookups continue from there
  uint64_t suv[BC_PER], skey[BC_PER];
  int32_t pa[BC_PER], pb[BC_PER];
#pragma unroll
  for (int i = 0; i < BC_PER; i++) {
    int64_t idx = base + tid + i * BS;
    suv[i] = idx < n ? lr_in[idx] : 0;
    skey[i] = idx < n ? lp_in[idx] : KEY_INF;
  }
#pragma unroll
  for (int i = 0; i < BC_PER; i++) {
    pa[i] = __hip_atomic_load(&parent[(int32_t)(uint32_t)suv[i]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    pb[i] = __hip_atomic_load(&parent[(int32_t)(suv[i] >> 32)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  int32_t ra[BC_PER], rb[BC_PER];
  for (int i = 0; i < BC_PER; i++) {
    int64_t idx = base + tid + i * BS;
    ra[i] = rb[i] = -1;
    if (idx < n) {
      ra[i] = uf_find_from(parent, (int32_t)(uint32_t)suv[i], pa[i]);
      rb[i] = uf_find_from(parent, (int32_t)(suv[i] >> 32), pb[i]);
    }
  }
  // Late rounds and hubs make one component's root the target of most
  // updates, and atomics on one address serialise.  The roots' current
  // values are loaded first (all items' loads together) and an update that
  // cannot lower cur (it only decreases) or change nxt (only ever set to
  // KEY_INF here) is skipped; besides, when at least a quarter of the
  // wavefront's live lanes share the first live lane's root on a side, they
  // fold their keys and one lane updates.
  uint64_t va[BC_PER], vb[BC_PER], na[BC_PER], nb[BC_PER];
#pragma unroll
  for (int i = 0; i < BC_PER; i++) {
    bool live = ra[i] != rb[i];
    va[i] = live ? __hip_atomic_load(&cur[ra[i]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    vb[i] = live ? __hip_atomic_load(&cur[rb[i]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    na[i] = live ? __hip_atomic_load(&nxt[ra[i]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : KEY_INF;
    nb[i] = live ? __hip_atomic_load(&nxt[rb[i]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : KEY_INF;
  }
  for (int i = 0; i < BC_PER; i++) {
    ruv[i] = 0;
    uint64_t key = skey[i];
    bool live = ra[i] != rb[i];
#pragma unroll
    for (int side = 0; side < 2; side++) {
      int32_t r = side ? rb[i] : ra[i];
      bool lower = live && key < (side ? vb[i] : va[i]);
      bool clear = live && (side ? nb[i] : na[i]) != KEY_INF;
      uint64_t lmask = __ballot(lower || clear);
      bool done = false;
      if (lmask) {
        int leader = __ffsll((long long)lmask) - 1;
        int32_t rl = __shfl(r, leader);
        bool same = (lower || clear) && r == rl;
        uint64_t smask = __ballot(same);
        if (4 * __popcll(smask) >= __popcll(lmask) && __popcll(smask) > 1) {
          uint64_t mn = wave_min<uint64_t>(same && lower ? key : KEY_INF);
          bool anyc = __ballot(same && clear) != 0;
          if (lane_id() == leader) {
            if (mn != KEY_INF) atomicMin((unsigned long long*)&cur[rl], (unsigned long long)mn);
            if (anyc) nxt[rl] = KEY_INF;
          }
          done = same;
        }
      }
      if (!done) {
        if (lower) atomicMin((unsigned long long*)&cur[r], (unsigned long long)key);
        if (clear) nxt[r] = KEY_INF;
      }
    }
    if (live) {
      ruv[i] = (uint64_t)(uint32_t)ra[i] | ((uint64_t)(uint32_t)rb[i] << 32);
      keep |= 1u << i;
      nk++;
    }
  }
  bool last = base + BC_CHUNK >= n;
  int64_t pos = block_reserve_lb<BS>(ts, blockIdx.x, last, nk, nullptr, cnt_out, &sbase, stmp);
  if (last && tid == 0) {
    atomicAdd(&stats[0], (unsigned long long)n);   // info[I_FIN]
    atomicAdd(&stats[1], *cnt_out);                // info[I_FKEPT]
    *msf_mark = *msf_now;                          // forest records before the next merge
    if (cnt_copy) *cnt_copy = *cnt_out;            // (this thread set *cnt_out)
  }
  // the block's records are staged in LDS, one array at a time, and written
  // out one word per lane, so every wave stores whole lines
  uint64_t ro[BC_PER];
#pragma unroll
  for (int i = 0; i < BC_PER; i++) ro[i] = (keep >> i & 1u) ? lo_in[base + tid + i * BS] : 0;
  int64_t bbase = (int64_t)sbase;
  int loc = (int)(pos - bbase);
  if (tid == BS - 1) stot = loc + nk;
  int q = loc;
#pragma unroll
  for (int i = 0; i < BC_PER; i++)
    if (keep >> i & 1u) sst[q++] = ruv[i];
  __syncthreads();
  int tot = stot;
  for (int k = tid; k < tot; k += BS) lr_out[bbase + k] = sst[k];
  __syncthreads();
  q = loc;
#pragma unroll
  for (int i = 0; i < BC_PER; i++)
    if (keep >> i & 1u) sst[q++] = skey[i];
  __syncthreads();
  for (int k = tid; k < tot; k += BS) lp_out[bbase + k] = sst[k];
  __syncthreads();
  q = loc;
#pragma unroll
  for (int i = 0; i < BC_PER; i++)
    if (keep >> i & 1u) sst[q++] = ro[i];
  __syncthreads();
  for (int k = tid; k < tot; k += BS) lo_out[bbase + k] = sst[k];
}

// After the cutoff selection, one launch: the components of the forest
// edges up to the cutoff T (union-find in cc, which holds the identity from
// the degree pass), the contraction's member counts and gather prefix set to
// zero, and with guarded keys the check that every forest edge sharing T's K
// bucket has exactly T's score (then the edge order inside the bucket is the
// exact one; keys null: no check).
__global__ void k_cutoff_union(const uint64_t* __restrict__ msfP, const uint64_t* __restrict__ msfO,
                               const unsigned long long* cnt, const SelState* st, const KeyND* __restrict__ keys,
                               const uint64_t* __restrict__ kexact, const unsigned long long* guard, int ebits,
                               int* viol, int32_t* cc, int32_t* __restrict__ zero_a,
                               int64_t* __restrict__ zero_b, int64_t nz) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t x = i0; x < nz; x += stride) {
    zero_a[x] = 0;
    zero_b[x] = 0;
  }
  int64_t n = (int64_t)*cnt;
  uint64_t T = st->prefix;
  bool check = keys && *guard;
  uint64_t emask = (1ull << ebits) - 1;
  for (int64_t i = i0; i < n; i += stride) {
    uint64_t p = msfP[i];
    if (p <= T) {
      uint64_t uv = msfO[i];
      uf_union(cc, (int32_t)(uint32_t)uv, (int32_t)(uv >> 32));
    }
    if (!check || p == T || (p >> ebits) != (T >> ebits)) continue;
    if (key_exact(kexact, p & emask) && key_exact(kexact, T & emask)) continue;   // equal scores
    KeyND x = keys[p & emask], y = keys[T & emask];
    if ((unsigned __int128)x.N * y.D != (unsigned __int128)y.N * x.D) *viol = 1;
  }
}

// ---------------------------------------------------------------------------
// components of the forest edges with key <= T, canonical numbering
// ---------------------------------------------------------------------------
__global__ void k_iota(int32_t* __restrict__ a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = (int32_t)i;
}


// Every node's root in the union-find uf (into root), and a flag on each
// root (its number among the roots in id order is the flags' exclusive scan).
__global__ void k_cc_flatten(int32_t* uf, int32_t* __restrict__ root, int32_t* __restrict__ flag, int64_t n) {
  int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < n) {
    int32_t r = uf_find(uf, (int32_t)x);
    root[x] = r;
    flag[x] = (r == (int32_t)x) ? 1 : 0;
  }
}


// ---------------------------------------------------------------------------
// radix select (declared in prim.hpp)
// ---------------------------------------------------------------------------
// Grid barrier: each block publishes its arrival epoch in its own flag line
// (after a release fence) and waits, one thread per block, until every flag
// has reached the epoch.  Flags start at zero (cleared with the level's
// info block) and every barrier of the level publishes a larger epoch than
// the one before, so a flag only ever moves forward.  Plain
// stores and no read-modify-write: atomics on one address serialise across
// the chip.  The wait is bounded; a timeout sets *err.
__device__ void sel_barrier(unsigned long long* flags, unsigned long long epoch, unsigned long long* err) {
  __syncthreads();
  int t = threadIdx.x;
  if (t == 0) {
    __threadfence();
    __hip_atomic_store(&flags[blockIdx.x * SEL_FLAG], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (t < (int)gridDim.x) {
    long spins = 0;
    while (__hip_atomic_load(&flags[t * SEL_FLAG], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
      if (++spins > SEL_SPIN) {
        __hip_atomic_store(err, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __syncthreads();
  if (t == 0) __threadfence();   // acquire: later plain loads see the other blocks' stores
  __syncthreads();
}

// Sum over blocks j = sub, sub + LANES, ... < G of a[j * stride + col]: the
// column of one bin (or group) in the per-block histograms, for LANES
// threads sharing it.  All of a thread's loads are issued before any is
// used (after a barrier they all go to memory).
template <int LANES>
__device__ __forceinline__ unsigned int col_part_sum(const unsigned int* a, int stride, int col, int G,
                                                     int sub) {
  constexpr int NV = SEL_MAXB / LANES;
  unsigned int v[NV];
#pragma unroll
  for (int q = 0; q < NV; q++) {
    int j = sub + q * LANES;
    v[q] = j < G ? a[(int64_t)j * stride + col] : 0u;
  }
  unsigned int s = 0;
#pragma unroll
  for (int q = 0; q < NV; q++) s += v[q];
  return s;
}

// A band threshold derived from a selected sample key (thr null: none).
// With c > 0 the level's key mode goes into info[I_GUARD] first (the packed
// key is inexact for some pair of edges only when Dmax^2 > 2^c, Dmax =
// largest d_u d_v).  Guarded keys order edges of one K bucket only
// approximately, so there the band is widened to the end of the sample's K
// bucket.  Samples are the keys of edges 0, s, 2s, ...; when the selected
// one is edge eq = q s itself, the band is (most likely) one tied K bucket
// read in edge order, i.e. a run of consecutive rows, whose forest has about
// one edge per row rather than per candidate: such a band is extended to
// edge e_tie (chosen to cover k rows).  Only the band's size changes.
// guess (nullable, two words): where the level's cutoff, the k-th lightest
// forest edge, most likely lies.  Forest keys lie at or below the band's
// threshold.  When fewer than qlo_max samples (fewer than about 0.9 k edges)
// lie below the selected sample's K bucket, the cutoff lies in that bucket,
// ties included; otherwise the guess is the smallest sample up to the
// threshold.
struct ThrSpec {
  unsigned long long* thr;
  unsigned long long* info;
  int c, ebits;
  unsigned long long eq, e_tie;
  unsigned long long* guess;
  unsigned long long qlo_max;
};

__device__ __forceinline__ void band_threshold(const ThrSpec& ts, uint64_t p, bool all) {
  uint64_t emask = (1ull << ts.ebits) - 1;
  if (ts.c > 0) {
    unsigned __int128 D2 = (unsigned __int128)ts.info[I_DMAXE] * ts.info[I_DMAXE];
    ts.info[I_GUARD] = ((D2 >> 64) != 0 || D2 > ((unsigned __int128)1 << ts.c)) ? 1ull : 0ull;
  }
  bool widen = ts.info[I_GUARD] != 0;
  if (all) *ts.thr = KEY_INF;
  else if (widen) *ts.thr = p | emask;
  else if ((p & emask) == ts.eq && ts.e_tie > (p & emask)) *ts.thr = (p & ~emask) | (ts.e_tie & emask);
  else *ts.thr = p;
}

__global__ void __launch_bounds__(SEL_BS)
    k_select(const uint64_t* __restrict__ keys, const unsigned long long* cnt_dev, int64_t cnt_host,
             const unsigned long long* k_dev, unsigned long long k_host, int bits, SelState* st,
             unsigned long long* flags, unsigned long long epoch0, unsigned long long* err, ThrSpec tsp,
             const unsigned long long* guess_lo, const unsigned long long* guess_hi) {
  static_assert(SEL_NGRP * 8 == SEL_BS && SEL_GBINS * 4 == SEL_BS, "pick layout");
  __shared__ unsigned int h[SEL_BINS];
  __shared__ uint64_t sbuf[SEL_SMALL];
  __shared__ uint64_t s2[LDS_SMALL2];
  __shared__ unsigned int s2cnt;
  __shared__ unsigned long long tmp[SEL_BS / WAVE];
  __shared__ unsigned long long red[2 * (SEL_BS / WAVE)];
  __shared__ unsigned long long spick[3];
  __shared__ unsigned int sgrp[2];
  __shared__ unsigned int slocal;
  int t = threadIdx.x;
  int G = gridDim.x, B = blockIdx.x;
  int64_t n = cnt_dev ? (int64_t)*cnt_dev : cnt_host;
  unsigned long long k = k_dev ? *k_dev : k_host;
  int64_t stride = (int64_t)G * SEL_BS;
  unsigned long long epoch = epoch0;   // barrier i publishes epoch0 + i + 1
  uint64_t prefix = 0, mask = 0;
  int hi = bits;
  int64_t cb = n;   // keys matching (prefix, mask)
  unsigned long long bstar = 0;   // bucket chosen by the last pass
  int p = 0;
  bool guessed = false, again = false;
  if (G > 1 && guess_lo && guess_hi) {
    uint64_t lo = *guess_lo, hk = *guess_hi;
    if (lo < hk) {
      int d = 63 - __clzll((long long)(lo ^ hk));   // highest bit the bounds differ in
      if (d + 1 < hi) {
        uint64_t low = (2ull << d) - 1;
        prefix = lo & ~low;
        mask = ~low;
        hi = d + 1;
        guessed = true;
      }
    }
  }
  if (G > 1) {
    for (; p == 0 || again || (cb > SEL_SMALL && hi > 0); p++) {
      again = false;
      int lo = hi - SEL_DIGIT > 0 ? hi - SEL_DIGIT : 0;
      int nb = 1 << (hi - lo);
      uint64_t dm = (uint64_t)(nb - 1);
      for (int b = t; b < SEL_BINS; b += SEL_BS) h[b] = 0;
      __syncthreads();
      uint64_t mn = ~0ull, mx = 0;
      unsigned long long nbelow = 0;   // keys below the guessed range (guessed pass)
      for (int64_t i0 = (int64_t)B * SEL_BS + t; i0 < n; i0 += stride * SEL_UNROLL) {
        uint64_t kk[SEL_UNROLL];
#pragma unroll
        for (int u = 0; u < SEL_UNROLL; u++) {
          int64_t i = i0 + u * stride;
          kk[u] = i < n ? keys[i] : 0;
        }
#pragma unroll
        for (int u = 0; u < SEL_UNROLL; u++) {
          bool in = i0 + u * stride < n;
          bool m = in && (kk[u] & mask) == prefix;
          nbelow += in && (kk[u] & mask) < prefix;
          hist_add(h, m, (uint32_t)((kk[u] >> lo) & dm));
          if (m) {
            mn = kk[u] < mn ? kk[u] : mn;
            mx = kk[u] > mx ? kk[u] : mx;
          }
        }
      }
      __syncthreads();
      if (guessed) {
        unsigned long long bt;
        (void)block_incl_scan<unsigned long long, SEL_BS, false>(nbelow, tmp, &bt);
        if (t == 0) st->bbelow[B] = bt;
      }
      unsigned int (*bh)[SEL_BINS] = st->bhist[p & 1];
      unsigned int (*gs)[SEL_NGRP] = st->gsum[p & 1];
      for (int b = t; b < SEL_BINS; b += SEL_BS) bh[B][b] = h[b];   // one contiguous row per block
      {
        // group sums: 8 threads per group of 64 bins
        int g = t / 8, sub = t % 8;
        unsigned int s = 0;
        for (int q = 0; q < SEL_GBINS / 8; q++) s += h[g * SEL_GBINS + sub + 8 * q];
        s += __shfl_xor((int)s, 1);
        s += __shfl_xor((int)s, 2);
        s += __shfl_xor((int)s, 4);
        if (sub == 0) gs[B][g] = s;
      }
      block_minmax(mn, mx, red);
      if (t == 0) {
        st->bmn[p & 1][B] = mn;
        st->bmx[p & 1][B] = mx;
      }
      sel_barrier(flags, ++epoch, err);
      mn = ~0ull;
      mx = 0;
      for (int j = t; j < G; j += SEL_BS) {
        uint64_t a = st->bmn[p & 1][j], c = st->bmx[p & 1][j];
        mn = a < mn ? a : mn;
        mx = c > mx ? c : mx;
      }
      block_minmax(mn, mx, red);
      // the group holding the k-th key: 8 threads per group's row
      unsigned long long gc;
      {
        int g = t / 8, sub = t % 8;
        unsigned int s = col_part_sum<8>(&gs[0][0], SEL_NGRP, g, G, sub);
        s += __shfl_xor((int)s, 1);
        s += __shfl_xor((int)s, 2);
        s += __shfl_xor((int)s, 4);
        gc = sub == 0 ? s : 0;
      }
      unsigned long long total;
      unsigned long long before = block_incl_scan<unsigned long long, SEL_BS, false>(gc, tmp, &total) - gc;
      if (guessed) {
        guessed = false;
        unsigned long long bs = 0;
        for (int j = t; j < G; j += SEL_BS) bs += st->bbelow[j];
        unsigned long long below;
        (void)block_incl_scan<unsigned long long, SEL_BS, false>(bs, tmp, &below);
        if (k >= below && k - below < total) {
          // the k-th key shares the guessed bits: rank it among those keys
          k -= below;
          cb = (int64_t)total;
        } else {
          // it lies outside the guessed bounds: a pass again over every key
          // (uniform: every block read the same counts), into the other
          // histogram buffers, which no block still reads
          prefix = 0;
          mask = 0;
          hi = bits;
          cb = n;
          again = true;
          __syncthreads();
          continue;
        }
      }
      if (t == 0) spick[0] = ~0ull;
      __syncthreads();
      if (gc && k >= before && k < before + gc) {
        sgrp[0] = (unsigned int)(t / 8);
        spick[1] = before;
        spick[0] = 0;
      }
      __syncthreads();
      if (spick[0] == ~0ull) {   // k >= the number of keys (uniform over the grid)
        if (B == 0 && t == 0) {
          __hip_atomic_store(err, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          st->prefix = ~0ull;
          if (tsp.thr) band_threshold(tsp, ~0ull, false);
        }
        return;
      }
      unsigned int gstar = sgrp[0];
      unsigned long long kg = k - spick[1];
      __syncthreads();
      // the bin inside that group: 4 threads per bin's row
      unsigned long long bc;
      {
        int bi = t / 4, sub = t % 4;
        unsigned int s = col_part_sum<4>(&bh[0][0], SEL_BINS, gstar * SEL_GBINS + bi, G, sub);
        s += __shfl_xor((int)s, 1);
        s += __shfl_xor((int)s, 2);
        bc = sub == 0 ? s : 0;
      }
      before = block_incl_scan<unsigned long long, SEL_BS, false>(bc, tmp, &total) - bc;
      if (bc && kg >= before && kg < before + bc) {
        spick[0] = (unsigned long long)(gstar * SEL_GBINS + t / 4);
        spick[1] = before + (k - kg);
        spick[2] = bc;
      }
      __syncthreads();
      bstar = spick[0];
      prefix |= bstar << lo;
      mask |= dm << lo;
      k -= spick[1];
      bool all_one = (int64_t)spick[2] == cb;
      cb = (int64_t)spick[2];
      hi = lo;
      __syncthreads();
      if (all_one) {
        // one bucket holds every matching key: the bits the extreme ones share
        // are decided
        uint64_t x = mn ^ mx;
        if (x == 0) {
          prefix = mn;
          mask = ~0ull;
          hi = 0;
        } else {
          int d = 63 - __clzll((long long)x);   // highest differing bit
          if (d + 1 < hi) {
            uint64_t low = (2ull << d) - 1;     // d < hi <= 63 here
            prefix = mn & ~low;
            mask = ~low;
            hi = d + 1;
          }
        }
      }
    }
  }
  if (hi == 0 || cb == 0) {
    if (B == 0 && t == 0) {
      st->prefix = prefix;
      st->mask = mask;
      if (tsp.thr) band_threshold(tsp, prefix, false);
    }
    return;
  }
  // at most SEL_SMALL keys match: gather them
  if (t == 0) slocal = 0;
  __syncthreads();
  if (G == 1) {
    // every key matches: copy them in order (the host sized this launch
    // for at most SEL_SMALL keys)
    if (n > SEL_SMALL) {
      if (t == 0) __hip_atomic_store(err, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      n = SEL_SMALL;
    }
    constexpr int PER = 16;
    for (int c0 = 0; c0 < n; c0 += PER * SEL_BS) {
      uint64_t v[PER];
#pragma unroll
      for (int q = 0; q < PER; q++) {
        int i = c0 + t + q * SEL_BS;
        v[q] = i < n ? keys[i] : 0;
      }
#pragma unroll
      for (int q = 0; q < PER; q++) {
        int i = c0 + t + q * SEL_BS;
        if (i < n) sbuf[i] = v[q];
      }
    }
    __syncthreads();
    uint64_t r = lds_select(sbuf, (int)n, k, h, tmp, red, spick, err, s2, &s2cnt, st->ext);
    uint64_t kb = r & ~((1ull << tsp.ebits) - 1);   // start of the selected key's K bucket
    unsigned long long nlo = 0;
    if (tsp.guess) {
      unsigned long long c = 0;
      for (int i = t; i < n; i += SEL_BS) c += sbuf[i] < kb;
      (void)block_incl_scan<unsigned long long, SEL_BS, false>(c, tmp, &nlo);
    }
    if (t == 0) {
      st->prefix = r;
      st->mask = ~0ull;
      if (tsp.thr) {
        band_threshold(tsp, r, false);
        if (tsp.guess) {
          bool bucket = nlo < tsp.qlo_max;
          tsp.guess[0] = bucket ? kb : st->ext[0];
          tsp.guess[1] = bucket ? (r | ((1ull << tsp.ebits) - 1)) : *tsp.thr;
        }
      }
    }
    return;
  }
  // this block's offset: the chosen bucket's counts of the blocks before it
  unsigned int (*bh)[SEL_BINS] = st->bhist[(p - 1) & 1];
  unsigned long long part = t < B ? bh[t][bstar] : 0;   // B < SEL_MAXB <= SEL_BS
  unsigned long long off;
  (void)block_incl_scan<unsigned long long, SEL_BS, false>(part, tmp, &off);
  for (int64_t i0 = (int64_t)B * SEL_BS; i0 < n; i0 += stride * SEL_UNROLL) {
    uint64_t kk[SEL_UNROLL];
#pragma unroll
    for (int u = 0; u < SEL_UNROLL; u++) {
      int64_t i = i0 + u * stride + t;
      kk[u] = i < n ? keys[i] : 0;
    }
#pragma unroll
    for (int u = 0; u < SEL_UNROLL; u++) {
      bool m = i0 + u * stride + t < n && (kk[u] & mask) == prefix;
      unsigned int q = wave_reserve(&slocal, m);
      if (m && q < (unsigned)SEL_SMALL) sbuf[q] = kk[u];
    }
  }
  __syncthreads();
  unsigned int cnt = slocal < (unsigned)SEL_SMALL ? slocal : (unsigned)SEL_SMALL;
  for (unsigned int i = t; i < cnt; i += SEL_BS)
    if (off + i < (unsigned long long)SEL_SMALL) st->buf[off + i] = sbuf[i];
  sel_barrier(flags, ++epoch, err);
  if (B != 0) return;
  cnt = (unsigned int)cb;
  {
    constexpr int PER = 16;
    for (unsigned int c0 = 0; c0 < cnt; c0 += PER * SEL_BS) {
      uint64_t v[PER];
#pragma unroll
      for (int q = 0; q < PER; q++) {
        unsigned int i = c0 + t + q * SEL_BS;
        v[q] = i < cnt ? st->buf[i] : 0;
      }
#pragma unroll
      for (int q = 0; q < PER; q++) {
        unsigned int i = c0 + t + q * SEL_BS;
        if (i < cnt) sbuf[i] = v[q];
      }
    }
  }
  __syncthreads();
  uint64_t r = lds_select(sbuf, (int)cnt, k, h, tmp, red, spick, err, s2, &s2cnt);
  if (t == 0) {
    st->prefix = r;
    st->mask = ~0ull;
    if (tsp.thr) band_threshold(tsp, r, false);
  }
}

int radix_select(spc_ctx* ctx, const uint64_t* keys, const unsigned long long* cnt_dev,
                 int64_t cnt_bound, const unsigned long long* k_dev, unsigned long long k_host,
                 int bits, SelState* st, unsigned long long* flags, unsigned long long* err,
                 const ThrSpec* thr, const unsigned long long* guess_lo, const unsigned long long* guess_hi) {
  unsigned long long epoch0 = ctx->sel_epoch;
  ctx->sel_epoch += 64;   // a select meets at most 2 + 64 / SEL_DIGIT times
  // 32 keys per thread and pass up to SEL_MAXB blocks (a barrier's cost
  // grows with the blocks that meet at it)
  int maxb = ctx->num_cus < SEL_MAXB ? ctx->num_cus : SEL_MAXB;
  if (ctx->tune.sel_blocks > 0 && ctx->tune.sel_blocks < maxb) maxb = ctx->tune.sel_blocks;
  int grid = cnt_bound <= SEL_SMALL ? 1 : grid_for(cnt_bound, SEL_BS * 32, maxb);
  if (grid < 2 && cnt_bound > SEL_SMALL) grid = 2;
  hipLaunchKernelGGL(k_select, dim3(grid), dim3(SEL_BS), 0, ctx->stream, keys, cnt_dev, cnt_bound, k_dev,
                     k_host, bits, st, flags, epoch0, err, thr ? *thr : ThrSpec{nullptr, nullptr, 0, 1, 0, 0, nullptr, 0},
                     guess_lo, guess_hi);
  SPC_LAUNCH_CHECK(ctx, "radix_select");
  return SPC_OK;
}

// ---------------------------------------------------------------------------
// host orchestration of A1-A4
// ---------------------------------------------------------------------------
__global__ void k_set_u64(unsigned long long* p, unsigned long long v) { *p = v; }

__global__ void k_clear(int32_t* a, int64_t na, uint64_t* b, int64_t nb, uint64_t* c, int64_t nc,
                        unsigned long long* info, uint32_t slots, unsigned long long* word) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = i0; i < na; i += stride) a[i] = 0;
  for (int64_t i = i0; i < nb; i += stride) b[i] = 0;
  for (int64_t i = i0; i < nc; i += stride) c[i] = 0;
  if (info && i0 < 32 && (slots >> i0 & 1u)) info[i0] = 0;
  if (word && i0 == 32) *word = 0;
}

void launch_clear(spc_ctx* ctx, int32_t* a, int64_t na, uint64_t* b, int64_t nb, unsigned long long* info,
                  uint32_t slots, uint64_t* c, int64_t nc, unsigned long long* word) {
  int64_t big = na > nb ? na : nb;
  if (nc > big) big = nc;
  if (big < 64) big = 64;
  hipLaunchKernelGGL(k_clear, dim3(grid_for(big, 256, ctx->num_cus * 4)), dim3(256), 0, ctx->stream, a, na,
                     b, nb, c, nc, info, slots, word);
}

__global__ void k_readback(const unsigned long long* info, int ninfo, const int64_t* x0,
                           const int32_t* x1, const uint64_t* x2, int64_t* out, int64_t token) {
  int t = threadIdx.x;
  if (info && t < ninfo) out[t] = (int64_t)info[t];
  if (t == 0) {
    out[I_NINFO] = x0 ? *x0 : 0;
    out[I_NINFO + 1] = x1 ? (int64_t)*x1 : 0;
    out[I_NINFO + 2] = x2 ? (int64_t)*x2 : 0;
  }
  __threadfence_system();
  __syncthreads();
  if (t == 0 && token) __hip_atomic_store(&out[I_NINFO + 3], token, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

int wait_token(spc_ctx* ctx, int64_t token) {
  int64_t* w = ctx->h_pinned + I_NINFO + 3;
  for (long spins = 1;; spins++) {
    if (__atomic_load_n(w, __ATOMIC_ACQUIRE) == token) return SPC_OK;
    if ((spins & 4095) == 0 && hipStreamQuery(ctx->stream) != hipErrorNotReady) {
      SPC_HIP(ctx, hipStreamSynchronize(ctx->stream));
      if (__atomic_load_n(w, __ATOMIC_ACQUIRE) == token) return SPC_OK;
      return set_error(ctx, SPC_EHIP, "a kernel ended without its readback");
    }
  }
}

int readback_wait(spc_ctx* ctx, const unsigned long long* info, int ninfo, const int64_t* x0, const int32_t* x1,
                  const uint64_t* x2) {
  int64_t token = ++ctx->rb_token;
  hipLaunchKernelGGL(k_readback, dim3(1), dim3(64), 0, ctx->stream, info, ninfo, x0, x1, x2, ctx->h_pinned,
                     token);
  SPC_LAUNCH_CHECK(ctx, "readback");
  return wait_token(ctx, token);
}

__global__ void k_copy_u64(unsigned long long* dst, const unsigned long long* src) { *dst = *src; }

__global__ void k_fill_u64(uint64_t* __restrict__ a, int64_t n, uint64_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_zero32(uint32_t* __restrict__ a, int64_t n) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = 0u;
}

void launch_zero(spc_ctx* ctx, void* p, size_t bytes) {
  int64_t n = (int64_t)(bytes / sizeof(uint32_t));
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_zero32, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, ctx->stream,
                     (uint32_t*)p, n);
}

// a band threshold without a selection ("everything")
__global__ void k_thr_all(ThrSpec ts) { band_threshold(ts, 0, true); }

// Info block (and up to three scalars) to the pinned host copy, then wait.
static int sync_info(spc_ctx* ctx, const LevelWork& W, const int64_t* x0 = nullptr,
                     const int32_t* x1 = nullptr, const uint64_t* x2 = nullptr) {
  return readback_wait(ctx, W.info, (int)I_NINFO, x0, x1, x2);
}

// checks of the level's input that the device reports (integer weight
// total; floating-point weights finite, positive and within the exact range)
static int check_total(spc_ctx* ctx) {
  uint64_t total = (uint64_t)ctx->h_pinned[I_TOTAL];
  if (total > 2147483647ull)
    return set_error(ctx, SPC_EOVERFLOW, "total integer weight %llu exceeds 2^31-1",
                     (unsigned long long)total);
  uint64_t bad = (uint64_t)ctx->h_pinned[I_FP_BAD];
  if (bad & 1)
    return set_error(ctx, SPC_EINVAL, "floating-point weights must be finite and positive "
                                      "(self-loops finite and non-negative)");
  if (bad & 2)
    return set_error(ctx, SPC_ERANGE, "floating-point weights span more than %d binades: their sums "
                                      "cannot be held exactly", FP_MAX_SPAN);
  return SPC_OK;
}

// Spanning forest of the live list lr[0]/lp[0]/lo[0] (count in info[I_LIVE0])
// on top of the components already in parent.  With fused_first, bestA
// already holds every node's lightest incident key (first round done by the
// key pass); otherwise both best arrays must be all-infinite on entry.
// Rounds are issued two at a time between host synchronisations: a round
// with no live edges is an empty launch.  The first batch runs before any
// count is known on the host, with grids for the list's capacity m (blocks
// past the device-side count return at once).  On return the host copy of
// the info block is current.
static int spanning_forest(spc_ctx* ctx, LevelWork& W, int64_t n, int64_t m, bool fused_first,
                           const KeyND* guard_keys, int ebits, int64_t& live0, bool speculate,
                           bool& first_complete) {
  unsigned long long* info = W.info;
  int64_t* hinfo = ctx->h_pinned;
  int rc;
  int64_t cnt = m;
  uint64_t* cur = W.bestA;
  uint64_t* nxt = W.bestB;
  int in = 0;
  if (fused_first) {
    TimedScope ts(ctx, "forest_merge", (double)cnt);
    launch_bv_merge(ctx, W, cnt, W.lr[0], W.lp[0], W.lr[0], &info[I_LIVE0], cur, n, guard_keys, ebits);
  }
  if (fused_first) {
    // the band's first records start where the previous band's ended
    TimedScope ts(ctx, "forest_shortcut", (double)cnt);
    hipLaunchKernelGGL(k_shortcut, dim3(grid_for(cnt, 256, 16 * ctx->num_cus)), dim3(256), 0, ctx->stream,
                       W.parent, W.msfC,
                       &info[I_MSF0], &info[I_MSF]);
    cur = W.bestB;
    nxt = W.bestA;
  }
  int64_t bound = cnt;   // live edges of the current list, at most
  bool lo0_is_lr = true;  // list 0 comes from the row pass: its endpoints are its roots
  for (int batch = 0; bound > 0; batch++) {
    // every round at least halves the components that still have live
    // edges, so this many rounds means corrupted state
    if (batch >= 40) return set_error(ctx, SPC_EINVAL, "internal: spanning forest did not converge");
    // the first batch issues as many rounds as the previous level needed
    // (each round past convergence is three empty launches, each batch a
    // host wait); later batches two
    int rounds = batch == 0 ? (speculate && ctx->speculate == 2 ? 1 : ctx->forest_batch) : 2;
    for (int r = 0; r < rounds; r++) {
      int out = in ^ 1;
      bool mark = false;
      int ci = in == 0 ? I_LIVE0 : I_LIVE1;
      int co = out == 0 ? I_LIVE0 : I_LIVE1;
      {
        TimedScope ts(ctx, "forest_candidates", (double)bound);
        // the last round of a batch the host does not wait for also leaves
        // its live count in info[I_SPEC]
        mark = speculate && batch == 0 && r == rounds - 1;
        hipLaunchKernelGGL(k_bv_candidates, dim3(grid_for(bound, BC_CHUNK)), dim3(BS), 0, ctx->stream,
                           W.lr[in], W.lp[in], (in == 0 && lo0_is_lr) ? W.lr[0] : W.lo[in], &info[ci],
                           W.lr[out], W.lp[out], W.lo[out], &info[co], cur, nxt, W.parent,
                           next_scan(ctx, W), &info[I_FIN], &info[I_MSF], &info[I_MSF0],
                           mark ? &info[I_SPEC] : (unsigned long long*)nullptr);
      }
      if (out == 0) lo0_is_lr = false;
      if (mark) {
        // not waited for: the forest counts as complete only when this
        // lookup left no live edge, so its hooking round would be empty
        SPC_LAUNCH_CHECK(ctx, "forest round");
        in = out;
        break;
      }
      {
        TimedScope ts(ctx, "forest_merge", (double)bound);
        launch_bv_merge(ctx, W, bound, W.lr[out], W.lp[out], W.lo[out], &info[co], cur, n, guard_keys, ebits);
      }
      {
        TimedScope ts(ctx, "forest_shortcut", (double)bound);
        hipLaunchKernelGGL(k_shortcut, dim3(grid_for(bound, 256, 16 * ctx->num_cus)), dim3(256), 0,
                           ctx->stream, W.parent, W.msfC, &info[I_MSF0], &info[I_MSF]);
      }
      SPC_LAUNCH_CHECK(ctx, "forest round");
      uint64_t* t = cur;
      cur = nxt;
      nxt = t;
      in = out;
    }
    if (speculate) {
      // no wait: the live edges left are in info[I_SPEC] for a later check
      live0 = 0;
      return SPC_OK;
    }
    rc = sync_info(ctx, W);
    if (rc) return rc;
    if (batch == 0) {
      rc = check_total(ctx);
      if (rc) return rc;
      live0 = hinfo[I_CAND];
    }
    if (hinfo[I_LBERR]) return set_error(ctx, SPC_EINVAL, "internal: look-back wait gave up");
    bound = hinfo[in == 0 ? I_LIVE0 : I_LIVE1];
    if (batch == 0) first_complete = bound == 0;
  }
  return SPC_OK;
}

// Key pass, bands of candidate edges, spanning forest, cutoff.  On return
// sel2->prefix holds the key of the k-th lightest forest edge; info[I_VIOL]
// (read at the level's next synchronisation) says whether a guarded
// decision failed.
static int order_and_select(spc_ctx* ctx, const LevelIn& g, int64_t t, int64_t k, int64_t m,
                            bool rank, LevelWork& W, LevelResult& R, const LevelInF* gf,
                            const Segments* seg, bool speculate) {
  hipStream_t st = ctx->stream;
  int64_t n = g.n;
  unsigned long long* info = W.info;
  int64_t* hinfo = ctx->h_pinned;
  int ebits = bitlen64((uint64_t)(m - 1));
  if (ebits < 1) ebits = 1;
  int c = 62 - ebits;
  const unsigned long long* guard = &info[I_GUARD];
  if (!rank) {
    launch_score(ctx, g, W, m, c, ebits, 0);   // timed inside, one scope per kernel
  }
  if (!rank) {
    SPC_LAUNCH_CHECK(ctx, "score");   // the first band's threshold kernel sets the key mode
    R.key_bits = 64;
  } else if (gf) {
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, &info[I_GUARD], 0ull);
    int rc = fp_rank_keys(ctx, *gf, W, m);
    if (rc) return rc;
    R.key_bits = bitlen64((uint64_t)(m - 1));
  } else {
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, &info[I_GUARD], 0ull);
    {
      launch_score(ctx, g, W, m, c, ebits, 1);
    }
    SPC_LAUNCH_CHECK(ctx, "score(rank)");
    KeyND* sorted = nullptr;
    {
      TimedScope ts(ctx, "rank_sort", (double)m);
      int rc = merge_sort<KeyND, LessND>(ctx, W.keysA, W.keysB, m, LessND(), &sorted);
      if (rc) return rc;
    }
    TimedScope ts(ctx, "rank_scatter", (double)m);
    launch_rank_scatter(ctx, g, W, m, sorted);
    SPC_LAUNCH_CHECK(ctx, "rank scatter");
    R.key_bits = bitlen64((uint64_t)(m - 1));
  }
  // exact records for guarded checks (only consulted when info[I_GUARD] is set)
  const KeyND* gk = rank ? nullptr : W.keysA;

  // A4: bands of the lightest edges; each band extends the forest built so far
  unsigned long long* thr_lo = &info[I_BAD];
  unsigned long long* thr_hi = &info[I_NC];
  int64_t target = k + k / 2 + 4096;
  int64_t done_cand = 0;
  bool sampled = false;   // a band threshold came from the key samples
  R.candidates = 0;
  for (int band = 0;; band++) {
    // a batch builds its forest in one band: each graph's own (each graph
    // needs its own count of forest edges), or every edge when a graph's
    // band fell short
    bool seg_band = seg && band == 0 && !rank && !gf && !ctx->seg_full_band && !ctx->force_full_filter &&
                    target < m;
    bool all = ctx->force_full_filter || target >= m || band >= 2 || (seg && !seg_band);
    R.seg_band = seg_band;
    int kc = (!rank && band == 0) ? c : 0;   // the first threshold kernel also sets the key mode
    if (band > 0) {
      hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, st, W.bestA, n, KEY_INF);
      hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, st, W.bestB, n, KEY_INF);
      // the previous band's upper bound is this band's lower bound
      hipLaunchKernelGGL(k_copy_u64, dim3(1), dim3(1), 0, st, thr_lo, thr_hi);
    }
    if (all || seg_band) {
      // (also the key mode of the level, read by the batch bands)
      hipLaunchKernelGGL(k_thr_all, dim3(1), dim3(1), 0, st, ThrSpec{thr_hi, info, kc, ebits, 0, 0, nullptr, 0});
      if (seg_band) {
        TimedScope ts(ctx, "batch_bands", (double)seg->G);
        int rc = seg_bands(ctx, g, W, *seg, ebits, ctx->seg_band_shrink != 0);
        if (rc) return rc;
      }
    } else if (!rank) {
      int sh = sample_shift(m);
      int64_t ns = ((m - 1) >> sh) + 1;
      int64_t q = (int64_t)((double)target / (double)(1ll << sh) * 1.05) + 16;
      if (q >= ns) {
        all = true;
        hipLaunchKernelGGL(k_thr_all, dim3(1), dim3(1), 0, st, ThrSpec{thr_hi, info, kc, ebits, 0, 0, nullptr, 0});
      } else {
        TimedScope ts(ctx, "select_threshold", (double)ns);
        // a tied band of consecutive rows needs about k rows: k m / n edges
        uint64_t e_tie = 0;
        if (band == 0) {
          double rows = 1.1 * (double)k * (double)m / (double)n + 4096.0;
          e_tie = rows >= (double)(m - 1) ? (uint64_t)(m - 1) : (uint64_t)rows;
        }
        // the cutoff is taken to lie in the selected sample's K bucket when
        // fewer than about 0.9 k edges lie below that bucket
        ThrSpec tsp{thr_hi, info, kc, ebits, (unsigned long long)q << sh, (unsigned long long)e_tie,
                    W.sel->guess, (unsigned long long)(0.9 * (double)k) >> sh};
        int rc = radix_select(ctx, W.samples, nullptr, ns, nullptr, (unsigned long long)q, 64, W.sel,
                              (unsigned long long*)W.selflag, &info[I_LBERR], &tsp);
        if (rc) return rc;
        sampled = true;
      }
    } else {
      hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, thr_hi, (unsigned long long)(target - 1));
    }
    {
      TimedScope ts(ctx, "rowpass", (double)g.nnz);
      hipLaunchKernelGGL(k_rowpass, dim3(grid_for(g.nnz, TILE_R)), dim3(BS), 0, st, g, W.lc, W.Pc,
                         thr_lo, thr_hi, band > 0 ? 1 : 0, band == 0 ? 1 : 0, W.bestA, W.lr[0],
                         W.lp[0], &info[I_LIVE0], &info[I_CAND], next_scan(ctx, W),
                         gf ? (const int32_t*)nullptr : W.ptrow,   // (the integer degree pass wrote it)
                         seg_band ? W.gid : (const int32_t*)nullptr, seg_band ? W.thrg : (const uint64_t*)nullptr);
    }
    SPC_LAUNCH_CHECK(ctx, "rowpass");
    int64_t live0 = 0;
    bool spec = speculate && band == 0 && !seg;
    bool first_complete = false;
    int rc = spanning_forest(ctx, W, n, m, band == 0, gk, ebits, live0, spec, first_complete);
    if (rc) return rc;
    R.bands = band + 1;
    if (spec) {
      // assumed complete with at least k edges; counts come with the
      // level's later read
      R.spec = true;
      R.msf = -1;
      break;
    }
    if (band == 0) R.first_batch_complete = first_complete;
    done_cand += live0;
    R.candidates = done_cand;
    R.msf = hinfo[I_MSF];
    if (seg || R.msf >= k) break;
    if (all)
      return set_error(ctx, SPC_EUNREACHABLE,
                       "only %lld merges possible, %lld requested (more than %lld components)",
                       (long long)R.msf, (long long)k, (long long)t);
    // candidates needed grow with the shortfall of forest edges per candidate
    double need = (double)done_cand * 1.3 * (double)k / (double)(R.msf > 0 ? R.msf : 1);
    int64_t nt = (int64_t)need + 4096;
    target = nt > 2 * target ? nt : 2 * target;
  }

  if (seg) return SPC_OK;   // each graph's cutoff: seg_cutoff_union in select_level
  // cutoff: the k-th lightest forest edge
  {
    TimedScope ts(ctx, "select_cutoff", (double)R.msf);
    int bits = rank ? bitlen64((uint64_t)(m - 1)) : 64;
    // sized for the forest's record count when the host read it (else for n)
    int64_t nf = R.spec ? n : R.msf > 1 ? R.msf : 1;
    // bounds the band's sample selection guessed for the cutoff (checked by
    // the selection)
    const unsigned long long* glo = sampled && !rank ? &W.sel->guess[0] : nullptr;
    if (glo && ctx->force_bad_guess) {
      // (a test option: bounds above every forest key, so that the
      // selection takes its start-over path)
      hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, &W.sel->guess[0], ~0ull - 1);
      hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, &W.sel->guess[1], ~0ull);
    }
    int rc = radix_select(ctx, W.msfP, &info[I_MSF], nf, nullptr, (unsigned long long)(k - 1), bits,
                          W.sel2, (unsigned long long*)W.selflag, &info[I_LBERR], nullptr, glo,
                          glo ? &W.sel->guess[1] : nullptr);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_cutoff_union, dim3(grid_for(n, 256, ctx->num_cus * 8)), dim3(256), 0, st, W.msfP,
                     W.msfO, &info[I_MSF], W.sel2, rank ? (const KeyND*)nullptr : (const KeyND*)W.keysA, W.kexact,
                     guard, ebits, (int*)&info[I_VIOL], W.root, W.mcount, W.gptr, t + 1);
  R.contract_zeroed = true;
  SPC_LAUNCH_CHECK(ctx, "cutoff check");
  return SPC_OK;
}

int select_level(spc_ctx* ctx, const LevelIn& g, int64_t t, int32_t* cluster_of, LevelWork& W,
                 LevelResult& R, const LevelInF* gf, const Segments* seg, bool defer, bool rank_only,
                 bool speculate) {
  if (seg && gf)
    return set_error(ctx, SPC_EINVAL, "batched coarsening takes integer weights");
  hipStream_t st = ctx->stream;
  int64_t n = g.n, m = g.nnz / 2;
  int64_t k = n - t;  // merges
  unsigned long long* info = W.info;
  int64_t* hinfo = ctx->h_pinned;
  ctx->lb_words = lb_words(n, g.nnz);
  ctx->lb_epoch = 0;
  ctx->sel_epoch = 0;
  // every level starts with the scan chain's error flag clear, so one
  // failed wait does not fail later calls on this context
  launch_clear(ctx, nullptr, 0, W.lbstate, ctx->lb_words, info, 0xffffffffu, W.selflag,
               (int64_t)SEL_MAXB * SEL_FLAG,
               ctx->scan_state ? (unsigned long long*)(ctx->scan_state + ctx->scan_cap - 1) : nullptr);
  if (ctx->force_scan_flag && ctx->scan_state) {
    // test option: this level finds the flag raised, as after a wait that gave up
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st,
                       (unsigned long long*)(ctx->scan_state + ctx->scan_cap - 1), 1ull);
    ctx->force_scan_flag = 0;
  }

  // A1
  int nb = grid_for(n, DEG_ROWS);
  if (gf) {
    TimedScope ts(ctx, "degree_fp", (double)n);
    launch_fp_degree(ctx, *gf, W);
  } else {
    {
      TimedScope ts(ctx, "degree", (double)n);
      hipLaunchKernelGGL(k_degree, dim3(nb), dim3(BS), 0, st, g, W.deg, W.lc, W.uptr, W.bestA, W.bestB,
                         W.parent, W.root, W.degpart, W.htab, info, next_scan(ctx, W), W.trow, W.ptrow);
    }
    TimedScope ts(ctx, "degree_total", (double)nb);
    // (with the long rows' position maps for the scores, when rows can be long)
    int sp_grid = 1 + (g.nnz > HUGE_T ? H_MAX * SP_MAP : 0);
    hipLaunchKernelGGL(k_sum_parts, dim3(sp_grid), dim3(SP_BS), 0, st, W.degpart, (int64_t)nb, g, W.htab, W.deg,
                       info, W.hmap);
  }
  SPC_LAUNCH_CHECK(ctx, "degree");
  int rc;
  if (gf) {
    // the floating-point degree pass leaves upper-entry counts (the integer
    // one stores their prefix itself)
    TimedScope ts(ctx, "scan_upper", (double)n);
    rc = exclusive_scan<int64_t>(ctx, W.uptr, W.uptr, n, (int64_t*)W.scan_partial);
    if (rc) return rc;
  }
  if (k <= 0 || m == 0) {
    rc = sync_info(ctx, W);
    if (rc) return rc;
    rc = check_total(ctx);
    if (rc) return rc;
    if (k > 0) return set_error(ctx, SPC_EUNREACHABLE, "graph has no edges");
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n, 256)), dim3(256), 0, st, cluster_of, n);
    R.n_c = n;
    R.eps = 0.0;
    return SPC_OK;
  }

  // A2-A4 and the labels; a guarded key that fails its exactness check
  // falls back to ranks
  bool rank = ctx->force_rank_mode != 0 || gf != nullptr || rank_only;
  for (int pass = 0; pass < 2; pass++) {
    if (pass == 1) {
      rank = true;
      uint32_t slots = (1u << I_MSF) | (1u << I_VIOL);
      for (int i = I_ROUNDS; i <= I_MSF0; i++) slots |= 1u << i;
      launch_clear(ctx, nullptr, 0, nullptr, 0, info, slots);
      hipLaunchKernelGGL(k_iota, dim3(grid_for(n, 256)), dim3(256), 0, st, W.parent, n);
      hipLaunchKernelGGL(k_iota, dim3(grid_for(n, 256)), dim3(256), 0, st, W.root, n);
      hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, st, W.bestA, n, KEY_INF);
      hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, st, W.bestB, n, KEY_INF);
    }
    R.k = k;
    rc = order_and_select(ctx, g, t, k, m, rank, W, R, gf, seg, speculate && defer && pass == 0);
    if (rc) return rc;
    int64_t msf_bound = R.msf >= 0 ? R.msf : n;
    {
      TimedScope ts(ctx, "components", (double)n);
      // (the whole-graph path joined its cutoff's forest edges in the
      // cutoff's launch; a batch joins each graph's here)
      if (seg) {
        int ebits = bitlen64((uint64_t)(m - 1));
        rc = seg_cutoff_union(ctx, g, W, R, *seg, ebits < 1 ? 1 : ebits, rank);
        if (rc) return rc;
      }
      // roots (into parent, free after the forest) and root flags
      hipLaunchKernelGGL(k_cc_flatten, dim3(grid_for(n, 256)), dim3(256), 0, st, W.root, W.parent,
                         W.flag, n);
    }
    SPC_LAUNCH_CHECK(ctx, "components");
    {
      TimedScope ts(ctx, "relabel", (double)n);
      // labels: the scan leaves the number of roots in flag[n]
      rc = exclusive_scan<int32_t>(ctx, W.flag, W.flag, n, (int32_t*)W.scan_partial);
      if (rc) return rc;
      launch_relabel_eps(ctx, g, W, cluster_of, t, gf || seg ? 0 : msf_bound, !gf && !seg);
    }
    if (gf) launch_eps_fp(ctx, W);
    if (ctx->force_redo_rank && !rank)
      hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, &info[I_VIOL], 1ull);
    SPC_LAUNCH_CHECK(ctx, "relabel");
    if (defer) {
      // labels are in [0, t) whatever the key mode: the cutoff joins exactly
      // k forest edges (keys are distinct), and the labelling clamps besides
      R.pending = true;
      R.pending_rank = rank;
      R.n_c = t;
      return SPC_OK;
    }
    rc = sync_info(ctx, W, nullptr, W.flag + n);
    if (rc) return rc;
    rc = finish_select(ctx, R, t, rank, gf != nullptr, seg);
    if (rc != SPC_REDO_RANK) return rc;
  }
  return set_error(ctx, SPC_EINVAL, "internal: rank keys redone twice");
}

int finish_select(spc_ctx* ctx, LevelResult& R, int64_t t, bool rank, bool fp, const Segments* seg) {
  int64_t* hinfo = ctx->h_pinned;
  R.pending = false;
  if (R.spec) {
    // the forest the host did not wait for: complete after its first batch
    // and with at least k edges?  Otherwise every later step used a wrong
    // forest, and the level is redone waiting
    R.spec = false;
    if (hinfo[I_SPEC] != 0 || hinfo[I_MSF] < R.k) {
      ctx->spec_ok = 0;
      return SPC_REDO_SPEC;
    }
    int rc = check_total(ctx);
    if (rc) return rc;
    R.msf = hinfo[I_MSF];
    R.candidates = hinfo[I_CAND];
    R.first_batch_complete = true;
  }
  ctx->spec_ok = R.bands == 1 && R.first_batch_complete ? 1 : 0;
  int64_t nc = (int32_t)hinfo[I_NINFO + 1];
  R.key_mode = fp ? 3 : rank ? 1 : (hinfo[I_GUARD] ? 2 : 0);
  R.rounds = hinfo[I_ROUNDS];
  {
    // rounds after the fused first one, plus the lookup that finds the
    // list empty
    int64_t need = R.rounds - (R.bands == 1 ? 1 : 0) + 1;
    ctx->forest_batch = need < 1 ? 1 : need > 8 ? 8 : (int)need;
  }
  R.forest_in = hinfo[I_FIN];
  R.forest_kept = hinfo[I_FKEPT];
  R.merge_in = hinfo[I_MIN];
  R.keys_written = (rank || hinfo[I_KEYS]) ? 1 : 0;
  if (hinfo[I_VIOL]) {
    if (rank) return set_error(ctx, SPC_EINVAL, "internal: exact rank order flagged as inexact");
    return SPC_REDO_RANK;
  }
  if (hinfo[I_LBERR]) return set_error(ctx, SPC_EINVAL, "internal: look-back wait gave up");
  if (seg && hinfo[I_SEG_SHORT]) {
    if (R.seg_band) return SPC_REDO_BAND;   // a band, not the graph, may have fallen short
    return set_error(ctx, SPC_EUNREACHABLE, "a graph of the batch has more components than its target");
  }
  double eps;
  memcpy(&eps, &hinfo[I_EPS], sizeof(double));
  R.eps = eps;
  R.n_c = nc;
  if (R.n_c != t)
    return set_error(ctx, SPC_EINVAL, "internal: %lld super-nodes produced, %lld expected",
                     (long long)R.n_c, (long long)t);
  return SPC_OK;
}

}  // namespace spc

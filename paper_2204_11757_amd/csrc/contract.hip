// A5: contraction of the fine graph into the coarsened graph of
// Definition 1.  Super-node a's weight towards b is the sum of w(x, y) over
// members x of a and y of b; pairs inside one super-node become a's
// self-loop weight together with the members' own self-loops; sizes add.
// Coarse rows are ascending in b with no diagonal entry.
//
// Two streaming passes put every super-node's inputs side by side, then
// one reduction per coarse row:
//   slots    each fine node x holds 1 + len(x) records of super-node c(x)
//            (a member record with its size and self-loop, then one record
//            (c(y), w) per entry x -> y); run-aggregated atomics on the
//            super-node's record count hand out x's slot range;
//   scatter  entry-parallel tiles write every entry's record, and the
//            member records, at those slots: super-node a's records are
//            then contiguous at rec[gptr[a], gptr[a + 1]);
//   reduce   by the record count E_a of the row:
//              E_a <= SMALL_CAP   one thread, a sorted register list;
//              E_a <= REG32_CAP   sixteen lanes, sums in an LDS hash table
//                                 and each distinct column's rank;
//              E_a <= WAVE_CAP    one wavefront, the same (a bitonic sort in
//                                 LDS above WAVE_CAP / 2 records);
//              E_a <= BLOCK_CAP   one 256-thread block, bitonic sort in LDS;
//              larger             dense accumulators over the coarse ids
//                                 (few such rows) or a merge sort of all
//                                 their records.
// A row's distinct (column, weight) pairs overwrite its own records (they
// are fewer), a scan of the row counts gives the coarse row pointer, and a
// tiled copy packs the entries.  Integer sums do not depend on the order in
// which the atomics placed the members, so the result is deterministic.
#include "level.hpp"

namespace spc {

constexpr int SMALL_CAP = 16;
constexpr int REG32_CAP = 32;
constexpr int SMALL_BS = 128;
constexpr int SMALL_RPT = 4;   // rows per thread, at most (fewer when there are few rows)
constexpr int WAVE_CAP = 512;
constexpr int BLOCK_CAP = 4096;

// Records: an entry x -> y of a member is (c(y) << 32) | w (c(y) < 2^31); a
// member record has bit 63 set, the member's size in bits 32..62 and its
// self-loop weight in bits 0..31 (both below 2^31 by the weight bound).
constexpr uint64_t REC_MEMBER = 1ull << 63;

__device__ __forceinline__ uint64_t member_record(uint32_t size, uint32_t self) {
  return REC_MEMBER | ((uint64_t)size << 32) | self;
}

// Lanes of a wavefront holding the same key in consecutive lanes form a
// run.  head: this lane starts its run; end: one past the run's last lane
// (meaningful on the head lane).  All 64 lanes must call it.
__device__ __forceinline__ void wave_runs(int32_t key, bool& head, int& end, uint64_t& heads) {
  int l = lane_id();
  int32_t prev = __shfl_up(key, 1);
  head = (l == 0) || (key != prev);
  heads = __ballot(head);
  uint64_t after = (l == WAVE - 1) ? 0ull : (heads & (~0ull << (l + 1)));
  end = after ? (__ffsll((long long)after) - 1) : WAVE;
}

__device__ __forceinline__ int run_head_of(uint64_t heads) {
  int l = lane_id();
  uint64_t upto = (l == WAVE - 1) ? heads : (heads & ((2ull << l) - 1));
  return 63 - __clzll((long long)upto);
}

// Member counting and scattering take one node per thread in blocks of
// CM_BS.  Consecutive nodes of one super-node form runs; a run inside a
// wavefront is summed with wavefront operations, and runs that continue
// across wavefront borders are chained by thread 0 so that a super-node
// spanning the whole block costs one global atomic (a giant super-node
// would otherwise serialise one atomic per wavefront on one address).
constexpr int CM_BS = 1024;
constexpr int CM_W = CM_BS / WAVE;

struct RunPieces {
  int32_t fk[CM_W], lk[CM_W];             // keys of each wavefront's first / last run
  int32_t fc[CM_W], lc[CM_W];             // their lengths in nodes
  unsigned long long fe[CM_W], le[CM_W];  // their summed values
  int32_t single[CM_W];                   // the wavefront is one run
  unsigned long long fb[CM_W], lb[CM_W];  // slot bases handed back
};

// Border pieces: piece 0 of wavefront w is its first run, piece 1 its last
// run (present when the wavefront holds more than one run).  A chain is a
// maximal sequence of pieces with one key that touch across wavefront
// borders.  Thread q < 2 * CM_W looks at piece (q / 2, q % 2); if that piece
// starts a chain, it returns true with the chain's key, node count and
// value sum, and its last piece in (wl, pl).
__device__ __forceinline__ bool chain_at(const RunPieces& P, int q, int32_t& key, int& cnt,
                                         unsigned long long& sum, int& wl, int& pl) {
  int w = q >> 1, p = q & 1;
  if (p == 1 && P.single[w]) return false;
  key = p ? P.lk[w] : P.fk[w];
  if (p == 0 && w > 0 && key == (P.single[w - 1] ? P.fk[w - 1] : P.lk[w - 1])) return false;
  cnt = p ? P.lc[w] : P.fc[w];
  sum = p ? P.le[w] : P.fe[w];
  wl = w;
  pl = p;
  // extend while the current piece ends its wavefront and the next
  // wavefront opens with the same key
  while ((pl == 1 || P.single[wl]) && wl + 1 < CM_W && P.fk[wl + 1] == key) {
    wl++;
    pl = 0;
    cnt += P.fc[wl];
    sum += P.fe[wl];
  }
  return true;
}

// ---- slots: each fine node's record range inside its super-node -----------
// Thread per node x (blocks of CM_BS): x needs 1 + len(x) slots of c(x).  A
// run of lanes with one super-node takes its slots with one atomic on the
// super-node's count; runs continuing across wavefront borders are chained
// by thread 0's pieces (one atomic per chain).  off[x] = x's first slot
// relative to its super-node's first record; ecnt[a] ends as a's record
// count.
__global__ void __launch_bounds__(CM_BS)
    k_slot_alloc(LevelIn g, const int32_t* __restrict__ c, unsigned long long* ecnt,
                 int64_t* __restrict__ off) {
  __shared__ RunPieces P;
  int64_t x = (int64_t)blockIdx.x * CM_BS + threadIdx.x;
  bool valid = x < g.n;
  int32_t a = valid ? c[x] : -1;
  int64_t len = valid ? 1 + (g.rp[x + 1] - g.rp[x]) : 0;
  // a super-node whose members are spread over the wavefront (a large
  // super-node of an irregular graph) would cost one atomic per member on
  // one address: the lanes of the first lane's super-node take their slots
  // together first, and drop out of the runs below (when they are one run
  // from lane 0 the runs already take them together, across wavefronts)
  int32_t hot = __shfl(a, 0);
  uint64_t hmask = __ballot(a == hot && hot >= 0);
  int64_t hot_off = -1;
  if (hot >= 0 && __popcll(hmask) > 1 && (hmask & (hmask + 1)) != 0) {
    bool mine = (hmask >> lane_id()) & 1ull;
    int64_t hl = mine ? len : 0;
    int64_t hinc = wave_incl_sum(hl);
    int64_t htot = __shfl(hinc, WAVE - 1);
    unsigned long long hb = 0;
    if (lane_id() == 0) hb = atomicAdd(&ecnt[hot], (unsigned long long)htot);
    hb = __shfl(hb, 0);
    if (mine) {
      hot_off = (int64_t)hb + hinc - hl;
      a = -1;
      len = 0;
    }
  }
  bool head;
  int end;
  uint64_t heads;
  wave_runs(a, head, end, heads);
  int64_t inc = wave_incl_sum(len);
  int64_t at_end = __shfl(inc, end - 1);
  int l = lane_id(), w = threadIdx.x / WAVE;
  unsigned long long base = 0;   // on head lanes of inner runs: the run's first slot
  if (head) {
    int cnt = end - l;
    unsigned long long e = (unsigned long long)(at_end - inc + len);
    bool first = l == 0, last = end == WAVE;
    if (first) {
      P.fk[w] = a;
      P.fc[w] = cnt;
      P.fe[w] = e;
      P.single[w] = last ? 1 : 0;
    } else if (last) {
      P.lk[w] = a;
      P.lc[w] = cnt;
      P.le[w] = e;
    } else if (a >= 0) {
      base = atomicAdd(&ecnt[a], e);
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * CM_W) {
    int32_t k;
    int cnt, wl, pl;
    unsigned long long e;
    if (chain_at(P, threadIdx.x, k, cnt, e, wl, pl) && k >= 0) {
      unsigned long long b = atomicAdd(&ecnt[k], e);
      // consecutive slot ranges to the chain's pieces in block order
      int v = threadIdx.x >> 1, q = threadIdx.x & 1;
      while (true) {
        if (q == 0) {
          P.fb[v] = b;
          b += P.fe[v];
        } else {
          P.lb[v] = b;
          b += P.le[v];
        }
        if (v == wl && q == pl) break;
        v++;
        q = 0;
      }
    }
  }
  __syncthreads();
  int h = run_head_of(heads);
  unsigned long long bh = __shfl(base, h);
  int endh = __shfl(end, h);
  int64_t before_h = __shfl(inc, h) - __shfl(len, h);   // the wavefront's slots before the run
  if (valid) {
    if (hot_off >= 0) {
      off[x] = hot_off;
    } else {
      if (h == 0) bh = P.fb[w];
      else if (endh == WAVE) bh = P.lb[w];
      off[x] = (int64_t)bh + (inc - len - before_h);
    }
  }
}

// ---- scatter: every record to its slot --------------------------------------
// Tiles of RT consecutive fine entries (mapped to rows by the load-balanced
// search, renumbered per XCD so that a tile's neighbours share its L2) write
// (c(y) << 32) | w at gptr[c(x)] + off[x] + 1 + (j - rp[x]); the member
// records are written by the tiles that take the per-row path, for the rows
// starting in them, and by the blocks past the tiles (RM nodes per block)
// for the other rows.
constexpr int RT = ENTRY_TILE;
constexpr int RT_BS = 256;
constexpr int RT_PER = RT / RT_BS;
constexpr int RM = 2048;

// A tile whose rows r0..r1 number at most RT: each row's record base
// gptr[c(x)] + off[x] + 1 - rp[x] is computed once, in the pass that marks
// the rows' first positions for the load-balanced search, and the entries'
// own loads are issued before it.  The same pass writes the member record
// (just before the row's first entry record) of every row that starts in
// the tile (the last tile: at or after its start), so it lands beside the
// row's entries.
__device__ __forceinline__ bool scatter_rows_tile(const int32_t* __restrict__ ptrow, int64_t t, int tiles,
                                                  int64_t n, int64_t& r0, int64_t& r1) {
  r0 = ptrow[t];
  r1 = t + 1 < tiles ? ptrow[t + 1] : n - 1;
  return r1 - r0 < RT;
}

__device__ __forceinline__ void scatter_tile_rows(const LevelIn& g, const int32_t* __restrict__ c,
                                                  const int64_t* __restrict__ gptr,
                                                  const int64_t* __restrict__ off, uint64_t* __restrict__ rec,
                                                  int64_t p0, int64_t r0, int64_t r1, bool last, int32_t* srow,
                                                  int64_t* sbase_row, int32_t* stmp) {
  using L = Lbs<RT, RT_BS>;
  int tid = threadIdx.x;
  int32_t yr[RT_PER];
  uint32_t wr[RT_PER];
#pragma unroll
  for (int i = 0; i < RT_PER; i++) {
    int64_t j = p0 + tid + i * RT_BS;
    bool in = j < g.nnz;
    yr[i] = in ? g.col[j] : 0;
    wr[i] = in ? (uint32_t)g.w[j] : 0u;
  }
  for (int k = tid; k < RT; k += RT_BS) srow[L::at(k)] = (int32_t)r0;
  __syncthreads();
  int nr = (int)(r1 - r0) + 1;   // at most RT
  for (int i = tid; i < nr; i += RT_BS) {
    int64_t r = r0 + i;
    int64_t pr = g.rp[r];
    int64_t b = gptr[c[r]] + off[r] + 1 - pr;
    int64_t q = pr - p0;
    if (i > 0 && q > 0 && q < RT) atomicMax(&srow[L::at((int)q)], (int32_t)r);
    sbase_row[i] = b;
    if (q >= 0 && (q < RT || last)) {
      uint32_t sz = g.size ? (uint32_t)g.size[r] : 1u;
      uint32_t sw = g.self ? (uint32_t)g.self[r] : 0u;
      rec[b + pr - 1] = member_record(sz, sw);
    }
  }
#pragma unroll
  for (int i = 0; i < RT_PER; i++) yr[i] = c[yr[i]];
  __syncthreads();
  // inclusive max-scan of the marks: every position's row
  constexpr int PER = L::PER;
  int32_t loc[PER];
  int32_t run = INT32_MIN;
#pragma unroll
  for (int i = 0; i < PER; i++) {
    int32_t v = srow[L::at(tid * PER + i)];
    run = v > run ? v : run;
    loc[i] = run;
  }
  int32_t tot;
  int32_t inc = block_incl_scan<int32_t, RT_BS, true>(run, stmp, &tot);
  int32_t prev = __shfl_up(inc, 1);
  if (lane_id() == 0) prev = (tid / WAVE > 0) ? stmp[tid / WAVE - 1] : INT32_MIN;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; i++) srow[L::at(tid * PER + i)] = loc[i] > prev ? loc[i] : prev;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RT_PER; i++) {
    int k = tid + i * RT_BS;
    int64_t j = p0 + k;
    if (j < g.nnz) {
      int32_t x = srow[L::at(k)];
      rec[sbase_row[x - r0] + j] = ((uint64_t)(uint32_t)yr[i] << 32) | wr[i];
    }
  }
}

__global__ void __launch_bounds__(RT_BS)
    k_record_scatter(LevelIn g, const int32_t* __restrict__ c, const int64_t* __restrict__ gptr,
                     const int64_t* __restrict__ off, uint64_t* __restrict__ rec, int tiles,
                     const int32_t* __restrict__ ptrow) {
  __shared__ int32_t srow[Lbs<RT, RT_BS>::SIZE];
  __shared__ int64_t sh[2];
  __shared__ int32_t stmp[RT_BS / WAVE];
  __shared__ int64_t sbase_row[RT];
  int tid = threadIdx.x;
  if ((int)blockIdx.x >= tiles) {
    // the member records the tiles did not write: rows whose tile (the one
    // holding the row's start; the last one for rows starting at the end)
    // took the per-entry path, or whose rows it does not span (an empty row
    // starting right at the tile's first position, before the row that
    // holds it)
    int64_t x0 = (int64_t)(blockIdx.x - tiles) * RM;
#pragma unroll
    for (int i = 0; i < RM / RT_BS; i++) {
      int64_t x = x0 + i * RT_BS + tid;
      if (x >= g.n) break;
      if (ptrow && tiles > 0) {
        int64_t t = g.rp[x] / RT;
        if (t > tiles - 1) t = tiles - 1;
        int64_t ra, rb;
        if (scatter_rows_tile(ptrow, t, tiles, g.n, ra, rb) && x >= ra && x <= rb) continue;
      }
      uint32_t sz = g.size ? (uint32_t)g.size[x] : 1u;
      uint32_t sw = g.self ? (uint32_t)g.self[x] : 0u;
      rec[gptr[c[x]] + off[x]] = member_record(sz, sw);
    }
    return;
  }
  int64_t t = xcd_tile(blockIdx.x, tiles);
  int64_t p0 = t * RT;
  if (ptrow) {
    // the tile's first row from the degree pass (uniform over the block)
    int64_t r0, r1;
    if (scatter_rows_tile(ptrow, t, tiles, g.n, r0, r1)) {
      scatter_tile_rows(g, c, gptr, off, rec, p0, r0, r1, t == tiles - 1, srow, (int64_t*)sbase_row, stmp);
      return;
    }
    lbs_fill<RT, RT_BS>(g.rp, r0, r1, p0, srow, stmp);
  } else {
    lbs_tile<RT, RT_BS>(g.rp, g.n, p0, srow, sh, stmp);
  }
  int32_t xr[RT_PER], yr[RT_PER];
  uint32_t wr[RT_PER];
  int64_t pr[RT_PER];
  // all loads of a stage issued before any is used
#pragma unroll
  for (int i = 0; i < RT_PER; i++) {
    int k = tid + i * RT_BS;
    int64_t j = p0 + k;
    bool in = j < g.nnz;
    xr[i] = in ? srow[Lbs<RT, RT_BS>::at(k)] : -1;
    yr[i] = in ? g.col[j] : 0;
    wr[i] = in ? (uint32_t)g.w[j] : 0u;
  }
#pragma unroll
  for (int i = 0; i < RT_PER; i++) {
    int64_t j = p0 + tid + i * RT_BS;
    int32_t x = xr[i];
    pr[i] = x >= 0 ? gptr[c[x]] + off[x] + 1 + (j - g.rp[x]) : 0;
    yr[i] = x >= 0 ? c[yr[i]] : 0;
  }
#pragma unroll
  for (int i = 0; i < RT_PER; i++)
    if (xr[i] >= 0) rec[pr[i]] = ((uint64_t)(uint32_t)yr[i] << 32) | wr[i];
}

// ---- rows of at most CAP records: one thread each ---------------------------
// The sorted distinct (column, weight) list is held in registers (every
// access uses a compile-time index), built by insertion with equal columns
// merged; records are loaded EB at a time.  Returns the row's member count.
template <int CAP>
__device__ __forceinline__ int reduce_row_regs(const uint64_t* __restrict__ rec_in, uint64_t* __restrict__ rec_out,
                                               const int64_t* __restrict__ gptr, int64_t* __restrict__ cnt,
                                               int64_t* __restrict__ self_out, int32_t* __restrict__ size_out,
                                               int32_t a) {
  int64_t self = 0;
  int32_t sz = 0;
  int mem = 0;
  int cntd = 0;
  int32_t kb[CAP];
  uint32_t kw[CAP];
#pragma unroll
  for (int q = 0; q < CAP; q++) {
    kb[q] = INT32_MAX;
    kw[q] = 0;
  }
  constexpr int EB = 8;
  int64_t g0 = gptr[a], g1 = gptr[a + 1];
#pragma unroll 1
  for (int64_t p = g0; p < g1; p += EB) {
    uint64_t r[EB];
#pragma unroll
    for (int q = 0; q < EB; q++) r[q] = p + q < g1 ? rec_in[p + q] : ~0ull;
#pragma unroll
    for (int q = 0; q < EB; q++) {
      if (r[q] == ~0ull) continue;
      if (r[q] & REC_MEMBER) {
        mem++;
        sz += (int32_t)((r[q] >> 32) & 0x7fffffffu);
        self += (uint32_t)r[q];
        continue;
      }
      int32_t b = (int32_t)(r[q] >> 32);
      uint32_t wv = (uint32_t)r[q];
      if (b == a) {
        self += wv;
        continue;
      }
      bool found = false;
      int ins = 0;
#pragma unroll
      for (int s = 0; s < CAP; s++) {
        bool hit = kb[s] == b;
        kw[s] += hit ? wv : 0u;   // sums stay below 2^31
        found |= hit;
        ins += kb[s] < b ? 1 : 0;
      }
      if (!found) {
#pragma unroll
        for (int s = CAP - 1; s >= 0; s--) {
          if (s > ins) {
            kb[s] = kb[s - 1];
            kw[s] = kw[s - 1];
          } else if (s == ins) {
            kb[s] = b;
            kw[s] = wv;
          }
        }
        cntd++;
      }
    }
  }
  // every record of the row is in registers: its slots may be overwritten
#pragma unroll
  for (int q = 0; q < CAP; q++)
    if (q < cntd) rec_out[g0 + q] = ((uint64_t)(uint32_t)kb[q] << 32) | kw[q];
  cnt[a] = cntd;
  self_out[a] = self;
  size_out[a] = sz;
  return mem;
}

// RPT rows per thread: 4 when the rows fill the chip many times over (fewer
// blocks on the class chains), fewer when there are few.  Rows above
// SMALL_CAP records go to their class's list.
template <int RPT>
__global__ void __launch_bounds__(SMALL_BS)
    k_contract_small(uint64_t* __restrict__ rec, const int64_t* __restrict__ gptr, int64_t* __restrict__ cnt,
                     int64_t* __restrict__ self_out, int32_t* __restrict__ size_out, int64_t n_c,
                     int32_t* __restrict__ r32list, int32_t* __restrict__ midlist,
                     int32_t* __restrict__ blocklist, int32_t* __restrict__ hugelist,
                     unsigned long long* info, TileScan ts, int lane_cap, int wave_cap) {
  __shared__ unsigned long long stmp[SMALL_BS / WAVE];
  __shared__ int64_t sbase[4];
  __shared__ int32_t smx[SMALL_BS / WAVE];
  int tid = threadIdx.x;
  int64_t base = (int64_t)blockIdx.x * SMALL_BS * RPT;
  uint32_t r32m = 0, midm = 0, blkm = 0, hugem = 0;
  int nr32 = 0, nmid = 0, nblk = 0, nhuge = 0;
  int32_t mx = 0;
  for (int r = 0; r < RPT; r++) {
    int64_t a = base + r * SMALL_BS + tid;
    if (a >= n_c) break;
    int64_t E = gptr[a + 1] - gptr[a];
    if (E > SMALL_CAP) {
      cnt[a] = 0;   // until its class's kernel writes it
      if (E <= lane_cap) {
        r32m |= 1u << r;
        nr32++;
      } else if (E <= wave_cap) {
        midm |= 1u << r;
        nmid++;
      } else if (E <= BLOCK_CAP) {
        blkm |= 1u << r;
        nblk++;
      } else {
        hugem |= 1u << r;
        nhuge++;
        self_out[a] = 0;   // the huge-row kernels add into these
        size_out[a] = 0;
      }
      continue;
    }
    int mem = reduce_row_regs<SMALL_CAP>(rec, rec, gptr, cnt, self_out, size_out, (int32_t)a);
    mx = mem > mx ? mem : mx;
  }
  mx = wave_max(mx);
  if (lane_id() == 0) smx[tid / WAVE] = mx;
  __syncthreads();
  if (tid == 0) {
    int32_t m2 = 0;
    for (int w = 0; w < SMALL_BS / WAVE; w++) m2 = smx[w] > m2 ? smx[w] : m2;
    // most blocks see the maximum already published and skip the atomic
    if ((unsigned long long)m2 >
        __hip_atomic_load(&info[I_MAXCL], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(&info[I_MAXCL], (unsigned long long)m2);
  }
  // the four class lists: per-thread counts (at most RPT each) packed
  // in 16-bit fields, one block scan, then one look-back chain per class
  // run by lanes 0-3
  unsigned long long mine = (unsigned long long)nr32 | ((unsigned long long)nmid << 16) |
                            ((unsigned long long)nblk << 32) | ((unsigned long long)nhuge << 48);
  unsigned long long tot;
  unsigned long long incl = block_incl_scan<unsigned long long, SMALL_BS, false>(mine, stmp, &tot);
  unsigned long long excl = incl - mine;
  // wavefront w runs the chains of classes w and w + 2
  static_assert(SMALL_BS == 2 * WAVE, "two wavefronts share the four chains");
  for (int q = 0; q < 2; q++) {
    int cls = tid / WAVE + 2 * q;
    int slot = cls == 0 ? I_R32 : cls == 1 ? I_MID : cls == 2 ? I_BLOCK : I_HUGE;
    uint64_t cnt_c = (tot >> (16 * cls)) & 0xffffull;
    TileScan t = ts;
    t.state += (int64_t)cls * gridDim.x;
    uint64_t ex = lb_exclusive_wave(t, blockIdx.x, cnt_c);
    if (lane_id() == 0) {
      sbase[cls] = (int64_t)ex;
      if (blockIdx.x == gridDim.x - 1) info[slot] = ex + cnt_c;
    }
  }
  __syncthreads();
  int64_t p0 = sbase[0] + (int64_t)(excl & 0xffff);
  int64_t p1 = sbase[1] + (int64_t)((excl >> 16) & 0xffff);
  int64_t p2 = sbase[2] + (int64_t)((excl >> 32) & 0xffff);
  int64_t p3 = sbase[3] + (int64_t)((excl >> 48) & 0xffff);
  for (int r = 0; r < RPT; r++) {
    int32_t a = (int32_t)(base + r * SMALL_BS + tid);
    if (r32m >> r & 1u) r32list[p0++] = a;
    if (midm >> r & 1u) midlist[p1++] = a;
    if (blkm >> r & 1u) blocklist[p2++] = a;
    if (hugem >> r & 1u) hugelist[p3++] = a;
  }
}

// ---- listed rows of at most REG32_CAP records: RG_L lanes each --------------
// Four rows per wavefront, each with RG_L lanes and a table of RG_T slots in
// LDS: the hashed reduction below (same table, compaction and ranks), run
// by lane groups.  One thread per row would insert every record into a
// sorted register list, a chain of dependent steps per record.
constexpr int RG_L = 16;
constexpr int RG_N = WAVE / RG_L;
constexpr int RG_T = 2 * REG32_CAP;   // >= 2 E: a free slot always exists
static_assert(RG_T % RG_L == 0 && RG_T == 64, "the hash below takes 6 bits");

template <typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = RG_L / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__global__ void __launch_bounds__(WAVE)
    k_contract_reg32(uint64_t* __restrict__ rec, const int64_t* __restrict__ gptr,
                     const int32_t* __restrict__ rows, int64_t nrows, const unsigned long long* nrows_dev,
                     int64_t* __restrict__ cnt, int64_t* __restrict__ self_out, int32_t* __restrict__ size_out,
                     unsigned long long* info) {
  __shared__ uint64_t tab[RG_N * RG_T];
  int l = lane_id(), gi = l / RG_L, gl = l % RG_L;
  uint64_t* t = tab + gi * RG_T;
  // (with nrows_dev the count is read here and the grid strides over it)
  int64_t nr = nrows_dev ? (int64_t)*nrows_dev : nrows;
  int mx = 0;
  for (int64_t base = (int64_t)blockIdx.x * RG_N; base < nr; base += (int64_t)gridDim.x * RG_N) {
    int64_t r = base + gi;
    bool has = r < nr;
    int32_t a = has ? rows[r] : 0;
    int64_t g0 = has ? gptr[a] : 0, g1 = has ? gptr[a + 1] : 0;
#pragma unroll
    for (int i = gl; i < RG_T; i += RG_L) t[i] = KEY_INF;
    __syncthreads();
    uint64_t self = 0;
    int32_t sz = 0, mem = 0;
    for (int64_t p = g0 + gl; p < g1; p += RG_L) {
      uint64_t v = rec[p];
      uint32_t b = (uint32_t)(v >> 32);
      if (v & REC_MEMBER) {
        mem++;
        sz += (int32_t)(b & 0x7fffffffu);
        self += (uint32_t)v;
      } else if ((int32_t)b == a) {
        self += (uint32_t)v;
      } else {
        uint32_t h = (b * 0x9E3779B1u) >> 26;
        while (true) {
          unsigned long long old = atomicCAS((unsigned long long*)&t[h], (unsigned long long)KEY_INF,
                                             (unsigned long long)v);
          if (old == KEY_INF) break;
          if ((uint32_t)(old >> 32) == b) {
            atomicAdd((unsigned long long*)&t[h], (unsigned long long)(uint32_t)v);
            break;
          }
          h = (h + 1) & (uint32_t)(RG_T - 1);
        }
      }
    }
    self = group_sum(self);
    sz = group_sum(sz);
    mem = group_sum(mem);
    __syncthreads();
    // compaction in place, as in the wavefront reduction (each write lands
    // at or below the writer's own slot of the step)
    int D = 0;
#pragma unroll
    for (int q = 0; q < RG_T; q += RG_L) {
      uint64_t x = t[q + gl];
      bool occ = x != KEY_INF;
      uint32_t gb = (uint32_t)(__ballot(occ) >> (gi * RG_L)) & ((1u << RG_L) - 1);
      if (occ) t[D + __popc(gb & ((1u << gl) - 1))] = x;
      D += __popc(gb);
    }
    __syncthreads();
    for (int i = gl; i < D; i += RG_L) {
      uint64_t x = t[i];
      uint32_t b = (uint32_t)(x >> 32);
      int rank = 0;
      for (int j = 0; j < D; j++) rank += (uint32_t)(t[j] >> 32) < b ? 1 : 0;
      rec[g0 + rank] = x;
    }
    if (has && gl == 0) {
      cnt[a] = D;
      self_out[a] = (int64_t)self;
      size_out[a] = sz;
    }
    mx = mem > mx ? mem : mx;
    __syncthreads();   // the next rows reuse the tables
  }
  mx = wave_max(mx);
  if (lane_id() == 0 && (unsigned long long)mx >
      __hip_atomic_load(&info[I_MAXCL], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    atomicMax(&info[I_MAXCL], (unsigned long long)mx);
}

// ---- a row of at most WAVE_CAP / 2 records, one wavefront ------------------
// The row's entries are summed per coarse column in an LDS hash table of
// T >= 2 E slots (open addressing; a slot holds column << 32 | weight sum,
// the sum below 2^31 by the weight bound), the occupied slots are compacted
// to the table's front, and each distinct column's place in the output is
// its rank among them: a row's distinct columns are few (about six on
// triangle meshes) against its records, so this replaces a sort of all the
// records with one of the distinct columns.  Returns the member count.
__device__ __forceinline__ int reduce_row_hashed(uint64_t* __restrict__ rec, int64_t g0, int64_t g1, int32_t a,
                                                 uint64_t* ent, int64_t* __restrict__ cnt,
                                                 int64_t* __restrict__ self_out, int32_t* __restrict__ size_out) {
  int l = lane_id();
  int E = (int)(g1 - g0);
  int lg = 6;
  while ((1 << lg) < 2 * E) lg++;
  int T = 1 << lg;   // a multiple of WAVE, at most WAVE_CAP
  for (int i = l; i < T; i += WAVE) ent[i] = KEY_INF;
  __syncthreads();
  uint64_t self = 0;
  int32_t sz = 0, mem = 0;
  for (int64_t p = g0 + l; p < g1; p += WAVE) {
    uint64_t v = rec[p];
    uint32_t b = (uint32_t)(v >> 32);
    if (v & REC_MEMBER) {
      mem++;
      sz += (int32_t)(b & 0x7fffffffu);
      self += (uint32_t)v;
    } else if ((int32_t)b == a) {
      self += (uint32_t)v;
    } else {
      // T > E >= distinct columns: a free slot always exists
      uint32_t h = (b * 0x9E3779B1u) >> (32 - lg);
      while (true) {
        unsigned long long old = atomicCAS((unsigned long long*)&ent[h], (unsigned long long)KEY_INF,
                                           (unsigned long long)v);
        if (old == KEY_INF) break;
        if ((uint32_t)(old >> 32) == b) {
          atomicAdd((unsigned long long*)&ent[h], (unsigned long long)(uint32_t)v);
          break;
        }
        h = (h + 1) & (uint32_t)(T - 1);
      }
    }
  }
  self = wave_sum(self);
  sz = wave_sum(sz);
  mem = wave_sum(mem);
  __syncthreads();
  // compaction in place: a write lands below the slots still to be read
  // (every lane reads slot q + l before any lane writes in that step)
  int D = 0;
  for (int q = 0; q < T; q += WAVE) {
    uint64_t x = ent[q + l];
    bool occ = x != KEY_INF;
    uint64_t bm = __ballot(occ);
    if (occ) ent[D + __popcll(bm & lanemask_lt())] = x;
    D += __popcll(bm);
  }
  __syncthreads();
  if (D <= WAVE) {
    if (l < D) {
      uint64_t x = ent[l];
      uint32_t b = (uint32_t)(x >> 32);
      int rank = 0;
      for (int j = 0; j < D; j++) rank += (uint32_t)(ent[j] >> 32) < b ? 1 : 0;
      rec[g0 + rank] = x;
    }
  } else {
    // more distinct columns than lanes: sort them (columns are distinct)
    int P2 = 1;
    while (P2 < D) P2 <<= 1;
    for (int i = D + l; i < P2; i += WAVE) ent[i] = KEY_INF;
    __syncthreads();
    for (int k = 2; k <= P2; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int p = l; p < P2 / 2; p += WAVE) {
          int i = 2 * j * (p / j) + (p % j);
          int r = i + j;
          bool asc = (i & k) == 0;
          uint64_t x = ent[i], y = ent[r];
          if (asc ? (y < x) : (x < y)) {
            ent[i] = y;
            ent[r] = x;
          }
        }
        __syncthreads();
      }
    }
    for (int i = l; i < D; i += WAVE) rec[g0 + i] = ent[i];
  }
  if (l == 0) {
    cnt[a] = D;
    self_out[a] = (int64_t)self;
    size_out[a] = sz;
  }
  __syncthreads();   // the next row reuses the table
  return mem;
}

// ---- listed rows of at most CAP records: one TB-thread block each -----------
// (one wavefront: rows of at most CAP / 2 records take the hashed reduction)
template <int TB, int CAP>
__global__ void __launch_bounds__(TB)
    k_contract_row(uint64_t* __restrict__ rec, const int64_t* __restrict__ gptr,
                   const int32_t* __restrict__ rowlist, const unsigned long long* nrows_dev,
                   int64_t* __restrict__ cnt, int64_t* __restrict__ self_out, int32_t* __restrict__ size_out,
                   unsigned long long* info) {
  __shared__ uint64_t ent[CAP];
  __shared__ int lcnt;
  __shared__ unsigned long long lself;
  __shared__ int lsize, lmem;
  __shared__ int32_t stmp[TB / WAVE];
  int tid = threadIdx.x;
  // one row per block, or (nrows_dev: the count is read here) the blocks
  // stride over the rows
  int64_t nr = nrows_dev ? (int64_t)*nrows_dev : (int64_t)gridDim.x;
  for (int64_t r = blockIdx.x; r < nr; r += gridDim.x) {
    int32_t a = rowlist[r];
    if constexpr (TB == WAVE) {
      int64_t h0 = gptr[a], h1 = gptr[a + 1];
      if (h1 - h0 <= CAP / 2) {   // (uniform over the block)
        int mem = reduce_row_hashed(rec, h0, h1, a, ent, cnt, self_out, size_out);
        if (tid == 0 && (unsigned long long)mem >
            __hip_atomic_load(&info[I_MAXCL], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
          atomicMax(&info[I_MAXCL], (unsigned long long)mem);
        continue;
      }
    }
    if (tid == 0) {
      lcnt = 0;
      lself = 0;
      lsize = 0;
      lmem = 0;
    }
    __syncthreads();
    int64_t g0 = gptr[a], g1 = gptr[a + 1];
    int64_t self = 0;
    int32_t sz = 0, mem = 0;
    for (int64_t p = g0 + tid; p < g1; p += TB) {
      uint64_t v = rec[p];
      if (v & REC_MEMBER) {
        mem++;
        sz += (int32_t)((v >> 32) & 0x7fffffffu);
        self += (uint32_t)v;
      } else if ((int32_t)(v >> 32) == a) {
        self += (uint32_t)v;
      } else {
        ent[atomicAdd(&lcnt, 1)] = v;
      }
    }
    self = wave_sum(self);
    sz = wave_sum(sz);
    mem = wave_sum(mem);
    if (lane_id() == 0) {
      atomicAdd(&lself, (unsigned long long)self);
      atomicAdd(&lsize, sz);
      atomicAdd(&lmem, mem);
    }
    __syncthreads();
    int K = lcnt;
    int P2 = 1;
    while (P2 < K) P2 <<= 1;
    for (int i = K + tid; i < P2; i += TB) ent[i] = KEY_INF;
    __syncthreads();
    for (int k = 2; k <= P2; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int p = tid; p < P2 / 2; p += TB) {
          int i = 2 * j * (p / j) + (p % j);
          int l = i + j;
          bool asc = (i & k) == 0;
          uint64_t x = ent[i], y = ent[l];
          if (asc ? (y < x) : (x < y)) {
            ent[i] = y;
            ent[l] = x;
          }
        }
        __syncthreads();
      }
    }
    // distinct columns in ascending order, weights summed, over the row's
    // own records (all of them are in LDS now)
    int carry = 0;
    for (int base = 0; base < K; base += TB) {
      int i = base + tid;
      bool head = false;
      uint32_t b = 0;
      if (i < K) {
        b = (uint32_t)(ent[i] >> 32);
        head = (i == 0) || ((uint32_t)(ent[i - 1] >> 32) != b);
      }
      int32_t tot;
      int32_t inc = block_incl_scan<int32_t, TB, false>(head ? 1 : 0, stmp, &tot);
      if (head) {
        uint64_t sum = 0;
        for (int q = i; q < K && (uint32_t)(ent[q] >> 32) == b; q++) sum += (uint32_t)ent[q];
        rec[g0 + carry + inc - 1] = ((uint64_t)b << 32) | sum;
      }
      carry += tot;
    }
    if (tid == 0) {
      cnt[a] = carry;
      self_out[a] = (int64_t)lself;
      size_out[a] = lsize;
      if ((unsigned long long)lmem >
          __hip_atomic_load(&info[I_MAXCL], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(&info[I_MAXCL], (unsigned long long)lmem);
    }
    __syncthreads();   // the next row reuses the block's LDS
  }
}

// ---- rows with more than BLOCK_CAP gathered entries ------------------------
struct KW {
  uint64_t key, w;
};
struct LessKW {
  __device__ __forceinline__ bool operator()(const KW& a, const KW& b) const { return a.key < b.key; }
};

// ---- rows of more than BLOCK_CAP records ("huge") ---------------------------
// hoff[h] = records of the listed huge rows before h (hoff[H] = all).  With
// H_dev (the count in device memory, launch bound H) rows past that count
// have no records, and a count above the bound sets *over and leaves every
// row empty.  At most 64 rows: one wavefront takes the prefix.
__global__ void k_huge_prefix_wave(const int32_t* __restrict__ hugelist, int64_t H,
                                   const int64_t* __restrict__ gptr, int64_t* __restrict__ hoff,
                                   const unsigned long long* H_dev, unsigned long long* over) {
  int h = threadIdx.x;
  int64_t Hn = H;
  if (H_dev) {
    Hn = (int64_t)*H_dev;
    if (Hn > H) {
      if (h == 0) *over = 1;
      Hn = 0;
    }
  }
  int64_t v = 0;
  if (h < Hn) {
    int32_t a = hugelist[h];
    v = gptr[a + 1] - gptr[a];
  }
  int64_t incl = wave_incl_sum(v);
  if (h < H) hoff[h] = incl - v;
  if (h == WAVE - 1) hoff[H] = incl;
}

// more rows (host-known count): per-row record counts, scanned afterwards
__global__ void k_huge_count(const int32_t* __restrict__ hugelist, int64_t H, const int64_t* __restrict__ gptr,
                             int64_t* __restrict__ hcount) {
  int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h < H) {
    int32_t a = hugelist[h];
    hcount[h] = gptr[a + 1] - gptr[a];
  }
}

// Record q (0 <= q < hoff[H]) of the huge rows in list order belongs to row
// srow's h; member records and intra entries add to the row's size, member
// count and self-loop (lanes of one row summed in registers, then in LDS: a
// tile of HD <= BLOCK_CAP records meets at most two rows, since every huge
// row has more), cross entries go to `cross(h, a, b, w)`.
constexpr int HT = 4096;
constexpr int HT_BS = 256;
static_assert(HT <= BLOCK_CAP, "a tile of records must meet at most two huge rows");

struct HugeSums {
  unsigned long long self[2];
  int32_t size[2];
  int32_t mem[2];
};

template <int HD, typename Cross>
__device__ __forceinline__ void huge_tile(const uint64_t* __restrict__ rec, const int64_t* __restrict__ gptr,
                                          const int32_t* __restrict__ hugelist, const int64_t* __restrict__ hoff,
                                          int64_t H, int64_t q0, int64_t total, int64_t* self_out,
                                          int32_t* size_out, int64_t* hmem, HugeSums& S, int32_t* srow,
                                          int64_t* sh, int32_t* stmp, Cross cross) {
  lbs_tile<HD, HT_BS>(hoff, H, q0, srow, sh, stmp);
  int tid = threadIdx.x;
  if (tid < 2) {
    S.self[tid] = 0;
    S.size[tid] = 0;
    S.mem[tid] = 0;
  }
  int32_t h0 = srow[0];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < HD / HT_BS; r++) {
    int k = tid + r * HT_BS;
    int64_t q = q0 + k;
    int32_t h = -1;
    int64_t self = 0;
    int32_t sz = 0, mem = 0;
    if (q < total) {
      h = srow[Lbs<HD, HT_BS>::at(k)];
      int32_t a = hugelist[h];
      uint64_t v = rec[gptr[a] + (q - hoff[h])];
      if (v & REC_MEMBER) {
        mem = 1;
        sz = (int32_t)((v >> 32) & 0x7fffffffu);
        self = (uint32_t)v;
      } else if ((int32_t)(v >> 32) == a) {
        self = (uint32_t)v;
      } else {
        cross(r, h, (int32_t)(v >> 32), (uint32_t)v);
      }
    }
    bool head;
    int end;
    uint64_t heads;
    wave_runs(h, head, end, heads);
    int64_t si = wave_incl_sum(self);
    int32_t zi = wave_incl_sum(sz), mi = wave_incl_sum(mem);
    int64_t se = __shfl(si, end - 1);
    int32_t ze = __shfl(zi, end - 1), me = __shfl(mi, end - 1);
    if (head && h >= 0) {
      if (se - si + self) atomicAdd(&S.self[h - h0], (unsigned long long)(se - si + self));
      if (ze - zi + sz) atomicAdd(&S.size[h - h0], ze - zi + sz);
      if (me - mi + mem) atomicAdd(&S.mem[h - h0], me - mi + mem);
    }
  }
  __syncthreads();
  if (tid < 2 && h0 + tid < H) {
    int32_t a = hugelist[h0 + tid];
    if (S.self[tid]) atomicAdd((unsigned long long*)&self_out[a], S.self[tid]);
    if (S.size[tid]) atomicAdd(&size_out[a], S.size[tid]);
    if (S.mem[tid]) atomicAdd((unsigned long long*)&hmem[h0 + tid], (unsigned long long)S.mem[tid]);
  }
}

// Dense path for few huge rows: row h's cross weights accumulate in
// dense[h * ncp + (b - base[h])] (u32; a row's total stays below 2^31), then
// a compaction in ascending b emits the row.  base is null (0) for one graph;
// in a batch it is the first coarse node of the row's graph, whose coarse
// range (at most ncp wide) holds every column of the row.  Tiles of HD
// records: 4096 on large levels, 1024 (4 per thread) on small ones.
constexpr int64_t HD_SMALL_NNZ = 4000000;   // levels up to this many entries use 1024-record tiles

template <int HD>
__global__ void __launch_bounds__(HT_BS)
    k_huge_dense(const uint64_t* __restrict__ rec, const int64_t* __restrict__ gptr,
                 const int32_t* __restrict__ hugelist, const int64_t* __restrict__ hoff, int64_t H,
                 int64_t* self_out, int32_t* size_out, int64_t* hmem, uint32_t* __restrict__ dense, int64_t ncp,
                 const int32_t* __restrict__ base, unsigned long long* bad) {
  __shared__ int32_t srow[Lbs<HD, HT_BS>::SIZE];
  __shared__ int64_t sh[2];
  __shared__ int32_t stmp[HT_BS / WAVE];
  __shared__ HugeSums S;
  static_assert(HD <= HT && HD % HT_BS == 0, "a dense tile meets at most two huge rows");
  int64_t q0 = (int64_t)blockIdx.x * HD;
  int64_t total = hoff[H];
  if (q0 >= total) return;
  huge_tile<HD>(rec, gptr, hugelist, hoff, H, q0, total, self_out, size_out, hmem, S, srow, sh, stmp,
                [&](int, int32_t h, int32_t b, uint32_t w) {
                  int64_t rel = (int64_t)b - (base ? base[h] : 0);
                  if ((uint64_t)rel < (uint64_t)ncp) atomicAdd(&dense[(int64_t)h * ncp + rel], w);
                  else *bad = 1;
                });
}

// Sort path: every cross record of the huge rows as ((h << 32) | b, w),
// compacted in tile order by a decoupled look-back (tiles past the records
// take part with nothing, so the chain's last tile stores the total).
__global__ void __launch_bounds__(HT_BS)
    k_huge_entries(const uint64_t* __restrict__ rec, const int64_t* __restrict__ gptr,
                   const int32_t* __restrict__ hugelist, const int64_t* __restrict__ hoff, int64_t H,
                   int64_t* self_out, int32_t* size_out, int64_t* hmem, KW* __restrict__ out,
                   unsigned long long* gcnt, TileScan ts) {
  __shared__ int32_t srow[Lbs<HT, HT_BS>::SIZE];
  __shared__ int64_t sh[2];
  __shared__ int32_t stmp[HT_BS / WAVE];
  __shared__ unsigned long long sbase;
  __shared__ HugeSums S;
  int64_t q0 = (int64_t)blockIdx.x * HT;
  int64_t total = hoff[H];
  if (q0 >= total) {
    block_reserve_lb<HT_BS>(ts, blockIdx.x, blockIdx.x == gridDim.x - 1, 0, nullptr, gcnt, &sbase, stmp);
    return;
  }
  uint32_t cross = 0;
  int ncross = 0;
  uint64_t keyv[HT / HT_BS];
  uint32_t wv[HT / HT_BS];
#pragma unroll
  for (int r = 0; r < HT / HT_BS; r++) {
    keyv[r] = 0;
    wv[r] = 0;
  }
  huge_tile<HT>(rec, gptr, hugelist, hoff, H, q0, total, self_out, size_out, hmem, S, srow, sh, stmp,
                [&](int r, int32_t h, int32_t b, uint32_t w) {
                  cross |= 1u << r;
                  ncross++;
                  keyv[r] = ((uint64_t)(uint32_t)h << 32) | (uint32_t)b;
                  wv[r] = w;
                });
  int64_t pos = block_reserve_lb<HT_BS>(ts, blockIdx.x, blockIdx.x == gridDim.x - 1, ncross, nullptr,
                                       gcnt, &sbase, stmp);
#pragma unroll
  for (int r = 0; r < HT / HT_BS; r++)
    if (cross >> r & 1u) out[pos++] = KW{keyv[r], (uint64_t)wv[r]};
}

// Compaction of the dense rows: tile t of row h covers b in
// [t * DC_T, (t + 1) * DC_T), 8 consecutive b per thread; each row is its
// own look-back chain, whose last tile writes the row's entry count.
constexpr int DC_BS = 256;
constexpr int DC_PER = 8;
constexpr int DC_T = DC_BS * DC_PER;

__global__ void __launch_bounds__(DC_BS)
    k_dense_compact(const uint32_t* __restrict__ dense, int64_t ncp, int64_t n_c, int64_t tpr,
                    const int32_t* __restrict__ hugelist, const int64_t* __restrict__ gptr,
                    uint64_t* __restrict__ temp, int64_t* cnt, TileScan ts,
                    const int32_t* __restrict__ base, const unsigned long long* H_dev, int64_t H,
                    const int64_t* __restrict__ hmem, unsigned long long* info) {
  __shared__ int stmp[DC_BS / WAVE];
  __shared__ unsigned long long sbase;
  int64_t h = blockIdx.x / tpr, t = blockIdx.x % tpr;
  if (H_dev) {
    // rows past the count in device memory (or all, above the bound H)
    unsigned long long Hn = *H_dev;
    if (Hn > (unsigned long long)H || h >= (int64_t)Hn) return;
  }
  int32_t a = hugelist[h];
  if (t == 0 && threadIdx.x == 0) atomicMax(&info[I_MAXCL], (unsigned long long)hmem[h]);
  int64_t cb = base ? base[h] : 0;   // column of the window's first slot
  n_c -= cb;                          // slots past the last coarse node stay unused
  int64_t b0 = t * DC_T + (int64_t)threadIdx.x * DC_PER;
  const uint4* src = (const uint4*)(dense + h * ncp + b0);
  uint4 v0 = src[0], v1 = src[1];
  uint32_t v[DC_PER] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
  int my = 0;
#pragma unroll
  for (int q = 0; q < DC_PER; q++) my += (v[q] != 0 && b0 + q < n_c) ? 1 : 0;
  TileScan tr = ts;
  tr.state += h * tpr;
  int64_t pos = block_reserve_lb<DC_BS>(tr, t, t == tpr - 1, my, nullptr,
                                        (unsigned long long*)&cnt[a], &sbase, stmp);
  uint64_t* o = temp + gptr[a];
#pragma unroll
  for (int q = 0; q < DC_PER; q++)
    if (v[q] != 0 && b0 + q < n_c) o[pos++] = ((uint64_t)(cb + b0 + q) << 32) | v[q];
}

// first coarse node of the graph holding huge row h (batches)
__global__ void k_huge_base(const int32_t* __restrict__ hugelist, int64_t H, const int64_t* __restrict__ coff,
                            int64_t G, int32_t* __restrict__ base) {
  int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= H) return;
  int64_t a = hugelist[h], lo = 0, hi = G - 1;
  while (lo < hi) {   // the last graph whose range starts at or before a
    int64_t mid = (lo + hi + 1) >> 1;
    if (coff[mid] <= a) lo = mid;
    else hi = mid - 1;
  }
  base[h] = (int32_t)coff[lo];
}

__global__ void k_head_flags(const KW* __restrict__ s, int64_t G, int32_t* __restrict__ flag,
                             uint64_t* __restrict__ wcol) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < G) {
    flag[i] = (i == 0 || s[i].key != s[i - 1].key) ? 1 : 0;
    wcol[i] = s[i].w;
  }
}

__global__ void k_head_index(const KW* __restrict__ s, int64_t G, const int32_t* __restrict__ pos,
                             int32_t* __restrict__ hstart) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < G && (i == 0 || s[i].key != s[i - 1].key)) hstart[pos[i]] = (int32_t)i;
}

// one (row, column) run per head: its weight sum from the scanned weights;
// its slot is the head's rank among the heads of its row
__global__ void k_huge_reduce(const KW* __restrict__ s, int64_t G, const int32_t* __restrict__ pos,
                              const int32_t* __restrict__ hstart, const uint64_t* __restrict__ wx,
                              const int32_t* __restrict__ hugelist, const int32_t* __restrict__ rowfirst,
                              const int64_t* __restrict__ gptr, uint64_t* __restrict__ temp) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G) return;
  if (!(i == 0 || s[i].key != s[i - 1].key)) return;
  int32_t r = pos[i];
  int64_t e = (r + 1 < pos[G]) ? hstart[r + 1] : G;
  uint64_t key = s[i].key;
  int32_t h = (int32_t)(key >> 32);
  uint32_t b = (uint32_t)key;
  uint64_t sum = wx[e] - wx[i];
  int32_t a = hugelist[h];
  temp[gptr[a] + (r - rowfirst[h])] = ((uint64_t)b << 32) | sum;
}

// rowfirst[h] = rank of huge row h's first head, hcount[h] = its heads
__global__ void k_huge_rowfirst(const KW* __restrict__ s, int64_t G, const int32_t* __restrict__ pos,
                                int32_t* __restrict__ rowfirst, int32_t* __restrict__ rowlast) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G) return;
  int32_t h = (int32_t)(s[i].key >> 32);
  if (i == 0 || (int32_t)(s[i - 1].key >> 32) != h) rowfirst[h] = pos[i];
  if (i == G - 1 || (int32_t)(s[i + 1].key >> 32) != h) rowlast[h] = pos[i + 1] - 1;
}

__global__ void k_huge_counts(const int32_t* __restrict__ hugelist, int64_t H,
                              const int32_t* __restrict__ rowfirst, const int32_t* __restrict__ rowlast,
                              int64_t* __restrict__ cnt, const int64_t* __restrict__ hmem,
                              unsigned long long* info) {
  int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h < H) {
    cnt[hugelist[h]] = rowlast[h] < 0 ? 0 : (int64_t)(rowlast[h] - rowfirst[h] + 1);
    atomicMax(&info[I_MAXCL], (unsigned long long)hmem[h]);
  }
}

__global__ void k_fill_i32(int32_t* __restrict__ a, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// ---- packing: tiles of output positions mapped to coarse rows -----------
constexpr int PACK_T = 1024;
constexpr int PACK_BS = 256;

__global__ void __launch_bounds__(PACK_BS)
    k_pack(const int64_t* __restrict__ rpc, int64_t n_c, const int64_t* __restrict__ gptr,
           const uint64_t* __restrict__ temp, int32_t* __restrict__ col_c, int32_t* __restrict__ w_c) {
  __shared__ int32_t srow[Lbs<PACK_T, PACK_BS>::SIZE];
  __shared__ int64_t sh[2];
  __shared__ int32_t stmp[PACK_BS / WAVE];
  int64_t p0 = (int64_t)blockIdx.x * PACK_T;
  int64_t total = rpc[n_c];
  if (p0 >= total) return;   // (a grid sized by a bound; uniform over the block)
  lbs_tile<PACK_T, PACK_BS>(rpc, n_c, p0, srow, sh, stmp);
  for (int i = 0; i < PACK_T / PACK_BS; i++) {
    int k = threadIdx.x + i * PACK_BS;
    int64_t p = p0 + k;
    if (p >= total) break;
    int32_t a = srow[Lbs<PACK_T, PACK_BS>::at(k)];
    uint64_t v = temp[gptr[a] + (p - rpc[a])];
    col_c[p] = (int32_t)(v >> 32);
    w_c[p] = (int32_t)(uint32_t)v;
  }
}

// Rows of the register, wavefront and block classes.  With dev the class
// counts stay in device memory (the kernels read them; grids cover a bound),
// otherwise hinfo holds them.
// Classes whose bit is clear in `launch` (dev only) are not launched: the
// caller checks their counts once read.
static int contract_classes(spc_ctx* ctx, int64_t n_c, spc_graph_out* out, LevelWork& W, bool dev,
                            int launch = 7) {
  hipStream_t st = ctx->stream;
  int64_t* hinfo = ctx->h_pinned;
  unsigned long long* info = W.info;
  int64_t* self_out = (int64_t*)out->self_w;
  int64_t nr32 = dev ? 0 : hinfo[I_R32], nmid = dev ? 0 : hinfo[I_MID], nblk = dev ? 0 : hinfo[I_BLOCK];
  int64_t cap = (int64_t)ctx->num_cus * 8;
  if (!(launch & 1)) nr32 = 0;
  if (!(launch & 2)) nmid = 0;
  if (!(launch & 4)) nblk = 0;
  if ((dev && (launch & 1)) || nr32 > 0) {
    TimedScope ts(ctx, "contract_reg32", (double)nr32);
    int64_t gr = dev ? std::min((int64_t)grid_for(n_c, RG_N), cap * 4) : (int64_t)grid_for(nr32, RG_N);
    hipLaunchKernelGGL(k_contract_reg32, dim3((unsigned)gr), dim3(WAVE), 0, st, W.temp, W.gptr, W.r32list,
                       nr32, dev ? &info[I_R32] : nullptr, W.cnt, self_out, out->size, info);
    SPC_LAUNCH_CHECK(ctx, "contract reg32");
  }
  if ((dev && (launch & 2)) || nmid > 0) {
    TimedScope ts(ctx, "contract_wave_rows", (double)nmid);
    int64_t gr = dev ? std::min(n_c, cap * 4) : nmid;
    hipLaunchKernelGGL((k_contract_row<WAVE, WAVE_CAP>), dim3((unsigned)gr), dim3(WAVE), 0, st, W.temp, W.gptr,
                       W.midlist, dev ? &info[I_MID] : nullptr, W.cnt, self_out, out->size, info);
    SPC_LAUNCH_CHECK(ctx, "contract wave rows");
  }
  if ((dev && (launch & 4)) || nblk > 0) {
    TimedScope ts(ctx, "contract_block_rows", (double)nblk);
    int64_t gr = dev ? std::min(n_c, cap) : nblk;
    hipLaunchKernelGGL((k_contract_row<256, BLOCK_CAP>), dim3((unsigned)gr), dim3(256), 0, st, W.temp, W.gptr,
                       W.blocklist, dev ? &info[I_BLOCK] : nullptr, W.cnt, self_out, out->size, info);
    SPC_LAUNCH_CHECK(ctx, "contract block rows");
  }
  return SPC_OK;
}

// Rows with more than BLOCK_CAP records ("huge").  H rows, or with dev at
// most H (the count in device memory; above H the kernels do nothing and
// set info[I_HOVER]); dev always takes the dense path, which the caller
// checked fits for H rows.  total_bound: records of all rows together (the
// launches that cover the huge rows' records, whose total stays on the
// device, are sized by it).
static int contract_huge(spc_ctx* ctx, const LevelIn& g, int64_t n_c, spc_graph_out* out, LevelWork& W,
                         const Segments* seg, int64_t H, bool dev) {
  hipStream_t st = ctx->stream;
  int64_t* hinfo = ctx->h_pinned;
  unsigned long long* info = W.info;
  int64_t* self_out = (int64_t*)out->self_w;
  const unsigned long long* Hd = dev ? &info[I_HUGE] : nullptr;
  int64_t total_bound = g.nnz + g.n;
  int rc;
  TimedScope ts(ctx, "contract_huge", (double)H);
  int64_t* hoff = W.hmoff;
  int64_t* hmem = W.hmrs;   // members per huge row
  // few huge rows: dense accumulators over the coarse ids (they fit in the
  // gather buffers when H * ncp <= 2 nnz); in a batch, per huge row only the
  // coarse range of its own graph
  int64_t win = seg ? seg->wmax : n_c;
  int64_t ncp = (win + DC_T - 1) / DC_T * DC_T;
  bool dense_path = dev || (!ctx->force_huge_sort && H * ncp <= 2 * g.nnz);
  uint32_t* dense = (uint32_t*)W.gkeyA;
  launch_clear(ctx, nullptr, 0, dense_path ? (uint64_t*)dense : nullptr, dense_path ? (H * ncp + 1) / 2 : 0,
               nullptr, 0, (uint64_t*)hmem, H);
  if (H <= WAVE) {
    hipLaunchKernelGGL(k_huge_prefix_wave, dim3(1), dim3(WAVE), 0, st, W.hugelist, H, W.gptr, hoff, Hd,
                       &info[I_HOVER]);
  } else {
    hipLaunchKernelGGL(k_huge_count, dim3(grid_for(H, 256)), dim3(256), 0, st, W.hugelist, H, W.gptr, hoff);
    rc = exclusive_scan<int64_t>(ctx, hoff, hoff, H, (int64_t*)W.scan_partial);
    if (rc) return rc;
  }
  if (dense_path) {
    int32_t* base = nullptr;
    if (seg) {
      base = W.hmnode;
      hipLaunchKernelGGL(k_huge_base, dim3(grid_for(H, 256)), dim3(256), 0, st, W.hugelist, H, seg->coff,
                         seg->G, base);
    }
    bool big_tiles = ctx->tune.huge_tile == 4096 || (ctx->tune.huge_tile != 1024 && g.nnz > HD_SMALL_NNZ);
    if (big_tiles)
      hipLaunchKernelGGL(k_huge_dense<HT>, dim3(grid_for(total_bound, HT)), dim3(HT_BS), 0, st, W.temp, W.gptr,
                         W.hugelist, hoff, H, self_out, out->size, hmem, dense, ncp, (const int32_t*)base,
                         &info[I_DENSE]);
    else
      hipLaunchKernelGGL(k_huge_dense<1024>, dim3(grid_for(total_bound, 1024)), dim3(HT_BS), 0, st, W.temp,
                         W.gptr, W.hugelist, hoff, H, self_out, out->size, hmem, dense, ncp, (const int32_t*)base,
                         &info[I_DENSE]);
    int64_t tpr = ncp / DC_T;
    hipLaunchKernelGGL(k_dense_compact, dim3((unsigned)(H * tpr)), dim3(DC_BS), 0, st, dense, ncp, n_c,
                       tpr, W.hugelist, W.gptr, W.temp, W.cnt, next_scan(ctx, W), (const int32_t*)base, Hd, H,
                       hmem, info);
    SPC_LAUNCH_CHECK(ctx, "huge dense");
    return SPC_OK;
  }
  launch_clear(ctx, nullptr, 0, nullptr, 0, info, 1u << I_LIVE1);
  KW* A = (KW*)W.gkeyA;
  KW* B = (KW*)W.gkeyB;
  hipLaunchKernelGGL(k_huge_entries, dim3(grid_for(total_bound, HT)), dim3(HT_BS), 0, st, W.temp, W.gptr,
                     W.hugelist, hoff, H, self_out, out->size, hmem, A, &info[I_LIVE1], next_scan(ctx, W));
  SPC_LAUNCH_CHECK(ctx, "huge gather");
  rc = readback_wait(ctx, nullptr, 0, (const int64_t*)&info[I_LIVE1]);
  if (rc) return rc;
  int64_t G = hinfo[I_NINFO];
  KW* sorted = A;
  if (G > 0) {
    rc = merge_sort<KW, LessKW>(ctx, A, B, G, LessKW(), &sorted);
    if (rc) return rc;
  }
  // scratch in the other buffer: scanned weights, head ranks, head starts
  char* scratch = (char*)(sorted == A ? B : A);
  uint64_t* wx = (uint64_t*)scratch;
  int32_t* pos = (int32_t*)(wx + G + 1);
  int32_t* hstart = pos + G + 1;
  int32_t* rowfirst = W.hmrow;
  int32_t* rowlast = W.hmnode;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(H, 256)), dim3(256), 0, st, rowlast, H, -1);
  if (G > 0) {
    hipLaunchKernelGGL(k_head_flags, dim3(grid_for(G, 256)), dim3(256), 0, st, sorted, G, pos, wx);
    rc = exclusive_scan<int32_t>(ctx, pos, pos, G, (int32_t*)W.scan_partial);
    if (rc) return rc;
    rc = exclusive_scan<uint64_t>(ctx, wx, wx, G, (uint64_t*)W.scan_partial);
    if (rc) return rc;
    hipLaunchKernelGGL(k_head_index, dim3(grid_for(G, 256)), dim3(256), 0, st, sorted, G, pos, hstart);
    hipLaunchKernelGGL(k_huge_rowfirst, dim3(grid_for(G, 256)), dim3(256), 0, st, sorted, G, pos,
                       rowfirst, rowlast);
    hipLaunchKernelGGL(k_huge_reduce, dim3(grid_for(G, 256)), dim3(256), 0, st, sorted, G, pos,
                       hstart, wx, W.hugelist, rowfirst, W.gptr, W.temp);
  }
  hipLaunchKernelGGL(k_huge_counts, dim3(grid_for(H, 256)), dim3(256), 0, st, W.hugelist, H, rowfirst,
                     rowlast, W.cnt, hmem, info);
  SPC_LAUNCH_CHECK(ctx, "huge reduce");
  return SPC_OK;
}

// Coarse row pointer from the row counts, then the info block, the entry
// total and the look-back error flags to the host.
// pack_bound > 0: the pack is launched right after the scan, before the
// wait, over pack_bound entries (at least the coarse entries, which the
// output must hold; the pack reads the total from the row pointer)
static int rowptr_and_read(spc_ctx* ctx, const LevelWork& W, spc_graph_out* out, int64_t n_c,
                           const int32_t* x1, int64_t pack_bound = 0) {
  if (n_c > 0) {
    // the scan's last tile writes the host's copy (one launch fewer) and
    // then a new token, which the host polls
    int64_t token = ++ctx->rb_token;
    {
      TimedScope ts(ctx, "contract_rowptr", (double)n_c);
      int rc = exclusive_scan<int64_t>(ctx, W.cnt, out->row_ptr, n_c, (int64_t*)W.scan_partial,
                                       ScanReadback{W.info, (int)I_NINFO, x1, ctx->h_pinned, token});
      if (rc) return rc;
      SPC_LAUNCH_CHECK(ctx, "row-pointer scan");
    }
    if (pack_bound > 0) {
      TimedScope ts(ctx, "contract_pack", (double)pack_bound);
      hipLaunchKernelGGL(k_pack, dim3(grid_for(pack_bound, PACK_T)), dim3(PACK_BS), 0, ctx->stream, out->row_ptr,
                         n_c, W.gptr, W.temp, out->col, (int32_t*)out->w);
      SPC_LAUNCH_CHECK(ctx, "pack");
    }
    return wait_token(ctx, token);
  }
  int rc = exclusive_scan<int64_t>(ctx, W.cnt, out->row_ptr, n_c, (int64_t*)W.scan_partial);
  if (rc) return rc;
  return readback_wait(ctx, W.info, (int)I_NINFO, (const int64_t*)(out->row_ptr + n_c), x1,
                       (const uint64_t*)(ctx->scan_state ? ctx->scan_state + ctx->scan_cap - 1 : nullptr));
}

// At most this many huge rows take the path without a host wait after the
// small rows (their dense accumulators are cleared for all of them).
constexpr int64_t H_DEV = 4;

int contract_level(spc_ctx* ctx, const LevelIn& g, const int32_t* c, int64_t n_c,
                   spc_graph_out* out, LevelWork& W, LevelResult& R, const Segments* seg,
                   const int32_t* ptrow) {
  hipStream_t st = ctx->stream;
  int64_t n = g.n;
  int64_t* hinfo = ctx->h_pinned;
  unsigned long long* info = W.info;
  int64_t* self_out = (int64_t*)out->self_w;
  int64_t* off = W.hpos;   // each fine node's first slot inside its super-node's records
  int rc;
  int64_t packed_bound = 0;   // entries a pack launched before the last wait covers
  {
    TimedScope ts(ctx, "contract_members", (double)n);
    // (the merge cutoff's launch zeroed the record counts already when it
    // ran; the class slots are still zero from the level's start then)
    if (!R.contract_zeroed)
      launch_clear(ctx, W.mcount, n_c + 1, (uint64_t*)W.gptr, n_c + 1, info,
                   (1u << I_MID) | (1u << I_HUGE) | (1u << I_MAXCL) | (1u << I_BLOCK) | (1u << I_R32) |
                       (1u << I_HOVER));
    hipLaunchKernelGGL(k_slot_alloc, dim3(grid_for(n, CM_BS)), dim3(CM_BS), 0, st, g, c,
                       (unsigned long long*)W.gptr, off);
    SPC_LAUNCH_CHECK(ctx, "slot_alloc");
    rc = exclusive_scan<int64_t>(ctx, W.gptr, W.gptr, n_c, (int64_t*)W.scan_partial);
    if (rc) return rc;
    int tiles = g.nnz > 0 ? grid_for(g.nnz, RT) : 0;
    hipLaunchKernelGGL(k_record_scatter, dim3(tiles + grid_for(n, RM)), dim3(RT_BS), 0, st, g, c, W.gptr, off,
                       W.temp, tiles, ptrow);
    SPC_LAUNCH_CHECK(ctx, "record_scatter");
  }
  {
    TimedScope ts(ctx, "contract_small", (double)g.nnz);
    // the fewest rows per thread that keep the grid within 1024 blocks, or
    // the tuned count when its four class chains fit the level's look-back
    // words
    TileScan tsc = next_scan(ctx, W);
    int rpt = n_c <= 1024 * SMALL_BS ? 1 : n_c <= 1024 * SMALL_BS * 2 ? 2 : SMALL_RPT;
    int want = ctx->tune.small_rpt;
    if ((want == 1 || want == 2 || want == 4) && 4 * (int64_t)grid_for(n_c, SMALL_BS * want) <= ctx->lb_words)
      rpt = want;
    int lane_max = ctx->tune.lane_max == 16 ? 16 : REG32_CAP;
    int wave_max = ctx->tune.wave_max >= 64 && ctx->tune.wave_max <= WAVE_CAP ? ctx->tune.wave_max : WAVE_CAP;
    if (rpt == 1)
      hipLaunchKernelGGL(k_contract_small<1>, dim3(grid_for(n_c, SMALL_BS)), dim3(SMALL_BS), 0, st, W.temp,
                         W.gptr, W.cnt, self_out, out->size, n_c, W.r32list, W.midlist, W.blocklist, W.hugelist,
                         info, tsc, lane_max, wave_max);
    else if (rpt == 2)
      hipLaunchKernelGGL(k_contract_small<2>, dim3(grid_for(n_c, SMALL_BS * 2)), dim3(SMALL_BS), 0, st, W.temp,
                         W.gptr, W.cnt, self_out, out->size, n_c, W.r32list, W.midlist, W.blocklist, W.hugelist,
                         info, tsc, lane_max, wave_max);
    else
      hipLaunchKernelGGL(k_contract_small<SMALL_RPT>, dim3(grid_for(n_c, SMALL_BS * SMALL_RPT)), dim3(SMALL_BS),
                         0, st, W.temp, W.gptr, W.cnt, self_out, out->size, n_c, W.r32list, W.midlist,
                         W.blocklist, W.hugelist, info, tsc, lane_max, wave_max);
  }
  SPC_LAUNCH_CHECK(ctx, "contract_small");
  // with a deferred selection, the first read also carries its super-node count
  const int32_t* x1 = R.pending ? (const int32_t*)(W.flag + n) : (const int32_t*)nullptr;
  int64_t ncp1 = (n_c + DC_T - 1) / DC_T * DC_T;
  // without the wait when the last level had a few huge rows and few rows
  // of the wavefront and block classes (their kernels then stride over
  // device-held counts on bounded grids, which is slower for many rows)
  bool dev = !seg && !ctx->force_huge_sort && ctx->contract_wait != 1 && H_DEV * ncp1 <= 2 * g.nnz &&
             (ctx->contract_wait >= 2 || ctx->contract_dev);
  if (dev) {
    // the class lists and up to H_DEV huge rows run on counts the device
    // holds; the one host wait is the coarse row pointer's.  Classes the
    // last level did not have are not launched; should this level have
    // rows of them after all, they run once the counts are read.
    int launch = ctx->contract_wait == 3 ? 0 : ctx->contract_classes_seen;
    rc = contract_classes(ctx, n_c, out, W, true, launch);
    if (rc) return rc;
    rc = contract_huge(ctx, g, n_c, out, W, seg, H_DEV, true);
    if (rc) return rc;
    rc = rowptr_and_read(ctx, W, out, n_c, x1);
    if (rc) return rc;
    if (R.pending) {
      rc = finish_select(ctx, R, n_c, R.pending_rank, false, seg);
      if (rc) return rc;
    }
    int missed = ((hinfo[I_R32] > 0) ? 1 : 0) | ((hinfo[I_MID] > 0) ? 2 : 0) | ((hinfo[I_BLOCK] > 0) ? 4 : 0);
    missed &= ~launch;
    if (hinfo[I_HOVER] || missed) {
      // more huge rows than H_DEV (they were left alone), or rows of a class
      // not launched: the host knows the counts now
      if (missed) {
        rc = contract_classes(ctx, n_c, out, W, false, missed);
        if (rc) return rc;
      }
      if (hinfo[I_HOVER]) {
        rc = contract_huge(ctx, g, n_c, out, W, seg, hinfo[I_HUGE], false);
        if (rc) return rc;
      }
      rc = rowptr_and_read(ctx, W, out, n_c, nullptr);
      if (rc) return rc;
    }
  } else {
    rc = readback_wait(ctx, info, (int)I_NINFO, nullptr, x1);
    if (rc) return rc;
    if (R.pending) {
      rc = finish_select(ctx, R, n_c, R.pending_rank, false, seg);
      if (rc) return rc;
    }
    int64_t H = hinfo[I_HUGE];
    rc = contract_classes(ctx, n_c, out, W, false);
    if (rc) return rc;
    if (H > 0) {
      rc = contract_huge(ctx, g, n_c, out, W, seg, H, false);
      if (rc) return rc;
    }
    // every row's entries are final here: when the output holds as many
    // entries as the fine graph (a bound on the coarse one), the pack goes
    // before the host's wait for the coarse count
    if (out->nnz_cap >= g.nnz && g.nnz > 0) packed_bound = g.nnz;
    rc = rowptr_and_read(ctx, W, out, n_c, nullptr, packed_bound);
    if (rc) return rc;
  }
  R.maxcl = hinfo[I_MAXCL];
  {
    int64_t H = hinfo[I_HUGE];
    ctx->contract_dev = H >= 1 && H <= H_DEV && hinfo[I_MID] + hinfo[I_BLOCK] <= 8192 && hinfo[I_R32] <= 65536;
    ctx->contract_classes_seen =
        ((hinfo[I_R32] > 0) ? 1 : 0) | ((hinfo[I_MID] > 0) ? 2 : 0) | ((hinfo[I_BLOCK] > 0) ? 4 : 0);
  }
  int64_t nnz_c = hinfo[I_NINFO];
  if (hinfo[I_DENSE]) return set_error(ctx, SPC_EINVAL, "internal: a huge row left its graph's coarse range");
  if (hinfo[I_LBERR] || hinfo[I_NINFO + 2])
    return set_error(ctx, SPC_EINVAL, "internal: look-back wait gave up");
  if (nnz_c > out->nnz_cap)
    return set_error(ctx, SPC_ECAPACITY, "coarse graph needs %lld entries, capacity %lld",
                     (long long)nnz_c, (long long)out->nnz_cap);
  if (nnz_c > 0 && packed_bound < nnz_c) {   // (not packed before the wait)
    TimedScope ts(ctx, "contract_pack", (double)nnz_c);
    hipLaunchKernelGGL(k_pack, dim3(grid_for(nnz_c, PACK_T)), dim3(PACK_BS), 0, st, out->row_ptr, n_c,
                       W.gptr, W.temp, out->col, (int32_t*)out->w);
    SPC_LAUNCH_CHECK(ctx, "pack");
  }
  R.nnz_c = nnz_c;
  return SPC_OK;
}

}  // namespace spc

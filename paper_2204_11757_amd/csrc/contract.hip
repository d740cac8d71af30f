// A5: contraction of the fine graph into the coarsened graph of
// Definition 1.  Super-node a's weight towards b is the sum of w(x, y) over
// members x of a and y of b; pairs inside one super-node become a's
// self-loop weight together with the members' own self-loops; sizes add.
// Coarse rows are ascending in b with no diagonal entry.
//
// Rows are grouped by the number E_a of fine entries their members hold:
//   E_a <= SMALL_CAP   one thread per coarse row, sorted insertion into a
//                      thread-private LDS list (merging equal columns);
//   E_a <= WAVE_CAP    one wavefront per row, bitonic sort in LDS;
//   E_a <= BLOCK_CAP   one 256-thread block per row, bitonic sort in LDS;
//   larger             all entries of such rows are gathered, merge-sorted
//                      by (row, column) and reduced.
// Each path writes its row's distinct (column, weight) pairs into a scratch
// region at the row's gathered-entry offset; a scan of the row counts then
// yields the coarse row_ptr and a tiled copy packs the entries.
#include "level.hpp"

namespace spc {

constexpr int SMALL_CAP = 32;
constexpr int SMALL_BS = 128;
constexpr int SMALL_RPT = 4;   // rows per thread
constexpr int WAVE_CAP = 512;
constexpr int BLOCK_CAP = 4096;

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

// member counts and gathered-entry counts per super-node; lanes of one
// wavefront that hit the same super-node add once
__global__ void k_cluster_count(LevelIn g, const int32_t* __restrict__ c, int32_t* mcount,
                                unsigned long long* ecnt) {
  int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool valid = x < g.n;
  int32_t a = valid ? c[x] : -1;
  int64_t len = valid ? g.rp[x + 1] - g.rp[x] : 0;
  bool head;
  int end;
  uint64_t heads;
  wave_runs(a, head, end, heads);
  int64_t inc = wave_incl_sum(len);
  int64_t at_end = __shfl(inc, end - 1);
  if (head && a >= 0) {
    atomicAdd(&mcount[a], end - lane_id());
    atomicAdd(&ecnt[a], (unsigned long long)(at_end - inc + len));
  }
}

__global__ void k_member_scatter(const int32_t* __restrict__ c, const int32_t* __restrict__ mptr,
                                 int32_t* mcount, int32_t* __restrict__ members, int64_t n) {
  int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool valid = x < n;
  int32_t a = valid ? c[x] : -1;
  bool head;
  int end;
  uint64_t heads;
  wave_runs(a, head, end, heads);
  int old = 0;
  if (head && a >= 0) old = atomicSub(&mcount[a], end - lane_id());
  int h = run_head_of(heads);
  int oldh = __shfl(old, h);
  int endh = __shfl(end, h);
  if (valid) {
    int s = endh - h;
    members[mptr[a] + oldh - s + (lane_id() - h)] = (int32_t)x;
  }
}

// ---- rows with at most SMALL_CAP gathered entries: one thread each --------
__global__ void __launch_bounds__(SMALL_BS)
    k_contract_small(LevelIn g, const int32_t* __restrict__ c, const int32_t* __restrict__ mptr,
                     const int32_t* __restrict__ members, const int64_t* __restrict__ gptr,
                     uint64_t* __restrict__ temp, int64_t* __restrict__ cnt,
                     int64_t* __restrict__ self_out, int32_t* __restrict__ size_out, int64_t n_c,
                     int32_t* __restrict__ midlist, int32_t* __restrict__ blocklist,
                     int32_t* __restrict__ hugelist, unsigned long long* info) {
  __shared__ uint64_t lst[SMALL_CAP * SMALL_BS];
  __shared__ int stmp[SMALL_BS / WAVE];
  __shared__ unsigned long long sbase;
  __shared__ int32_t smx[SMALL_BS / WAVE];
  int tid = threadIdx.x;
  int64_t base = (int64_t)blockIdx.x * SMALL_BS * SMALL_RPT;
  uint32_t midm = 0, blkm = 0, hugem = 0;
  int nmid = 0, nblk = 0, nhuge = 0;
  int32_t mx = 0;
  for (int r = 0; r < SMALL_RPT; r++) {
    int64_t a = base + r * SMALL_BS + tid;
    if (a >= n_c) break;
    int64_t E = gptr[a + 1] - gptr[a];
    int32_t msz = mptr[a + 1] - mptr[a];
    mx = msz > mx ? msz : mx;
    if (E > SMALL_CAP) {
      if (E <= WAVE_CAP) {
        midm |= 1u << r;
        nmid++;
      } else if (E <= BLOCK_CAP) {
        blkm |= 1u << r;
        nblk++;
      } else {
        hugem |= 1u << r;
        nhuge++;
        self_out[a] = 0;
        size_out[a] = 0;
      }
      continue;
    }
    int64_t self = 0;
    int32_t sz = 0;
    int cntd = 0;
    int32_t a32 = (int32_t)a;
    for (int32_t p = mptr[a]; p < mptr[a + 1]; p++) {
      int32_t x = members[p];
      sz += g.size ? g.size[x] : 1;
      if (g.self) self += g.self[x];
      for (int64_t j = g.rp[x]; j < g.rp[x + 1]; j++) {
        int32_t b = c[g.col[j]];
        uint32_t wv = (uint32_t)g.w[j];
        if (b == a32) {
          self += wv;
          continue;
        }
        int i = cntd - 1;
        while (i >= 0 && (int32_t)(lst[i * SMALL_BS + tid] >> 32) > b) i--;
        if (i >= 0 && (int32_t)(lst[i * SMALL_BS + tid] >> 32) == b) {
          lst[i * SMALL_BS + tid] += wv;  // sums stay below 2^31: no carry into the column
        } else {
          for (int q = cntd; q > i + 1; q--) lst[q * SMALL_BS + tid] = lst[(q - 1) * SMALL_BS + tid];
          lst[(i + 1) * SMALL_BS + tid] = ((uint64_t)(uint32_t)b << 32) | wv;
          cntd++;
        }
      }
    }
    int64_t o = gptr[a];
    for (int q = 0; q < cntd; q++) temp[o + q] = lst[q * SMALL_BS + tid];
    cnt[a] = cntd;
    self_out[a] = self;
    size_out[a] = sz;
  }
  mx = wave_max(mx);
  if (lane_id() == 0) smx[tid / WAVE] = mx;
  __syncthreads();
  if (tid == 0) {
    int32_t m2 = 0;
    for (int w = 0; w < SMALL_BS / WAVE; w++) m2 = smx[w] > m2 ? smx[w] : m2;
    if (m2) atomicMax(&info[I_MAXCL], (unsigned long long)m2);
  }
  int64_t p1 = block_reserve<SMALL_BS>(&info[I_MID], nmid, &sbase, stmp);
  int64_t p2 = block_reserve<SMALL_BS>(&info[I_BLOCK], nblk, &sbase, stmp);
  int64_t p3 = block_reserve<SMALL_BS>(&info[I_HUGE], nhuge, &sbase, stmp);
  for (int r = 0; r < SMALL_RPT; r++) {
    int32_t a = (int32_t)(base + r * SMALL_BS + tid);
    if (midm >> r & 1u) midlist[p1++] = a;
    if (blkm >> r & 1u) blocklist[p2++] = a;
    if (hugem >> r & 1u) hugelist[p3++] = a;
  }
}

// ---- rows with at most CAP gathered entries: one BS-thread block each ----
template <int TB, int CAP>
__global__ void __launch_bounds__(TB)
    k_contract_row(LevelIn g, const int32_t* __restrict__ c, const int32_t* __restrict__ mptr,
                   const int32_t* __restrict__ members, const int64_t* __restrict__ gptr,
                   const int32_t* __restrict__ rowlist, uint64_t* __restrict__ temp,
                   int64_t* __restrict__ cnt, int64_t* __restrict__ self_out,
                   int32_t* __restrict__ size_out) {
  __shared__ uint64_t ent[CAP];
  __shared__ int lcnt;
  __shared__ unsigned long long lself;
  __shared__ int lsize;
  __shared__ int32_t stmp[TB / WAVE];
  int tid = threadIdx.x;
  int32_t a = rowlist[blockIdx.x];
  if (tid == 0) {
    lcnt = 0;
    lself = 0;
    lsize = 0;
  }
  __syncthreads();
  int64_t self = 0;
  int32_t sz = 0;
  for (int32_t p = mptr[a] + tid; p < mptr[a + 1]; p += TB) {
    int32_t x = members[p];
    sz += g.size ? g.size[x] : 1;
    if (g.self) self += g.self[x];
    for (int64_t j = g.rp[x]; j < g.rp[x + 1]; j++) {
      int32_t b = c[g.col[j]];
      uint32_t wv = (uint32_t)g.w[j];
      if (b == a) {
        self += wv;
      } else {
        int pos = atomicAdd(&lcnt, 1);
        ent[pos] = ((uint64_t)(uint32_t)b << 32) | wv;
      }
    }
  }
  self = wave_sum(self);
  sz = wave_sum(sz);
  if (lane_id() == 0) {
    atomicAdd(&lself, (unsigned long long)self);
    atomicAdd(&lsize, sz);
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
  // distinct columns in ascending order, weights summed
  int64_t o = gptr[a];
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
      temp[o + carry + inc - 1] = ((uint64_t)b << 32) | sum;
    }
    carry += tot;
  }
  if (tid == 0) {
    cnt[a] = carry;
    self_out[a] = (int64_t)lself;
    size_out[a] = lsize;
  }
}

// ---- rows with more than BLOCK_CAP gathered entries ------------------------
struct KW {
  uint64_t key, w;
};
struct LessKW {
  __device__ __forceinline__ bool operator()(const KW& a, const KW& b) const { return a.key < b.key; }
};

__global__ void k_huge_members_count(const int32_t* __restrict__ hugelist, int64_t H,
                                     const int32_t* __restrict__ mptr, int64_t* __restrict__ hcount) {
  int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h < H) {
    int32_t a = hugelist[h];
    hcount[h] = mptr[a + 1] - mptr[a];
  }
}

__global__ void k_huge_members_fill(const int32_t* __restrict__ hugelist,
                                    const int32_t* __restrict__ mptr,
                                    const int32_t* __restrict__ members,
                                    const int64_t* __restrict__ hoff, int32_t* __restrict__ hmrow,
                                    int32_t* __restrict__ hmnode) {
  int h = blockIdx.x;
  int32_t a = hugelist[h];
  int32_t s = mptr[a], e = mptr[a + 1];
  int64_t o = hoff[h];
  for (int32_t p = s + threadIdx.x; p < e; p += blockDim.x) {
    hmrow[o + (p - s)] = h;
    hmnode[o + (p - s)] = members[p];
  }
}

// per huge member: count cross entries; add self-loop and intra weight, and
// sizes, to the super-node with integer atomics (order-independent), once
// per run of lanes that share a super-node
__global__ void k_huge_member_pass1(LevelIn g, const int32_t* __restrict__ c,
                                    const int32_t* __restrict__ hugelist,
                                    const int32_t* __restrict__ hmrow,
                                    const int32_t* __restrict__ hmnode, int64_t HM,
                                    int64_t* __restrict__ hcnt, int64_t* self_out,
                                    int32_t* size_out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool valid = i < HM;
  int32_t h = valid ? hmrow[i] : -1;
  int64_t self = 0, k = 0;
  int32_t sz = 0;
  if (valid) {
    int32_t x = hmnode[i];
    int32_t a = hugelist[h];
    self = g.self ? g.self[x] : 0;
    sz = g.size ? g.size[x] : 1;
    for (int64_t j = g.rp[x]; j < g.rp[x + 1]; j++) {
      if (c[g.col[j]] == a) self += g.w[j];
      else k++;
    }
    hcnt[i] = k;
  }
  bool head;
  int end;
  uint64_t heads;
  wave_runs(h, head, end, heads);
  int64_t si = wave_incl_sum(self);
  int32_t zi = wave_incl_sum(sz);
  int64_t se = __shfl(si, end - 1);
  int32_t ze = __shfl(zi, end - 1);
  if (head && h >= 0) {
    int32_t a = hugelist[h];
    atomicAdd((unsigned long long*)&self_out[a], (unsigned long long)(se - si + self));
    atomicAdd(&size_out[a], ze - zi + sz);
  }
}

__global__ void k_huge_member_pass2(LevelIn g, const int32_t* __restrict__ c,
                                    const int32_t* __restrict__ hugelist,
                                    const int32_t* __restrict__ hmrow,
                                    const int32_t* __restrict__ hmnode, int64_t HM,
                                    const int64_t* __restrict__ hpos, KW* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= HM) return;
  int32_t x = hmnode[i];
  int32_t h = hmrow[i];
  int32_t a = hugelist[h];
  int64_t o = hpos[i];
  for (int64_t j = g.rp[x]; j < g.rp[x + 1]; j++) {
    int32_t b = c[g.col[j]];
    if (b != a) out[o++] = KW{((uint64_t)(uint32_t)h << 32) | (uint32_t)b, (uint64_t)(uint32_t)g.w[j]};
  }
}

__global__ void k_head_flags(const KW* __restrict__ s, int64_t G, int32_t* __restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < G) flag[i] = (i == 0 || s[i].key != s[i - 1].key) ? 1 : 0;
}

__global__ void k_huge_reduce(const KW* __restrict__ s, int64_t G, const int32_t* __restrict__ pos,
                              const int32_t* __restrict__ hugelist, const int64_t* __restrict__ hoff,
                              const int64_t* __restrict__ hpos, const int64_t* __restrict__ gptr,
                              uint64_t* __restrict__ temp) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G) return;
  if (!(i == 0 || s[i].key != s[i - 1].key)) return;
  uint64_t key = s[i].key;
  int32_t h = (int32_t)(key >> 32);
  uint32_t b = (uint32_t)key;
  uint64_t sum = 0;
  for (int64_t q = i; q < G && s[q].key == key; q++) sum += s[q].w;
  int64_t seg0 = hpos[hoff[h]];
  int32_t a = hugelist[h];
  int64_t r = pos[i] - pos[seg0];
  temp[gptr[a] + r] = ((uint64_t)b << 32) | sum;
}

__global__ void k_huge_counts(const int32_t* __restrict__ hugelist, int64_t H,
                              const int64_t* __restrict__ hoff, const int64_t* __restrict__ hpos,
                              const int32_t* __restrict__ pos, int64_t* __restrict__ cnt) {
  int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h < H) cnt[hugelist[h]] = pos[hpos[hoff[h + 1]]] - pos[hpos[hoff[h]]];
}

// ---- packing: tiles of output positions mapped to coarse rows -----------
constexpr int PACK_T = 1024;
constexpr int PACK_BS = 256;

__global__ void __launch_bounds__(PACK_BS)
    k_pack(const int64_t* __restrict__ rpc, int64_t n_c, const int64_t* __restrict__ gptr,
           const uint64_t* __restrict__ temp, int32_t* __restrict__ col_c, int32_t* __restrict__ w_c) {
  __shared__ int32_t srow[PACK_T];
  __shared__ int64_t sh[2];
  __shared__ int32_t stmp[PACK_BS / WAVE];
  int64_t p0 = (int64_t)blockIdx.x * PACK_T;
  lbs_tile<PACK_T, PACK_BS>(rpc, n_c, p0, srow, sh, stmp);
  int64_t total = rpc[n_c];
  for (int i = 0; i < PACK_T / PACK_BS; i++) {
    int k = threadIdx.x + i * PACK_BS;
    int64_t p = p0 + k;
    if (p >= total) break;
    int32_t a = srow[k];
    uint64_t v = temp[gptr[a] + (p - rpc[a])];
    col_c[p] = (int32_t)(v >> 32);
    w_c[p] = (int32_t)(uint32_t)v;
  }
}

int contract_level(spc_ctx* ctx, const LevelIn& g, const int32_t* c, int64_t n_c,
                   spc_graph_out* out, LevelWork& W, LevelResult& R) {
  hipStream_t st = ctx->stream;
  int64_t n = g.n;
  int64_t* hinfo = ctx->h_pinned;
  unsigned long long* info = W.info;
  int64_t* self_out = (int64_t*)out->self_w;
  int rc;
  {
    TimedScope ts(ctx, "contract_members", (double)n);
    SPC_HIP(ctx, hipMemsetAsync(W.mcount, 0, sizeof(int32_t) * (n_c + 1), st));
    SPC_HIP(ctx, hipMemsetAsync(W.gptr, 0, sizeof(int64_t) * (n_c + 1), st));
    hipLaunchKernelGGL(k_cluster_count, dim3(grid_for(n, 256)), dim3(256), 0, st, g, c, W.mcount,
                       (unsigned long long*)W.gptr);
    SPC_LAUNCH_CHECK(ctx, "cluster_count");
    rc = exclusive_scan<int32_t>(ctx, W.mcount, W.mptr, n_c, (int32_t*)W.scan_partial);
    if (rc) return rc;
    rc = exclusive_scan<int64_t>(ctx, W.gptr, W.gptr, n_c, (int64_t*)W.scan_partial);
    if (rc) return rc;
    hipLaunchKernelGGL(k_member_scatter, dim3(grid_for(n, 256)), dim3(256), 0, st, c, W.mptr,
                       W.mcount, W.members, n);
  }
  SPC_HIP(ctx, hipMemsetAsync(&info[I_MID], 0, sizeof(unsigned long long) * 2, st));
  SPC_HIP(ctx, hipMemsetAsync(&info[I_MAXCL], 0, sizeof(unsigned long long), st));
  SPC_HIP(ctx, hipMemsetAsync(&info[I_BLOCK], 0, sizeof(unsigned long long), st));
  {
    TimedScope ts(ctx, "contract_small", (double)g.nnz);
    hipLaunchKernelGGL(k_contract_small, dim3(grid_for(n_c, SMALL_BS * SMALL_RPT)), dim3(SMALL_BS), 0,
                       st, g, c, W.mptr, W.members, W.gptr, W.temp, W.cnt, self_out, out->size, n_c,
                       W.midlist, W.blocklist, W.hugelist, info);
  }
  SPC_LAUNCH_CHECK(ctx, "contract_small");
  SPC_HIP(ctx, hipMemcpyAsync(hinfo, info, sizeof(unsigned long long) * I_NINFO,
                              hipMemcpyDeviceToHost, st));
  SPC_HIP(ctx, hipStreamSynchronize(st));
  int64_t nmid = hinfo[I_MID], nblk = hinfo[I_BLOCK], H = hinfo[I_HUGE];
  R.maxcl = hinfo[I_MAXCL];
  if (nmid > 0) {
    TimedScope ts(ctx, "contract_wave_rows", (double)nmid);
    hipLaunchKernelGGL((k_contract_row<WAVE, WAVE_CAP>), dim3((unsigned)nmid), dim3(WAVE), 0, st, g, c,
                       W.mptr, W.members, W.gptr, W.midlist, W.temp, W.cnt, self_out, out->size);
    SPC_LAUNCH_CHECK(ctx, "contract wave rows");
  }
  if (nblk > 0) {
    TimedScope ts(ctx, "contract_block_rows", (double)nblk);
    hipLaunchKernelGGL((k_contract_row<256, BLOCK_CAP>), dim3((unsigned)nblk), dim3(256), 0, st, g, c,
                       W.mptr, W.members, W.gptr, W.blocklist, W.temp, W.cnt, self_out, out->size);
    SPC_LAUNCH_CHECK(ctx, "contract block rows");
  }
  if (H > 0) {
    TimedScope ts(ctx, "contract_huge", (double)H);
    hipLaunchKernelGGL(k_huge_members_count, dim3(grid_for(H, 256)), dim3(256), 0, st, W.hugelist, H,
                       W.mptr, W.hmoff);
    rc = exclusive_scan<int64_t>(ctx, W.hmoff, W.hmoff, H, (int64_t*)W.scan_partial);
    if (rc) return rc;
    int64_t HM = 0;
    SPC_HIP(ctx, hipMemcpyAsync(&HM, W.hmoff + H, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SPC_HIP(ctx, hipStreamSynchronize(st));
    hipLaunchKernelGGL(k_huge_members_fill, dim3((unsigned)H), dim3(256), 0, st, W.hugelist, W.mptr,
                       W.members, W.hmoff, W.hmrow, W.hmnode);
    int64_t* hpos = W.hpos;
    hipLaunchKernelGGL(k_huge_member_pass1, dim3(grid_for(HM, 256)), dim3(256), 0, st, g, c,
                       W.hugelist, W.hmrow, W.hmnode, HM, hpos, self_out, out->size);
    rc = exclusive_scan<int64_t>(ctx, hpos, hpos, HM, (int64_t*)W.scan_partial);
    if (rc) return rc;
    int64_t G = 0;
    SPC_HIP(ctx, hipMemcpyAsync(&G, hpos + HM, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SPC_HIP(ctx, hipStreamSynchronize(st));
    KW* A = (KW*)W.gkeyA;
    KW* B = (KW*)W.gkeyB;
    hipLaunchKernelGGL(k_huge_member_pass2, dim3(grid_for(HM, 256)), dim3(256), 0, st, g, c,
                       W.hugelist, W.hmrow, W.hmnode, HM, hpos, A);
    SPC_LAUNCH_CHECK(ctx, "huge gather");
    KW* sorted = A;
    if (G > 0) {
      rc = merge_sort<KW, LessKW>(ctx, A, B, G, LessKW(), &sorted);
      if (rc) return rc;
    }
    int32_t* pos = (int32_t*)(sorted == A ? B : A);
    hipLaunchKernelGGL(k_head_flags, dim3(grid_for(G, 256)), dim3(256), 0, st, sorted, G, pos);
    rc = exclusive_scan<int32_t>(ctx, pos, pos, G, (int32_t*)W.scan_partial);
    if (rc) return rc;
    hipLaunchKernelGGL(k_huge_reduce, dim3(grid_for(G, 256)), dim3(256), 0, st, sorted, G, pos,
                       W.hugelist, W.hmoff, hpos, W.gptr, W.temp);
    hipLaunchKernelGGL(k_huge_counts, dim3(grid_for(H, 256)), dim3(256), 0, st, W.hugelist, H, W.hmoff,
                       hpos, pos, W.cnt);
    SPC_LAUNCH_CHECK(ctx, "huge reduce");
  }
  {
    TimedScope ts(ctx, "contract_rowptr", (double)n_c);
    rc = exclusive_scan<int64_t>(ctx, W.cnt, out->row_ptr, n_c, (int64_t*)W.scan_partial);
    if (rc) return rc;
  }
  int64_t nnz_c = 0;
  SPC_HIP(ctx, hipMemcpyAsync(&nnz_c, out->row_ptr + n_c, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  SPC_HIP(ctx, hipStreamSynchronize(st));
  if (nnz_c > out->nnz_cap)
    return set_error(ctx, SPC_ECAPACITY, "coarse graph needs %lld entries, capacity %lld",
                     (long long)nnz_c, (long long)out->nnz_cap);
  if (nnz_c > 0) {
    TimedScope ts(ctx, "contract_pack", (double)nnz_c);
    hipLaunchKernelGGL(k_pack, dim3(grid_for(nnz_c, PACK_T)), dim3(PACK_BS), 0, st, out->row_ptr, n_c,
                       W.gptr, W.temp, out->col, (int32_t*)out->w);
    SPC_LAUNCH_CHECK(ctx, "pack");
  }
  R.nnz_c = nnz_c;
  return SPC_OK;
}

}  // namespace spc

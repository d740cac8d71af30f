// Floating-point path of one coarsening level: FP32 weights (an input level)
// or FP64 weights (coarse levels), FP64 self-loops.
//
// * Degrees (the row sums after Theorem 1) and coarse weights (Definition 1's
//   sums) are the correctly rounded values of the exact real sums, so they
//   do not depend on summation order.  Every weight of a level is an integer
//   multiple of 2^L, L the smallest ulp exponent among them; sums are held
//   exactly as 192-bit integers in units of 2^L and rounded once, to nearest
//   with ties to even.  A level whose weights span more than FP_MAX_SPAN
//   binades above 2^L is rejected.
// * The merge score of edge (u, v) (Theorem 1) is evaluated in FP64 in the
//   common-support form 2 - 2 t, t = sum of min(a_ux / d_u, a_vx / d_v) over
//   the common support in ascending x (the diagonal positions x = u and
//   x = v included when the self-loop weight is positive), each quotient
//   correctly rounded and t summed left to right.
// * The order (Algorithm 1's sort) is (score, edge id), by a merge sort; the
//   rest of the selection runs on the ranks exactly as on the integer path.
#include "level.hpp"

namespace spc {

__device__ __forceinline__ double fp_w(const LevelInF& g, int64_t j) {
  return g.w32 ? (double)((const float*)g.w)[j] : ((const double*)g.w)[j];
}

// v > 0 and finite: v = mant * 2^lsb with mant < 2^53
__device__ __forceinline__ void fp_split(double v, uint64_t& mant, int& lsb) {
  uint64_t b = (uint64_t)__double_as_longlong(v);
  int E = (int)((b >> 52) & 0x7ff);
  uint64_t f = b & ((1ull << 52) - 1);
  if (E == 0) {
    mant = f;
    lsb = -1074;
  } else {
    mant = f | (1ull << 52);
    lsb = E - 1075;
  }
}

// ---------------------------------------------------------------------------
// 192-bit unsigned fixed point (three 64-bit limbs, least significant first)
// ---------------------------------------------------------------------------
struct Fx {
  uint64_t l0, l1, l2;
};

__device__ __forceinline__ uint64_t fx_limb(const Fx& a, int i) {
  return i == 0 ? a.l0 : i == 1 ? a.l1 : i == 2 ? a.l2 : 0ull;
}

__device__ __forceinline__ void fx_add3(Fx& a, uint64_t b0, uint64_t b1, uint64_t b2) {
  uint64_t s0 = a.l0 + b0;
  uint64_t c0 = s0 < b0;
  uint64_t s1 = a.l1 + b1;
  uint64_t c1 = s1 < b1;
  uint64_t s1c = s1 + c0;
  c1 |= s1c < c0;
  a.l0 = s0;
  a.l1 = s1c;
  a.l2 = a.l2 + b2 + c1;
}

// mant << s as three limbs (0 <= s; bits beyond 192 are dropped, which the
// span bound excludes)
__device__ __forceinline__ Fx fx_of(uint64_t mant, int s) {
  int q = s >> 6, r = s & 63;
  uint64_t lo = mant << r;
  uint64_t hi = r ? (mant >> (64 - r)) : 0ull;
  Fx x;
  x.l0 = q == 0 ? lo : 0ull;
  x.l1 = q == 0 ? hi : (q == 1 ? lo : 0ull);
  x.l2 = q == 1 ? hi : (q == 2 ? lo : 0ull);
  return x;
}

__device__ __forceinline__ void fx_add_value(Fx& a, double v, int L) {
  if (!(v > 0.0)) return;
  uint64_t mant;
  int lsb;
  fp_split(v, mant, lsb);
  Fx x = fx_of(mant, lsb - L);
  fx_add3(a, x.l0, x.l1, x.l2);
}

// (a >> s) & (2^64 - 1) for 0 <= s < 192
__device__ __forceinline__ uint64_t fx_shr64(const Fx& a, int s) {
  int q = s >> 6, r = s & 63;
  uint64_t x0 = fx_limb(a, q), x1 = fx_limb(a, q + 1);
  return r ? ((x0 >> r) | (x1 << (64 - r))) : x0;
}

__device__ __forceinline__ int fx_bit(const Fx& a, int b) { return (int)((fx_limb(a, b >> 6) >> (b & 63)) & 1ull); }

// any bit below position p (p >= 0)
__device__ __forceinline__ bool fx_any_below(const Fx& a, int p) {
  int q = p >> 6, r = p & 63;
  bool any = false;
  if (q > 0) any |= a.l0 != 0;
  if (q > 1) any |= a.l1 != 0;
  if (q > 2) any |= a.l2 != 0;
  if (q < 3 && r) any |= (fx_limb(a, q) & ((1ull << r) - 1)) != 0;
  return any;
}

// a * 2^L rounded to nearest, ties to even
__device__ __forceinline__ double fx_round(const Fx& a, int L) {
  int h = a.l2 ? 128 + 63 - __clzll((long long)a.l2)
                : a.l1 ? 64 + 63 - __clzll((long long)a.l1) : a.l0 ? 63 - __clzll((long long)a.l0) : -1;
  if (h < 0) return 0.0;
  if (h <= 52) return ldexp((double)a.l0, L);
  int s = h - 52;
  uint64_t mant = fx_shr64(a, s) & ((1ull << 53) - 1);
  int guard = fx_bit(a, s - 1);
  bool sticky = s >= 2 && fx_any_below(a, s - 1);
  if (guard && (sticky || (mant & 1ull))) mant += 1;   // 2^53 stays exact
  return ldexp((double)mant, L + s);
}

// six 32-bit chunks of a fixed-point value, for chunk-wise atomic sums
__device__ __forceinline__ uint32_t fx_chunk(const Fx& a, int c) {
  uint64_t l = c < 2 ? a.l0 : c < 4 ? a.l1 : a.l2;
  return (uint32_t)(l >> (32 * (c & 1)));
}

// sums of chunks (each slot at most 2^32 terms) back to a fixed-point value
__device__ __forceinline__ Fx fx_from_chunks(const uint64_t* s, int64_t stride, int64_t idx) {
  uint32_t out[FP_LIMBS];
  uint64_t carry = 0;
#pragma unroll
  for (int c = 0; c < FP_LIMBS; c++) {
    uint64_t v = s[c * stride + idx];
    uint64_t lo = (v & 0xffffffffull) + carry;
    out[c] = (uint32_t)lo;
    carry = (lo >> 32) + (v >> 32);
  }
  Fx x;
  x.l0 = (uint64_t)out[0] | ((uint64_t)out[1] << 32);
  x.l1 = (uint64_t)out[2] | ((uint64_t)out[3] << 32);
  x.l2 = (uint64_t)out[4] | ((uint64_t)out[5] << 32);
  return x;
}

__device__ __forceinline__ int fp_level_L(const unsigned long long* info) {
  return (int)((int64_t)info[I_FP_LMIN] - FP_EBIAS);
}

// ---------------------------------------------------------------------------
// validation and exponent range of a level's weights
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(BS) k_fp_range(LevelInF g, unsigned long long* info) {
  __shared__ int sl[BS / WAVE], sh[BS / WAVE], sb[BS / WAVE];
  int lmin = 1 << 20, hmax = -(1 << 20), bad = 0;
  int64_t stride = (int64_t)gridDim.x * BS;
  for (int64_t j = (int64_t)blockIdx.x * BS + threadIdx.x; j < g.nnz + g.n; j += stride) {
    double v;
    bool positive_required = j < g.nnz;
    if (j < g.nnz) v = fp_w(g, j);
    else if (g.self) v = g.self[j - g.nnz];
    else continue;
    if (!isfinite(v) || v < 0.0 || (positive_required && v == 0.0)) {
      bad = 1;
      continue;
    }
    if (v == 0.0) continue;
    uint64_t mant;
    int lsb;
    fp_split(v, mant, lsb);
    lmin = lsb < lmin ? lsb : lmin;
    int msb = lsb + 63 - __clzll((long long)mant);
    hmax = msb > hmax ? msb : hmax;
  }
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    int a = __shfl_xor(lmin, o), b = __shfl_xor(hmax, o), c = __shfl_xor(bad, o);
    lmin = a < lmin ? a : lmin;
    hmax = b > hmax ? b : hmax;
    bad |= c;
  }
  if (lane_id() == 0) {
    sl[threadIdx.x / WAVE] = lmin;
    sh[threadIdx.x / WAVE] = hmax;
    sb[threadIdx.x / WAVE] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < BS / WAVE; w++) {
      lmin = sl[w] < lmin ? sl[w] : lmin;
      hmax = sh[w] > hmax ? sh[w] : hmax;
      bad |= sb[w];
    }
    if (bad) atomicOr(&info[I_FP_BAD], 1ull);
    if (lmin < (1 << 20)) atomic_min_lazy(&info[I_FP_LMIN], (unsigned long long)(lmin + FP_EBIAS));
    if (hmax > -(1 << 20)) atomic_max_lazy(&info[I_FP_HMAX], (unsigned long long)(hmax + FP_EBIAS));
  }
}

__global__ void k_fp_range_init(unsigned long long* info) {
  info[I_FP_LMIN] = ~0ull;
  info[I_FP_HMAX] = 0;
  info[I_FP_BAD] = 0;
}

// span check after the range pass: flag 2 when the fixed point cannot hold
// the level's sums exactly
__global__ void k_fp_span(unsigned long long* info) {
  if (info[I_FP_LMIN] == ~0ull) {   // no nonzero weight at all
    info[I_FP_LMIN] = FP_EBIAS;
    info[I_FP_HMAX] = FP_EBIAS;
  }
  int64_t span = (int64_t)info[I_FP_HMAX] - (int64_t)info[I_FP_LMIN];
  if (span > FP_MAX_SPAN) atomicOr(&info[I_FP_BAD], 2ull);
}

// ---------------------------------------------------------------------------
// A1: degrees (exact row sums, rounded once) and the per-level setup the
// selection kernels expect (lower counts, upper counts, forest state)
// ---------------------------------------------------------------------------
constexpr int FD_PER = 16;
constexpr int FD_ROWS = BS * FD_PER;
constexpr int FD_SHORT = 64;

__global__ void __launch_bounds__(BS)
    k_fp_degree(LevelInF g, double* __restrict__ deg, int32_t* __restrict__ lc, int64_t* __restrict__ ucnt,
                uint64_t* __restrict__ bestA, uint64_t* __restrict__ bestB, int32_t* __restrict__ parent,
                int32_t* __restrict__ cc, const unsigned long long* info) {
  __shared__ int stmp[BS / WAVE];
  __shared__ int32_t slong[FD_ROWS];
  __shared__ uint64_t schunk[BS / WAVE][FP_LIMBS];
  int tid = threadIdx.x;
  int L = fp_level_L(info);
  int64_t base = (int64_t)blockIdx.x * FD_ROWS;
  uint32_t longmask = 0;
  int nlong = 0;
  for (int i = 0; i < FD_PER; i++) {
    int64_t u = base + i * BS + tid;
    if (u >= g.n) break;
    int64_t s = g.rp[u], e = g.rp[u + 1];
    int64_t lo = s, hi = e;   // entries with col < u
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (g.col[mid] < u) lo = mid + 1;
      else hi = mid;
    }
    lc[u] = (int32_t)(lo - s);
    ucnt[u] = e - lo;
    if (e - s <= FD_SHORT) {
      Fx a{0, 0, 0};
      if (g.self) fx_add_value(a, g.self[u], L);
      for (int64_t j = s; j < e; j++) fx_add_value(a, fp_w(g, j), L);
      deg[u] = fx_round(a, L);
    } else {
      longmask |= 1u << i;
      nlong++;
    }
    bestA[u] = KEY_INF;
    bestB[u] = KEY_INF;
    parent[u] = (int32_t)u;
    cc[u] = (int32_t)u;
  }
  int total_long;
  int p = block_incl_scan<int, BS, false>(nlong, stmp, &total_long) - nlong;
  for (int i = 0; i < FD_PER; i++)
    if (longmask >> i & 1u) slong[p++] = (int32_t)(base + i * BS + tid);
  __syncthreads();
  for (int r = 0; r < total_long; r++) {
    int64_t u = slong[r];
    int64_t s = g.rp[u], e = g.rp[u + 1];
    Fx a{0, 0, 0};
    for (int64_t j = s + tid; j < e; j += BS) fx_add_value(a, fp_w(g, j), L);
#pragma unroll
    for (int c = 0; c < FP_LIMBS; c++) {
      uint64_t v = wave_sum<uint64_t>((uint64_t)fx_chunk(a, c));
      if (lane_id() == 0) schunk[tid / WAVE][c] = v;
    }
    __syncthreads();
    if (tid == 0) {
      uint64_t tot[FP_LIMBS];
#pragma unroll
      for (int c = 0; c < FP_LIMBS; c++) {
        tot[c] = 0;
        for (int w = 0; w < BS / WAVE; w++) tot[c] += schunk[w][c];
      }
      Fx x = fx_from_chunks(tot, 1, 0);
      if (g.self) fx_add_value(x, g.self[u], L);
      deg[u] = fx_round(x, L);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// A2: FP64 scores, one thread per edge (u < v), 4 edges per thread, tiles
// of consecutive edge ids mapped to rows through the upper-entry prefix
// ---------------------------------------------------------------------------
constexpr int FS_TILE = 1024;

__device__ __forceinline__ double fp_min(double p, double q) { return p < q ? p : q; }

__global__ void __launch_bounds__(BS)
    k_fp_score(LevelInF g, const double* __restrict__ deg, const int32_t* __restrict__ lc,
               const int64_t* __restrict__ uptr, int64_t m, KeyFD* __restrict__ keys) {
  __shared__ int32_t srow[Lbs<FS_TILE, BS>::SIZE];
  __shared__ int64_t sh[2];
  __shared__ int32_t stmp[BS / WAVE];
  int64_t e0 = (int64_t)blockIdx.x * FS_TILE;
  lbs_tile<FS_TILE, BS>(uptr, g.n, e0, srow, sh, stmp);
  for (int it = 0; it < FS_TILE / BS; it++) {
    int k = threadIdx.x + it * BS;
    int64_t e = e0 + k;
    if (e >= m) break;
    int32_t u = srow[Lbs<FS_TILE, BS>::at(k)];
    int64_t j = g.rp[u] + lc[u] + (e - uptr[u]);
    int32_t v = g.col[j];
    double wuv = fp_w(g, j);
    double du = deg[u], dv = deg[v];
    double su = g.self ? g.self[u] : 0.0, sv = g.self ? g.self[v] : 0.0;
    bool doneU = !(su > 0.0), doneV = !(sv > 0.0);
    int64_t a = g.rp[u], ae = g.rp[u + 1], b = g.rp[v], be = g.rp[v + 1];
    double t = 0.0;
    while (true) {
      // next common neighbour in ascending order (INT32_MAX: none left)
      int32_t xc = INT32_MAX;
      double wa = 0.0, wb = 0.0;
      while (a < ae && b < be) {
        int32_t x = g.col[a], y = g.col[b];
        if (x < y) a++;
        else if (x > y) b++;
        else {
          xc = x;
          wa = fp_w(g, a);
          wb = fp_w(g, b);
          a++;
          b++;
          break;
        }
      }
      // the diagonal positions take their place in the ascending order
      if (!doneU && u < xc) {   // x = u: a_uu = self_u, a_vu = w_uv
        t = t + fp_min(su / du, wuv / dv);
        doneU = true;
      }
      if (!doneV && v < xc) {   // x = v: a_uv = w_uv, a_vv = self_v
        t = t + fp_min(wuv / du, sv / dv);
        doneV = true;
      }
      if (xc == INT32_MAX) break;
      t = t + fp_min(wa / du, wb / dv);
    }
    keys[e] = KeyFD{2.0 - 2.0 * t, (uint64_t)e};
  }
}

__global__ void k_fd_scatter(const KeyFD* __restrict__ sorted, int64_t m, uint64_t* __restrict__ P) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < m) P[sorted[r].e] = (uint64_t)r;
}

__global__ void k_fp_eps(const KeyFD* __restrict__ sorted, const unsigned long long* msf,
                         const SelState* st, double* out) {
  if (*msf == 0) return;
  *out = sorted[st->prefix].s;
}

// ---------------------------------------------------------------------------
// A5: exact coarse sums.  The coarse structure comes from the integer
// contraction run on unit weights; every fine entry then adds its weight to
// its coarse entry (binary search in the coarse row) or to its super-node's
// self-loop, as 32-bit chunks of the fixed-point value.  A block first
// combines equal targets in an LDS table, so a giant super-node's self-loop
// costs a few global atomics per block.
// ---------------------------------------------------------------------------
__global__ void k_fill_ones(int32_t* __restrict__ a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 1;
}

constexpr int SC_T = 512;          // fine entries per block
constexpr int SC_SLOTS = 1024;     // LDS table slots (load factor <= 1/2)

__global__ void __launch_bounds__(BS)
    k_fp_scatter(LevelInF g, const int32_t* __restrict__ c, const int64_t* __restrict__ rpc,
                 const int32_t* __restrict__ colc, int64_t nnz_c, int32_t* __restrict__ emap,
                 uint64_t* acc, uint64_t* selfacc, int64_t n_c, const unsigned long long* info) {
  __shared__ int32_t srow[Lbs<SC_T, BS>::SIZE];
  __shared__ int64_t sh[2];
  __shared__ int32_t stmp[BS / WAVE];
  __shared__ unsigned long long skey[SC_SLOTS];   // ~0: empty
  __shared__ unsigned long long ssum[FP_LIMBS][SC_SLOTS];
  int tid = threadIdx.x;
  int L = fp_level_L(info);
  int64_t j0 = (int64_t)blockIdx.x * SC_T;
  for (int s = tid; s < SC_SLOTS; s += BS) {
    skey[s] = ~0ull;
#pragma unroll
    for (int q = 0; q < FP_LIMBS; q++) ssum[q][s] = 0;
  }
  lbs_tile<SC_T, BS>(g.rp, g.n, j0, srow, sh, stmp);   // synchronises
  for (int it = 0; it < SC_T / BS; it++) {
    int k = tid + it * BS;
    int64_t j = j0 + k;
    if (j >= g.nnz) break;
    int32_t x = srow[Lbs<SC_T, BS>::at(k)];
    int32_t a = c[x], b = c[g.col[j]];
    unsigned long long key;
    if (a == b) {
      key = (unsigned long long)(nnz_c + a);
      emap[j] = -1 - a;
    } else {
      int64_t lo = rpc[a], hi = rpc[a + 1];
      while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (colc[mid] < b) lo = mid + 1;
        else hi = mid;
      }
      key = (unsigned long long)lo;
      emap[j] = (int32_t)lo;
    }
    double v = fp_w(g, j);
    uint64_t mant;
    int lsb;
    fp_split(v, mant, lsb);
    Fx f = fx_of(mant, lsb - L);
    uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 54) & (SC_SLOTS - 1);
    while (true) {
      unsigned long long old = atomicCAS(&skey[h], ~0ull, key);
      if (old == ~0ull || old == key) break;
      h = (h + 1) & (SC_SLOTS - 1);
    }
#pragma unroll
    for (int q = 0; q < FP_LIMBS; q++) {
      uint32_t ch = fx_chunk(f, q);
      if (ch) atomicAdd(&ssum[q][h], (unsigned long long)ch);
    }
  }
  __syncthreads();
  for (int s = tid; s < SC_SLOTS; s += BS) {
    unsigned long long key = skey[s];
    if (key == ~0ull) continue;
    bool cross = (int64_t)key < nnz_c;
    uint64_t* dst = cross ? acc : selfacc;
    int64_t idx = cross ? (int64_t)key : (int64_t)key - nnz_c;
    int64_t stride = cross ? nnz_c : n_c;
#pragma unroll
    for (int q = 0; q < FP_LIMBS; q++) {
      unsigned long long v = ssum[q][s];
      if (v) atomicAdd((unsigned long long*)&dst[q * stride + idx], v);
    }
  }
}

// members' own self-loops into their super-node's (runs of one super-node
// in a wavefront add once)
__global__ void k_fp_self_scatter(LevelInF g, const int32_t* __restrict__ c, uint64_t* selfacc, int64_t n_c,
                                  const unsigned long long* info) {
  int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int L = fp_level_L(info);
  bool valid = x < g.n;
  int32_t a = valid ? c[x] : -1;
  double v = valid ? g.self[x] : 0.0;
  Fx f{0, 0, 0};
  fx_add_value(f, v, L);
  bool head;
  int end;
  uint64_t heads;
  int l = lane_id();
  int32_t prev = __shfl_up(a, 1);
  head = (l == 0) || (a != prev);
  heads = __ballot(head);
  uint64_t after = (l == WAVE - 1) ? 0ull : (heads & (~0ull << (l + 1)));
  end = after ? (__ffsll((long long)after) - 1) : WAVE;
#pragma unroll
  for (int q = 0; q < FP_LIMBS; q++) {
    uint64_t ch = fx_chunk(f, q);
    uint64_t inc = wave_incl_sum<uint64_t>(ch);
    uint64_t at_end = __shfl(inc, end - 1);
    uint64_t run = at_end - inc + ch;
    if (head && a >= 0 && run) atomicAdd((unsigned long long*)&selfacc[q * n_c + a], (unsigned long long)run);
  }
}

__global__ void k_fp_finalize(const uint64_t* __restrict__ acc, int64_t nnz_c, const uint64_t* __restrict__ selfacc,
                              int64_t n_c, double* __restrict__ w_c, double* __restrict__ self_c,
                              const unsigned long long* info) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int L = fp_level_L(info);
  if (i < nnz_c) w_c[i] = fx_round(fx_from_chunks(acc, nnz_c, i), L);
  else if (i < nnz_c + n_c) self_c[i - nnz_c] = fx_round(fx_from_chunks(selfacc, n_c, i - nnz_c), L);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
void launch_fp_degree(spc_ctx* ctx, const LevelInF& g, LevelWork& W) {
  hipStream_t st = ctx->stream;
  hipLaunchKernelGGL(k_fp_range_init, dim3(1), dim3(1), 0, st, W.info);
  hipLaunchKernelGGL(k_fp_range, dim3(grid_for(g.nnz + g.n, BS * 8, ctx->num_cus * 8)), dim3(BS), 0, st, g,
                     W.info);
  hipLaunchKernelGGL(k_fp_span, dim3(1), dim3(1), 0, st, W.info);
  hipLaunchKernelGGL(k_fp_degree, dim3(grid_for(g.n, FD_ROWS)), dim3(BS), 0, st, g, (double*)W.deg, W.lc,
                     W.uptr, W.bestA, W.bestB, W.parent, W.root, W.info);
}

int fp_rank_keys(spc_ctx* ctx, const LevelInF& g, LevelWork& W, int64_t m) {
  hipStream_t st = ctx->stream;
  KeyFD* A = (KeyFD*)W.keysA;
  KeyFD* B = (KeyFD*)W.keysB;
  {
    TimedScope ts(ctx, "score_fp", (double)m);
    hipLaunchKernelGGL(k_fp_score, dim3(grid_for(m, FS_TILE)), dim3(BS), 0, st, g, (const double*)W.deg,
                       W.lc, W.uptr, m, A);
  }
  SPC_LAUNCH_CHECK(ctx, "fp score");
  KeyFD* sorted = nullptr;
  {
    TimedScope ts(ctx, "rank_sort", (double)m);
    int rc = merge_sort<KeyFD, LessFD>(ctx, A, B, m, LessFD(), &sorted);
    if (rc) return rc;
  }
  W.fd_sorted = sorted;
  TimedScope ts(ctx, "rank_scatter", (double)m);
  hipLaunchKernelGGL(k_fd_scatter, dim3(grid_for(m, 256)), dim3(256), 0, st, sorted, m, W.P);
  LevelIn gs{g.n, g.nnz, g.rp, g.col, nullptr, nullptr, g.size};
  launch_rank_mirror(ctx, gs, W, m);
  SPC_LAUNCH_CHECK(ctx, "fp rank scatter");
  return SPC_OK;
}

void launch_eps_fp(spc_ctx* ctx, LevelWork& W) {
  hipLaunchKernelGGL(k_fp_eps, dim3(1), dim3(1), 0, ctx->stream, W.fd_sorted, &W.info[I_MSF], W.sel2,
                     (double*)&W.info[I_EPS]);
}

int contract_level_fp(spc_ctx* ctx, const LevelInF& g, const int32_t* c, int64_t n_c, spc_graph_out* out,
                      LevelWork& W, LevelResult& R) {
  hipStream_t st = ctx->stream;
  // structure: the integer contraction on unit weights (weights into scratch)
  hipLaunchKernelGGL(k_fill_ones, dim3(grid_for(g.nnz, 256)), dim3(256), 0, st, W.ones, g.nnz);
  LevelIn gs{g.n, g.nnz, g.rp, g.col, W.ones, nullptr, g.size};
  spc_graph_out so = *out;
  so.w = W.wtmp;
  so.self_w = W.selftmp;
  int rc = contract_level(ctx, gs, c, n_c, &so, W, R);
  if (rc) return rc;
  int64_t nnz_c = R.nnz_c;
  TimedScope ts(ctx, "contract_fp_sums", (double)g.nnz);
  launch_zero(ctx, W.acc, sizeof(uint64_t) * (size_t)(FP_LIMBS * std::max<int64_t>(nnz_c, 1)));
  launch_zero(ctx, W.selfacc, sizeof(uint64_t) * (size_t)(FP_LIMBS * n_c));
  if (g.nnz > 0)
    hipLaunchKernelGGL(k_fp_scatter, dim3(grid_for(g.nnz, SC_T)), dim3(BS), 0, st, g, c, out->row_ptr,
                       out->col, nnz_c, W.emap, W.acc, W.selfacc, n_c, W.info);
  if (g.self)
    hipLaunchKernelGGL(k_fp_self_scatter, dim3(grid_for(g.n, 256)), dim3(256), 0, st, g, c, W.selfacc, n_c,
                       W.info);
  hipLaunchKernelGGL(k_fp_finalize, dim3(grid_for(nnz_c + n_c, 256)), dim3(256), 0, st, W.acc, nnz_c,
                     W.selfacc, n_c, (double*)out->w, (double*)out->self_w, W.info);
  SPC_LAUNCH_CHECK(ctx, "fp contraction sums");
  return SPC_OK;
}

}  // namespace spc

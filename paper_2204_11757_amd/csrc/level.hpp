// One coarsening level: shared types between the selection kernels
// (degrees, scores, order, merge selection) and the contraction kernels.
#pragma once

#include "prim.hpp"


// Hierarchy produced by spc_coarsen_to: level l (1-based) holds the coarse
// graph after l levels and the map from level l-1 nodes to its super-nodes.
struct spc_hier {
  spc_ctx* ctx = nullptr;
  int64_t n0 = 0;
  // batched hierarchies: node offsets of the batch's graphs at every level
  // (entry 0: the input); empty for a single graph
  std::vector<std::vector<int64_t>> goff;
  struct Level {
    int64_t n = 0, nnz = 0, n_prev = 0;
    int64_t* rp = nullptr;
    int32_t* col = nullptr;
    void* w = nullptr;        // int32 (integer path) or double (floating-point path)
    void* self = nullptr;     // int64 or double
    int32_t* size = nullptr;
    int32_t* cluster_of = nullptr;
    spc_wtype wtype = SPC_W_I32;
    spc_level_stats st{};
    void* block = nullptr;    // the one allocation the arrays above live in
    hipEvent_t ev[2] = {nullptr, nullptr};   // level timing, read once the hierarchy is built
  };
  std::vector<Level> levels;
  // the levels' timing events are read (a wait for the last level) when
  // stats are first asked for, so a call returns once its work is queued
  bool timing_pending = false;
};

namespace spc {

constexpr int BS = 256;   // block size of the selection kernels
// Rows longer than HUGE_T are registered by the degree pass; the first H_MAX
// of them get a dense column -> position map, so the score of each of their
// edges looks columns up instead of searching the long row.
constexpr int HUGE_T = 1024;
constexpr int H_MAX = 4;
// edges per tile of the score kernel (three per thread)
constexpr int SCORE_TILE = 768;
// CSR entries per tile of the row pass and of the contraction's record scatter
constexpr int ENTRY_TILE = 2048;

// Device view of an integer-path input graph.
struct LevelIn {
  int64_t n, nnz;
  const int64_t* rp;
  const int32_t* col;
  const int32_t* w;
  const int64_t* self;   // nullable
  const int32_t* size;   // nullable
};

// Device view of a floating-point input graph: FP32 weights (an input
// level) or FP64 weights (coarse levels), FP64 self-loops.
struct LevelInF {
  int64_t n, nnz;
  const int64_t* rp;
  const int32_t* col;
  const void* w;
  int w32;               // 1: w is float[nnz], 0: double[nnz]
  const double* self;    // nullable
  const int32_t* size;   // nullable
};

// Sort record of the floating-point order: FP64 score, ties by edge index.
struct KeyFD {
  double s;
  uint64_t e;
};

struct LessFD {
  __device__ __forceinline__ bool operator()(const KeyFD& a, const KeyFD& b) const {
    return a.s < b.s || (a.s == b.s && a.e < b.e);
  }
};

// A batch of independent graphs coarsened as one block-diagonal graph:
// graph i owns nodes [off[i], off[i+1]) and needs k[i] merges this level.
// Device arrays.
struct Segments {
  int64_t G;
  const int64_t* off;   // [G + 1] node ranges of the graphs
  const int64_t* k;     // [G] merges per graph
  const int64_t* coff;  // [G + 1] the graphs' coarse node ranges after the level
  int64_t wmax;         // largest coarse range
};

// Exact sort key of the rank-mode order: score N / D, ties by edge index.
struct KeyND {
  uint64_t N, D, e;
};

// bit e of the exactness map (set by the score pass for edges whose packed
// key was computed without remainder)
__device__ __forceinline__ bool key_exact(const uint64_t* __restrict__ kexact, uint64_t e) {
  return (kexact[e >> 6] >> (e & 63)) & 1ull;
}

__device__ __forceinline__ bool exact_less(const KeyND& x, const KeyND& y) {
  return (unsigned __int128)x.N * y.D < (unsigned __int128)y.N * x.D;
}

struct LessND {
  __device__ __forceinline__ bool operator()(const KeyND& a, const KeyND& b) const {
    unsigned __int128 l = (unsigned __int128)a.N * b.D;
    unsigned __int128 r = (unsigned __int128)b.N * a.D;
    if (l != r) return l < r;
    return a.e < b.e;
  }
};

// Indices into the per-level device info block.
enum Info : int {
  I_DMAX = 0,
  I_TOTAL = 1,
  I_LIVE0 = 2,
  I_LIVE1 = 3,
  I_MSF = 4,
  I_MID = 5,
  I_HUGE = 6,
  I_LONGROW = 7,  // rows longer than HUGE_T (the first H_MAX get a position map)
  I_BAD = 8,
  I_NC = 9,
  I_MAXCL = 10,
  I_EPS = 11,
  I_DMAXE = 12,   // largest D = d_u d_v over edges
  I_VIOL = 13,    // a guarded-key decision was not exact
  I_BLOCK = 14,   // contraction rows for the block-per-row class
  I_R32 = 15,     // contraction rows for the 32-entry register class
  I_LBERR = 16,   // a look-back wait gave up (internal error)
  I_GUARD = 17,   // packed keys are guarded (not exact for every pair)
  I_ROUNDS = 18,  // spanning-forest rounds that merged something
  I_FIN = 19,     // live edges read by root-lookup rounds
  I_FKEPT = 20,   // live edges kept by root-lookup rounds
  I_MIN = 21,     // live edges read by hooking rounds
  I_KEYS = 22,    // exact per-edge records were written
  I_MSF0 = 23,    // forest records before the current hooking round
  I_FP_LMIN = 24, // floating-point path: smallest weight ulp exponent + FP_EBIAS
  I_FP_HMAX = 25, // floating-point path: largest weight exponent + FP_EBIAS
  I_FP_BAD = 26,  // floating-point path: a weight is not finite / not positive
  I_SEG_SHORT = 27, // batch: a graph has fewer forest edges than merges needed
  I_CAND = 28,    // live edges the band's row pass produced (a copy of I_LIVE0)
  I_DENSE = 29,   // a dense row accumulator index fell outside its window (internal error)
  I_HOVER = 30,   // more huge contraction rows than the path without a host wait takes
  I_SPEC = 31,    // live edges left after the first forest batch (checked later when not waited for)
  I_NINFO = 32
};

// Block-wide reservation of `my` consecutive slots per thread behind a
// global counter with one atomic per block.  All BS threads must call it.
// tmp: LDS int[BS/64]; sh_base: LDS scalar.
template <int BS>
__device__ __forceinline__ int64_t block_reserve(unsigned long long* counter, int my,
                                                 unsigned long long* sh_base, int* tmp) {
  int total;
  int incl = block_incl_scan<int, BS, false>(my, tmp, &total);
  if (threadIdx.x == 0) *sh_base = total ? atomicAdd(counter, (unsigned long long)total) : 0ull;
  __syncthreads();
  int64_t base = (int64_t)*sh_base + (incl - my);
  __syncthreads();
  return base;
}

struct LevelWork {
  unsigned long long* info;  // [I_NINFO]
  uint64_t* lbstate;         // look-back words, lb_words(n, nnz)
  uint64_t* deg;             // [n]
  uint64_t* degpart;         // [n / 4096 + 2] per-block weight sums
  int32_t* lc;               // [n]  entries with col < row
  int64_t* uptr;             // [n+1] upper-edge prefix (edge ids)
  int32_t* trow;             // [m / SCORE_TILE + 2] row holding each score tile's first edge
  int32_t* ptrow;            // [nnz / ENTRY_TILE + 2] row holding each entry tile's first entry
                             // (both written by the integer degree pass)
  int32_t* gid;              // [n] batch: each node's graph
  uint64_t* thrg;            // [n] batch: each graph's band threshold (at most n graphs)
  uint64_t* P;               // [m]  order key per edge (sorted-rank order)
  uint64_t* Pc;              // [nnz] order key per CSR entry (both directions)
  uint64_t* samples;         // [m/64 + 2], keys of edges 0, s, 2s, ... (s = 2^sample_shift(m))
  uint64_t* kexact;          // [m/64 + 2] bit e: edge e's packed key has no remainder
  uint64_t* bestA;           // [n]
  uint64_t* bestB;           // [n]
  int32_t* parent;           // [n]
  uint64_t* lr[2];           // [m] live edges: current roots (lo | hi << 32)
  uint64_t* lp[2];           // [m] live edges: key
  uint64_t* lo[2];           // [m] live edges: original endpoints
  uint64_t* msfP;            // [n]
  uint64_t* msfO;            // [n]
  int32_t* msfC;             // [n]  root hooked by each forest edge
  int32_t* root;             // [n] union-find of the merge cutoff's components
  int32_t* flag;             // [n+1]
  SelState* sel;
  SelState* sel2;
  uint64_t* selflag;         // [SEL_MAXB * SEL_FLAG] radix-select barrier flags
  void* scan_partial;        // SCAN_MAXB * 8 bytes
  KeyND* keysA;              // [m] rank mode
  KeyND* keysB;              // [m]
  // contraction
  int32_t* mcount;           // [n+1]
  int32_t* mptr;             // [n+1]
  int32_t* members;          // [n]
  int64_t* gptr;             // [n+1] super-node record counts, then their prefix
  uint64_t* temp;            // [nnz + n] records grouped by super-node, reduced in place
  int64_t* cnt;              // [n+1]
  int32_t* r32list;          // [n]
  int32_t* midlist;          // [n]
  int32_t* blocklist;        // [n]
  int32_t* hugelist;         // [n]
  int64_t* hmoff;            // [n+1] record prefix over the huge rows
  int32_t* hmrow;            // [n]  sort path: each huge row's first head rank
  int32_t* hmnode;           // [n]  sort path: last head rank; batches: graph base per huge row
  int64_t* hpos;             // [n+1] fine node -> its first slot in its super-node's records
  int64_t* hmrs;             // [n]  members per huge row
  int32_t* htab;             // [H_MAX] rows longer than HUGE_T, in registration order
  int32_t* hmap;             // [H_MAX * n] per such row: column -> position in the row
  uint64_t* gkeyA;           // [nnz] (key, w) pairs, 16 bytes each
  uint64_t* gkeyB;           // [nnz]
  // floating-point path only (null on the integer path)
  int32_t* ones;             // [nnz]  unit weights for the structure pass
  int32_t* wtmp;             // [nnz]  structure pass's integer coarse weights
  int64_t* selftmp;          // [n]
  uint64_t* acc;             // [FP_LIMBS * nnz] coarse entry sums, 32-bit limbs
  uint64_t* selfacc;         // [FP_LIMBS * n]
  int32_t* emap;             // [nnz]  fine entry -> coarse entry (>= 0) or -1 - self node
  KeyFD* fd_sorted;          // sorted FP order records (points into keysA or keysB)
};

constexpr int FP_LIMBS = 6;     // 192-bit fixed point in 32-bit limbs
constexpr int FP_EBIAS = 4096;  // bias of the exponents kept in the info block
// FP sums: every weight of a level is an integer multiple of 2^L (L the
// smallest ulp exponent among them) and below 2^(H+1) (H the largest
// exponent); a sum of at most 2^31 of them in units of 2^L stays below
// 2^(H - L + 32), inside the 192-bit fixed point when H - L <= 159.
constexpr int FP_MAX_SPAN = 192 - 33;

// look-back words a level needs: the most tiles any compaction launch uses
// Edges between two key samples: 64, or more so that at most about 4096
// samples (one block's in-LDS selection) pick a band's threshold.
inline int sample_shift(int64_t m) {
  int s = 6;
  while ((m >> s) > 4096) s++;
  return s;
}

inline int64_t lb_words(int64_t n, int64_t nnz) { return nnz / 1024 + 4 * (n / 256) + 4096; }

void plan_level(Arena& A, int64_t n, int64_t nnz, LevelWork& W, bool fp = false);

// A fresh look-back chain for one launch, words from `off` of the level's
// array; the array is zeroed again when the epochs run out.
inline TileScan next_scan(spc_ctx* ctx, const LevelWork& W, int64_t off = 0) {
  if (ctx->lb_epoch >= LB_MAX_EPOCH) {
    launch_zero(ctx, W.lbstate, sizeof(uint64_t) * (size_t)ctx->lb_words);
    ctx->lb_epoch = 0;
  }
  return TileScan{W.lbstate + off, ++ctx->lb_epoch, &W.info[I_LBERR]};
}

struct LevelResult {
  int64_t n_c = 0, nnz_c = 0, msf = 0, rounds = 0, candidates = 0, maxcl = 0;
  int key_mode = 0, key_bits = 0, bands = 0, keys_written = 0;
  int64_t forest_in = 0, forest_kept = 0, merge_in = 0;
  double eps = 0.0;
  // the selection's checks wait for the contraction's first synchronisation
  // (n_c is the target until then); rank: the labels came from rank keys
  bool pending = false, pending_rank = false;
  // spec: the host did not wait for the first forest batch (the forest was
  // assumed complete, with at least k edges); checked with the others
  bool spec = false;
  int64_t k = 0;       // merges of the level
  bool first_batch_complete = false;
  // the selection zeroed the contraction's member counts and gather prefix
  bool contract_zeroed = false;
  // a batch's forest was built over per-graph bands (not every edge)
  bool seg_band = false;
};

// internal return codes (never reach the caller): a guarded key decision
// failed after a deferred check, the level is redone with rank keys; the
// forest was not complete after its first batch (or had too few edges)
// although the host did not wait for it, the level is redone waiting
constexpr int SPC_REDO_RANK = 1;
constexpr int SPC_REDO_SPEC = 2;
// a graph of a batch had fewer forest edges inside its band than merges:
// the level is redone over every edge
constexpr int SPC_REDO_BAND = 3;

// A2 and A3 launches (score.hip).  mode 0: packed keys into Pc and the
// samples (exact records too when the key is not surely exact); mode 1:
// exact records only, for the sorted-rank order.
void launch_score(spc_ctx* ctx, const LevelIn& g, const LevelWork& W, int64_t m, int c, int ebits,
                  int mode);
// rank order: P from the sorted exact records, mirrored into Pc
void launch_rank_scatter(spc_ctx* ctx, const LevelIn& g, const LevelWork& W, int64_t m,
                         const KeyND* sorted);
// Pc from P (an edge's rank into both of its CSR entries)
void launch_rank_mirror(spc_ctx* ctx, const LevelIn& g, const LevelWork& W, int64_t m);
// cluster_of[x] = label of x's component root (W.parent, labels in W.flag,
// clamped to [0, t)); with eps, also info[I_EPS] = exact score of the forest
// edge whose key equals sel2's cutoff.  One launch.
void launch_relabel_eps(spc_ctx* ctx, const LevelIn& g, const LevelWork& W, int32_t* cluster_of, int64_t t,
                        int64_t msf_bound, bool eps);

// Floating-point path pieces (fp.hip).
// A1: validates the weights, records their exponent range, computes the
// degrees as correctly rounded exact sums (into W.deg as doubles) and the
// per-level initialisation of the integer path's k_degree.
void launch_fp_degree(spc_ctx* ctx, const LevelInF& g, LevelWork& W);
// A2 + A3: FP64 scores in the common-support form, sorted with ties by edge
// id, ranks scattered into P and Pc.
int fp_rank_keys(spc_ctx* ctx, const LevelInF& g, LevelWork& W, int64_t m);
// info[I_EPS] = score of the cutoff rank
void launch_eps_fp(spc_ctx* ctx, LevelWork& W);
// A5 with correctly rounded exact FP64 sums; also fills W.emap.
int contract_level_fp(spc_ctx* ctx, const LevelInF& g, const int32_t* cluster_of, int64_t n_c,
                      spc_graph_out* out, LevelWork& W, LevelResult& R);

// Batched merge cutoff (batch.hip): forest edges sorted by (graph, key);
// each graph's first k[i] are joined in `parent` (which must hold the
// identity); info[I_EPS] receives the largest accepted score, info[I_VIOL]
// a failed guarded decision, info[I_SEG_SHORT] a graph short of edges.
// Batch bands: gid[u] = u's graph, and each graph's band threshold: about
// 2 k_g of its edges (from a sorted sample of its keys; whole K buckets
// when keys are guarded; a tied bucket is extended to cover about 1.1 k_g
// rows).  shrink (a test option) aims at k_g / 4 instead.
int seg_bands(spc_ctx* ctx, const LevelIn& g, LevelWork& W, const Segments& seg, int ebits, bool shrink);
int seg_cutoff_union(spc_ctx* ctx, const LevelIn& g, LevelWork& W, const LevelResult& R,
                     const Segments& seg, int ebits, bool rank);

// Steps A1-A4: degrees, scores, order, merge selection -> cluster_of.  With
// gf the weights are floating point (g then carries the structure only);
// with seg the input is a batch and every graph has its own target.
// With defer, the host does not wait for the labels: R.pending is set and
// finish_select runs at the contraction's first synchronisation; with
// rank_only the level starts in rank-key mode.
// With speculate (only with defer) the host does not wait for the first
// forest batch either.
int select_level(spc_ctx* ctx, const LevelIn& g, int64_t t, int32_t* cluster_of, LevelWork& W,
                 LevelResult& R, const LevelInF* gf = nullptr, const Segments* seg = nullptr,
                 bool defer = false, bool rank_only = false, bool speculate = false);
// Checks and results of the selection from the host copy of the info block
// (super-node count in slot I_NINFO + 1): SPC_OK, an error, or
// SPC_REDO_RANK when packed keys took an inexact decision, SPC_REDO_SPEC
// when a forest the host did not wait for turned out incomplete.
int finish_select(spc_ctx* ctx, LevelResult& R, int64_t t, bool rank, bool fp, const Segments* seg);

// Step A5: contraction of Definition 1 into caller buffers.
// ptrow: the entry tiles' first rows of g (W.ptrow after the integer degree
// pass on g), or null to search for them.
int contract_level(spc_ctx* ctx, const LevelIn& g, const int32_t* cluster_of, int64_t n_c,
                   spc_graph_out* out, LevelWork& W, LevelResult& R, const Segments* seg = nullptr,
                   const int32_t* ptrow = nullptr);

}  // namespace spc

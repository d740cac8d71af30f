/*
 * spc.h -- C ABI of the MI355X (gfx950) spectrum-preserving graph
 * coarsening library (method of Brissette, Huang, Slota, "Parallel
 * coarsening of graph data with spectral guarantees", arXiv 2204.11757).
 *
 * Problem (introduction, before Definition 1): given a weighted graph
 * G = (V, E) with n nodes and a target n_c, merge nodes into n_c
 * super-nodes.  One level follows Algorithm 1: score every edge by the
 * 1-norm distance of the endpoints' normalised adjacency rows
 * (Theorem 1), order the edges by that score, and merge along edges in
 * that order, skipping edges whose ends already share a super-node, until
 * n_c super-nodes remain; then build the coarsened graph of Definition 1.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Graphs are symmetric CSR in DEVICE memory: row_ptr int64[n+1],
 * col int32[nnz] strictly ascending per row with no diagonal entry, and
 * weights w[nnz].  nnz = 2m counts both directions of each undirected edge.
 * A node's self-loop weight (the diagonal of the weighted adjacency; zero
 * on input graphs, the intra-cluster weight on coarse graphs) lives in
 * self_w[n]; size[n] counts the original nodes a super-node stands for.
 *
 * Weight types: SPC_W_I32 (integer path, exact: w int32 > 0, self_w
 * int64 >= 0, the total weight sum(w) + sum(self_w) at most 2^31 - 1), or
 * SPC_W_F32 / SPC_W_F64 (floating-point path: scores in FP64, self_w and
 * coarse weights in FP64; every weight and degree sum is the correctly
 * rounded value of the exact sum).
 *
 * Edge order: by score, then the smaller endpoint id, then the larger one.
 * Super-nodes are numbered by ascending smallest member.  Results are
 * bit-for-bit deterministic.
 *
 * All device pointers are caller-owned unless stated otherwise.  Calls are
 * ordered on the context's HIP stream; a call that returns host scalars
 * synchronises that stream before returning.  No C++ exception crosses
 * this boundary.  Return value: SPC_OK or a negative error code; the
 * detail of the last error is available from spc_last_error(ctx).
 */
#ifndef SPC_H
#define SPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPC_OK 0
#define SPC_EINVAL (-1)       /* bad argument or malformed graph            */
#define SPC_EUNREACHABLE (-2) /* target below the number of components      */
#define SPC_EOVERFLOW (-3)    /* integer weight total exceeds 2^31 - 1      */
#define SPC_ECAPACITY (-4)    /* a caller-provided output is too small      */
#define SPC_ENOMEM (-5)       /* device or host allocation failed           */
#define SPC_EHIP (-6)         /* a HIP runtime call failed                  */
#define SPC_ERANGE (-7)       /* FP weights span too wide an exponent range */

typedef struct spc_ctx spc_ctx;
typedef struct spc_hier spc_hier;

typedef enum { SPC_W_I32 = 0, SPC_W_F32 = 1, SPC_W_F64 = 2 } spc_wtype;

/* Input graph view (device pointers).  self_w is int64 on the integer path
 * and double on the floating-point path; self_w and size may be NULL
 * (all zero / all one). */
typedef struct {
  int64_t n, nnz;
  const int64_t* row_ptr;
  const int32_t* col;
  const void* w;
  const void* self_w;
  const int32_t* size;
  int32_t wtype;
} spc_graph;

/* Caller-allocated output graph (device pointers).  The coarse weight type
 * is int32 (integer path) or double (floating-point path); self_w is int64
 * or double.  Capacities equal to the input's n and nnz always suffice. */
typedef struct {
  int64_t* row_ptr;   /* [n_cap + 1] */
  int32_t* col;       /* [nnz_cap]   */
  void* w;            /* [nnz_cap]   */
  void* self_w;       /* [n_cap]     */
  int32_t* size;      /* [n_cap]     */
  int64_t n_cap, nnz_cap;
} spc_graph_out;

/* Per-level statistics (host struct, filled when non-NULL). */
typedef struct {
  int64_t n_in, m_in, n_out, nnz_out, merges, largest_cluster;
  int64_t boruvka_rounds;   /* spanning-forest rounds that merged something   */
  int64_t candidate_edges;  /* edges that entered the spanning-forest phase   */
  int32_t key_mode;   /* 0: exact packed fixed-point key, 1: sorted rank,
                         2: guarded packed key (checked, exact on success) */
  int32_t key_bits;
  double eps_max;     /* largest accepted score (Theorem 2's epsilon)    */
  float ms_total;
  int32_t bands;            /* candidate bands (row passes) used             */
  int64_t forest_in;        /* live edges read by the root-lookup rounds     */
  int64_t forest_kept;      /* live edges those rounds kept                  */
  int64_t merge_in;         /* live edges read by the hooking rounds         */
  int64_t forest_edges;     /* spanning-forest edges found                   */
  int32_t keys_written;     /* exact per-edge score records were written     */
} spc_level_stats;

/* Create a context on a device; hip_stream is a hipStream_t (NULL: the
 * null stream).  The context owns its workspace. */
int spc_create(spc_ctx** ctx, int device, void* hip_stream);
int spc_destroy(spc_ctx* ctx);
/* Make hip_stream the context's stream.  When it differs from the current
 * one, the new stream first waits (on the device, no host wait) for what
 * was queued on the old one, since that work still uses the context's
 * workspace. */
int spc_set_stream(spc_ctx* ctx, void* hip_stream);

/* Route the library's device allocations (workspace, hierarchy levels)
 * through caller-supplied functions, e.g. a framework's caching allocator.
 * alloc(bytes, user) returns a device pointer or NULL; free(ptr, user).
 * Passing NULL restores hipMalloc / hipFree. */
int spc_set_allocator(spc_ctx* ctx, void* (*alloc)(size_t, void*), void (*free_)(void*, void*),
                      void* user);

/* Context options (for tests and tuning; results never depend on them, but
 * "scan_flag" makes one level fail on purpose):
 *   "rank_order"  1: always order edges by a full sort into ranks, even when
 *                 the exact packed fixed-point key fits in 64 bits.
 *   "full_forest" 1: build the spanning forest over every edge instead of
 *                 only the lightest candidates.
 *   "huge_sort"   1: contract coarse rows above the block capacity by a
 *                 sort even when dense accumulators would fit.
 *   "redo_rank"   1: treat every packed-key level as if one of its guarded
 *                 decisions had failed, so that it is redone with rank keys
 *                 (the fallback path).
 *   "bad_select_guess" 1: give the merge cutoff's selection key bounds above
 *                 every forest key, so that the cutoff lies below them and the
 *                 selection starts over (its fallback path).
 *   "batch_band_short" 1: in a batch, each graph's merge-cutoff candidate
 *                 band aims at a quarter of that graph's merges, so that
 *                 bands fall short and the level is redone over every edge
 *                 (the batched selection's fallback path).
 *   "scan_flag"   1: the next level (once) finds the error flag of the
 *                 context's scan chain raised, as after a look-back wait that
 *                 gave up, and fails with SPC_EINVAL; later levels start with
 *                 the flag clear.
 *   "speculate"   whether the host waits for the first batch of spanning-
 *                 forest rounds: 0 (default) not when the previous level's
 *                 forest was complete after it, 1 always, 2 never (and that
 *                 batch is one round, so a longer forest takes the path that
 *                 redoes the level waiting).
 *   "contract_wait" how the contraction launches its row-class kernels:
 *                 0 (default) as the previous level's classes suggest, 1
 *                 always after reading the class counts on the host, 2
 *                 always on counts the kernels read from device memory
 *                 (when the huge rows' accumulators fit), 3 as 2 but with
 *                 no class kernel launched before the counts are read.
 *   "timing"      1: record a HIP event pair on the context stream around
 *                 every kernel launch, for spc_timing_report.
 *   Launch settings (0 = the tuned or built-in choice; a value fixes it for
 *   every later call): "lane_max" 16 or 32 (contraction rows of 17..lane_max
 *   records take one thread each, larger ones a wavefront), "wave_max"
 *   64..512 (rows up to it take a wavefront, larger ones a 256-thread
 *   block), "small_rpt" 1, 2 or 4 (rows per thread of the small-row pass),
 *   "huge_tile" 1024 or 4096 (records per tile of the dense huge rows),
 *   "sel_blocks" 1..128 (blocks of the radix select), "bv_short" (live
 *   lists up to this length use the 4-items-per-thread hooking pass).
 * Unknown names return SPC_EINVAL. */
int spc_set_option(spc_ctx* ctx, const char* name, int64_t value);

/* Per-kernel timing collected while the "timing" option was on, as text:
 * one line per kernel, "name launches total_ms work_units\n" (work units:
 * edges for edge-parallel kernels, nodes for node-parallel ones).  Clears
 * the collected events; synchronises the stream.  SPC_ECAPACITY if cap is
 * too small. */
int spc_timing_report(spc_ctx* ctx, char* buf, size_t cap);

/* Human-readable description of the last error on this context. */
const char* spc_last_error(const spc_ctx* ctx);
const char* spc_strerror(int code);

/* One level of Algorithm 1 (fitness loop, sort, merge loop) followed by
 * the contraction of Definition 1.
 *   g           input graph (device), validated for basic shape only.
 *   n_target    number of super-nodes; n_target >= n gives the identity.
 *   cluster_of  device int32[n]: super-node of every node (output).
 *   coarse      caller-allocated coarse graph (output), n_cap >= n_target,
 *               nnz_cap >= g->nnz.
 *   nnz_c       host: number of coarse CSR entries written.
 *   st          host stats or NULL.
 * Errors: SPC_EINVAL (bad sizes / null pointers / n_target < 1),
 * SPC_EUNREACHABLE, SPC_EOVERFLOW, SPC_ECAPACITY, SPC_EHIP, SPC_ENOMEM. */
int spc_coarsen_level(spc_ctx* ctx, const spc_graph* g, int64_t n_target, int32_t* cluster_of,
                      spc_graph_out* coarse, int64_t* nnz_c, spc_level_stats* st);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * level as spc_coarsen_level, computed in the library's own fixed scratch
 * array instead of an allocated workspace.  The call makes no allocation
 * (no hipMalloc, hipFree, allocator hook, event or pinned-memory
 * creation); the caller passes inputs and outputs as for
 * spc_coarsen_level, and st->ms_total is 0 (not timed).
 *   Scratch: SPC_NOALLOC_SCRATCH_BYTES per device, a static device array
 *   held from the library's load until the process ends, its address
 *   resolved once per device by spc_create.  The level needs about 100
 *   bytes per CSR entry plus 170 per node (FP weights: about 160 more per
 *   entry), so graphs up to roughly a million CSR entries fit; a larger one
 *   gets SPC_ECAPACITY with the bytes it would need.
 *   Every call on a device shares that device's array, which keeps the last
 *   call's contents (the level clears what must start at zero).  Calls that
 *   overlap on one device -- from two streams or two contexts on it --
 *   race on the array; calls ordered on one stream do not.
 * Errors: those of spc_coarsen_level, SPC_ECAPACITY for a graph too large
 * for the array, SPC_EHIP if the array's address could not be resolved. */
#define SPC_NOALLOC_SCRATCH_BYTES (134217728)
int spc_coarsen_level_noalloc(spc_ctx* ctx, const spc_graph* g, int64_t n_target, int32_t* cluster_of,
                              spc_graph_out* coarse, int64_t* nnz_c, spc_level_stats* st);

/* The graph under a node relabeling: node u becomes perm[u] (perm: device
 * int32[n], a permutation of [0, n)), so out's row perm[u] holds row u's
 * entries with their columns relabeled, ascending; self-loops and sizes
 * move with their nodes.  This is Definition 1's contraction with one
 * member per super-node.  Every score is unchanged (the measure of
 * Theorem 1 does not depend on node names), so coarsening the relabeled
 * graph changes only the tie-break of Algorithm 1's sort: equal scores
 * fall by (perm[u], perm[v]) instead of (u, v), and with a seeded random
 * perm the ties are broken by a seeded hash instead of the lowest ids.
 * out: capacities n and nnz; *nnz_out = nnz.  Weight types as the input's
 * (FP weights come out as FP64).  SPC_EINVAL if perm is not a permutation.
 * Waits for the permutation check. */
int spc_relabel(spc_ctx* ctx, const spc_graph* g, const int32_t* perm, spc_graph_out* out, int64_t* nnz_out);

/* Autotuner: times the call (spc_coarsen_to(g, n_c, schedule), or with
 * G > 0 spc_coarsen_batched(G, g, graph_off, n_c_graph, schedule)) under
 * launch settings chosen by coordinate descent -- contraction rows per
 * thread, thread- versus wavefront- versus block-per-row boundaries, dense
 * tile size, radix-select blocks, hooking-pass width; each setting in turn
 * with the others at their best so far, two runs each, a change kept when
 * it saves 2 percent -- and keeps the fastest for the input's size class
 * (bit length of nnz; batches apart).  Later calls on inputs of that class
 * use it.  Results never depend on these settings.  report (nullable):
 * the trials as text, "setting=value ms" per line.  Waits for every trial. */
int spc_autotune(spc_ctx* ctx, const spc_graph* g, int64_t n_c, int schedule, int32_t G, const int64_t* graph_off,
                 const int64_t* n_c_graph, char* report, size_t cap);

/* Coarsen to n_c super-nodes level by level, re-scoring each level (the
 * multilevel refinement the conclusion proposes).  schedule 0: halve the
 * node count per level, t = max(n_c, ceil(n_l / 2)); schedule 1: a single
 * level straight to n_c (Algorithm 1 as printed); schedule -j (j >= 1): j
 * merges per level, t = max(n_c, n_l - j), i.e. the scores are recomputed
 * after every j merges -- the re-scoring cadence of the conclusion, with
 * j = 1 the explicit greedy algorithm of the introduction, which recomputes
 * every norm after each merge.  Other values: SPC_EINVAL.  The hierarchy owns every
 * level's graph and cluster map; free it with spc_hier_free.  The call
 * returns once the last level's work is queued on the context's stream
 * (each level waits inside the call for its coarse size): read the arrays
 * in that stream's order. */
int spc_coarsen_to(spc_ctx* ctx, const spc_graph* g, int64_t n_c, int schedule, spc_hier** out);

/* Batched coarsening: G independent graphs packed block-diagonally in one
 * graph g (graph i owns nodes [graph_off[i], graph_off[i+1]) and only edges
 * among them; host int64[G+1]), each coarsened to its own n_c[i] (host
 * int64[G]) with the level schedule of spc_coarsen_to applied per graph.
 * Every graph's result equals what spc_coarsen_to gives for it alone (the
 * merge loop of Algorithm 1 runs per graph; the graphs only share the
 * launches).  Level l of the returned hierarchy is the packed union of the
 * graphs' level-l graphs (a graph already at its target is carried over
 * unchanged); spc_hier_graph_offsets gives each level's node offsets.
 * Integer weights only (SPC_W_I32).  SPC_EUNREACHABLE if some graph has
 * more connected components than its target. */
int spc_coarsen_batched(spc_ctx* ctx, int32_t G, const spc_graph* g, const int64_t* graph_off,
                        const int64_t* n_c, int schedule, spc_hier** out);
/* Node offsets (host int64[G+1], cap >= G+1) of a batched hierarchy's
 * graphs at level lvl (0 = the input).  SPC_EINVAL for a hierarchy that
 * does not come from spc_coarsen_batched. */
int spc_hier_graph_offsets(const spc_hier* h, int lvl, int64_t* off, int64_t cap);

int spc_hier_num_levels(const spc_hier* h);
/* Level lvl (1-based; level 0 is the input, not stored).  view receives
 * device pointers owned by the hierarchy; cluster_of maps level lvl-1
 * nodes to level lvl super-nodes.  stats may be NULL; the first request
 * for stats waits until the hierarchy's work has run (its level times are
 * read then). */
int spc_hier_level(const spc_hier* h, int lvl, spc_graph* view, const int32_t** cluster_of,
                   spc_level_stats* stats);
/* Copy level lvl (1-based) into caller-allocated device buffers, ordered on
 * the context's stream: the coarse graph into dst (capacities must hold
 * the level's n and nnz) and, when cluster_of is non-NULL, its cluster map
 * (int32[n of level lvl-1]). */
int spc_hier_export_level(spc_ctx* ctx, const spc_hier* h, int lvl, spc_graph_out* dst,
                          int32_t* cluster_of);
void spc_hier_free(spc_hier* h);

/* Lift (Definition 2) of k coarse vectors from level to_lvl down to level
 * from_lvl <= to_lvl (0 = the input graph).  x_c: device double[n_to * k],
 * column-major; x_f: device double[n_from * k].  c(u) is the level-to_lvl
 * super-node holding level-from_lvl node u (the cluster maps composed) and
 * s(.) the number of input nodes a node stands for (its size).
 * mode 0: piecewise constant, x_f[u] = x_c[c(u)];
 * mode 1: orthonormal, x_f[u] = x_c[c(u)] / sqrt(s(c(u)) / s(u)): the
 * coordinates, in level from_lvl's orthonormal basis, of the orthonormal
 * lift Q = B S^-1/2 (B the input-node membership matrix, S = diag(s)).
 * From level 0 this is x_c[c(u)] / sqrt(s(c(u))); the columns of the map
 * are orthonormal, and lifting to_lvl -> from_lvl -> 0 equals lifting
 * to_lvl -> 0.  Stream-ordered.  SPC_EINVAL unless 0 <= from_lvl <= to_lvl
 * <= levels. */
int spc_lift(spc_ctx* ctx, const spc_hier* h, int from_lvl, int to_lvl, int mode,
             const double* x_c, int k, double* x_f);

/* Spectral error of level lvl's lift against k eigenpairs of the input
 * graph's normalised Laplacian (Theorem 1's Lambda; the lift of
 * Definition 2).  prec (SPC_W_F64 or SPC_W_F32) is the type of U, R and
 * every intermediate: U device prec[n0 * k] column-major, unit-norm
 * eigenvectors; lambda: device double[k].  For each i, with Q the
 * orthonormal lift, t = D_c^{-1/2} Q^T u_i, R_i = 1 - t^T W_c t (the lift's
 * Rayleigh quotient at u_i; W_c includes the self-loops).  Writes R
 * (device prec[k], nullable) and the host scalar
 * loss = sum_i (R_i - lambda_i)^2 (summed in double).  Synchronises.
 * SPC_EINVAL for another prec. */
int spc_spectral_error(spc_ctx* ctx, const spc_hier* h, int lvl, const void* U,
                       const double* lambda, int k, int prec, void* R, double* loss);

/* Composed cluster map of level lvl: cmap[x] (device int32[n0]) is the
 * level-lvl super-node holding input node x (lvl = 0: the identity). */
int spc_hier_cluster_map(spc_ctx* ctx, const spc_hier* h, int lvl, int32_t* cmap);

/* Spectral error (as spc_spectral_error) of an explicit coarse graph, e.g.
 * one whose FP64 weights are being refined after coarsening.  coarse:
 * device graph with SPC_W_I32 or SPC_W_F64 weights, its size[] the number
 * of input nodes per super-node; cmap: device int32[n0], input node ->
 * super-node of coarse.  prec, U and R as for spc_spectral_error.  Writes R
 * (nullable) and the host loss.  Synchronises. */
int spc_spectral_error_graph(spc_ctx* ctx, const spc_graph* coarse, const int32_t* cmap, int64_t n0,
                             const void* U, const double* lambda, int k, int prec, void* R, double* loss);

/* Gradient of that loss with respect to the coarse weights, computed in
 * prec (SPC_W_F64 or SPC_W_F32, also the type of U, d_wc and d_selfc).
 * The weight of an undirected coarse edge {a, b} is one parameter held at
 * both CSR entries (a, b) and (b, a); d_wc[j] (device prec[nnz]) receives
 * d loss / d w_ab at both of them, so a step that updates both entries
 * alike keeps the graph symmetric.  d_selfc (device prec[n_c]) receives
 * d loss / d self_w[a].  With z = W_c t:
 *   d(t^T W_c t)/d w_ab   = 2 t_a t_b - t_a z_a / d_a - t_b z_b / d_b,
 *   d(t^T W_c t)/d self_a = t_a^2 - t_a z_a / d_a,
 * and d loss / d(t_i^T W_c t_i) = -2 (R_i - lambda_i).  Stream-ordered. */
int spc_spectral_error_backward(spc_ctx* ctx, const spc_graph* coarse, const int32_t* cmap, int64_t n0,
                                const void* U, const double* lambda, int k, int prec, void* d_wc,
                                void* d_selfc);

/* Entry map of a contraction (Definition 1): for every fine CSR entry j of
 * `fine` (device int32[nnz]), the position of its coarse entry
 * (c(x), c(y)) in `coarse`, or -1 - c(x) when c(x) = c(y) (the entry adds
 * to that super-node's self-loop).  Stream-ordered. */
int spc_entry_map(spc_ctx* ctx, const spc_graph* fine, const int32_t* cluster_of,
                  const spc_graph* coarse, int32_t* entry_map);

/* Adjoint of the contraction of Definition 1 (coarse weights are sums of
 * fine weights, so their adjoint is a gather): d_wf[j] = d_wc[map[j]] or
 * d_selfc[-1 - map[j]]; when d_selff is non-NULL, d_selff[x] =
 * d_selfc[cluster_of[x]] (fine self-loops add to their super-node's).
 * All device double arrays.  Stream-ordered. */
int spc_contract_backward(spc_ctx* ctx, const int32_t* entry_map, const int32_t* cluster_of,
                          int64_t nnz_f, int64_t n_f, const double* d_wc, const double* d_selfc,
                          double* d_wf, double* d_selff);

/* Host-side structural validation of a graph held in HOST memory: sorted
 * unique columns, no diagonal entries, symmetric weights, positive
 * weights, and the integer total bound.  No GPU needed. */
int spc_validate_graph(const spc_graph* host_view);

#ifdef __cplusplus
}
#endif
#endif /* SPC_H */

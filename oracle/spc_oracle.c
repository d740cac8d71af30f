/*
 * Serial CPU oracle for spectrum-preserving graph coarsening
 * (Brissette, Huang, Slota: "Parallel coarsening of graph data with
 * spectral guarantees", arXiv 2204.11757).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, plain, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the package smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header or helper with the GPU library.
 *
 * Every loop below runs serially, in the order the paper states, with no
 * blocking, fusion or reordering.  Build: gcc -O2 -ffp-contract=off.
 *
 * Graph layout (both paths): symmetric CSR, row_ptr int64[n+1], col int32
 * ascending per row with no diagonal entries, weights w per entry, an
 * optional per-node self-loop weight self_w (the diagonal of the weighted
 * adjacency, nonzero on coarse graphs) and an optional per-node size (the
 * number of original nodes a super-node stands for).
 *
 * Readings of the paper that this file fixes:
 *  - w_x is node x's full weighted adjacency row, diagonal included, and
 *    d_x is its row sum (Theorem 1 and the notation following it).
 *  - The coarsened graph keeps the intra-cluster weight as a self-loop
 *    (Definition 1 lets the neighbour range over every node, including
 *    members of the same super-node).
 *  - Algorithm 1's merge loop runs while the super-node count exceeds the
 *    target, walks the sorted fitness list in order, and skips an edge
 *    whose ends are already merged (its running time is stated as
 *    O(n - n_c) merges).  Ties in the sort are broken by the smaller
 *    endpoint, then the larger one.
 *
 * Return codes: 0 ok, -1 invalid input, -2 target unreachable, -3 integer
 * weight total too large for exact 64-bit arithmetic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_EUNREACHABLE (-2)
#define OR_EOVERFLOW (-3)
#define OR_ENOMEM (-5)

/* ======================================================================
 * Exact sums of non-negative doubles.
 *
 * A fixed-point accumulator with 64-bit limbs: bit b of the accumulator has
 * value 2^(b - XBIAS).  Every finite double is an integer multiple of
 * 2^-1074 below 2^1024, so the sum is exact; rounding to double happens
 * once, to nearest with ties to even.  Coarse floating-point weights and
 * degrees are defined as the correctly rounded value of the exact real sum,
 * which makes them independent of summation order.
 * ====================================================================== */
#define XLIMBS 40
#define XBIAS 1152
typedef struct {
  uint64_t l[XLIMBS];
} xacc;

static void xacc_clear(xacc* a) { memset(a, 0, sizeof(*a)); }

static void xacc_add_bits(xacc* a, uint64_t mant, int pos) {
  /* add mant * 2^(pos - XBIAS) */
  int limb = pos / 64, sh = pos % 64;
  u128 v = ((u128)mant) << sh;
  uint64_t lo = (uint64_t)v, hi = (uint64_t)(v >> 64);
  uint64_t old = a->l[limb];
  a->l[limb] = old + lo;
  uint64_t carry = (a->l[limb] < old);
  int k = limb + 1;
  uint64_t add = hi;
  while (k < XLIMBS && (add || carry)) {
    uint64_t o = a->l[k];
    uint64_t s1 = o + add;
    uint64_t c1 = s1 < o;
    uint64_t s2 = s1 + carry;
    uint64_t c2 = s2 < s1;
    a->l[k] = s2;
    carry = c1 | c2;
    add = 0;
    k++;
  }
}

static int xacc_add(xacc* a, double v) {
  if (!(v >= 0.0) || isinf(v)) return -1;
  if (v == 0.0) return 0;
  int e;
  double f = frexp(v, &e); /* v = f * 2^e, 0.5 <= f < 1 */
  uint64_t mant = (uint64_t)ldexp(f, 53); /* exact: f has at most 53 bits */
  int pos = (e - 53) + XBIAS;
  xacc_add_bits(a, mant, pos);
  return 0;
}

static int xacc_bit(const xacc* a, int b) { return (int)((a->l[b / 64] >> (b % 64)) & 1u); }

static double xacc_round(const xacc* a) {
  int h = -1;
  for (int b = XLIMBS * 64 - 1; b >= 0; b--) {
    if (xacc_bit(a, b)) {
      h = b;
      break;
    }
  }
  if (h < 0) return 0.0;
  int lo = h - 52; /* lowest kept bit */
  if (lo < 0) lo = 0;
  uint64_t mant = 0;
  for (int b = h; b >= lo; b--) mant = (mant << 1) | (uint64_t)xacc_bit(a, b);
  if (lo > 0) {
    int rbit = xacc_bit(a, lo - 1);
    int sticky = 0;
    for (int b = lo - 2; b >= 0 && !sticky; b--) sticky = xacc_bit(a, b);
    if (rbit && (sticky || (mant & 1u))) mant += 1; /* may become 2^53: still exact */
  }
  return ldexp((double)mant, lo - XBIAS);
}

/* exported for the tests: correctly rounded sum of k non-negative doubles */
int or_exact_sum(int64_t k, const double* x, double* out) {
  xacc a;
  xacc_clear(&a);
  for (int64_t i = 0; i < k; i++)
    if (xacc_add(&a, x[i])) return OR_EINVAL;
  *out = xacc_round(&a);
  return OR_OK;
}

/* ======================================================================
 * Graph access.  wi/self_i are used on the integer path, wf/self_f on the
 * floating-point path; size may be NULL (every node stands for one node).
 * ====================================================================== */
typedef struct {
  int64_t n;
  const int64_t* rp;
  const int32_t* col;
  const int32_t* wi;
  const double* wf;
  const int64_t* self_i;
  const double* self_f;
  const int32_t* size;
} graph_t;

static int64_t max_row_len(const graph_t* g) {
  int64_t mx = 0;
  for (int64_t u = 0; u < g->n; u++) {
    int64_t d = g->rp[u + 1] - g->rp[u];
    if (d > mx) mx = d;
  }
  return mx;
}

/* Validation of the paper's standing assumptions on G (introduction, before
 * Definition 1): a simple weighted graph given as a symmetric CSR with
 * positive weights.  Connectivity is not required here; a disconnected
 * input is rejected later only if the target cannot be reached. */
static int validate(const graph_t* g, int fp, int64_t* total_out) {
  int64_t n = g->n;
  if (n < 1) return OR_EINVAL;
  if (g->rp[0] != 0) return OR_EINVAL;
  for (int64_t u = 0; u < n; u++)
    if (g->rp[u + 1] < g->rp[u]) return OR_EINVAL;
  u128 total = 0;
  for (int64_t u = 0; u < n; u++) {
    for (int64_t j = g->rp[u]; j < g->rp[u + 1]; j++) {
      int64_t v = g->col[j];
      if (v < 0 || v >= n || v == u) return OR_EINVAL;
      if (j > g->rp[u] && g->col[j - 1] >= v) return OR_EINVAL;
      if (fp) {
        if (!(g->wf[j] > 0.0) || isinf(g->wf[j])) return OR_EINVAL;
      } else {
        if (g->wi[j] <= 0) return OR_EINVAL;
        total += (u128)g->wi[j];
      }
      /* the mirror entry must exist with the same weight */
      int64_t lo = g->rp[v], hi = g->rp[v + 1] - 1, found = -1;
      while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (g->col[mid] == u) {
          found = mid;
          break;
        }
        if (g->col[mid] < u) lo = mid + 1;
        else hi = mid - 1;
      }
      if (found < 0) return OR_EINVAL;
      if (fp ? (g->wf[found] != g->wf[j]) : (g->wi[found] != g->wi[j])) return OR_EINVAL;
    }
    if (fp) {
      if (g->self_f && (!(g->self_f[u] >= 0.0) || isinf(g->self_f[u]))) return OR_EINVAL;
    } else if (g->self_i) {
      if (g->self_i[u] < 0) return OR_EINVAL;
      total += (u128)g->self_i[u];
    }
    if (g->size && g->size[u] < 1) return OR_EINVAL;
  }
  if (!fp && total > (u128)2147483647) return OR_EOVERFLOW;
  if (total_out) *total_out = (int64_t)total;
  return OR_OK;
}

/* Node u's full adjacency row w_u in ascending x, with the diagonal entry
 * (x = u, weight self_w[u]) placed in order when it is nonzero. */
static int64_t full_row_i(const graph_t* g, int64_t u, int64_t* xs, int64_t* as) {
  int64_t k = 0;
  int64_t s = g->self_i ? g->self_i[u] : 0;
  int placed = (s == 0);
  for (int64_t j = g->rp[u]; j < g->rp[u + 1]; j++) {
    if (!placed && g->col[j] > u) {
      xs[k] = u;
      as[k] = s;
      k++;
      placed = 1;
    }
    xs[k] = g->col[j];
    as[k] = g->wi[j];
    k++;
  }
  if (!placed) {
    xs[k] = u;
    as[k] = s;
    k++;
  }
  return k;
}

static int64_t full_row_f(const graph_t* g, int64_t u, int64_t* xs, double* as) {
  int64_t k = 0;
  double s = g->self_f ? g->self_f[u] : 0.0;
  int placed = (s == 0.0);
  for (int64_t j = g->rp[u]; j < g->rp[u + 1]; j++) {
    if (!placed && g->col[j] > u) {
      xs[k] = u;
      as[k] = s;
      k++;
      placed = 1;
    }
    xs[k] = g->col[j];
    as[k] = g->wf[j];
    k++;
  }
  if (!placed) {
    xs[k] = u;
    as[k] = s;
    k++;
  }
  return k;
}

/* ======================================================================
 * Degrees d_x: the row sum of w_x (notation after Theorem 1).
 * Integer path: exact int64.  Floating-point path: correctly rounded exact
 * sum of the diagonal and the row entries.
 * ====================================================================== */
int or_degrees_i(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* w,
                 const int64_t* self_w, int64_t* deg) {
  (void)col;
  for (int64_t u = 0; u < n; u++) {
    int64_t d = self_w ? self_w[u] : 0;
    for (int64_t j = rp[u]; j < rp[u + 1]; j++) d += w[j];
    deg[u] = d;
  }
  return OR_OK;
}

int or_degrees_f(int64_t n, const int64_t* rp, const int32_t* col, const double* w,
                 const double* self_w, double* deg) {
  (void)col;
  xacc a;
  for (int64_t u = 0; u < n; u++) {
    xacc_clear(&a);
    if (self_w && xacc_add(&a, self_w[u])) return OR_EINVAL;
    for (int64_t j = rp[u]; j < rp[u + 1]; j++)
      if (xacc_add(&a, w[j])) return OR_EINVAL;
    deg[u] = xacc_round(&a);
  }
  return OR_OK;
}

/* ======================================================================
 * Merge scores: the 1-norm distance between normalised adjacency rows,
 * || w_u/d_u - w_v/d_v ||_1 (Theorem 1), evaluated once per edge as in
 * Algorithm 1's fitness loop.  Edges u < v are enumerated in lexicographic
 * order; eu/ev receive the endpoints.
 *
 * Integer path, exact: with D = d_u d_v the score is N / D where
 *   N = sum_x | a_ux d_v - a_vx d_u |   over the union of both supports.
 * Because both normalised rows sum to one, the same N also equals
 *   2 D - 2 sum_{x in both supports} min(a_ux d_v, a_vx d_u);
 * both are computed and must agree.
 *
 * Floating-point path: p_x = a_ux / d_u and q_x = a_vx / d_v (each a
 * correctly rounded division), t = sum of min(p_x, q_x) over the common
 * support taken left to right in ascending x, score = 2 - 2 t.  The literal
 * sum of |p_x - q_x| over the union is returned alongside it.
 * ====================================================================== */
int64_t or_count_edges(int64_t n, const int64_t* rp, const int32_t* col) {
  int64_t m = 0;
  for (int64_t u = 0; u < n; u++)
    for (int64_t j = rp[u]; j < rp[u + 1]; j++)
      if (col[j] > u) m++;
  return m;
}

int or_scores_i(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* w,
                const int64_t* self_w, const int64_t* deg, int64_t* eu, int64_t* ev,
                uint64_t* N_out, uint64_t* D_out) {
  graph_t g = {n, rp, col, w, NULL, self_w, NULL, NULL};
  int64_t L = max_row_len(&g) + 1;
  int64_t* xu = malloc(sizeof(int64_t) * L);
  int64_t* au = malloc(sizeof(int64_t) * L);
  int64_t* xv = malloc(sizeof(int64_t) * L);
  int64_t* av = malloc(sizeof(int64_t) * L);
  if (!xu || !au || !xv || !av) return OR_ENOMEM;
  int64_t e = 0;
  int rc = OR_OK;
  for (int64_t u = 0; u < n && rc == OR_OK; u++) {
    int64_t ku = full_row_i(&g, u, xu, au);
    for (int64_t j = rp[u]; j < rp[u + 1]; j++) {
      int64_t v = col[j];
      if (v <= u) continue;
      int64_t kv = full_row_i(&g, v, xv, av);
      uint64_t du = (uint64_t)deg[u], dv = (uint64_t)deg[v];
      uint64_t D = du * dv;
      /* intersection form */
      uint64_t M = 0;
      int64_t a = 0, b = 0;
      while (a < ku && b < kv) {
        if (xu[a] < xv[b]) a++;
        else if (xu[a] > xv[b]) b++;
        else {
          uint64_t l = (uint64_t)au[a] * dv, r = (uint64_t)av[b] * du;
          M += (l < r) ? l : r;
          a++;
          b++;
        }
      }
      uint64_t N = 2 * D - 2 * M;
      /* literal union form */
      uint64_t Nl = 0;
      a = 0;
      b = 0;
      while (a < ku || b < kv) {
        uint64_t l = 0, r = 0;
        if (b >= kv || (a < ku && xu[a] < xv[b])) {
          l = (uint64_t)au[a] * dv;
          a++;
        } else if (a >= ku || xv[b] < xu[a]) {
          r = (uint64_t)av[b] * du;
          b++;
        } else {
          l = (uint64_t)au[a] * dv;
          r = (uint64_t)av[b] * du;
          a++;
          b++;
        }
        Nl += (l > r) ? (l - r) : (r - l);
      }
      if (Nl != N) {
        rc = OR_EINVAL; /* cannot happen for a valid graph; reported loudly */
        break;
      }
      eu[e] = u;
      ev[e] = v;
      N_out[e] = N;
      D_out[e] = D;
      e++;
    }
  }
  free(xu);
  free(au);
  free(xv);
  free(av);
  return rc;
}

int or_scores_f(int64_t n, const int64_t* rp, const int32_t* col, const double* w,
                const double* self_w, const double* deg, int64_t* eu, int64_t* ev,
                double* score, double* score_literal) {
  graph_t g = {n, rp, col, NULL, w, NULL, self_w, NULL};
  int64_t L = max_row_len(&g) + 1;
  int64_t* xu = malloc(sizeof(int64_t) * L);
  double* au = malloc(sizeof(double) * L);
  int64_t* xv = malloc(sizeof(int64_t) * L);
  double* av = malloc(sizeof(double) * L);
  if (!xu || !au || !xv || !av) return OR_ENOMEM;
  int64_t e = 0;
  for (int64_t u = 0; u < n; u++) {
    int64_t ku = full_row_f(&g, u, xu, au);
    for (int64_t j = rp[u]; j < rp[u + 1]; j++) {
      int64_t v = col[j];
      if (v <= u) continue;
      int64_t kv = full_row_f(&g, v, xv, av);
      double du = deg[u], dv = deg[v];
      double t = 0.0;
      int64_t a = 0, b = 0;
      while (a < ku && b < kv) {
        if (xu[a] < xv[b]) a++;
        else if (xu[a] > xv[b]) b++;
        else {
          double p = au[a] / du, q = av[b] / dv;
          t = t + ((p < q) ? p : q);
          a++;
          b++;
        }
      }
      double lit = 0.0;
      a = 0;
      b = 0;
      while (a < ku || b < kv) {
        double p = 0.0, q = 0.0;
        if (b >= kv || (a < ku && xu[a] < xv[b])) {
          p = au[a] / du;
          a++;
        } else if (a >= ku || xv[b] < xu[a]) {
          q = av[b] / dv;
          b++;
        } else {
          p = au[a] / du;
          q = av[b] / dv;
          a++;
          b++;
        }
        lit = lit + fabs(p - q);
      }
      eu[e] = u;
      ev[e] = v;
      score[e] = 2.0 - 2.0 * t;
      score_literal[e] = lit;
      e++;
    }
  }
  free(xu);
  free(au);
  free(xv);
  free(av);
  return OR_OK;
}

/* ======================================================================
 * Sort of the fitness list (Algorithm 1).  Strict total order on edges:
 * the score first, then the smaller endpoint, then the larger endpoint.
 * The integer comparison is exact: N1/D1 < N2/D2  <=>  N1 D2 < N2 D1.
 * ====================================================================== */
typedef struct {
  uint64_t N, D;
  double s;
  int64_t u, v, e;
} rec_t;

static int cmp_rec_i(const void* pa, const void* pb) {
  const rec_t* a = pa;
  const rec_t* b = pb;
  u128 l = (u128)a->N * b->D, r = (u128)b->N * a->D;
  if (l < r) return -1;
  if (l > r) return 1;
  if (a->u != b->u) return a->u < b->u ? -1 : 1;
  if (a->v != b->v) return a->v < b->v ? -1 : 1;
  return 0;
}

static int cmp_rec_f(const void* pa, const void* pb) {
  const rec_t* a = pa;
  const rec_t* b = pb;
  if (a->s < b->s) return -1;
  if (a->s > b->s) return 1;
  if (a->u != b->u) return a->u < b->u ? -1 : 1;
  if (a->v != b->v) return a->v < b->v ? -1 : 1;
  return 0;
}

/* order[r] = index of the edge at sorted position r */
int or_order_i(int64_t m, const int64_t* eu, const int64_t* ev, const uint64_t* N,
               const uint64_t* D, int64_t* order) {
  rec_t* r = malloc(sizeof(rec_t) * (m ? m : 1));
  if (!r) return OR_ENOMEM;
  for (int64_t e = 0; e < m; e++) {
    r[e].N = N[e];
    r[e].D = D[e];
    r[e].s = 0;
    r[e].u = eu[e];
    r[e].v = ev[e];
    r[e].e = e;
  }
  qsort(r, (size_t)m, sizeof(rec_t), cmp_rec_i);
  for (int64_t k = 0; k < m; k++) order[k] = r[k].e;
  free(r);
  return OR_OK;
}

int or_order_f(int64_t m, const int64_t* eu, const int64_t* ev, const double* s,
               int64_t* order) {
  rec_t* r = malloc(sizeof(rec_t) * (m ? m : 1));
  if (!r) return OR_ENOMEM;
  for (int64_t e = 0; e < m; e++) {
    if (isnan(s[e])) {
      free(r);
      return OR_EINVAL;
    }
    r[e].N = 0;
    r[e].D = 1;
    r[e].s = s[e];
    r[e].u = eu[e];
    r[e].v = ev[e];
    r[e].e = e;
  }
  qsort(r, (size_t)m, sizeof(rec_t), cmp_rec_f);
  for (int64_t k = 0; k < m; k++) order[k] = r[k].e;
  free(r);
  return OR_OK;
}

/* ======================================================================
 * Merge loop of Algorithm 1 with a union-find forest.  The super-node
 * count s starts at n; edges are visited in sorted order; an edge whose
 * ends already lie in one super-node is skipped; otherwise the two
 * super-nodes merge (the larger root is hooked under the smaller, so a
 * root is always the smallest member) and s drops by one.  The loop stops
 * when s reaches the target t.
 *
 * Super-nodes are then numbered by ascending smallest member.
 * accepted (nullable) receives the merged edges in merge order.
 * ====================================================================== */
static int64_t uf_find(int64_t* parent, int64_t x) {
  int64_t r = x;
  while (parent[r] != r) r = parent[r];
  while (parent[x] != r) {
    int64_t nx = parent[x];
    parent[x] = r;
    x = nx;
  }
  return r;
}

int or_merge(int64_t n, int64_t m, const int64_t* eu, const int64_t* ev, const int64_t* order,
             int64_t t, int32_t* cluster_of, int64_t* accepted, int64_t* n_accepted) {
  if (t < 1) return OR_EINVAL;
  int64_t* parent = malloc(sizeof(int64_t) * n);
  if (!parent) return OR_ENOMEM;
  for (int64_t x = 0; x < n; x++) parent[x] = x;
  int64_t s = n, k = 0;
  for (int64_t r = 0; r < m && s > t; r++) {
    int64_t e = order[r];
    int64_t a = uf_find(parent, eu[e]), b = uf_find(parent, ev[e]);
    if (a == b) continue;
    if (a < b) parent[b] = a;
    else parent[a] = b;
    s--;
    if (accepted) accepted[k] = e;
    k++;
  }
  if (n_accepted) *n_accepted = k;
  if (s > t) {
    free(parent);
    return OR_EUNREACHABLE;
  }
  /* number super-nodes by ascending smallest member (= root) */
  int64_t next = 0;
  int64_t* id = malloc(sizeof(int64_t) * n);
  if (!id) {
    free(parent);
    return OR_ENOMEM;
  }
  for (int64_t x = 0; x < n; x++) {
    if (uf_find(parent, x) == x) id[x] = next++;
  }
  for (int64_t x = 0; x < n; x++) cluster_of[x] = (int32_t)id[uf_find(parent, x)];
  free(id);
  free(parent);
  return OR_OK;
}

/* ======================================================================
 * Contraction (Definition 1): super-node a's weight towards super-node b
 * is the sum of w(x, y) over members x of a and y of b.  Pairs with a = b
 * become a's self-loop weight, which also absorbs the members' own
 * self-loops; sizes add.  Rows come out ascending in b with no diagonal.
 *
 * Every directed fine entry (and every member self-loop) becomes a tuple
 * (a, b, x, y, w); the tuples are sorted and equal (a, b) runs are summed,
 * exactly in int64 or as a correctly rounded exact sum in floating point.
 * ====================================================================== */
typedef struct {
  int64_t a, b, x, y;
  int64_t wi;
  double wf;
} tup_t;

static int cmp_tup(const void* pa, const void* pb) {
  const tup_t* p = pa;
  const tup_t* q = pb;
  if (p->a != q->a) return p->a < q->a ? -1 : 1;
  if (p->b != q->b) return p->b < q->b ? -1 : 1;
  if (p->x != q->x) return p->x < q->x ? -1 : 1;
  if (p->y != q->y) return p->y < q->y ? -1 : 1;
  return 0;
}

static int contract_common(const graph_t* g, int fp, const int32_t* c, int64_t n_c,
                           int64_t* rp_c, int32_t* col_c, int32_t* w_ci, double* w_cf,
                           int64_t* self_ci, double* self_cf, int32_t* size_c, int64_t* nnz_c) {
  int64_t n = g->n, nnz = g->rp[n];
  tup_t* T = malloc(sizeof(tup_t) * (size_t)(nnz + n + 1));
  if (!T) return OR_ENOMEM;
  int64_t k = 0;
  for (int64_t x = 0; x < n; x++) {
    if (c[x] < 0 || c[x] >= n_c) {
      free(T);
      return OR_EINVAL;
    }
    for (int64_t j = g->rp[x]; j < g->rp[x + 1]; j++) {
      T[k].a = c[x];
      T[k].b = c[g->col[j]];
      T[k].x = x;
      T[k].y = g->col[j];
      T[k].wi = fp ? 0 : g->wi[j];
      T[k].wf = fp ? g->wf[j] : 0.0;
      k++;
    }
    int has_self = fp ? (g->self_f && g->self_f[x] != 0.0) : (g->self_i && g->self_i[x] != 0);
    if (has_self) {
      T[k].a = c[x];
      T[k].b = c[x];
      T[k].x = x;
      T[k].y = x;
      T[k].wi = fp ? 0 : g->self_i[x];
      T[k].wf = fp ? g->self_f[x] : 0.0;
      k++;
    }
  }
  qsort(T, (size_t)k, sizeof(tup_t), cmp_tup);
  for (int64_t a = 0; a < n_c; a++) {
    if (fp) self_cf[a] = 0.0;
    else self_ci[a] = 0;
    size_c[a] = 0;
  }
  for (int64_t x = 0; x < n; x++) size_c[c[x]] += g->size ? g->size[x] : 1;
  for (int64_t a = 0; a < n_c; a++)
    if (size_c[a] == 0) { /* cluster ids must be a surjection */
      free(T);
      return OR_EINVAL;
    }
  int64_t out = 0, i = 0;
  int64_t row = 0;
  rp_c[0] = 0;
  xacc acc;
  while (i < k) {
    int64_t a = T[i].a, b = T[i].b;
    int64_t s_i = 0;
    xacc_clear(&acc);
    int64_t j = i;
    while (j < k && T[j].a == a && T[j].b == b) {
      if (fp) {
        if (xacc_add(&acc, T[j].wf)) {
          free(T);
          return OR_EINVAL;
        }
      } else {
        s_i += T[j].wi;
      }
      j++;
    }
    while (row < a) rp_c[++row] = out;
    if (a == b) {
      if (fp) self_cf[a] = xacc_round(&acc);
      else self_ci[a] = s_i;
    } else {
      col_c[out] = (int32_t)b;
      if (fp) w_cf[out] = xacc_round(&acc);
      else {
        if (s_i > 2147483647) {
          free(T);
          return OR_EOVERFLOW;
        }
        w_ci[out] = (int32_t)s_i;
      }
      out++;
    }
    i = j;
  }
  while (row < n_c) rp_c[++row] = out;
  *nnz_c = out;
  free(T);
  return OR_OK;
}

int or_contract_i(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* w,
                  const int64_t* self_w, const int32_t* size, const int32_t* cluster_of,
                  int64_t n_c, int64_t* rp_c, int32_t* col_c, int32_t* w_c, int64_t* self_c,
                  int32_t* size_c, int64_t* nnz_c) {
  graph_t g = {n, rp, col, w, NULL, self_w, NULL, size};
  return contract_common(&g, 0, cluster_of, n_c, rp_c, col_c, w_c, NULL, self_c, NULL, size_c,
                         nnz_c);
}

int or_contract_f(int64_t n, const int64_t* rp, const int32_t* col, const double* w,
                  const double* self_w, const int32_t* size, const int32_t* cluster_of,
                  int64_t n_c, int64_t* rp_c, int32_t* col_c, double* w_c, double* self_c,
                  int32_t* size_c, int64_t* nnz_c) {
  graph_t g = {n, rp, col, NULL, w, NULL, self_w, size};
  return contract_common(&g, 1, cluster_of, n_c, rp_c, col_c, NULL, w_c, NULL, self_c, size_c,
                         nnz_c);
}

/* ======================================================================
 * One coarsening level = Algorithm 1 with target t: degrees, fitness,
 * sort, merge loop, then the contraction of Definition 1.
 * Output arrays are sized by the caller for the fine graph (n, nnz).
 * eps_max receives the largest accepted score (Theorem 2's epsilon).
 * ====================================================================== */
int or_coarsen_level_i(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* w,
                       const int64_t* self_w, const int32_t* size, int64_t t, int32_t* cluster_of,
                       int64_t* n_c, int64_t* rp_c, int32_t* col_c, int32_t* w_c, int64_t* self_c,
                       int32_t* size_c, int64_t* nnz_c, double* eps_max) {
  graph_t g = {n, rp, col, w, NULL, self_w, NULL, size};
  int rc = validate(&g, 0, NULL);
  if (rc) return rc;
  if (t < 1) return OR_EINVAL;
  if (t > n) t = n;
  int64_t m = or_count_edges(n, rp, col);
  int64_t* deg = malloc(sizeof(int64_t) * n);
  int64_t* eu = malloc(sizeof(int64_t) * (m ? m : 1));
  int64_t* ev = malloc(sizeof(int64_t) * (m ? m : 1));
  uint64_t* N = malloc(sizeof(uint64_t) * (m ? m : 1));
  uint64_t* D = malloc(sizeof(uint64_t) * (m ? m : 1));
  int64_t* order = malloc(sizeof(int64_t) * (m ? m : 1));
  int64_t* acc = malloc(sizeof(int64_t) * (n ? n : 1));
  if (!deg || !eu || !ev || !N || !D || !order || !acc) return OR_ENOMEM;
  or_degrees_i(n, rp, col, w, self_w, deg);
  rc = or_scores_i(n, rp, col, w, self_w, deg, eu, ev, N, D);
  if (!rc) rc = or_order_i(m, eu, ev, N, D, order);
  int64_t na = 0;
  if (!rc) rc = or_merge(n, m, eu, ev, order, t, cluster_of, acc, &na);
  if (!rc) {
    double mx = 0.0;
    for (int64_t k = 0; k < na; k++) {
      double s = (double)N[acc[k]] / (double)D[acc[k]];
      if (s > mx) mx = s;
    }
    if (eps_max) *eps_max = mx;
    *n_c = t;
    rc = or_contract_i(n, rp, col, w, self_w, size, cluster_of, t, rp_c, col_c, w_c, self_c,
                       size_c, nnz_c);
  }
  free(deg);
  free(eu);
  free(ev);
  free(N);
  free(D);
  free(order);
  free(acc);
  return rc;
}

int or_coarsen_level_f(int64_t n, const int64_t* rp, const int32_t* col, const double* w,
                       const double* self_w, const int32_t* size, int64_t t, int32_t* cluster_of,
                       int64_t* n_c, int64_t* rp_c, int32_t* col_c, double* w_c, double* self_c,
                       int32_t* size_c, int64_t* nnz_c, double* eps_max) {
  graph_t g = {n, rp, col, NULL, w, NULL, self_w, size};
  int rc = validate(&g, 1, NULL);
  if (rc) return rc;
  if (t < 1) return OR_EINVAL;
  if (t > n) t = n;
  int64_t m = or_count_edges(n, rp, col);
  double* deg = malloc(sizeof(double) * n);
  int64_t* eu = malloc(sizeof(int64_t) * (m ? m : 1));
  int64_t* ev = malloc(sizeof(int64_t) * (m ? m : 1));
  double* s = malloc(sizeof(double) * (m ? m : 1));
  double* sl = malloc(sizeof(double) * (m ? m : 1));
  int64_t* order = malloc(sizeof(int64_t) * (m ? m : 1));
  int64_t* acc = malloc(sizeof(int64_t) * (n ? n : 1));
  if (!deg || !eu || !ev || !s || !sl || !order || !acc) return OR_ENOMEM;
  rc = or_degrees_f(n, rp, col, w, self_w, deg);
  if (!rc) rc = or_scores_f(n, rp, col, w, self_w, deg, eu, ev, s, sl);
  if (!rc) rc = or_order_f(m, eu, ev, s, order);
  int64_t na = 0;
  if (!rc) rc = or_merge(n, m, eu, ev, order, t, cluster_of, acc, &na);
  if (!rc) {
    double mx = -INFINITY;
    for (int64_t k = 0; k < na; k++)
      if (s[acc[k]] > mx) mx = s[acc[k]];
    if (eps_max) *eps_max = na ? mx : 0.0;
    *n_c = t;
    rc = or_contract_f(n, rp, col, w, self_w, size, cluster_of, t, rp_c, col_c, w_c, self_c,
                       size_c, nnz_c);
  }
  free(deg);
  free(eu);
  free(ev);
  free(s);
  free(sl);
  free(order);
  free(acc);
  return rc;
}

int or_validate(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* wi,
                const double* wf, const int64_t* self_i, const double* self_f,
                const int32_t* size, int fp) {
  graph_t g = {n, rp, col, wi, wf, self_i, self_f, size};
  return validate(&g, fp, NULL);
}

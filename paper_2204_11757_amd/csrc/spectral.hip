// The lift of Definition 2 applied to vectors, the spectral error of a
// level's lift against eigenpairs of the input graph, and host-side
// validation of a graph.
#include <cmath>

#include "level.hpp"

using namespace spc;


namespace {

constexpr int MAXCHAIN = 64;
struct MapChain {
  const int32_t* maps[MAXCHAIN];
  int count;
};

struct LessU64 {
  __device__ __forceinline__ bool operator()(const uint64_t& a, const uint64_t& b) const { return a < b; }
};

__global__ void k_compose(MapChain ch, int64_t n, int32_t* __restrict__ out) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  int32_t a = (int32_t)u;
  for (int i = 0; i < ch.count; i++) a = ch.maps[i][a];
  out[u] = a;
}

__global__ void k_lift(const int32_t* __restrict__ cmap, const int32_t* __restrict__ size_from,
                       const int32_t* __restrict__ size_to, int mode, const double* __restrict__ xc,
                       int64_t n_to, int k, double* __restrict__ xf, int64_t n_from) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n_from) return;
  int32_t a = cmap[u];
  double s = 1.0;
  if (mode == 1) {
    // orthonormal lift in level from's own orthonormal basis: the super-node's
    // size relative to u's (from the input level, u's size is 1)
    double sf = size_from ? (double)size_from[u] : 1.0;
    double st = size_to ? (double)size_to[a] : 1.0;
    s = sqrt(st / sf);
  }
  for (int c = 0; c < k; c++) {
    double v = xc[a + n_to * (int64_t)c];
    xf[u + n_from * (int64_t)c] = (mode == 1) ? v / s : v;
  }
}

__global__ void k_pair_keys(const int32_t* __restrict__ cmap, int64_t n, uint64_t* __restrict__ keys) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) keys[u] = ((uint64_t)(uint32_t)cmap[u] << 32) | (uint64_t)u;
}

__global__ void k_count_clusters(const int32_t* __restrict__ cmap, int64_t n, int32_t* cnt) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) atomicAdd(&cnt[cmap[u]], 1);
}

// Weights of a coarse graph as FP64: int32 or double entries, int64 or
// double self-loops (integer levels convert exactly).
struct CoarseView {
  int64_t nc, nnz;
  const int64_t* rp;
  const int32_t* col;
  const void* w;
  const void* self;   // nullable
  const int32_t* size;
  int fp;             // 1: double weights and self-loops
};

__device__ __forceinline__ double cv_w(const CoarseView& g, int64_t j) {
  return g.fp ? ((const double*)g.w)[j] : (double)((const int32_t*)g.w)[j];
}
__device__ __forceinline__ double cv_self(const CoarseView& g, int64_t a) {
  if (!g.self) return 0.0;
  return g.fp ? ((const double*)g.self)[a] : (double)((const int64_t*)g.self)[a];
}

// Sums over a super-node's members and over a coarse row run in a fixed
// order, so results are reproducible: one thread walks a short list in
// order; a list longer than LONG_LIST is summed by one block with a fixed
// shape (strided partial sums, then a tree), in a separate launch.  Every
// quantity is computed in the type T (double, or float for the FP32 form).
constexpr int LONG_LIST = 2048;
constexpr int SP_BS = 256;

template <typename T>
__device__ __forceinline__ T block_sum_fixed(T v, T* tmp) {
  tmp[threadIdx.x] = v;
  __syncthreads();
  for (int o = SP_BS / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) tmp[threadIdx.x] += tmp[threadIdx.x + o];
    __syncthreads();
  }
  T r = tmp[0];
  __syncthreads();
  return r;
}

// y = Q^T u_i (members summed in ascending fine id), d = W_c row sums with
// the diagonal, t = D_c^{-1/2} y; short lists here, long ones in k_restrict_long
template <typename T>
__global__ void k_restrict_scale(const uint64_t* __restrict__ sorted, const int32_t* __restrict__ mptr,
                                 const T* __restrict__ U, int64_t n0, int k, CoarseView g,
                                 T* __restrict__ t, T* __restrict__ dc) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.nc * k) return;
  int64_t a = idx % g.nc;
  int i = (int)(idx / g.nc);
  if (mptr[a + 1] - mptr[a] > LONG_LIST || g.rp[a + 1] - g.rp[a] > LONG_LIST) return;
  T y = 0;
  for (int32_t p = mptr[a]; p < mptr[a + 1]; p++) {
    int64_t u = (int64_t)(sorted[p] & 0xffffffffull);
    y += U[u + n0 * i];
  }
  y = y / sqrt((T)(g.size ? g.size[a] : 1));
  T d = (T)cv_self(g, a);
  for (int64_t j = g.rp[a]; j < g.rp[a + 1]; j++) d += (T)cv_w(g, j);
  t[a + g.nc * i] = y / sqrt(d);
  if (i == 0) dc[a] = d;
}

// one block per super-node with a long member list or a long row
template <typename T>
__global__ void __launch_bounds__(SP_BS)
    k_restrict_long(const uint64_t* __restrict__ sorted, const int32_t* __restrict__ mptr,
                    const T* __restrict__ U, int64_t n0, int k, CoarseView g, T* __restrict__ t,
                    T* __restrict__ dc) {
  __shared__ T tmp[SP_BS];
  int64_t a = blockIdx.x;
  int32_t m0 = mptr[a], m1 = mptr[a + 1];
  int64_t r0 = g.rp[a], r1 = g.rp[a + 1];
  if (m1 - m0 <= LONG_LIST && r1 - r0 <= LONG_LIST) return;
  T part = 0;
  for (int64_t j = r0 + threadIdx.x; j < r1; j += SP_BS) part += (T)cv_w(g, j);
  T d = (T)cv_self(g, a) + block_sum_fixed(part, tmp);
  for (int i = 0; i < k; i++) {
    part = 0;
    for (int32_t p = m0 + threadIdx.x; p < m1; p += SP_BS)
      part += U[(int64_t)(sorted[p] & 0xffffffffull) + n0 * i];
    T y = block_sum_fixed(part, tmp) / sqrt((T)(g.size ? g.size[a] : 1));
    if (threadIdx.x == 0) t[a + g.nc * i] = y / sqrt(d);
  }
  if (threadIdx.x == 0) dc[a] = d;
}

// z = W_c t (W_c with its diagonal, summed in ascending column), prod = t z;
// short rows here, long ones in k_quad_long
template <typename T>
__global__ void k_quad(CoarseView g, int k, const T* __restrict__ t, T* __restrict__ z, T* __restrict__ prod) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.nc * k) return;
  int64_t a = idx % g.nc;
  int i = (int)(idx / g.nc);
  if (g.rp[a + 1] - g.rp[a] > LONG_LIST) return;
  const T* ti = t + g.nc * i;
  T s = (T)cv_self(g, a);
  T acc = 0;
  bool placed = (s == (T)0);
  for (int64_t j = g.rp[a]; j < g.rp[a + 1]; j++) {
    int32_t b = g.col[j];
    if (!placed && b > a) {
      acc += s * ti[a];
      placed = true;
    }
    acc += (T)cv_w(g, j) * ti[b];
  }
  if (!placed) acc += s * ti[a];
  z[idx] = acc;
  prod[idx] = ti[a] * acc;
}

template <typename T>
__global__ void __launch_bounds__(SP_BS)
    k_quad_long(CoarseView g, int k, const T* __restrict__ t, T* __restrict__ z, T* __restrict__ prod) {
  __shared__ T tmp[SP_BS];
  int64_t a = blockIdx.x;
  int64_t r0 = g.rp[a], r1 = g.rp[a + 1];
  if (r1 - r0 <= LONG_LIST) return;
  for (int i = 0; i < k; i++) {
    const T* ti = t + g.nc * i;
    T part = 0;
    for (int64_t j = r0 + threadIdx.x; j < r1; j += SP_BS) part += (T)cv_w(g, j) * ti[g.col[j]];
    T acc = block_sum_fixed(part, tmp) + (T)cv_self(g, a) * ti[a];
    if (threadIdx.x == 0) {
      z[a + g.nc * i] = acc;
      prod[a + g.nc * i] = ti[a] * acc;
    }
  }
}

// f_i = sum_a prod[a, i]: one block per i, fixed reduction shape
template <typename T>
__global__ void __launch_bounds__(256) k_colsum(const T* __restrict__ prod, int64_t nc, T* __restrict__ R) {
  __shared__ T tmp[256];
  int i = blockIdx.x;
  T s = 0;
  for (int64_t a = threadIdx.x; a < nc; a += 256) s += prod[a + nc * i];
  tmp[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) tmp[threadIdx.x] += tmp[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) R[i] = (T)1 - tmp[0];
}

// Gradient of loss = sum_i (R_i - lambda_i)^2, R_i = 1 - t_i^T W_c t_i,
// t_i = D_c^{-1/2} y_i, with respect to the undirected weight w_ab = w_ba
// (written at both of its CSR entries) and to the self-loop weights:
//   d(t^T W t)/d w_ab   = 2 t_a t_b - t_a z_a / d_a - t_b z_b / d_b
//   d(t^T W t)/d self_a = t_a^2 - t_a z_a / d_a          (z = W t)
template <typename T>
__global__ void k_spectral_grad(CoarseView g, int k, const T* __restrict__ t, const T* __restrict__ z,
                                const T* __restrict__ dc, const T* __restrict__ coef, T* __restrict__ d_w,
                                T* __restrict__ d_self) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < g.nnz) {
    // the row of entry idx: binary search in rp
    int64_t lo = 0, hi = g.nc - 1;
    while (lo < hi) {
      int64_t mid = (lo + hi + 1) >> 1;
      if (g.rp[mid] <= idx) lo = mid;
      else hi = mid - 1;
    }
    int64_t a = lo, b = g.col[idx];
    T s = 0;
    for (int i = 0; i < k; i++) {
      const T* ti = t + g.nc * i;
      const T* zi = z + g.nc * i;
      T f = (T)2 * ti[a] * ti[b] - ti[a] * zi[a] / dc[a] - ti[b] * zi[b] / dc[b];
      s += coef[i] * f;
    }
    d_w[idx] = s;
  } else if (idx < g.nnz + g.nc) {
    int64_t a = idx - g.nnz;
    T s = 0;
    for (int i = 0; i < k; i++) {
      const T* ti = t + g.nc * i;
      const T* zi = z + g.nc * i;
      s += coef[i] * (ti[a] * ti[a] - ti[a] * zi[a] / dc[a]);
    }
    d_self[a] = s;
  }
}

template <typename T>
__global__ void k_loss_coef(const T* __restrict__ R, const double* __restrict__ lam, int k, T* __restrict__ coef) {
  int i = threadIdx.x;
  if (i < k) coef[i] = (T)-2 * (R[i] - (T)lam[i]);   // d loss / d f_i, f_i = t_i^T W t_i
}

int compose_map(spc_ctx* ctx, const spc_hier* h, int from_lvl, int to_lvl, int32_t* out, int64_t n_from) {
  MapChain ch;
  ch.count = 0;
  for (int l = from_lvl + 1; l <= to_lvl; l++) {
    if (ch.count >= MAXCHAIN) return set_error(ctx, SPC_EINVAL, "hierarchy deeper than %d", MAXCHAIN);
    ch.maps[ch.count++] = h->levels[l - 1].cluster_of;
  }
  hipLaunchKernelGGL(k_compose, dim3(grid_for(n_from, 256)), dim3(256), 0, ctx->stream, ch, n_from, out);
  SPC_LAUNCH_CHECK(ctx, "compose");
  return SPC_OK;
}

// Forward (and, when d_w is non-NULL, backward) of the spectral error of a
// coarse graph whose super-nodes are given by cmap (fine id -> coarse id,
// n0 entries; cmap may live in the workspace when own_cmap is false).
template <typename T>
static int spectral_t(spc_ctx* ctx, const CoarseView& g, const int32_t* cmap_in, const spc_hier* h, int lvl,
                      int64_t n0, const T* U, const double* lambda, int k, T* R, double* loss, T* d_w,
                      T* d_self) {
  int64_t nc = g.nc;
  Arena A;
  A.counting = true;
  for (int pass = 0; pass < 2; pass++) {
    A.off = 0;
    if (pass == 1) {
      int rc = ensure_workspace(ctx, A.cap + 256);
      if (rc) return rc;
      A.counting = false;
      A.base = (char*)ctx->ws;
      A.cap = ctx->ws_cap;
    }
    int32_t* cmap = A.take<int32_t>(n0);
    uint64_t* ka = A.take<uint64_t>(n0);
    uint64_t* kb = A.take<uint64_t>(n0);
    int32_t* mptr = A.take<int32_t>(nc + 1);
    T* t = A.take<T>(nc * k);
    T* z = A.take<T>(nc * k);
    T* prod = A.take<T>(nc * k);
    T* dc = A.take<T>(nc);
    T* Rd = A.take<T>(k);
    T* coef = A.take<T>(k);
    if (pass == 0) {
      A.cap = A.off;
      continue;
    }
    hipStream_t st = ctx->stream;
    int rc;
    if (cmap_in) {
      SPC_HIP(ctx, hipMemcpyAsync(cmap, cmap_in, sizeof(int32_t) * n0, hipMemcpyDeviceToDevice, st));
    } else {
      rc = compose_map(ctx, h, 0, lvl, cmap, n0);
      if (rc) return rc;
    }
    hipLaunchKernelGGL(k_pair_keys, dim3(grid_for(n0, 256)), dim3(256), 0, st, cmap, n0, ka);
    uint64_t* sorted = nullptr;
    rc = merge_sort<uint64_t, LessU64>(ctx, ka, kb, n0, LessU64(), &sorted);
    if (rc) return rc;
    launch_zero(ctx, mptr, sizeof(int32_t) * (nc + 1));
    hipLaunchKernelGGL(k_count_clusters, dim3(grid_for(n0, 256)), dim3(256), 0, st, cmap, n0, mptr);
    rc = exclusive_scan<int32_t>(ctx, mptr, mptr, nc, nullptr);
    if (rc) return rc;
    int64_t nk = nc * k;
    T* Rout = R ? R : Rd;
    hipLaunchKernelGGL(k_restrict_scale<T>, dim3(grid_for(nk, 256)), dim3(256), 0, st, sorted, mptr, U, n0, k,
                       g, t, dc);
    hipLaunchKernelGGL(k_restrict_long<T>, dim3((unsigned)nc), dim3(SP_BS), 0, st, sorted, mptr, U, n0, k, g,
                       t, dc);
    hipLaunchKernelGGL(k_quad<T>, dim3(grid_for(nk, 256)), dim3(256), 0, st, g, k, t, z, prod);
    hipLaunchKernelGGL(k_quad_long<T>, dim3((unsigned)nc), dim3(SP_BS), 0, st, g, k, t, z, prod);
    hipLaunchKernelGGL(k_colsum<T>, dim3(k), dim3(256), 0, st, prod, nc, Rout);
    if (d_w) {
      hipLaunchKernelGGL(k_loss_coef<T>, dim3(1), dim3(256), 0, st, Rout, lambda, k, coef);
      hipLaunchKernelGGL(k_spectral_grad<T>, dim3(grid_for(g.nnz + nc, 256)), dim3(256), 0, st, g, k, t, z,
                         dc, coef, d_w, d_self);
    }
    SPC_LAUNCH_CHECK(ctx, "spectral_error");
    if (loss) {
      std::vector<T> hR(k);
      std::vector<double> hl(k);
      SPC_HIP(ctx, hipMemcpyAsync(hR.data(), Rout, sizeof(T) * k, hipMemcpyDeviceToHost, st));
      SPC_HIP(ctx, hipMemcpyAsync(hl.data(), lambda, sizeof(double) * k, hipMemcpyDeviceToHost, st));
      SPC_HIP(ctx, hipStreamSynchronize(st));
      double s = 0.0;
      for (int i = 0; i < k; i++) s += ((double)hR[i] - hl[i]) * ((double)hR[i] - hl[i]);
      *loss = s;
    }
  }
  return SPC_OK;
}

// The spectral error (and, with d_w, its gradient) in FP64 or FP32.
int spectral_impl(spc_ctx* ctx, const CoarseView& g, const int32_t* cmap_in, const spc_hier* h, int lvl,
                  int64_t n0, const void* U, const double* lambda, int k, int prec, void* R, double* loss,
                  void* d_w, void* d_self) {
  if (prec == SPC_W_F64)
    return spectral_t<double>(ctx, g, cmap_in, h, lvl, n0, (const double*)U, lambda, k, (double*)R, loss,
                              (double*)d_w, (double*)d_self);
  if (prec == SPC_W_F32)
    return spectral_t<float>(ctx, g, cmap_in, h, lvl, n0, (const float*)U, lambda, k, (float*)R, loss,
                             (float*)d_w, (float*)d_self);
  return set_error(ctx, SPC_EINVAL, "spectral precision must be SPC_W_F32 or SPC_W_F64");
}

CoarseView view_of_level(const spc_hier::Level& L) {
  CoarseView g;
  g.nc = L.n;
  g.nnz = L.nnz;
  g.rp = L.rp;
  g.col = L.col;
  g.w = L.w;
  g.self = L.self;
  g.size = L.size;
  g.fp = L.wtype != SPC_W_I32;
  return g;
}

int view_of_graph(spc_ctx* ctx, const spc_graph* c, CoarseView& g) {
  if (!c || c->n < 1 || c->nnz < 0 || !c->row_ptr || (c->nnz > 0 && (!c->col || !c->w)))
    return set_error(ctx, SPC_EINVAL, "bad coarse graph");
  if (c->wtype != SPC_W_I32 && c->wtype != SPC_W_F64)
    return set_error(ctx, SPC_EINVAL, "coarse weights must be int32 or float64");
  g.nc = c->n;
  g.nnz = c->nnz;
  g.rp = c->row_ptr;
  g.col = c->col;
  g.w = c->w;
  g.self = c->self_w;
  g.size = c->size;
  g.fp = c->wtype == SPC_W_F64;
  return SPC_OK;
}

// fine entry -> its coarse entry (>= 0) or -1 - super-node for an
// intra-super-node entry
__global__ void k_entry_map(const int64_t* __restrict__ rp, const int32_t* __restrict__ col, int64_t n,
                            int64_t nnz, const int32_t* __restrict__ c, const int64_t* __restrict__ rpc,
                            const int32_t* __restrict__ colc, int32_t* __restrict__ emap) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nnz) return;
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) >> 1;
    if (rp[mid] <= j) lo = mid;
    else hi = mid - 1;
  }
  int32_t a = c[lo], b = c[col[j]];
  if (a == b) {
    emap[j] = -1 - a;
    return;
  }
  int64_t l = rpc[a], h = rpc[a + 1];
  while (l < h) {
    int64_t mid = (l + h) >> 1;
    if (colc[mid] < b) l = mid + 1;
    else h = mid;
  }
  emap[j] = (int32_t)l;
}

// adjoint of the contraction (a gather): fine entries take their coarse
// entry's gradient, intra-super-node entries and fine self-loops take the
// super-node's self-loop gradient
__global__ void k_contract_backward(const int32_t* __restrict__ emap, int64_t nnz_f, const int32_t* __restrict__ c,
                                    int64_t n_f, const double* __restrict__ d_wc, const double* __restrict__ d_selfc,
                                    double* __restrict__ d_wf, double* __restrict__ d_selff) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nnz_f) {
    int32_t e = emap[i];
    d_wf[i] = e >= 0 ? d_wc[e] : d_selfc[-1 - e];
  } else if (i < nnz_f + n_f && d_selff) {
    d_selff[i - nnz_f] = d_selfc[c[i - nnz_f]];
  }
}

}  // namespace

extern "C" {

int spc_lift(spc_ctx* ctx, const spc_hier* h, int from_lvl, int to_lvl, int mode, const double* x_c,
             int k, double* x_f) {
  if (!ctx) return SPC_EINVAL;
  if (!h || from_lvl < 0 || to_lvl > (int)h->levels.size() || from_lvl > to_lvl || k < 0 ||
      (mode != 0 && mode != 1))
    return set_error(ctx, SPC_EINVAL, "bad lift arguments");
  if (k == 0) return SPC_OK;
  if (!x_c || !x_f) return set_error(ctx, SPC_EINVAL, "lift vectors are NULL");
  int64_t n_from = from_lvl == 0 ? h->n0 : h->levels[from_lvl - 1].n;
  int64_t n_to = to_lvl == 0 ? h->n0 : h->levels[to_lvl - 1].n;
  const int32_t* size_from = from_lvl == 0 ? nullptr : h->levels[from_lvl - 1].size;
  const int32_t* size_to = to_lvl == 0 ? nullptr : h->levels[to_lvl - 1].size;
  int rc = ensure_workspace(ctx, sizeof(int32_t) * n_from + 256);
  if (rc) return rc;
  int32_t* cmap = (int32_t*)ctx->ws;
  rc = compose_map(ctx, h, from_lvl, to_lvl, cmap, n_from);
  if (rc) return rc;
  hipLaunchKernelGGL(k_lift, dim3(grid_for(n_from, 256)), dim3(256), 0, ctx->stream, cmap, size_from,
                     size_to, mode, x_c, n_to, k, x_f, n_from);
  SPC_LAUNCH_CHECK(ctx, "lift");
  return SPC_OK;
}

int spc_spectral_error(spc_ctx* ctx, const spc_hier* h, int lvl, const void* U,
                       const double* lambda, int k, int prec, void* R, double* loss) {
  if (!ctx) return SPC_EINVAL;
  if (!h || lvl < 0 || lvl > (int)h->levels.size() || k < 1 || !U || !lambda || !loss)
    return set_error(ctx, SPC_EINVAL, "bad spectral_error arguments");
  if (lvl == 0) return set_error(ctx, SPC_EINVAL, "level 0 is the input graph; pass lvl >= 1");
  return spectral_impl(ctx, view_of_level(h->levels[lvl - 1]), nullptr, h, lvl, h->n0, U, lambda, k, prec, R,
                       loss, nullptr, nullptr);
}

int spc_hier_cluster_map(spc_ctx* ctx, const spc_hier* h, int lvl, int32_t* cmap) {
  if (!ctx) return SPC_EINVAL;
  if (!h || lvl < 0 || lvl > (int)h->levels.size() || !cmap)
    return set_error(ctx, SPC_EINVAL, "bad cluster map arguments");
  return compose_map(ctx, h, 0, lvl, cmap, h->n0);
}

int spc_spectral_error_graph(spc_ctx* ctx, const spc_graph* coarse, const int32_t* cmap, int64_t n0,
                             const void* U, const double* lambda, int k, int prec, void* R, double* loss) {
  if (!ctx) return SPC_EINVAL;
  if (!cmap || n0 < 1 || k < 1 || !U || !lambda || !loss)
    return set_error(ctx, SPC_EINVAL, "bad spectral_error arguments");
  CoarseView g;
  int rc = view_of_graph(ctx, coarse, g);
  if (rc) return rc;
  return spectral_impl(ctx, g, cmap, nullptr, 0, n0, U, lambda, k, prec, R, loss, nullptr, nullptr);
}

int spc_spectral_error_backward(spc_ctx* ctx, const spc_graph* coarse, const int32_t* cmap, int64_t n0,
                                const void* U, const double* lambda, int k, int prec, void* d_wc,
                                void* d_selfc) {
  if (!ctx) return SPC_EINVAL;
  if (!cmap || n0 < 1 || k < 1 || !U || !lambda || !d_wc || !d_selfc)
    return set_error(ctx, SPC_EINVAL, "bad spectral_error_backward arguments");
  CoarseView g;
  int rc = view_of_graph(ctx, coarse, g);
  if (rc) return rc;
  return spectral_impl(ctx, g, cmap, nullptr, 0, n0, U, lambda, k, prec, nullptr, nullptr, d_wc, d_selfc);
}

int spc_entry_map(spc_ctx* ctx, const spc_graph* fine, const int32_t* cluster_of, const spc_graph* coarse,
                  int32_t* entry_map) {
  if (!ctx) return SPC_EINVAL;
  if (!fine || !coarse || !cluster_of || !entry_map || fine->n < 1 || fine->nnz < 0 || !fine->row_ptr ||
      !coarse->row_ptr || (fine->nnz > 0 && !fine->col) || (coarse->nnz > 0 && !coarse->col))
    return set_error(ctx, SPC_EINVAL, "bad entry_map arguments");
  if (fine->nnz == 0) return SPC_OK;
  hipLaunchKernelGGL(k_entry_map, dim3(grid_for(fine->nnz, 256)), dim3(256), 0, ctx->stream, fine->row_ptr,
                     fine->col, fine->n, fine->nnz, cluster_of, coarse->row_ptr, coarse->col, entry_map);
  SPC_LAUNCH_CHECK(ctx, "entry_map");
  return SPC_OK;
}

int spc_contract_backward(spc_ctx* ctx, const int32_t* entry_map, const int32_t* cluster_of, int64_t nnz_f,
                          int64_t n_f, const double* d_wc, const double* d_selfc, double* d_wf, double* d_selff) {
  if (!ctx) return SPC_EINVAL;
  if (nnz_f < 0 || n_f < 1 || (nnz_f > 0 && (!entry_map || !d_wf)) || !d_selfc || (d_selff && !cluster_of))
    return set_error(ctx, SPC_EINVAL, "bad contract_backward arguments");
  int64_t tot = nnz_f + (d_selff ? n_f : 0);
  if (tot == 0) return SPC_OK;
  hipLaunchKernelGGL(k_contract_backward, dim3(grid_for(tot, 256)), dim3(256), 0, ctx->stream, entry_map, nnz_f,
                     cluster_of, n_f, d_wc, d_selfc, d_wf, d_selff);
  SPC_LAUNCH_CHECK(ctx, "contract_backward");
  return SPC_OK;
}

int spc_validate_graph(const spc_graph* g) {
  if (!g || g->n < 1 || g->nnz < 0 || (g->nnz & 1) || !g->row_ptr) return SPC_EINVAL;
  if (g->nnz > 0 && (!g->col || !g->w)) return SPC_EINVAL;
  const int64_t* rp = g->row_ptr;
  if (rp[0] != 0 || rp[g->n] != g->nnz) return SPC_EINVAL;
  bool fp = g->wtype != SPC_W_I32;
  if (g->wtype < 0 || g->wtype > 2) return SPC_EINVAL;
  auto wv = [&](int64_t j) -> double {
    if (g->wtype == SPC_W_I32) return (double)((const int32_t*)g->w)[j];
    if (g->wtype == SPC_W_F32) return (double)((const float*)g->w)[j];
    return ((const double*)g->w)[j];
  };
  unsigned long long total = 0;
  for (int64_t u = 0; u < g->n; u++) {
    if (rp[u + 1] < rp[u]) return SPC_EINVAL;
    for (int64_t j = rp[u]; j < rp[u + 1]; j++) {
      int64_t v = g->col[j];
      if (v < 0 || v >= g->n || v == u) return SPC_EINVAL;
      if (j > rp[u] && g->col[j - 1] >= v) return SPC_EINVAL;
      double x = wv(j);
      if (!(x > 0.0) || std::isinf(x)) return SPC_EINVAL;
      if (!fp) total += (unsigned long long)((const int32_t*)g->w)[j];
      // mirror entry with an identical weight
      int64_t lo = rp[v], hi = rp[v + 1];
      while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (g->col[mid] < u) lo = mid + 1;
        else hi = mid;
      }
      if (lo >= rp[v + 1] || g->col[lo] != u || wv(lo) != x) return SPC_EINVAL;
    }
    if (g->self_w) {
      if (fp) {
        double s = ((const double*)g->self_w)[u];
        if (!(s >= 0.0) || std::isinf(s)) return SPC_EINVAL;
      } else {
        int64_t s = ((const int64_t*)g->self_w)[u];
        if (s < 0) return SPC_EINVAL;
        total += (unsigned long long)s;
      }
    }
    if (g->size && g->size[u] < 1) return SPC_EINVAL;
    if (!fp && total > 2147483647ull) return SPC_EOVERFLOW;
  }
  return SPC_OK;
}

}  // extern "C"

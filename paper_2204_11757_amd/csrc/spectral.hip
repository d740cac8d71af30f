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
    // |c(u)| relative to u's own size; from the input level this is |c(u)|
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

// y = Q^T u_i (members summed in ascending fine id), t = D_c^{-1/2} y
__global__ void k_restrict_scale(const uint64_t* __restrict__ sorted, const int32_t* __restrict__ mptr,
                                 const double* __restrict__ U, int64_t n0, int k,
                                 const int64_t* __restrict__ rp, const int32_t* __restrict__ w,
                                 const int64_t* __restrict__ self, const int32_t* __restrict__ size,
                                 int64_t nc, double* __restrict__ t) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nc * k) return;
  int64_t a = idx % nc;
  int i = (int)(idx / nc);
  double y = 0.0;
  for (int32_t p = mptr[a]; p < mptr[a + 1]; p++) {
    int64_t u = (int64_t)(sorted[p] & 0xffffffffull);
    y += U[u + n0 * i];
  }
  y = y / sqrt((double)(size ? size[a] : 1));
  int64_t d = self ? self[a] : 0;
  for (int64_t j = rp[a]; j < rp[a + 1]; j++) d += w[j];
  t[a + nc * i] = y / sqrt((double)d);
}

// prod = t * (W_c t), W_c with its diagonal, summed in ascending column
__global__ void k_quad(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                       const int32_t* __restrict__ w, const int64_t* __restrict__ self, int64_t nc,
                       int k, const double* __restrict__ t, double* __restrict__ prod) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nc * k) return;
  int64_t a = idx % nc;
  int i = (int)(idx / nc);
  const double* ti = t + nc * i;
  double s = self ? (double)self[a] : 0.0;
  double z = 0.0;
  bool placed = (s == 0.0);
  for (int64_t j = rp[a]; j < rp[a + 1]; j++) {
    int32_t b = col[j];
    if (!placed && b > a) {
      z += s * ti[a];
      placed = true;
    }
    z += (double)w[j] * ti[b];
  }
  if (!placed) z += s * ti[a];
  prod[idx] = ti[a] * z;
}

// f_i = sum_a prod[a, i]: one block per i, fixed reduction shape
__global__ void __launch_bounds__(256) k_colsum(const double* __restrict__ prod, int64_t nc,
                                                double* __restrict__ R) {
  __shared__ double tmp[256];
  int i = blockIdx.x;
  double s = 0.0;
  for (int64_t a = threadIdx.x; a < nc; a += 256) s += prod[a + nc * i];
  tmp[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) tmp[threadIdx.x] += tmp[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) R[i] = 1.0 - tmp[0];
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

int spc_spectral_error(spc_ctx* ctx, const spc_hier* h, int lvl, const double* U,
                       const double* lambda, int k, double* R, double* loss) {
  if (!ctx) return SPC_EINVAL;
  if (!h || lvl < 0 || lvl > (int)h->levels.size() || k < 1 || !U || !lambda || !loss)
    return set_error(ctx, SPC_EINVAL, "bad spectral_error arguments");
  if (lvl == 0) return set_error(ctx, SPC_EINVAL, "level 0 is the input graph; pass lvl >= 1");
  const auto& L = h->levels[lvl - 1];
  int64_t n0 = h->n0, nc = L.n;
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
    int32_t* partial = A.take<int32_t>(SCAN_MAXB);
    double* t = A.take<double>(nc * k);
    double* prod = A.take<double>(nc * k);
    double* Rd = A.take<double>(k);
    if (pass == 0) {
      A.cap = A.off;
      continue;
    }
    hipStream_t st = ctx->stream;
    int rc = compose_map(ctx, h, 0, lvl, cmap, n0);
    if (rc) return rc;
    hipLaunchKernelGGL(k_pair_keys, dim3(grid_for(n0, 256)), dim3(256), 0, st, cmap, n0, ka);
    uint64_t* sorted = nullptr;
    rc = merge_sort<uint64_t, LessU64>(ctx, ka, kb, n0, LessU64(), &sorted);
    if (rc) return rc;
    SPC_HIP(ctx, hipMemsetAsync(mptr, 0, sizeof(int32_t) * (nc + 1), st));
    hipLaunchKernelGGL(k_count_clusters, dim3(grid_for(n0, 256)), dim3(256), 0, st, cmap, n0, mptr);
    rc = exclusive_scan<int32_t>(ctx, mptr, mptr, nc, partial);
    if (rc) return rc;
    int64_t nk = nc * k;
    hipLaunchKernelGGL(k_restrict_scale, dim3(grid_for(nk, 256)), dim3(256), 0, st, sorted, mptr, U, n0,
                       k, L.rp, L.w, L.self, L.size, nc, t);
    hipLaunchKernelGGL(k_quad, dim3(grid_for(nk, 256)), dim3(256), 0, st, L.rp, L.col, L.w, L.self, nc,
                       k, t, prod);
    hipLaunchKernelGGL(k_colsum, dim3(k), dim3(256), 0, st, prod, nc, R ? R : Rd);
    SPC_LAUNCH_CHECK(ctx, "spectral_error");
    std::vector<double> hR(k), hl(k);
    SPC_HIP(ctx, hipMemcpyAsync(hR.data(), R ? R : Rd, sizeof(double) * k, hipMemcpyDeviceToHost, st));
    SPC_HIP(ctx, hipMemcpyAsync(hl.data(), lambda, sizeof(double) * k, hipMemcpyDeviceToHost, st));
    SPC_HIP(ctx, hipStreamSynchronize(st));
    double s = 0.0;
    for (int i = 0; i < k; i++) s += (hR[i] - hl[i]) * (hR[i] - hl[i]);
    *loss = s;
  }
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

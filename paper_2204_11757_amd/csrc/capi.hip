// C ABI of the coarsening library (declared in include/spc.h): context,
// allocation hooks, error reporting, the level / multilevel entry points,
// the hierarchy, the lift (Definition 2) and the spectral error.
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <mutex>
#include <new>

#include "level.hpp"

using namespace spc;

namespace spc {

int set_error(spc_ctx* ctx, int code, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->err = buf;
    ctx->err_code = code;
  }
  return code;
}

int hip_error(spc_ctx* ctx, hipError_t e, const char* where) {
  return set_error(ctx, SPC_EHIP, "HIP error %d (%s) at %s", (int)e, hipGetErrorString(e), where);
}

void* dev_alloc(spc_ctx* ctx, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (ctx->alloc_fn) return ctx->alloc_fn(bytes, ctx->alloc_user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void dev_free(spc_ctx* ctx, void* p) {
  if (!p) return;
  if (ctx->free_fn) ctx->free_fn(p, ctx->alloc_user);
  else (void)hipFree(p);
}

int ensure_workspace(spc_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->ws_cap) return SPC_OK;
  if (ctx->no_alloc)
    return set_error(ctx, SPC_ECAPACITY, "the level needs %zu bytes of workspace, the scratch array holds %zu",
                     bytes, ctx->ws_cap);
  if (ctx->ws) {
    SPC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    dev_free(ctx, ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_cap = 0;
  }
  void* p = dev_alloc(ctx, bytes);
  if (!p) return set_error(ctx, SPC_ENOMEM, "workspace allocation of %zu bytes failed", bytes);
  ctx->ws = p;
  ctx->ws_cap = bytes;
  return SPC_OK;
}

int readback(spc_ctx* ctx, const void* dev, size_t bytes, void* host) {
  SPC_HIP(ctx, hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, ctx->stream));
  SPC_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return SPC_OK;
}

uint32_t scan_state_reserve(spc_ctx* ctx, int64_t words) {
  words += 1;   // the last word is the error flag
  if (words > ctx->scan_cap || ctx->scan_epoch >= LB_MAX_EPOCH) {
    if (words > ctx->scan_cap && ctx->no_alloc) {
      set_error(ctx, SPC_ECAPACITY, "a scan needs %lld look-back words, the scratch array holds %lld",
                (long long)words, (long long)ctx->scan_cap);
      return 0;
    }
    if (words > ctx->scan_cap) {
      int64_t cap = words > (1 << 16) ? words : (1 << 16);
      if (ctx->scan_state) {
        if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
          set_error(ctx, SPC_EHIP, "stream synchronisation failed");
          return 0;
        }
        dev_free(ctx, ctx->scan_state);
      }
      ctx->scan_state = (uint64_t*)dev_alloc(ctx, sizeof(uint64_t) * (size_t)cap);
      if (!ctx->scan_state) {
        ctx->scan_cap = 0;
        set_error(ctx, SPC_ENOMEM, "scan state allocation failed");
        return 0;
      }
      ctx->scan_cap = cap;
    }
    launch_zero(ctx, ctx->scan_state, sizeof(uint64_t) * (size_t)ctx->scan_cap);
    if (hipGetLastError() != hipSuccess) {
      set_error(ctx, SPC_EHIP, "scan state clear failed");
      return 0;
    }
    ctx->scan_epoch = 0;
  }
  return ++ctx->scan_epoch;
}

static int plan_and_bind(spc_ctx* ctx, int64_t n, int64_t nnz, LevelWork& W, bool fp) {
  Arena count;
  count.counting = true;
  plan_level(count, n, nnz, W, fp);
  int rc = ensure_workspace(ctx, count.off + 256);
  if (rc) return rc;
  Arena real;
  real.base = (char*)ctx->ws;
  real.cap = ctx->ws_cap;
  plan_level(real, n, nnz, W, fp);
  return SPC_OK;
}

__global__ void k_iota32(int32_t* a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = (int32_t)i;
}

__global__ void k_identity_aux(const int64_t* __restrict__ self_in, const int32_t* __restrict__ size_in,
                               int64_t* __restrict__ self_out, int32_t* __restrict__ size_out,
                               int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    self_out[i] = self_in ? self_in[i] : 0;
    size_out[i] = size_in ? size_in[i] : 1;
  }
}

static int check_graph(spc_ctx* ctx, const spc_graph* g) {
  if (!g) return set_error(ctx, SPC_EINVAL, "graph is NULL");
  if (g->n < 1 || g->n > INT32_MAX) return set_error(ctx, SPC_EINVAL, "n=%lld out of range", (long long)g->n);
  if (g->nnz < 0 || (g->nnz & 1) || g->nnz > INT32_MAX)
    return set_error(ctx, SPC_EINVAL, "nnz=%lld must be even and below 2^31", (long long)g->nnz);
  if (!g->row_ptr || (g->nnz > 0 && (!g->col || !g->w)))
    return set_error(ctx, SPC_EINVAL, "graph arrays are NULL");
  if (g->wtype != SPC_W_I32 && g->wtype != SPC_W_F32 && g->wtype != SPC_W_F64)
    return set_error(ctx, SPC_EINVAL, "unknown weight type %d", (int)g->wtype);
  return SPC_OK;
}

static LevelInF level_in_f(const spc_graph* g) {
  LevelInF L;
  L.n = g->n;
  L.nnz = g->nnz;
  L.rp = g->row_ptr;
  L.col = g->col;
  L.w = g->w;
  L.w32 = g->wtype == SPC_W_F32 ? 1 : 0;
  L.self = (const double*)g->self_w;
  L.size = g->size;
  return L;
}

// identity level of a floating-point graph: weights widened to FP64
__global__ void k_identity_fp(const void* __restrict__ w, int w32, int64_t nnz, const double* __restrict__ self_in,
                              const int32_t* __restrict__ size_in, int64_t n, double* __restrict__ w_out,
                              double* __restrict__ self_out, int32_t* __restrict__ size_out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nnz) w_out[i] = w32 ? (double)((const float*)w)[i] : ((const double*)w)[i];
  if (i < n) {
    self_out[i] = self_in ? self_in[i] : 0.0;
    size_out[i] = size_in ? size_in[i] : 1;
  }
}

// seen[perm[i]] counts the preimages of every target; a target out of
// range or hit twice sets *bad
__global__ void k_perm_mark(const int32_t* __restrict__ perm, int64_t n, int32_t* seen, unsigned long long* bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t p = perm[i];
  if (p < 0 || p >= n || atomicAdd(&seen[p], 1) != 0) *bad = 1;
}

static LevelIn level_in(const spc_graph* g) {
  LevelIn L;
  L.n = g->n;
  L.nnz = g->nnz;
  L.rp = g->row_ptr;
  L.col = g->col;
  L.w = (const int32_t*)g->w;
  L.self = (const int64_t*)g->self_w;
  L.size = g->size;
  return L;
}

// one level into caller buffers
// With ev non-null the level's start and end events are recorded there and
// not waited for (st->ms_total is filled in later); otherwise the call waits
// for the level's end to time it.
static int level_impl(spc_ctx* ctx, const spc_graph* g, int64_t t, int32_t* cluster_of,
                      spc_graph_out* out, int64_t* nnz_c, spc_level_stats* st,
                      const Segments* seg = nullptr, hipEvent_t* ev = nullptr) {
  int rc = check_graph(ctx, g);
  if (rc) return rc;
  if (t < 1) return set_error(ctx, SPC_EINVAL, "n_target must be >= 1");
  if (!cluster_of || !out || !nnz_c) return set_error(ctx, SPC_EINVAL, "output is NULL");
  if (t > g->n) t = g->n;
  if (!out->row_ptr || !out->self_w || !out->size || (g->nnz > 0 && (!out->col || !out->w)))
    return set_error(ctx, SPC_EINVAL, "output arrays are NULL");
  if (out->n_cap < t) return set_error(ctx, SPC_ECAPACITY, "n_cap %lld < %lld", (long long)out->n_cap, (long long)t);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (st && !ctx->no_alloc) {
    // events from the context's pool (creating one is a runtime call the
    // level boundary need not wait for)
    e0 = ev_get(ctx);
    e1 = ev_get(ctx);
    if (!e0 || !e1) return set_error(ctx, SPC_EHIP, "event creation failed");
    SPC_HIP(ctx, hipEventRecord(e0, ctx->stream));
  }
  bool fp = g->wtype != SPC_W_I32;
  LevelIn L = level_in(g);
  LevelInF LF = level_in_f(g);
  if (fp) {
    L.w = nullptr;      // the structure only: every weight read goes through LF
    L.self = nullptr;
  }
  LevelWork W;
  LevelResult R;
  rc = plan_and_bind(ctx, g->n, g->nnz, W, fp);
  if (rc) return rc;
  // the integer path checks the selection at the contraction's first
  // synchronisation (one wait per level fewer); a batch waits, since a graph
  // short of forest edges leaves more super-nodes than the target
  bool defer = !fp && !seg && t < g->n;
  // nor for the first forest batch when the last level's forest was complete
  // after it, in one band
  bool spec = defer && (ctx->speculate == 2 || (ctx->speculate == 0 && ctx->spec_ok));
  // the first batch of forest rounds as long as the last level of this size
  // class needed (else as the previous level's); launch counts only
  int cls = bitlen64((uint64_t)g->nnz);
  if (ctx->forest_batch_cls[cls] > 0) ctx->forest_batch = ctx->forest_batch_cls[cls];
  rc = select_level(ctx, L, t, cluster_of, W, R, fp ? &LF : nullptr, seg, defer, false, spec);
  if (rc == SPC_REDO_BAND) {
    // a graph of the batch had fewer forest edges inside its band than
    // merges: the selection again over every edge
    R = LevelResult();
    ctx->seg_full_band = 1;
    rc = select_level(ctx, L, t, cluster_of, W, R, fp ? &LF : nullptr, seg, defer, false, spec);
    ctx->seg_full_band = 0;
  }
  if (rc) return rc;
  if (fp && R.n_c == g->n) {
    if (out->nnz_cap < g->nnz) return set_error(ctx, SPC_ECAPACITY, "nnz_cap too small");
    SPC_HIP(ctx, hipMemcpyAsync(out->row_ptr, g->row_ptr, sizeof(int64_t) * (g->n + 1),
                                hipMemcpyDeviceToDevice, ctx->stream));
    if (g->nnz)
      SPC_HIP(ctx, hipMemcpyAsync(out->col, g->col, sizeof(int32_t) * g->nnz, hipMemcpyDeviceToDevice,
                                  ctx->stream));
    hipLaunchKernelGGL(k_identity_fp, dim3(grid_for(std::max(g->n, g->nnz), 256)), dim3(256), 0, ctx->stream,
                       g->w, LF.w32, g->nnz, LF.self, g->size, g->n, (double*)out->w, (double*)out->self_w,
                       out->size);
    SPC_LAUNCH_CHECK(ctx, "identity");
    R.nnz_c = g->nnz;
    R.maxcl = 1;
  } else if (fp) {
    rc = contract_level_fp(ctx, LF, cluster_of, R.n_c, out, W, R);
    if (rc) return rc;
  } else if (R.n_c == g->n) {
    // identity: copy the graph
    if (out->nnz_cap < g->nnz) return set_error(ctx, SPC_ECAPACITY, "nnz_cap too small");
    SPC_HIP(ctx, hipMemcpyAsync(out->row_ptr, g->row_ptr, sizeof(int64_t) * (g->n + 1),
                                hipMemcpyDeviceToDevice, ctx->stream));
    if (g->nnz) {
      SPC_HIP(ctx, hipMemcpyAsync(out->col, g->col, sizeof(int32_t) * g->nnz, hipMemcpyDeviceToDevice,
                                  ctx->stream));
      SPC_HIP(ctx, hipMemcpyAsync(out->w, g->w, sizeof(int32_t) * g->nnz, hipMemcpyDeviceToDevice,
                                  ctx->stream));
    }
    hipLaunchKernelGGL(k_identity_aux, dim3(grid_for(g->n, 256)), dim3(256), 0, ctx->stream,
                       (const int64_t*)g->self_w, g->size, (int64_t*)out->self_w, out->size, g->n);
    SPC_LAUNCH_CHECK(ctx, "identity");
    R.nnz_c = g->nnz;
    R.maxcl = 1;
  } else {
    // (the level's integer degree pass left the entry tiles' first rows)
    rc = contract_level(ctx, L, cluster_of, R.n_c, out, W, R, seg, W.ptrow);
    if (rc == SPC_REDO_SPEC) {
      // the forest needed more than its first batch: the level again, waiting
      R = LevelResult();
      rc = select_level(ctx, L, t, cluster_of, W, R, nullptr, seg, defer, false, false);
      if (rc) return rc;
      rc = contract_level(ctx, L, cluster_of, R.n_c, out, W, R, seg, W.ptrow);
    }
    if (rc == SPC_REDO_RANK) {
      // a guarded key decision failed: the level again with rank keys
      R = LevelResult();
      rc = select_level(ctx, L, t, cluster_of, W, R, nullptr, seg, false, true);
      if (rc) return rc;
      rc = contract_level(ctx, L, cluster_of, R.n_c, out, W, R, seg, W.ptrow);
    }
    if (rc) return rc;
  }
  *nnz_c = R.nnz_c;
  ctx->forest_batch_cls[cls] = ctx->forest_batch;   // (this level's need, from its selection)
  if (st) {
    float ms = 0;
    if (!e0) {
      // no events (the call that allocates nothing): not timed
    } else if (ev) {
      SPC_HIP(ctx, hipEventRecord(e1, ctx->stream));
      ev[0] = e0;
      ev[1] = e1;
    } else {
      SPC_HIP(ctx, hipEventRecord(e1, ctx->stream));
      SPC_HIP(ctx, hipEventSynchronize(e1));
      SPC_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
      ctx->ev_pool.push_back(e0);
      ctx->ev_pool.push_back(e1);
    }
    st->n_in = g->n;
    st->m_in = g->nnz / 2;
    st->n_out = R.n_c;
    st->nnz_out = R.nnz_c;
    st->merges = g->n - R.n_c;
    st->largest_cluster = R.maxcl;
    st->boruvka_rounds = R.rounds;
    st->candidate_edges = R.candidates;
    st->key_mode = R.key_mode;
    st->key_bits = R.key_bits;
    st->eps_max = R.eps;
    st->ms_total = ms;
    st->bands = R.bands;
    st->forest_in = R.forest_in;
    st->forest_kept = R.forest_kept;
    st->merge_in = R.merge_in;
    st->forest_edges = R.msf;
    st->keys_written = R.keys_written;
  }
  return SPC_OK;
}

}  // namespace spc

// ===========================================================================
// scratch of the entry point that allocates nothing
// ===========================================================================

// One array per device, in the library's code object: the workspace of
// spc_coarsen_level_noalloc (its first SPC_NOALLOC_SCAN_WORDS 8-byte words
// from the end hold the scan chain's look-back words).  In host code the
// name stands for a host-side shadow, not a device address: kernels only
// ever receive the address hipGetSymbolAddress resolves for the current
// device (kept per device in g_scratch).
static __device__ __align__(256) char scratch[SPC_NOALLOC_SCRATCH_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
constexpr int64_t SPC_NOALLOC_SCAN_WORDS = 1 << 16;
static std::mutex g_scratch_mu;
static void* g_scratch[SCRATCH_MAX_DEVICES];

// Device address of `scratch` on `device`, which must be current; resolved
// once per device.  Null when the lookup fails.
static void* resolve_scratch(int device) {
  if (device < 0 || device >= SCRATCH_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p) g_scratch[device] = p;
  }
  return g_scratch[device];
}

// ===========================================================================
// hierarchy
// ===========================================================================

// Target of the next level from n_l nodes (n_l > n_c).  schedule 0: halve,
// max(n_c, ceil(n_l / 2)); 1: straight to n_c (Algorithm 1 as printed, one
// scoring); -j (j >= 1): j merges per level, max(n_c, n_l - j), i.e. the
// scores are recomputed after every j merges (j = 1 is the explicit greedy
// algorithm, which recomputes every norm after each merge).
static int64_t level_target(int64_t n, int64_t n_c, int schedule) {
  if (schedule == 1) return n_c;
  if (schedule < 0) return std::max(n_c, n + (int64_t)schedule);
  return std::max(n_c, (n + 1) / 2);
}

// Launch settings for a call on input g: the tuned ones of its size class
// (unless spc_autotune is running a trial), else the built-in rules.
static int size_class(int64_t nnz, bool batched) { return bitlen64((uint64_t)nnz) + (batched ? 64 : 0); }

static void apply_tune(spc_ctx* ctx, int64_t nnz, bool batched) {
  if (ctx->tune_forced) return;
  ctx->tune = spc_tune();
  int key = size_class(nnz, batched);
  for (auto& kv : ctx->tuned)
    if (kv.first == key) ctx->tune = kv.second;
  const spc_tune& f = ctx->tune_set;
  if (f.lane_max) ctx->tune.lane_max = f.lane_max;
  if (f.wave_max) ctx->tune.wave_max = f.wave_max;
  if (f.small_rpt) ctx->tune.small_rpt = f.small_rpt;
  if (f.huge_tile) ctx->tune.huge_tile = f.huge_tile;
  if (f.sel_blocks) ctx->tune.sel_blocks = f.sel_blocks;
  if (f.bv_short) ctx->tune.bv_short = f.bv_short;
}

static void free_level(spc_ctx* ctx, spc_hier::Level& L) {
  dev_free(ctx, L.block);
  for (hipEvent_t& e : L.ev)
    if (e) ctx->ev_pool.push_back(e);
  L = spc_hier::Level();
}

// One allocation per level (each allocation may be a call into the host
// program's allocator), carved into the level's arrays at 256-byte offsets.
static bool alloc_level(spc_ctx* ctx, spc_hier::Level& L, int64_t t, int64_t nnz_cap, int64_t n_prev,
                        size_t wsz) {
  size_t sz[6] = {sizeof(int64_t) * (size_t)(t + 1), sizeof(int32_t) * (size_t)nnz_cap, wsz * (size_t)nnz_cap,
                  sizeof(int64_t) * (size_t)t, sizeof(int32_t) * (size_t)t, sizeof(int32_t) * (size_t)n_prev};
  size_t off[6], tot = 0;
  for (int i = 0; i < 6; i++) {
    off[i] = tot;
    tot += (sz[i] + 255) & ~(size_t)255;
  }
  L.block = dev_alloc(ctx, tot);
  if (!L.block) return false;
  char* b = (char*)L.block;
  L.rp = (int64_t*)(b + off[0]);
  L.col = (int32_t*)(b + off[1]);
  L.w = b + off[2];
  L.self = b + off[3];
  L.size = (int32_t*)(b + off[4]);
  L.cluster_of = (int32_t*)(b + off[5]);
  return true;
}

// Per-level times recorded without waiting: read after the last level.
static int finish_timing(spc_ctx* ctx, spc_hier* h) {
  for (auto& L : h->levels) {
    if (!L.ev[0]) continue;
    SPC_HIP(ctx, hipEventSynchronize(L.ev[1]));
    float ms = 0;
    SPC_HIP(ctx, hipEventElapsedTime(&ms, L.ev[0], L.ev[1]));
    L.st.ms_total = ms;
    ctx->ev_pool.push_back(L.ev[0]);
    ctx->ev_pool.push_back(L.ev[1]);
    L.ev[0] = L.ev[1] = nullptr;
  }
  h->timing_pending = false;
  return SPC_OK;
}

extern "C" {

const char* spc_strerror(int code) {
  switch (code) {
    case SPC_OK: return "ok";
    case SPC_EINVAL: return "invalid argument or malformed graph";
    case SPC_EUNREACHABLE: return "target below the number of connected components";
    case SPC_EOVERFLOW: return "integer weight total exceeds 2^31-1";
    case SPC_ECAPACITY: return "output capacity too small";
    case SPC_ENOMEM: return "allocation failed";
    case SPC_EHIP: return "HIP runtime error";
    case SPC_ERANGE: return "floating-point weights span too wide a range";
    default: return "unknown error";
  }
}

int spc_create(spc_ctx** out, int device, void* stream) {
  if (!out) return SPC_EINVAL;
  spc_ctx* ctx = new (std::nothrow) spc_ctx();
  if (!ctx) return SPC_ENOMEM;
  ctx->device = device;
  ctx->stream = (hipStream_t)stream;
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return SPC_EHIP;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
    ctx->num_cus = cus;
  // with the device current: this device's scratch array (a failure only
  // disables the entry point that allocates nothing)
  ctx->scratch = resolve_scratch(device);
  // coherent: the host polls a word that a running kernel writes
  if (hipHostMalloc((void**)&ctx->h_pinned, 4096, hipHostMallocCoherent) != hipSuccess) {
    delete ctx;
    return SPC_ENOMEM;
  }
  *out = ctx;
  return SPC_OK;
}

int spc_destroy(spc_ctx* ctx) {
  if (!ctx) return SPC_OK;
  (void)hipStreamSynchronize(ctx->stream);
  dev_free(ctx, ctx->ws);
  dev_free(ctx, ctx->scan_state);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->h_pinned) (void)hipHostFree(ctx->h_pinned);
  delete ctx;
  return SPC_OK;
}

int spc_set_stream(spc_ctx* ctx, void* stream) {
  if (!ctx) return SPC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (s == ctx->stream) return SPC_OK;
  // Work queued by earlier calls on the old stream still uses the context's
  // workspace, look-back words and pinned readback area: the new stream
  // waits for it on the device (no host wait).
  hipEvent_t e = ev_get(ctx);
  if (!e) return set_error(ctx, SPC_EHIP, "event creation failed");
  hipError_t r = hipEventRecord(e, ctx->stream);
  if (r == hipSuccess) r = hipStreamWaitEvent(s, e, 0);
  ctx->ev_pool.push_back(e);
  if (r != hipSuccess) return hip_error(ctx, r, "ordering the new stream after the old one");
  ctx->stream = s;
  return SPC_OK;
}

int spc_set_allocator(spc_ctx* ctx, void* (*alloc)(size_t, void*), void (*free_)(void*, void*),
                      void* user) {
  if (!ctx) return SPC_EINVAL;
  if ((alloc == nullptr) != (free_ == nullptr)) return set_error(ctx, SPC_EINVAL, "allocator pair incomplete");
  if (ctx->ws || ctx->scan_state) {
    (void)hipStreamSynchronize(ctx->stream);
    dev_free(ctx, ctx->ws);
    dev_free(ctx, ctx->scan_state);
    ctx->ws = nullptr;
    ctx->ws_cap = 0;
    ctx->scan_state = nullptr;
    ctx->scan_cap = 0;
  }
  ctx->alloc_fn = alloc;
  ctx->free_fn = free_;
  ctx->alloc_user = user;
  return SPC_OK;
}

const char* spc_last_error(const spc_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

int spc_set_option(spc_ctx* ctx, const char* name, int64_t value) {
  if (!ctx || !name) return SPC_EINVAL;
  if (!strcmp(name, "rank_order")) ctx->force_rank_mode = value ? 1 : 0;
  else if (!strcmp(name, "full_forest")) ctx->force_full_filter = value ? 1 : 0;
  else if (!strcmp(name, "batch_band_short")) ctx->seg_band_shrink = value ? 1 : 0;
  else if (!strcmp(name, "timing")) ctx->timing = value ? 1 : 0;
  else if (!strcmp(name, "huge_sort")) ctx->force_huge_sort = value ? 1 : 0;
  else if (!strcmp(name, "redo_rank")) ctx->force_redo_rank = value ? 1 : 0;
  else if (!strcmp(name, "bad_select_guess")) ctx->force_bad_guess = value ? 1 : 0;
  else if (!strcmp(name, "scan_flag")) ctx->force_scan_flag = value ? 1 : 0;
  else if (!strcmp(name, "lane_max")) {
    if (value != 0 && value != 16 && value != 32) return set_error(ctx, SPC_EINVAL, "lane_max takes 0, 16 or 32");
    ctx->tune_set.lane_max = (int)value;
  } else if (!strcmp(name, "wave_max")) {
    if (value != 0 && (value < 64 || value > 512)) return set_error(ctx, SPC_EINVAL, "wave_max takes 0 or 64..512");
    ctx->tune_set.wave_max = (int)value;
  } else if (!strcmp(name, "small_rpt")) {
    if (value != 0 && value != 1 && value != 2 && value != 4)
      return set_error(ctx, SPC_EINVAL, "small_rpt takes 0, 1, 2 or 4");
    ctx->tune_set.small_rpt = (int)value;
  } else if (!strcmp(name, "huge_tile")) {
    if (value != 0 && value != 1024 && value != 4096)
      return set_error(ctx, SPC_EINVAL, "huge_tile takes 0, 1024 or 4096");
    ctx->tune_set.huge_tile = (int)value;
  } else if (!strcmp(name, "sel_blocks")) {
    if (value < 0 || value > 128) return set_error(ctx, SPC_EINVAL, "sel_blocks takes 0..128");
    ctx->tune_set.sel_blocks = (int)value;
  } else if (!strcmp(name, "bv_short")) {
    if (value < 0) return set_error(ctx, SPC_EINVAL, "bv_short takes a length >= 0");
    ctx->tune_set.bv_short = value;
  }
  else if (!strcmp(name, "speculate")) {
    if (value < 0 || value > 2) return set_error(ctx, SPC_EINVAL, "speculate takes 0, 1 or 2");
    ctx->speculate = (int)value;
  } else if (!strcmp(name, "contract_wait")) {
    if (value < 0 || value > 3) return set_error(ctx, SPC_EINVAL, "contract_wait takes 0 to 3");
    ctx->contract_wait = (int)value;
  }
  else return set_error(ctx, SPC_EINVAL, "unknown option '%s'", name);
  return SPC_OK;
}

int spc_timing_report(spc_ctx* ctx, char* buf, size_t cap) {
  if (!ctx || !buf || cap == 0) return SPC_EINVAL;
  SPC_HIP(ctx, hipStreamSynchronize(ctx->stream));
  struct Agg {
    std::string name;
    int64_t count = 0;
    double ms = 0.0, units = 0.0;
  };
  std::vector<Agg> agg;
  for (auto& m : ctx->marks) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, m.a, m.b) != hipSuccess) ms = 0.f;
    size_t i = 0;
    while (i < agg.size() && agg[i].name != m.name) i++;
    if (i == agg.size()) {
      agg.push_back(Agg());
      agg.back().name = m.name;
    }
    agg[i].count++;
    agg[i].ms += ms;
    agg[i].units += m.units;
    ctx->ev_pool.push_back(m.a);
    ctx->ev_pool.push_back(m.b);
  }
  ctx->marks.clear();
  std::string out;
  char line[256];
  for (auto& a : agg) {
    snprintf(line, sizeof(line), "%s %lld %.6f %.0f\n", a.name.c_str(), (long long)a.count, a.ms, a.units);
    out += line;
  }
  if (out.size() + 1 > cap) return set_error(ctx, SPC_ECAPACITY, "timing report needs %zu bytes", out.size() + 1);
  memcpy(buf, out.c_str(), out.size() + 1);
  return SPC_OK;
}

int spc_coarsen_level(spc_ctx* ctx, const spc_graph* g, int64_t n_target, int32_t* cluster_of,
                      spc_graph_out* coarse, int64_t* nnz_c, spc_level_stats* st) {
  if (!ctx) return SPC_EINVAL;
  ctx->spec_ok = 0;   // a new graph: its first level waits for its forest
  if (g) apply_tune(ctx, g->nnz, false);
  return level_impl(ctx, g, n_target, cluster_of, coarse, nnz_c, st);
}

int spc_coarsen_level_noalloc(spc_ctx* ctx, const spc_graph* g, int64_t n_target, int32_t* cluster_of,
                              spc_graph_out* coarse, int64_t* nnz_c, spc_level_stats* st) {
  if (!ctx) return SPC_EINVAL;
  if (!ctx->scratch)
    return set_error(ctx, SPC_EHIP, "the scratch array of device %d could not be resolved", ctx->device);
  int rc = check_graph(ctx, g);
  if (rc) return rc;
  const size_t scan_bytes = sizeof(uint64_t) * (size_t)SPC_NOALLOC_SCAN_WORDS;
  const size_t ws_bytes = (size_t)SPC_NOALLOC_SCRATCH_BYTES - scan_bytes;
  {
    Arena count;
    count.counting = true;
    LevelWork W;
    plan_level(count, g->n, g->nnz, W, g->wtype != SPC_W_I32);
    if (count.off + 256 > ws_bytes)
      return set_error(ctx, SPC_ECAPACITY,
                       "n=%lld nnz=%lld needs %zu bytes of workspace; the scratch array holds %zu",
                       (long long)g->n, (long long)g->nnz, (size_t)(count.off + 256), ws_bytes);
  }
  // the context's workspace and scan chain stand aside for the scratch
  // array's; the scan words start cleared (the first scan clears them, as
  // with a fresh chain), the level clears the rest of what must start at zero
  void* ws = ctx->ws;
  size_t ws_cap = ctx->ws_cap;
  uint64_t* scan = ctx->scan_state;
  int64_t scan_cap = ctx->scan_cap;
  uint32_t scan_epoch = ctx->scan_epoch;
  int timing = ctx->timing;
  ctx->ws = ctx->scratch;
  ctx->ws_cap = ws_bytes;
  ctx->scan_state = (uint64_t*)((char*)ctx->scratch + ws_bytes);
  ctx->scan_cap = SPC_NOALLOC_SCAN_WORDS;
  ctx->scan_epoch = LB_MAX_EPOCH;
  ctx->timing = 0;
  ctx->no_alloc = 1;
  ctx->spec_ok = 0;
  apply_tune(ctx, g->nnz, false);
  rc = level_impl(ctx, g, n_target, cluster_of, coarse, nnz_c, st);
  ctx->no_alloc = 0;
  ctx->timing = timing;
  ctx->ws = ws;
  ctx->ws_cap = ws_cap;
  ctx->scan_state = scan;
  ctx->scan_cap = scan_cap;
  ctx->scan_epoch = scan_epoch;
  ctx->spec_ok = 0;
  return rc;
}

int spc_relabel(spc_ctx* ctx, const spc_graph* g, const int32_t* perm, spc_graph_out* out, int64_t* nnz_out) {
  if (!ctx) return SPC_EINVAL;
  int rc = check_graph(ctx, g);
  if (rc) return rc;
  if (!perm || !out || !nnz_out) return set_error(ctx, SPC_EINVAL, "relabel arguments are NULL");
  if (!out->row_ptr || !out->self_w || !out->size || (g->nnz > 0 && (!out->col || !out->w)))
    return set_error(ctx, SPC_EINVAL, "output arrays are NULL");
  if (out->n_cap < g->n || out->nnz_cap < g->nnz)
    return set_error(ctx, SPC_ECAPACITY, "relabel output needs n_cap >= n and nnz_cap >= nnz");
  bool fp = g->wtype != SPC_W_I32;
  apply_tune(ctx, g->nnz, false);
  LevelWork W;
  rc = plan_and_bind(ctx, g->n, g->nnz, W, fp);
  if (rc) return rc;
  // perm must be a permutation of [0, n): every target hit exactly once
  launch_clear(ctx, W.mcount, g->n + 1, nullptr, 0, W.info, 0xffffffffu);
  hipLaunchKernelGGL(k_perm_mark, dim3(grid_for(g->n, 256)), dim3(256), 0, ctx->stream, perm, g->n, W.mcount,
                     &W.info[I_VIOL]);
  SPC_LAUNCH_CHECK(ctx, "permutation check");
  // FP weights: their exponent range fixes the fixed-point unit of the
  // exact sums (and is checked like a level's input)
  if (fp) launch_fp_degree(ctx, level_in_f(g), W);
  rc = readback_wait(ctx, W.info, (int)I_NINFO);
  if (rc) return rc;
  if (ctx->h_pinned[I_VIOL]) return set_error(ctx, SPC_EINVAL, "perm is not a permutation of [0, n)");
  if (fp && (ctx->h_pinned[I_FP_BAD] & 1))
    return set_error(ctx, SPC_EINVAL, "floating-point weights must be finite and positive");
  if (fp && (ctx->h_pinned[I_FP_BAD] & 2))
    return set_error(ctx, SPC_ERANGE, "floating-point weights span more than %d binades", FP_MAX_SPAN);
  // the contraction of Definition 1 with singleton super-nodes c(u) = perm[u]
  LevelResult R;
  if (fp) rc = contract_level_fp(ctx, level_in_f(g), perm, g->n, out, W, R);
  else rc = contract_level(ctx, level_in(g), perm, g->n, out, W, R, nullptr);
  if (rc) return rc;
  *nnz_out = R.nnz_c;
  return SPC_OK;
}

int spc_coarsen_to(spc_ctx* ctx, const spc_graph* g, int64_t n_c, int schedule, spc_hier** out) {
  if (!ctx) return SPC_EINVAL;
  if (!out) return set_error(ctx, SPC_EINVAL, "out is NULL");
  *out = nullptr;
  ctx->spec_ok = 0;   // a new graph: its first level waits for its forest
  int rc = check_graph(ctx, g);
  if (rc) return rc;
  if (n_c < 1) return set_error(ctx, SPC_EINVAL, "n_c must be >= 1");
  if (schedule > 1) return set_error(ctx, SPC_EINVAL, "unknown schedule %d", schedule);
  apply_tune(ctx, g->nnz, false);
  spc_hier* h = new (std::nothrow) spc_hier();
  if (!h) return SPC_ENOMEM;
  h->ctx = ctx;
  h->n0 = g->n;
  spc_graph cur = *g;
  int64_t n = g->n;
  bool fp = g->wtype != SPC_W_I32;
  size_t wsz = fp ? sizeof(double) : sizeof(int32_t);
  while (n > n_c) {
    int64_t t = level_target(n, n_c, schedule);
    spc_hier::Level L;
    L.n_prev = n;
    L.wtype = fp ? SPC_W_F64 : SPC_W_I32;
    if (!alloc_level(ctx, L, t, std::max<int64_t>(cur.nnz, 1), n, wsz)) {
      spc_hier_free(h);
      return set_error(ctx, SPC_ENOMEM, "hierarchy allocation failed");
    }
    spc_graph_out o{L.rp, L.col, L.w, L.self, L.size, t, std::max<int64_t>(cur.nnz, 1)};
    int64_t nnz_c = 0;
    rc = level_impl(ctx, &cur, t, L.cluster_of, &o, &nnz_c, &L.st, nullptr, L.ev);
    if (rc) {
      free_level(ctx, L);
      spc_hier_free(h);
      return rc;
    }
    L.n = t;
    L.nnz = nnz_c;
    h->levels.push_back(L);
    cur.n = t;
    cur.nnz = nnz_c;
    cur.row_ptr = L.rp;
    cur.col = L.col;
    cur.w = L.w;
    cur.self_w = L.self;
    cur.size = L.size;
    cur.wtype = L.wtype;
    n = t;
  }
  h->timing_pending = true;
  *out = h;
  return SPC_OK;
}

int spc_coarsen_batched(spc_ctx* ctx, int32_t G, const spc_graph* g, const int64_t* graph_off,
                        const int64_t* n_c, int schedule, spc_hier** out) {
  if (!ctx) return SPC_EINVAL;
  if (!out) return set_error(ctx, SPC_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_graph(ctx, g);
  if (rc) return rc;
  if (g->wtype != SPC_W_I32) return set_error(ctx, SPC_EINVAL, "batched coarsening takes int32 weights");
  if (G < 1 || !graph_off || !n_c) return set_error(ctx, SPC_EINVAL, "bad batch description");
  if (schedule > 1) return set_error(ctx, SPC_EINVAL, "unknown schedule %d", schedule);
  if (graph_off[0] != 0 || graph_off[G] != g->n)
    return set_error(ctx, SPC_EINVAL, "graph offsets must run from 0 to n");
  apply_tune(ctx, g->nnz, true);
  std::vector<int64_t> ng(G), nc(G), off(graph_off, graph_off + G + 1);
  for (int32_t i = 0; i < G; i++) {
    ng[i] = off[i + 1] - off[i];
    if (ng[i] < 1) return set_error(ctx, SPC_EINVAL, "graph %d of the batch is empty", (int)i);
    if (n_c[i] < 1) return set_error(ctx, SPC_EINVAL, "n_c of graph %d must be >= 1", (int)i);
    nc[i] = std::min(n_c[i], ng[i]);
  }
  int64_t* d_off = (int64_t*)dev_alloc(ctx, sizeof(int64_t) * (G + 1));
  int64_t* d_k = (int64_t*)dev_alloc(ctx, sizeof(int64_t) * G);
  int64_t* d_coff = (int64_t*)dev_alloc(ctx, sizeof(int64_t) * (G + 1));
  spc_hier* h = new (std::nothrow) spc_hier();
  if (!h || !d_off || !d_k || !d_coff) {
    dev_free(ctx, d_off);
    dev_free(ctx, d_k);
    dev_free(ctx, d_coff);
    delete h;
    return set_error(ctx, SPC_ENOMEM, "batch allocation failed");
  }
  auto fail = [&](int code) {
    dev_free(ctx, d_off);
    dev_free(ctx, d_k);
    dev_free(ctx, d_coff);
    spc_hier_free(h);
    return code;
  };
  h->ctx = ctx;
  h->n0 = g->n;
  h->goff.push_back(off);
  spc_graph cur = *g;
  while (true) {
    std::vector<int64_t> tg(G), kk(G), noff(G + 1);
    int64_t T = 0;
    bool more = false;
    for (int32_t i = 0; i < G; i++) {
      tg[i] = ng[i] <= nc[i] ? ng[i] : level_target(ng[i], nc[i], schedule);
      kk[i] = ng[i] - tg[i];
      more |= kk[i] > 0;
      noff[i] = T;
      T += tg[i];
    }
    noff[G] = T;
    if (!more) break;
    SPC_HIP(ctx, hipMemcpyAsync(d_off, off.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, ctx->stream));
    SPC_HIP(ctx, hipMemcpyAsync(d_k, kk.data(), sizeof(int64_t) * G, hipMemcpyHostToDevice, ctx->stream));
    SPC_HIP(ctx, hipMemcpyAsync(d_coff, noff.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice,
                                ctx->stream));
    Segments seg{G, d_off, d_k, d_coff, *std::max_element(tg.begin(), tg.end())};
    spc_hier::Level L;
    L.n_prev = cur.n;
    L.wtype = SPC_W_I32;
    if (!alloc_level(ctx, L, T, std::max<int64_t>(cur.nnz, 1), cur.n, sizeof(int32_t))) {
      set_error(ctx, SPC_ENOMEM, "hierarchy allocation failed");
      return fail(SPC_ENOMEM);
    }
    spc_graph_out o{L.rp, L.col, L.w, L.self, L.size, T, std::max<int64_t>(cur.nnz, 1)};
    int64_t nnz_c = 0;
    rc = level_impl(ctx, &cur, T, L.cluster_of, &o, &nnz_c, &L.st, &seg, L.ev);
    if (rc) {
      free_level(ctx, L);
      return fail(rc);
    }
    L.n = T;
    L.nnz = nnz_c;
    h->levels.push_back(L);
    h->goff.push_back(noff);
    cur.n = T;
    cur.nnz = nnz_c;
    cur.row_ptr = L.rp;
    cur.col = L.col;
    cur.w = L.w;
    cur.self_w = L.self;
    cur.size = L.size;
    off = noff;
    ng = tg;
  }
  h->timing_pending = true;
  dev_free(ctx, d_off);
  dev_free(ctx, d_k);
  dev_free(ctx, d_coff);
  *out = h;
  return SPC_OK;
}

int spc_autotune(spc_ctx* ctx, const spc_graph* g, int64_t n_c, int schedule, int32_t G, const int64_t* graph_off,
                 const int64_t* n_c_graph, char* report, size_t cap) {
  if (!ctx) return SPC_EINVAL;
  int rc = check_graph(ctx, g);
  if (rc) return rc;
  bool batched = G > 0;
  // one trial: the whole call, freed, on a drained stream; the best of two
  auto trial = [&](const spc_tune& t, double& ms) -> int {
    ctx->tune = t;
    ctx->tune_forced = 1;
    ms = 1e30;
    for (int rep = 0; rep < 2; rep++) {
      int r = hipStreamSynchronize(ctx->stream) == hipSuccess ? SPC_OK : SPC_EHIP;
      if (r) break;
      auto t0 = std::chrono::steady_clock::now();
      spc_hier* h = nullptr;
      r = batched ? spc_coarsen_batched(ctx, G, g, graph_off, n_c_graph, schedule, &h)
                  : spc_coarsen_to(ctx, g, n_c, schedule, &h);
      if (r == SPC_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) r = SPC_EHIP;
      double dt = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      if (h) spc_hier_free(h);
      if (r) {
        ctx->tune_forced = 0;
        return r;
      }
      ms = std::min(ms, dt);
    }
    ctx->tune_forced = 0;
    return SPC_OK;
  };
  std::string log;
  char line[160];
  spc_tune best;
  int key = size_class(g->nnz, batched);
  for (auto& kv : ctx->tuned)
    if (kv.first == key) best = kv.second;
  double best_ms;
  rc = trial(best, best_ms);
  if (rc) return rc;
  snprintf(line, sizeof(line), "start %.3f ms\n", best_ms);
  log += line;
  // coordinate descent: each setting in turn, the others at their best so
  // far; a change is kept when it saves at least 2 percent
  struct Knob {
    const char* name;
    int64_t spc_tune::*i64;
    int spc_tune::*i32;
    int64_t vals[4];
    int nv;
  };
  const Knob knobs[] = {
      {"lane_max", nullptr, &spc_tune::lane_max, {16, 32}, 2},
      {"wave_max", nullptr, &spc_tune::wave_max, {128, 256, 512}, 3},
      {"small_rpt", nullptr, &spc_tune::small_rpt, {1, 2, 4}, 3},
      {"huge_tile", nullptr, &spc_tune::huge_tile, {1024, 4096}, 2},
      {"sel_blocks", nullptr, &spc_tune::sel_blocks, {32, 64, 128}, 3},
      {"bv_short", &spc_tune::bv_short, nullptr, {1 << 18, 1 << 20, 1 << 22}, 3},
  };
  for (const Knob& k : knobs) {
    for (int v = 0; v < k.nv; v++) {
      spc_tune t = best;
      int64_t cur = k.i64 ? best.*(k.i64) : (int64_t)(best.*(k.i32));
      if (cur == k.vals[v]) continue;
      if (k.i64) t.*(k.i64) = k.vals[v];
      else t.*(k.i32) = (int)k.vals[v];
      double ms;
      rc = trial(t, ms);
      if (rc) return rc;
      snprintf(line, sizeof(line), "%s=%lld %.3f ms\n", k.name, (long long)k.vals[v], ms);
      log += line;
      if (ms < 0.98 * best_ms) {
        best = t;
        best_ms = ms;
      }
    }
  }
  bool found = false;
  for (auto& kv : ctx->tuned)
    if (kv.first == key) {
      kv.second = best;
      found = true;
    }
  if (!found) ctx->tuned.push_back({key, best});
  snprintf(line, sizeof(line),
           "best %.3f ms: lane_max=%d wave_max=%d small_rpt=%d huge_tile=%d sel_blocks=%d bv_short=%lld\n",
           best_ms, best.lane_max, best.wave_max, best.small_rpt, best.huge_tile, best.sel_blocks,
           (long long)best.bv_short);
  log += line;
  if (report && cap > 0) {
    size_t k = std::min(cap - 1, log.size());
    memcpy(report, log.data(), k);
    report[k] = 0;
  }
  return SPC_OK;
}

int spc_hier_graph_offsets(const spc_hier* h, int lvl, int64_t* off, int64_t cap) {
  if (!h || lvl < 0 || lvl > (int)h->levels.size() || !off) return SPC_EINVAL;
  if (h->goff.empty()) return SPC_EINVAL;
  const auto& o = h->goff[lvl];
  if ((int64_t)o.size() > cap) return SPC_ECAPACITY;
  for (size_t i = 0; i < o.size(); i++) off[i] = o[i];
  return SPC_OK;
}

int spc_hier_num_levels(const spc_hier* h) { return h ? (int)h->levels.size() : 0; }

int spc_hier_level(const spc_hier* h, int lvl, spc_graph* view, const int32_t** cluster_of,
                   spc_level_stats* stats) {
  if (!h || lvl < 1 || lvl > (int)h->levels.size()) return SPC_EINVAL;
  const spc_hier::Level& L = h->levels[lvl - 1];
  if (view) {
    view->n = L.n;
    view->nnz = L.nnz;
    view->row_ptr = L.rp;
    view->col = L.col;
    view->w = L.w;
    view->self_w = L.self;
    view->size = L.size;
    view->wtype = L.wtype;
  }
  if (cluster_of) *cluster_of = L.cluster_of;
  if (stats) {
    if (h->timing_pending) {
      int rc = finish_timing(h->ctx, const_cast<spc_hier*>(h));
      if (rc) return rc;
    }
    *stats = h->levels[lvl - 1].st;
  }
  return SPC_OK;
}

int spc_hier_export_level(spc_ctx* ctx, const spc_hier* h, int lvl, spc_graph_out* dst,
                          int32_t* cluster_of) {
  if (!ctx) return SPC_EINVAL;
  if (!h || lvl < 1 || lvl > (int)h->levels.size() || !dst)
    return set_error(ctx, SPC_EINVAL, "bad export arguments");
  const spc_hier::Level& L = h->levels[lvl - 1];
  if (dst->n_cap < L.n || dst->nnz_cap < L.nnz)
    return set_error(ctx, SPC_ECAPACITY, "export buffers too small");
  hipStream_t st = ctx->stream;
  SPC_HIP(ctx, hipMemcpyAsync(dst->row_ptr, L.rp, sizeof(int64_t) * (L.n + 1), hipMemcpyDeviceToDevice, st));
  if (L.nnz) {
    SPC_HIP(ctx, hipMemcpyAsync(dst->col, L.col, sizeof(int32_t) * L.nnz, hipMemcpyDeviceToDevice, st));
    size_t wsz = L.wtype == SPC_W_I32 ? sizeof(int32_t) : sizeof(double);
    SPC_HIP(ctx, hipMemcpyAsync(dst->w, L.w, wsz * L.nnz, hipMemcpyDeviceToDevice, st));
  }
  SPC_HIP(ctx, hipMemcpyAsync(dst->self_w, L.self, sizeof(int64_t) * L.n, hipMemcpyDeviceToDevice, st));
  SPC_HIP(ctx, hipMemcpyAsync(dst->size, L.size, sizeof(int32_t) * L.n, hipMemcpyDeviceToDevice, st));
  if (cluster_of)
    SPC_HIP(ctx, hipMemcpyAsync(cluster_of, L.cluster_of, sizeof(int32_t) * L.n_prev,
                                hipMemcpyDeviceToDevice, st));
  return SPC_OK;
}

void spc_hier_free(spc_hier* h) {
  if (!h) return;
  // no wait: blocks go back to the allocator hook (which reuses them in the
  // context's stream order) or to hipFree (which waits for the device); a
  // level event still pending returns to the context's pool, where the next
  // record replaces it
  for (auto& L : h->levels) free_level(h->ctx, L);
  delete h;
}

}  // extern "C"

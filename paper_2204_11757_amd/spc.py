"""Python binding of libspc, the gfx950 coarsening library (include/spc.h).

Argument marshalling only: every step of the coarsening runs in the HIP
kernels behind the C ABI.  PyTorch provides device memory (tensors and, via
the allocator hook, the library's own workspace) and the HIP stream.  If
the shared library has not been built this module raises at first use; it
never falls back to another implementation.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspc.so")

SPC_OK, SPC_EINVAL, SPC_EUNREACHABLE, SPC_EOVERFLOW = 0, -1, -2, -3
SPC_ECAPACITY, SPC_ENOMEM, SPC_EHIP, SPC_ERANGE = -4, -5, -6, -7
SPC_W_I32, SPC_W_F32, SPC_W_F64 = 0, 1, 2

# every symbol declared in include/spc.h
EXPORTS = [
    "spc_create", "spc_destroy", "spc_set_stream", "spc_set_allocator", "spc_set_option",
    "spc_last_error",
    "spc_strerror", "spc_coarsen_level", "spc_coarsen_to", "spc_hier_num_levels",
    "spc_hier_level", "spc_hier_export_level", "spc_hier_free", "spc_lift",
    "spc_spectral_error", "spc_validate_graph", "spc_timing_report", "spc_hier_cluster_map",
    "spc_spectral_error_graph", "spc_spectral_error_backward", "spc_entry_map",
    "spc_contract_backward", "spc_coarsen_batched", "spc_hier_graph_offsets",
    "spc_coarsen_level_noalloc", "spc_relabel", "spc_autotune",
]


class SpcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"spc error {code}: {msg}")
        self.code = code


class _Graph(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p), ("col", C.c_void_p),
                ("w", C.c_void_p), ("self_w", C.c_void_p), ("size", C.c_void_p),
                ("wtype", C.c_int32)]


class _GraphOut(C.Structure):
    _fields_ = [("row_ptr", C.c_void_p), ("col", C.c_void_p), ("w", C.c_void_p),
                ("self_w", C.c_void_p), ("size", C.c_void_p), ("n_cap", C.c_int64),
                ("nnz_cap", C.c_int64)]


class LevelStats(C.Structure):
    _fields_ = [("n_in", C.c_int64), ("m_in", C.c_int64), ("n_out", C.c_int64),
                ("nnz_out", C.c_int64), ("merges", C.c_int64), ("largest_cluster", C.c_int64),
                ("boruvka_rounds", C.c_int64), ("candidate_edges", C.c_int64),
                ("key_mode", C.c_int32), ("key_bits", C.c_int32), ("eps_max", C.c_double),
                ("ms_total", C.c_float), ("bands", C.c_int32), ("forest_in", C.c_int64),
                ("forest_kept", C.c_int64), ("merge_in", C.c_int64), ("forest_edges", C.c_int64),
                ("keys_written", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libspc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python -m paper_2204_11757_amd.build")
        L = C.CDLL(LIB_PATH)
        p, i64, i32 = C.c_void_p, C.c_int64, C.c_int
        sig = {
            "spc_create": [C.POINTER(C.c_void_p), i32, p],
            "spc_destroy": [p],
            "spc_set_stream": [p, p],
            "spc_set_allocator": [p, p, p, p],
            "spc_set_option": [p, C.c_char_p, i64],
            "spc_coarsen_level": [p, C.POINTER(_Graph), i64, p, C.POINTER(_GraphOut),
                                  C.POINTER(C.c_int64), C.POINTER(LevelStats)],
            "spc_coarsen_level_noalloc": [p, C.POINTER(_Graph), i64, p, C.POINTER(_GraphOut),
                                          C.POINTER(C.c_int64), C.POINTER(LevelStats)],
            "spc_relabel": [p, C.POINTER(_Graph), p, C.POINTER(_GraphOut), C.POINTER(C.c_int64)],
            "spc_autotune": [p, C.POINTER(_Graph), i64, i32, i32, p, p, C.c_char_p, C.c_size_t],
            "spc_coarsen_to": [p, C.POINTER(_Graph), i64, i32, C.POINTER(C.c_void_p)],
            "spc_hier_num_levels": [p],
            "spc_hier_level": [p, i32, C.POINTER(_Graph), C.POINTER(C.c_void_p),
                               C.POINTER(LevelStats)],
            "spc_hier_export_level": [p, p, i32, C.POINTER(_GraphOut), p],
            "spc_lift": [p, p, i32, i32, i32, p, i32, p],
            "spc_spectral_error": [p, p, i32, p, p, i32, i32, p, C.POINTER(C.c_double)],
            "spc_validate_graph": [C.POINTER(_Graph)],
            "spc_timing_report": [p, C.c_char_p, C.c_size_t],
            "spc_hier_cluster_map": [p, p, i32, p],
            "spc_spectral_error_graph": [p, C.POINTER(_Graph), p, i64, p, p, i32, i32, p,
                                         C.POINTER(C.c_double)],
            "spc_spectral_error_backward": [p, C.POINTER(_Graph), p, i64, p, p, i32, i32, p, p],
            "spc_entry_map": [p, C.POINTER(_Graph), p, C.POINTER(_Graph), p],
            "spc_contract_backward": [p, p, p, i64, i64, p, p, p, p],
            "spc_coarsen_batched": [p, i32, C.POINTER(_Graph), p, p, i32, C.POINTER(C.c_void_p)],
            "spc_hier_graph_offsets": [p, i32, p, i64],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.spc_hier_free.argtypes = [p]
        L.spc_hier_free.restype = None
        L.spc_last_error.argtypes = [p]
        L.spc_last_error.restype = C.c_char_p
        L.spc_strerror.argtypes = [C.c_int]
        L.spc_strerror.restype = C.c_char_p
        _lib = L
    return _lib


# ----------------------------------------------------------------------------
# graphs in device memory
# ----------------------------------------------------------------------------

@dataclass
class DeviceGraph:
    """Symmetric CSR graph held in torch tensors on a GPU."""

    n: int
    row_ptr: torch.Tensor          # int64[n+1]
    col: torch.Tensor              # int32[nnz]
    w: torch.Tensor                # int32[nnz]
    self_w: Optional[torch.Tensor] = None   # int64[n]
    size: Optional[torch.Tensor] = None     # int32[n]

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @property
    def wtype(self) -> int:
        return {torch.int32: SPC_W_I32, torch.float32: SPC_W_F32,
                torch.float64: SPC_W_F64}[self.w.dtype]

    @staticmethod
    def from_host(g, device="cuda") -> "DeviceGraph":
        """From a host graph (anything with n, row_ptr, col, w, self_w, size)."""
        t = lambda a, dt: None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)
        wdt = np.int32 if np.asarray(g.w).dtype.kind in "iu" else np.asarray(g.w).dtype
        sdt = np.int64 if wdt == np.int32 else np.float64
        return DeviceGraph(n=int(g.n), row_ptr=t(g.row_ptr, np.int64), col=t(g.col, np.int32),
                           w=t(g.w, wdt), self_w=t(g.self_w, sdt), size=t(g.size, np.int32))

    def to_host(self):
        from meshgen import Graph
        c = lambda x: None if x is None else x.cpu().numpy()
        return Graph(n=self.n, row_ptr=c(self.row_ptr), col=c(self.col), w=c(self.w),
                     self_w=c(self.self_w), size=c(self.size))

    def _c(self) -> _Graph:
        ptr = lambda x: None if x is None else x.data_ptr()
        for x in (self.row_ptr, self.col, self.w, self.self_w, self.size):
            if x is not None and not x.is_contiguous():
                raise ValueError("graph tensors must be contiguous")
        return _Graph(self.n, self.nnz, ptr(self.row_ptr), ptr(self.col), ptr(self.w),
                      ptr(self.self_w), ptr(self.size), self.wtype)


def _empty_out(n: int, nnz: int, device, fp: bool = False):
    wdt = torch.float64 if fp else torch.int32
    sdt = torch.float64 if fp else torch.int64
    return DeviceGraph(n=n, row_ptr=torch.empty(n + 1, dtype=torch.int64, device=device),
                       col=torch.empty(max(nnz, 1), dtype=torch.int32, device=device),
                       w=torch.empty(max(nnz, 1), dtype=wdt, device=device),
                       self_w=torch.empty(max(n, 1), dtype=sdt, device=device),
                       size=torch.empty(max(n, 1), dtype=torch.int32, device=device))


def _out_c(o: DeviceGraph, n_cap: int, nnz_cap: int) -> _GraphOut:
    return _GraphOut(o.row_ptr.data_ptr(), o.col.data_ptr(), o.w.data_ptr(), o.self_w.data_ptr(),
                     o.size.data_ptr(), n_cap, nnz_cap)


# ----------------------------------------------------------------------------
# context: one per device, workspace through torch's caching allocator
# ----------------------------------------------------------------------------

_ALLOC_T = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_T = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Context:
    def __init__(self, device: int = 0):
        self.device = device
        h = C.c_void_p()
        rc = lib().spc_create(C.byref(h), device, None)
        if rc != SPC_OK:
            raise SpcError(rc, "spc_create failed")
        self.h = h

        def _alloc(size, user):
            try:
                return torch.cuda.caching_allocator_alloc(int(size), self.device,
                                                          torch.cuda.current_stream(self.device))
            except Exception:  # out of memory: report NULL, the library returns SPC_ENOMEM
                return None

        def _free(ptr, user):
            torch.cuda.caching_allocator_delete(ptr)

        self._alloc = _ALLOC_T(_alloc)
        self._free = _FREE_T(_free)
        self.check(lib().spc_set_allocator(self.h, C.cast(self._alloc, C.c_void_p),
                                           C.cast(self._free, C.c_void_p), None))

    def bind_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        self.check(lib().spc_set_stream(self.h, C.c_void_p(s)))

    def check(self, rc: int):
        if rc != SPC_OK:
            msg = lib().spc_last_error(self.h).decode() or lib().spc_strerror(rc).decode()
            raise SpcError(rc, msg)

    def close(self):
        """Destroy the library context (waits for its stream, returns its
        workspace through the allocator hook), then drop the callbacks."""
        if getattr(self, "h", None):
            lib().spc_destroy(self.h)
            self.h = None
        self._alloc = self._free = None


_contexts = {}
_live = weakref.WeakSet()     # hierarchies whose library handle is still held
_shutting_down = False


def _teardown():
    """At interpreter exit, while torch (whose allocator the library calls
    back into) is still intact: free every live hierarchy, then destroy the
    contexts.  Registered after torch's own exit handlers, so it runs before
    them; afterwards Hierarchy.__del__ does nothing."""
    global _shutting_down
    try:
        for h in list(_live):
            h.free()
        for ctx in list(_contexts.values()):
            ctx.close()
        _contexts.clear()
    finally:
        _shutting_down = True


atexit.register(_teardown)


def context(device=None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    if isinstance(device, torch.device):
        device = device.index if device.index is not None else torch.cuda.current_device()
    if device not in _contexts:
        _contexts[device] = Context(device)
    ctx = _contexts[device]
    ctx.bind_stream()
    return ctx


def set_option(name: str, value: int, device=None):
    """Context option (tests / tuning), by the names the C header lists."""
    ctx = context(device)
    ctx.check(lib().spc_set_option(ctx.h, name.encode(), int(value)))


def timing_report(device=None) -> dict:
    """Per-kernel timings collected while the "timing" option was on:
    {name: (launches, total_ms, work_units)}.  Clears the collection."""
    ctx = context(device)
    buf = C.create_string_buffer(1 << 16)
    ctx.check(lib().spc_timing_report(ctx.h, buf, len(buf)))
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms, units = line.split()
        out[name] = (int(cnt), float(ms), float(units))
    return out


def _dev(t: torch.Tensor) -> int:
    return t.device.index if t.device.index is not None else torch.cuda.current_device()


# ----------------------------------------------------------------------------
# entry points (same names as the C ABI without the prefix)
# ----------------------------------------------------------------------------

def coarsen_level(g: DeviceGraph, n_target: int):
    """One level of Algorithm 1 plus the contraction of Definition 1.
    Returns (cluster_of int32[n], coarse DeviceGraph, LevelStats)."""
    ctx = context(_dev(g.row_ptr))
    dev = g.row_ptr.device
    t = max(1, min(int(n_target), g.n))
    out = _empty_out(t, g.nnz, dev, fp=g.wtype != SPC_W_I32)
    cl = torch.empty(g.n, dtype=torch.int32, device=dev)
    nnz = C.c_int64()
    st = LevelStats()
    gc = g._c()
    oc = _out_c(out, t, max(g.nnz, 1))
    ctx.check(lib().spc_coarsen_level(ctx.h, C.byref(gc), int(n_target), cl.data_ptr(), C.byref(oc),
                                      C.byref(nnz), C.byref(st)))
    k = nnz.value
    n_c = st.n_out
    coarse = DeviceGraph(n=n_c, row_ptr=out.row_ptr[: n_c + 1], col=out.col[:k], w=out.w[:k],
                         self_w=out.self_w[:n_c], size=out.size[:n_c])
    return cl, coarse, st


def relabel(g: DeviceGraph, perm) -> DeviceGraph:
    """The graph with node u renamed perm[u] (a permutation of [0, n)).
    Scores do not depend on node names, so coarsening the result changes
    only how ties fall: by (perm[u], perm[v]) instead of (u, v) -- with a
    seeded random perm, a hash tie-break."""
    ctx = context(_dev(g.row_ptr))
    dev = g.row_ptr.device
    pt = torch.as_tensor(np.ascontiguousarray(perm, dtype=np.int32)).to(dev) if not torch.is_tensor(perm) \
        else perm.to(device=dev, dtype=torch.int32).contiguous()
    if pt.numel() != g.n:
        raise ValueError("perm must have n entries")
    out = _empty_out(g.n, g.nnz, dev, fp=g.wtype != SPC_W_I32)
    nnz = C.c_int64()
    gc = g._c()
    oc = _out_c(out, g.n, max(g.nnz, 1))
    ctx.check(lib().spc_relabel(ctx.h, C.byref(gc), pt.data_ptr(), C.byref(oc), C.byref(nnz)))
    k = nnz.value
    return DeviceGraph(n=g.n, row_ptr=out.row_ptr, col=out.col[:k], w=out.w[:k], self_w=out.self_w,
                       size=out.size)


def autotune(g: DeviceGraph, n_c=None, schedule: int = 0, graph_off=None, n_c_graph=None) -> str:
    """Tune the launch settings for inputs of g's size class (see
    spc_autotune): a plain call to n_c, or with graph_off and n_c_graph the
    batched call.  Returns the trials' report."""
    ctx = context(_dev(g.row_ptr))
    buf = C.create_string_buffer(1 << 14)
    gc = g._c()
    if graph_off is not None:
        off = np.ascontiguousarray(graph_off, dtype=np.int64)
        nc = np.ascontiguousarray(n_c_graph, dtype=np.int64)
        ctx.check(lib().spc_autotune(ctx.h, C.byref(gc), 0, int(schedule), int(off.shape[0] - 1),
                                     off.ctypes.data, nc.ctypes.data, buf, len(buf)))
    else:
        ctx.check(lib().spc_autotune(ctx.h, C.byref(gc), int(n_c), int(schedule), 0, None, None, buf, len(buf)))
    return buf.value.decode()


SPC_NOALLOC_SCRATCH_BYTES = 134217728


def coarsen_level_noalloc(g: DeviceGraph, n_target: int, cluster_of: torch.Tensor, out: DeviceGraph):
    """coarsen_level for callers that cannot allocate: the library works in
    its fixed per-device scratch array (SPC_NOALLOC_SCRATCH_BYTES) and
    allocates nothing; the caller provides cluster_of (int32[n]) and the
    output graph's tensors (capacities: out.n nodes, out.col.numel()
    entries).  Returns (number of coarse entries, LevelStats)."""
    ctx = context(_dev(g.row_ptr))
    nnz = C.c_int64()
    st = LevelStats()
    gc = g._c()
    oc = _out_c(out, out.n, int(out.col.numel()))
    ctx.check(lib().spc_coarsen_level_noalloc(ctx.h, C.byref(gc), int(n_target), cluster_of.data_ptr(),
                                              C.byref(oc), C.byref(nnz), C.byref(st)))
    return nnz.value, st


class Hierarchy:
    """Levels produced by coarsen_to; owns the library's hierarchy handle."""

    def __init__(self, ctx: Context, handle: C.c_void_p, n0: int):
        self.ctx = ctx
        self.h = handle
        self.n0 = n0
        _live.add(self)

    @property
    def num_levels(self) -> int:
        return lib().spc_hier_num_levels(self.h)

    def stats(self, lvl: int) -> LevelStats:
        st = LevelStats()
        view = _Graph()
        self.ctx.check(lib().spc_hier_level(self.h, lvl, C.byref(view), None, C.byref(st)))
        return st

    def level(self, lvl: int):
        """(cluster_of, coarse DeviceGraph, LevelStats) of level lvl (1-based),
        copied into fresh tensors."""
        st = LevelStats()
        view = _Graph()
        self.ctx.check(lib().spc_hier_level(self.h, lvl, C.byref(view), None, C.byref(st)))
        dev = torch.device("cuda", self.ctx.device)
        out = _empty_out(view.n, view.nnz, dev, fp=view.wtype != SPC_W_I32)
        n_prev = self.n0 if lvl == 1 else self.stats(lvl - 1).n_out
        cl = torch.empty(n_prev, dtype=torch.int32, device=dev)
        oc = _out_c(out, view.n, max(view.nnz, 1))
        self.ctx.bind_stream()
        self.ctx.check(lib().spc_hier_export_level(self.ctx.h, self.h, lvl, C.byref(oc), cl.data_ptr()))
        g = DeviceGraph(n=view.n, row_ptr=out.row_ptr, col=out.col[: view.nnz], w=out.w[: view.nnz],
                        self_w=out.self_w[: view.n], size=out.size[: view.n])
        return cl, g, st

    def free(self):
        if self.h:
            if self.ctx.h is None:
                raise RuntimeError("the hierarchy's context was destroyed")
            lib().spc_hier_free(self.h)
            self.h = None
        _live.discard(self)

    def __del__(self):
        if _shutting_down:
            return
        try:
            self.free()
        except Exception:
            pass


def coarsen_to(g: DeviceGraph, n_c: int, schedule: int = 0) -> Hierarchy:
    """Multilevel coarsening to n_c super-nodes.  schedule 0 halves the node
    count per level, 1 is a single level, -j takes j merges per level (the
    scores recomputed after every j merges; -1 is the explicit greedy)."""
    ctx = context(_dev(g.row_ptr))
    h = C.c_void_p()
    gc = g._c()
    ctx.check(lib().spc_coarsen_to(ctx.h, C.byref(gc), int(n_c), int(schedule), C.byref(h)))
    return Hierarchy(ctx, h, g.n)


def pack_graphs(graphs):
    """Host block-diagonal union of host graphs (node ids shifted) and the
    node offsets (int64[G+1])."""
    from meshgen import Graph
    offs = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        offs[i + 1] = offs[i] + g.n
    eoffs = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        eoffs[i + 1] = eoffs[i] + g.nnz
    rp = np.empty(offs[-1] + 1, dtype=np.int64)
    col = np.empty(eoffs[-1], dtype=np.int32)
    w = np.empty(eoffs[-1], dtype=graphs[0].w.dtype)
    for i, g in enumerate(graphs):
        rp[offs[i]: offs[i + 1]] = g.row_ptr[:-1] + eoffs[i]
        col[eoffs[i]: eoffs[i + 1]] = g.col + offs[i]
        w[eoffs[i]: eoffs[i + 1]] = g.w
    rp[-1] = eoffs[-1]
    has_self = any(g.self_w is not None for g in graphs)
    has_size = any(g.size is not None for g in graphs)
    sw = np.concatenate([g.self_w_or_zero() for g in graphs]) if has_self else None
    sz = np.concatenate([g.size_or_one() for g in graphs]) if has_size else None
    return Graph(n=int(offs[-1]), row_ptr=rp, col=col, w=w, self_w=sw, size=sz), offs


class BatchHierarchy(Hierarchy):
    """Hierarchy of a batch: level l is the packed union of the graphs'
    level-l graphs."""

    def __init__(self, ctx, handle, n0, G):
        super().__init__(ctx, handle, n0)
        self.G = G

    def offsets(self, lvl: int) -> np.ndarray:
        out = np.zeros(self.G + 1, dtype=np.int64)
        self.ctx.check(lib().spc_hier_graph_offsets(self.h, lvl, out.ctypes.data, self.G + 1))
        return out


def coarsen_batched(g: DeviceGraph, graph_off, n_c, schedule: int = 0) -> BatchHierarchy:
    """Coarsen a packed batch (graph i owns nodes graph_off[i]..graph_off[i+1])
    graph by graph to n_c[i], in shared launches."""
    ctx = context(_dev(g.row_ptr))
    off = np.ascontiguousarray(graph_off, dtype=np.int64)
    nc = np.ascontiguousarray(n_c, dtype=np.int64)
    G = off.shape[0] - 1
    h = C.c_void_p()
    gc = g._c()
    ctx.check(lib().spc_coarsen_batched(ctx.h, G, C.byref(gc), off.ctypes.data, nc.ctypes.data,
                                        int(schedule), C.byref(h)))
    return BatchHierarchy(ctx, h, g.n, G)


def lift(h: Hierarchy, from_lvl: int, to_lvl: int, mode: int, x_c: torch.Tensor) -> torch.Tensor:
    """Lift coarse vectors (n_to x k, float64) from level to_lvl to level from_lvl."""
    ctx = context(h.ctx.device)
    x = x_c.to(torch.float64)
    if x.dim() == 1:
        x = x[:, None]
    k = x.shape[1]
    xc = x.t().contiguous()           # column-major = transpose row-major
    n_from = h.n0 if from_lvl == 0 else h.stats(from_lvl).n_out
    xf = torch.empty((k, n_from), dtype=torch.float64, device=x.device)
    ctx.check(lib().spc_lift(ctx.h, h.h, from_lvl, to_lvl, mode, xc.data_ptr(), k, xf.data_ptr()))
    out = xf.t()
    return out[:, 0] if x_c.dim() == 1 else out


def _prec(U: torch.Tensor):
    """The spectral computation's type follows U's: float32 runs the FP32
    form, anything else FP64."""
    return (SPC_W_F32, torch.float32) if U.dtype == torch.float32 else (SPC_W_F64, torch.float64)


def spectral_error(h: Hierarchy, lvl: int, U: torch.Tensor, lam: torch.Tensor):
    """(loss, R): R_i = 1 - t_i^T W_c t_i, loss = sum (R_i - lambda_i)^2.
    Computed in U's precision (float32 or float64)."""
    ctx = context(h.ctx.device)
    prec, dt = _prec(U)
    Uc = U.to(dt).t().contiguous()
    k = Uc.shape[0]
    lamd = lam.to(torch.float64).contiguous()
    R = torch.empty(k, dtype=dt, device=U.device)
    loss = C.c_double()
    ctx.check(lib().spc_spectral_error(ctx.h, h.h, lvl, Uc.data_ptr(), lamd.data_ptr(), k, prec,
                                       R.data_ptr(), C.byref(loss)))
    return loss.value, R


def cluster_map(h: Hierarchy, lvl: int) -> torch.Tensor:
    """Input node -> level-lvl super-node (int32[n0])."""
    ctx = context(h.ctx.device)
    out = torch.empty(h.n0, dtype=torch.int32, device=torch.device("cuda", h.ctx.device))
    ctx.check(lib().spc_hier_cluster_map(ctx.h, h.h, lvl, out.data_ptr()))
    return out


def _colmajor(U: torch.Tensor) -> torch.Tensor:
    return U.to(_prec(U)[1]).t().contiguous()


def spectral_error_graph(coarse: DeviceGraph, cmap: torch.Tensor, U: torch.Tensor, lam: torch.Tensor):
    """(loss, R) of an explicit coarse graph (int32 or float64 weights) whose
    super-nodes are cmap (input node -> super-node), in U's precision."""
    ctx = context(_dev(coarse.row_ptr))
    prec, dt = _prec(U)
    Uc = _colmajor(U)
    k = Uc.shape[0]
    lamd = lam.to(torch.float64).contiguous()
    R = torch.empty(k, dtype=dt, device=U.device)
    loss = C.c_double()
    gc = coarse._c()
    ctx.check(lib().spc_spectral_error_graph(ctx.h, C.byref(gc), cmap.data_ptr(), int(cmap.numel()),
                                             Uc.data_ptr(), lamd.data_ptr(), k, prec, R.data_ptr(),
                                             C.byref(loss)))
    return loss.value, R


def spectral_error_backward(coarse: DeviceGraph, cmap: torch.Tensor, U: torch.Tensor, lam: torch.Tensor):
    """(d loss / d w_c at every CSR entry, d loss / d self_c), computed in
    U's precision (float32 gives the FP32 gradients)."""
    ctx = context(_dev(coarse.row_ptr))
    prec, dt = _prec(U)
    Uc = _colmajor(U)
    k = Uc.shape[0]
    lamd = lam.to(torch.float64).contiguous()
    dev = coarse.row_ptr.device
    dw = torch.empty(max(coarse.nnz, 1), dtype=dt, device=dev)
    ds = torch.empty(coarse.n, dtype=dt, device=dev)
    gc = coarse._c()
    ctx.check(lib().spc_spectral_error_backward(ctx.h, C.byref(gc), cmap.data_ptr(), int(cmap.numel()),
                                                Uc.data_ptr(), lamd.data_ptr(), k, prec, dw.data_ptr(),
                                                ds.data_ptr()))
    return dw[: coarse.nnz], ds


def entry_map(fine: DeviceGraph, cluster_of: torch.Tensor, coarse: DeviceGraph) -> torch.Tensor:
    """Fine CSR entry -> coarse entry position, or -1 - super-node."""
    ctx = context(_dev(fine.row_ptr))
    out = torch.empty(max(fine.nnz, 1), dtype=torch.int32, device=fine.row_ptr.device)
    gf, gc = fine._c(), coarse._c()
    ctx.check(lib().spc_entry_map(ctx.h, C.byref(gf), cluster_of.data_ptr(), C.byref(gc), out.data_ptr()))
    return out[: fine.nnz]


def contract_backward(emap: torch.Tensor, cluster_of: torch.Tensor, d_wc: torch.Tensor,
                      d_selfc: torch.Tensor, n_f: int, want_self: bool = True):
    """Adjoint of the contraction: (d_wf, d_selff or None)."""
    ctx = context(_dev(d_selfc))
    nnz_f = int(emap.numel())
    dev = d_selfc.device
    dwf = torch.empty(max(nnz_f, 1), dtype=torch.float64, device=dev)
    dsf = torch.empty(n_f, dtype=torch.float64, device=dev) if want_self else None
    d_wc = d_wc.to(torch.float64).contiguous()
    d_selfc = d_selfc.to(torch.float64).contiguous()
    ctx.check(lib().spc_contract_backward(ctx.h, emap.data_ptr() if nnz_f else None, cluster_of.data_ptr(),
                                          nnz_f, int(n_f), d_wc.data_ptr(), d_selfc.data_ptr(),
                                          dwf.data_ptr(), dsf.data_ptr() if dsf is not None else None))
    return dwf[:nnz_f], dsf


class SpectralError(torch.autograd.Function):
    """loss(w_c, self_c) = sum_i (R_i - lambda_i)^2 of a coarse graph whose
    FP64 weights w_c (one value per CSR entry, symmetric) and self-loops
    self_c are the differentiable inputs; the structure, cmap, U and lambda
    are fixed.  Forward and backward run in the library's kernels.

    An undirected weight w_ab is held at two entries; each entry receives
    half of d loss / d w_ab, so the gradient is exact for every change that
    keeps the graph symmetric (a parameter shared by both entries gets the
    full derivative)."""

    @staticmethod
    def forward(ctx_, w_c, self_c, structure: DeviceGraph, cmap, U, lam):
        g = DeviceGraph(n=structure.n, row_ptr=structure.row_ptr, col=structure.col,
                        w=w_c.detach().to(torch.float64).contiguous(),
                        self_w=self_c.detach().to(torch.float64).contiguous(), size=structure.size)
        loss, _ = spectral_error_graph(g, cmap, U, lam)
        ctx_.save_for_backward(w_c.detach(), self_c.detach())
        ctx_.g = g
        ctx_.cmap, ctx_.U, ctx_.lam = cmap, U, lam
        return torch.tensor(loss, dtype=torch.float64, device=w_c.device)

    @staticmethod
    def backward(ctx_, grad):
        w_c, self_c = ctx_.saved_tensors
        dw, ds = spectral_error_backward(ctx_.g, ctx_.cmap, ctx_.U, ctx_.lam)
        return (grad * (0.5 * dw)).to(w_c.dtype), (grad * ds).to(self_c.dtype), None, None, None, None


def spectral_error_loss(w_c, self_c, structure: DeviceGraph, cmap, U, lam):
    return SpectralError.apply(w_c, self_c, structure, cmap, U, lam)


def validate_graph(g) -> int:
    """Host-side structural validation (no GPU).  g: host arrays with
    n, row_ptr, col, w, self_w, size.  Returns an SPC_* code."""
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    w = np.ascontiguousarray(g.w)
    if w.dtype.kind in "iu":
        w = w.astype(np.int32)
        wt = SPC_W_I32
        sw = None if g.self_w is None else np.ascontiguousarray(g.self_w, dtype=np.int64)
    else:
        wt = SPC_W_F32 if w.dtype == np.float32 else SPC_W_F64
        sw = None if g.self_w is None else np.ascontiguousarray(g.self_w, dtype=np.float64)
    sz = None if g.size is None else np.ascontiguousarray(g.size, dtype=np.int32)
    p = lambda a: None if a is None else a.ctypes.data
    gc = _Graph(int(g.n), int(rp[-1]), p(rp), p(col), p(w), p(sw), p(sz), wt)
    return lib().spc_validate_graph(C.byref(gc))

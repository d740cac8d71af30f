"""Digests of coarsening results, for comparing a large result with a stored
reference without storing the arrays.

Each array is hashed (SHA-256) as the little-endian bytes of its canonical
type: cluster maps int32, row pointers int64 (rebased to start at 0), columns
int32, weights int32 (integer graphs) or float64, self-loops int64 or
float64, sizes int32.  Long arrays also get one short digest per chunk of
CHUNK elements, so that a mismatch can be located.  Nothing here computes
any part of the method; it only hashes arrays.
"""
from __future__ import annotations

import hashlib

import numpy as np

CHUNK = 1 << 22
FIELDS = ("cluster_of", "row_ptr", "col", "w", "self_w", "size")


def canonical(name: str, a, fp: bool) -> np.ndarray:
    """The canonical little-endian array of field `name`."""
    a = np.asarray(a)
    if name in ("cluster_of", "col", "size"):
        dt = np.dtype("<i4")
    elif name == "row_ptr":
        dt = np.dtype("<i8")
        a = a.astype(np.int64) - int(a[0]) if a.shape[0] else a
    elif name == "w":
        dt = np.dtype("<f8") if fp else np.dtype("<i4")
    elif name == "self_w":
        dt = np.dtype("<f8") if fp else np.dtype("<i8")
    else:
        raise KeyError(name)
    return np.ascontiguousarray(a, dtype=dt)


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(memoryview(a).cast("B")).hexdigest()


def chunk_shas(a: np.ndarray, chunk: int = CHUNK):
    return [sha(a[i:i + chunk])[:16] for i in range(0, a.shape[0], chunk)]


def level_fields(cluster_of, g) -> dict:
    """Field name -> array of one level: its cluster map and coarse graph
    (anything with row_ptr, col, w, self_w, size)."""
    return {"cluster_of": cluster_of, "row_ptr": g.row_ptr, "col": g.col, "w": g.w,
            "self_w": g.self_w, "size": g.size}


def level_digest(cluster_of, g, fp: bool, chunks: bool = True) -> dict:
    out = {"n": int(np.asarray(g.row_ptr).shape[0] - 1), "nnz": int(np.asarray(g.col).shape[0]),
           "sha": {}, "chunks": {}}
    for name, a in level_fields(cluster_of, g).items():
        c = canonical(name, a, fp)
        out["sha"][name] = sha(c)
        if chunks and c.shape[0] > CHUNK:
            out["chunks"][name] = chunk_shas(c)
    return out


def first_mismatch(name: str, got: np.ndarray, want_chunks) -> str:
    """Describe the first chunk of `got` whose digest differs."""
    have = chunk_shas(got)
    for i, (a, b) in enumerate(zip(have, want_chunks)):
        if a != b:
            return f"{name}: first differing chunk {i} (elements {i * CHUNK}..{(i + 1) * CHUNK - 1})"
    if len(have) != len(want_chunks):
        return f"{name}: {len(have)} chunks against {len(want_chunks)}"
    return f"{name}: chunks agree but the whole digest differs"


class GraphHasher:
    """Streaming SHA-256 of the per-graph level arrays of a batch, in graph
    order, equal to the digest of their block-diagonal union (cluster maps
    and columns shifted by the graph's node offset at that level, row
    pointers by its entry offset)."""

    def __init__(self, fp: bool):
        self.fp = fp
        self.h = {name: hashlib.sha256() for name in FIELDS}
        self.node_in = 0
        self.node_out = 0
        self.entries = 0
        self.nnz_total = 0

    def add(self, cluster_of, g):
        rp = np.asarray(g.row_ptr).astype(np.int64)
        parts = {
            "cluster_of": np.asarray(cluster_of).astype(np.int64) + self.node_out,
            "row_ptr": rp[:-1] - rp[0] + self.entries,
            "col": np.asarray(g.col).astype(np.int64) + self.node_out,
            "w": g.w, "self_w": g.self_w, "size": g.size,
        }
        for name, a in parts.items():
            c = np.ascontiguousarray(a, dtype=canonical_dtype(name, self.fp))
            self.h[name].update(memoryview(c).cast("B"))
        self.node_in += int(np.asarray(cluster_of).shape[0])
        self.node_out += int(rp.shape[0] - 1)
        self.entries += int(rp[-1] - rp[0])

    def digest(self) -> dict:
        last = np.array([self.entries], dtype="<i8")
        h = self.h["row_ptr"].copy()
        h.update(memoryview(last).cast("B"))
        out = {name: self.h[name].hexdigest() for name in FIELDS}
        out["row_ptr"] = h.hexdigest()
        return out


def canonical_dtype(name: str, fp: bool) -> np.dtype:
    if name in ("cluster_of", "col", "size"):
        return np.dtype("<i4")
    if name == "row_ptr":
        return np.dtype("<i8")
    if name == "w":
        return np.dtype("<f8") if fp else np.dtype("<i4")
    if name == "self_w":
        return np.dtype("<f8") if fp else np.dtype("<i8")
    raise KeyError(name)


def graph_levels_digest(levels, fp: bool) -> str:
    """One short digest over all levels of one graph: (cluster_of, coarse
    graph) pairs, arrays in FIELDS order, row pointers rebased."""
    h = hashlib.sha256()
    for cl, g in levels:
        for name, a in level_fields(cl, g).items():
            h.update(memoryview(canonical(name, a, fp)).cast("B"))
    return h.hexdigest()[:16]

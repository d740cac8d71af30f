"""CPU checks of the C ABI boundary: the library loads, exports every symbol
include/spc.h declares, and host-side validation matches the paper's
preconditions (and agrees with the oracle's).  No compute call is made."""
import os
import re

import numpy as np
import pytest

import oracle
from meshgen import Graph, from_edges, random_graph

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "spc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spc_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def spc():
    import paper_2204_11757_amd.build as B
    from paper_2204_11757_amd import spc as S
    if not os.path.exists(S.LIB_PATH):
        B.build()
    return S


def test_library_exports_every_declared_symbol(spc):
    import subprocess
    syms = header_symbols()
    assert len(syms) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", spc.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (spc_\w+)", out))
    missing = [s for s in syms if s not in exported]
    assert not missing, missing
    assert sorted(spc.EXPORTS) == syms
    L = spc.lib()
    for s in syms:
        assert hasattr(L, s)


def test_library_is_gfx950(spc):
    import subprocess
    out = subprocess.run(["strings", spc.LIB_PATH], capture_output=True, text=True).stdout
    assert "gfx950" in out


def test_strerror(spc):
    L = spc.lib()
    assert L.spc_strerror(0) == b"ok"
    assert b"components" in L.spc_strerror(-2)


@pytest.mark.parametrize("seed", range(5))
def test_validate_matches_oracle(spc, seed):
    g = random_graph(9, p=0.4, seed=seed, self_loops=seed % 2 == 1)
    assert spc.validate_graph(g) == 0 == oracle.validate(g)
    r = np.random.default_rng(seed)
    for kind in range(4):
        b = Graph(g.n, g.row_ptr.copy(), g.col.copy(), g.w.copy(),
                  None if g.self_w is None else g.self_w.copy())
        j = int(r.integers(0, g.nnz))
        if kind == 0:
            b.w[j] += 1                       # asymmetric
        elif kind == 1:
            b.w[j] = -1                       # negative weight
        elif kind == 2:
            row = int(np.searchsorted(b.row_ptr, j, side="right") - 1)
            b.col[j] = row                    # diagonal entry
        else:
            if b.self_w is None:
                continue
            b.self_w[0] = -3                  # negative self-loop
        assert spc.validate_graph(b) == oracle.validate(b) == spc.SPC_EINVAL


def test_validate_overflow(spc):
    g = from_edges(3, [0, 1], [1, 2], np.array([2 ** 30, 5], np.int32))
    assert spc.validate_graph(g) == spc.SPC_EOVERFLOW == oracle.validate(g)
    g = from_edges(3, [0, 1], [1, 2], np.array([2 ** 29, 5], np.int32))
    assert spc.validate_graph(g) == 0


def test_validate_float_weights(spc):
    g = random_graph(8, p=0.5, seed=2, float_weights=True, self_loops=True)
    assert spc.validate_graph(g) == 0
    g.w[3] = np.float32(np.inf)
    assert spc.validate_graph(g) == spc.SPC_EINVAL

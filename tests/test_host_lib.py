"""Host-side checks of the product library (no GPU needed): it loads, exports
every entry point include/pcot.h declares, validates arguments, and its
planner emits exactly the leaf orders the oracle enumerates from the paper's
description, each a legal order by brute force."""
import ctypes
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(pcot_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    import paper_1802_00166_amd as pc
    lib = ctypes.CDLL(pc.LIB_PATH)
    names = _declared()
    assert "pcot_stencil_run" in names and "pcot_dp_run" in names
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert missing == []


def test_version_and_validation_without_gpu():
    import paper_1802_00166_amd as pc
    assert b"gfx950" in pc.pcot_version()
    # invalid kind / dims / tile are rejected on the host
    with pytest.raises(pc.PcotError):
        pc.workspace_bytes("jacobi2d", "f64", (2, 10), 5, (4, 8, 64), "slt_wave")
    assert pc.pcot_stencil_workspace(9, 0, pc._dims((10, 10)), 5, None, 0) == 0
    assert not pc.tile_supported("jacobi2d", "f64", (4, 8, 96))   # 96 columns: not 64*C
    assert pc.tile_supported("jacobi2d", "f64", (16, 32, 128))
    t = pc.make_tile(4, 1, 64)
    assert pc.pcot_stencil_tile_supported(2, 0, ctypes.byref(t)) == -1   # s < 2: invalid


@pytest.mark.parametrize("kind,dims,T,tile", [
    ("jacobi1d", (10,), 7, (3, 4)),
    ("jacobi1d", (40,), 30, (8, 16)),
    ("jacobi2d", (12, 9), 5, (2, 3, 4)),
    ("jacobi2d", (20, 17), 9, (4, 8, 5)),
    ("jacobi2d", (9, 8), 6, (4, 2, 2)),
    ("heat3d", (6, 7, 5), 3, (2, 2, 3, 2)),
    ("heat3d", (9, 8, 10), 5, (2, 4, 3, 5)),
])
def test_planner_orders_match_oracle_enumeration(kind, dims, T, tile):
    import paper_1802_00166_amd as pc
    want = {
        "slt_lex": oracle.slt_leaves(dims, T, tile),
        "slt_wave": oracle.slt_leaves(dims, T, tile, wavefront=True),
        "cot_seq": oracle.cot_leaves(dims, T, tile),
        "cot_par": oracle.cot_leaves(dims, T, tile, parallel_groups=True),
    }
    for sched, order in want.items():
        got = pc.plan(kind, dims, T, tile, sched)
        assert got == [tuple(k) for k in order], sched
        assert oracle.check_plan(got, dims, T, tile) == []


def test_planner_full_size_leaf_counts():
    """Leaf counts at the headline size against the closed form: per time
    band, the skewed rows/columns a band touches."""
    import paper_1802_00166_amd as pc
    n, T, bt, bs = 4096, 512, 16, 64
    got = len(pc.plan("jacobi2d", (n, n), T, (bt, bs, bs), "slt_wave"))
    want = 0
    for kt in range(T // bt):
        t0, t1 = kt * bt, kt * bt + bt - 1
        lo, hi = 1 + t0, n - 2 + t1          # skewed range touched by the band
        k = (hi - 1) // bs - (lo - 1) // bs + 1
        want += k * k
    assert got == want
    assert len(pc.plan("jacobi2d", (n, n), T, (bt, bs, bs), "cot_par")) == want

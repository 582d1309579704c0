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


# Fields the tiled executors cannot address (32-bit byte offsets, stores
# masked at offset 0x7FFFFFF0) are refused on the host; nothing here touches
# a GPU: validation fails before any pointer is used.
@pytest.mark.parametrize("kind,dtype,dims", [
    ("jacobi2d", "f64", (16400, 16400)),     # 2.0 GiB
    ("heat3d", "f64", (700, 700, 700)),      # 2.6 GiB
    ("jacobi2d", "f32", (40000, 40000)),     # 6.0 GiB (past 4 GiB: a 32-bit size would wrap)
    ("jacobi1d", "bf16", (1 << 30,)),        # 2 GiB of bf16
])
def test_tiled_fields_past_the_offset_limit_are_refused(kind, dtype, dims):
    import paper_1802_00166_amd as pc
    tile = {"jacobi1d": (16, 256), "jacobi2d": (16, 64, 256), "heat3d": (2, 64, 16, 64)}[kind]
    tp = pc.make_tile(*tile)
    for sched in ("slt_lex", "slt_wave", "cot_seq", "cot_par"):
        n = pc.pcot_stencil_workspace(pc.KINDS[kind], pc.DTYPES[dtype], pc._dims(dims), 8,
                                      ctypes.byref(tp), pc.SCHEDULES[sched])
        assert n == 0
        assert "0x7FFFFFF0" in pc.last_error() or "below" in pc.last_error()
        st = pc.pcot_stencil_run(pc.KINDS[kind], pc.DTYPES[dtype], pc._dims(dims), 8, ctypes.byref(tp),
                                 pc.SCHEDULES[sched], ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000),
                                 ctypes.c_void_p(0x3000), ctypes.c_size_t(1 << 40), None)
        assert st == -2  # PCOT_ERR_UNSUPPORTED, before any device work
    # the batched form validates every instance the same way
    dims3 = (ctypes.c_int64 * 3)(*(list(dims) + [0] * (3 - len(dims))))
    Ts = (ctypes.c_int64 * 1)(8)
    tiles = (pc.pcot_tile * 1)(tp)
    assert pc.pcot_stencil_workspace_batched(pc.KINDS[kind], pc.DTYPES[dtype], 1, dims3, Ts, tiles,
                                             pc.SLT_WAVE) == 0
    # the untiled schedule has no such limit
    assert pc.pcot_stencil_workspace(pc.KINDS[kind], pc.DTYPES[dtype], pc._dims(dims), 8, None, pc.NAIVE) > 0


def test_tiled_field_just_under_the_offset_limit_is_accepted():
    import paper_1802_00166_amd as pc
    # f64 16000^2 = 1.91 GiB (+ two rows + 4 KiB) < 0x7FFFFFF0
    assert pc.workspace_bytes("jacobi2d", "f64", (16000, 16000), 8, (16, 64, 256), "slt_wave") > 0
    # the largest benchmark field, Heat-3D 512^3 f64 (1 GiB)
    assert pc.workspace_bytes("heat3d", "f64", (512, 512, 512), 128, (2, 64, 16, 64), "slt_wave") > 0
    with pytest.raises(pc.PcotError):
        pc.workspace_bytes("jacobi2d", "f64", (16400, 16400), 8, (16, 64, 256), "slt_wave")


def test_dp_plan_item_count_limit():
    import paper_1802_00166_amd as pc
    # N = 65536 at b = 32, k-chunk 16: about 2.9e9 k-chunk items, past int offsets
    tp = pc.make_tile(0, 32, 32, 16)
    assert pc.pcot_dp_workspace(65536, ctypes.byref(tp), pc.SLT_WAVE) == 0
    assert "items" in pc.last_error()
    # the same N with larger chunks stays under the limit (workspace only: no plan is built)
    tp = pc.make_tile(0, 64, 64, 256)
    assert pc.pcot_dp_workspace(65536, ctypes.byref(tp), pc.SLT_WAVE) > 0


def test_planner_matches_hand_enumerated_2d_orders():
    """The product planner against the hand-enumerated 2D golden (no oracle in between)."""
    import json
    import paper_1802_00166_amd as pc
    with open(os.path.join(ROOT, "tests", "golden", "cot_order_2d.json")) as f:
        g = json.load(f)
    pr = g["problem"]
    for sched in ("slt_lex", "slt_wave", "cot_seq", "cot_par"):
        got = pc.plan("jacobi2d", tuple(pr["dims"]), pr["T"], tuple(pr["tile"]), sched)
        assert [list(k) for k in got] == g[sched], sched


# ------------------------------------------------ trapezoid plans (host) ---
@pytest.mark.parametrize("sched", ["trap", "diamond"])
@pytest.mark.parametrize("shape,T,tile", [
    ((130, 300), 40, (16, 64, 128)),
    ((61, 77), 29, (8, 64, 128)),
    ((300, 520), 33, (8, 32, 128)),
    ((3, 3), 5, (8, 64, 128)),
    ((4, 700), 17, (16, 64, 128)),
    ((700, 5), 9, (8, 64, 128)),
    ((200, 200), 64, (8, 20, 30)),     # planner geometry at any footprint
])
def test_trap_plan_legal_by_brute_force(shape, T, tile, sched):
    import oracle
    import paper_1802_00166_amd as pc
    tiles, edges, traffic = pc.trap_plan(shape, T, tile, sched)
    assert oracle.check_trap_plan(shape, T, tiles, edges, tile[1:]) == []
    assert traffic[1] >= (shape[0] - 2) * (shape[1] - 2)   # every point stored at least at the end


def test_trap_plan_checker_catches_planted_mistakes():
    """The brute-force checker flags a dropped dependence, a range off by one
    and a tile out of queue order (mistakes planted in the plan it is given)."""
    import oracle
    import paper_1802_00166_amd as pc
    shape, T, tile = (130, 300), 40, (16, 64, 128)
    tiles, edges, _ = pc.trap_plan(shape, T, tile, "trap")
    assert oracle.check_trap_plan(shape, T, tiles, edges, tile[1:]) == []
    probs = oracle.check_trap_plan(shape, T, tiles, edges[1:], tile[1:])
    assert any(p[0] == "dependence" for p in probs)
    bad = tiles.copy()
    bad[0, 1] += 1                      # upright tile one row taller: overlaps its neighbour
    assert oracle.check_trap_plan(shape, T, bad, edges, tile[1:])
    rev = edges.copy()
    rev[0] = rev[0][::-1]
    assert any(p[0] == "edge order" for p in oracle.check_trap_plan(shape, T, tiles, rev, tile[1:]))


def test_trap_plan_refused_for_other_kinds_and_small_footprints():
    import paper_1802_00166_amd as pc
    with pytest.raises(pc.PcotError):
        pc.trap_plan((100, 100), 10, (16, 30, 128), "trap")    # F_y < 2 b_t + 2
    with pytest.raises(pc.PcotError):
        pc.trap_plan((100, 100), 10, (16, 64, 128), "slt_wave")


def test_motiv_workspace_is_linear_in_N_and_T():
    """O(N) memory: interior second buffer plus the two boundary arrays, not
    the (T+1) N of a full expansion."""
    import paper_1802_00166_amd as pc
    N, T = 4096, 8192
    ws = pc.workspace_bytes("motiv1d", "f64", (N,), T, (64, 256), "slt_wave")
    assert ws < 8 * (N + 2 * (T + 1)) + 64 * 1024 + 4 * 1024 * 4
    assert ws < 8 * N * (T + 1) / 100


def test_trap_plan_size_bound():
    """A concurrent-start plan is listed tile by tile on the host: plans of
    more than 2^24 tiles are refused before any is built."""
    import paper_1802_00166_amd as pc
    with pytest.raises(pc.PcotError) as e:
        pc.trap_plan((4096, 4096), 1 << 20, (8, 64, 128))
    assert "2^24" in str(e.value)
    with pytest.raises(pc.PcotError):   # the workspace query returns 0 for it
        pc.workspace_bytes("jacobi2d", "f64", (4096, 4096), 1 << 20, (8, 64, 128), "trap")

"""GPU parity of the concurrent-start trapezoid schedules (PCOT_TRAP,
PCOT_DIAMOND) of the 2D stencil against the oracle, through the C ABI: every
plan only reorders the points of the nest, so the result must equal the
oracle's bits exactly."""
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import field, run

pytestmark = pytest.mark.gpu

TILES = [(16, 64, 128), (8, 64, 128), (8, 32, 128)]


@pytest.mark.parametrize("sched", ["trap", "diamond"])
@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("shape,T", [
    ((130, 300), 40),     # several tiles per axis, T a multiple of some band heights
    ((61, 77), 29),       # ragged, a partial last band
    ((300, 520), 33),     # many tiles, walls on both sides of both axes
    ((3, 3), 5),          # one interior point
    ((4, 700), 17),       # two interior rows
    ((700, 5), 9),        # three interior columns
    ((45, 90), 1),        # one step
])
def test_trap_jacobi2d_f64_bit_exact(gpu, shape, T, tile, sched):
    u0 = field("jacobi2d", shape, "f64", 11)
    want = oracle.stencil("jacobi2d", "f64", u0, T)
    got = run("jacobi2d", "f64", u0, T, tile, sched)
    assert np.array_equal(got, want), (shape, T, tile, sched, np.abs(got - want).max())


def test_trap_repeated_runs_reuse_workspace(gpu):
    import torch
    import paper_1802_00166_amd as pc
    u0 = field("jacobi2d", (257, 391), "f64", 12)
    x = torch.from_numpy(u0).to(gpu)
    want = oracle.stencil("jacobi2d", "f64", u0, 48)
    ws = pc.alloc_workspace(pc.workspace_bytes("jacobi2d", "f64", u0.shape, 48, (16, 64, 128), "diamond"))
    out = torch.empty_like(x)
    for _ in range(3):
        pc.stencil_run("jacobi2d", "f64", x, 48, (16, 64, 128), "diamond", out=out, workspace=ws)
        torch.cuda.synchronize()
        assert pc.stream_status(ws) == 0
        assert np.array_equal(out.cpu().numpy(), want)


def test_trap_rejects_unsupported(gpu):
    import paper_1802_00166_amd as pc
    import torch
    x = torch.zeros((40, 40), dtype=torch.float32, device=gpu)
    with pytest.raises(pc.PcotError):   # f32 has no trapezoid executor
        pc.stencil_run("jacobi2d", "f32", x, 4, (16, 64, 128), "trap")
    x = torch.zeros((40, 40), dtype=torch.float64, device=gpu)
    with pytest.raises(pc.PcotError):   # footprint smaller than 2 b_t + 2
        pc.stencil_run("jacobi2d", "f64", x, 4, (32, 64, 128), "trap")


@pytest.mark.slow
@pytest.mark.parametrize("sched", ["trap", "diamond"])
def test_trap_full_size_headline(gpu, sched):
    """Jacobi-2D 4096^2, T=512, f64 at the trapezoid tiles the benchmark
    times: the whole field against the threaded (bit-identical) oracle."""
    u0 = synth.jacobi2d_input(4096, 4096)
    key = "_want_full"
    want = getattr(test_trap_full_size_headline, key, None)
    if want is None:
        want = oracle.stencil("jacobi2d", "f64", u0, 512, threads=min(16, os.cpu_count() or 1))
        setattr(test_trap_full_size_headline, key, want)
    for tile in [(16, 64, 128), (8, 64, 128)]:
        got = run("jacobi2d", "f64", u0, 512, tile, sched)
        assert np.array_equal(got, want), (tile, sched)

"""GPU parity of the nests with dependences inside a time step, through the
C ABI: in-place Gauss-Seidel-2D and the three-statement FDTD-2D update after
the embedding transformation, under every box-tile schedule.  Tiling only
reorders the points of a fully permutable nest, so every schedule and tile
must give the oracle's bits (the oracle runs the plain loop nests in program
order)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import field

pytestmark = pytest.mark.gpu

SCHEDS = ["slt_lex", "slt_wave", "cot_seq", "cot_par"]


def _gs_run(u0, T, tile, sched):
    import torch
    import paper_1802_00166_amd as pc
    x = torch.from_numpy(u0).to("cuda:0")
    y = pc.stencil_run("gs2d", "f64", x, T, tile, sched)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def _fdtd_fields(shape, seed):
    s = synth.test_rng(seed)
    n = shape[0] * shape[1]
    return [synth.uniform_f64(s, n, offset=k * n).reshape(shape) - 0.5 for k in range(3)]


def _fdtd_run(fields, T, tile, sched):
    import torch
    import paper_1802_00166_amd as pc
    x = torch.from_numpy(np.ascontiguousarray(np.stack(fields))).to("cuda:0")
    y = pc.stencil_run("fdtd2d", "f64", x, T, tile, sched)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("shape,T,tile", [
    ((70, 200), 17, (4, 8, 64)),
    ((130, 300), 40, (16, 32, 64)),
    ((61, 77), 29, (7, 5, 13)),        # odd sizes, ragged everywhere
    ((40, 140), 12, (32, 16, 32)),     # T < b_t
    ((33, 70), 9, (1, 2, 2)),          # smallest tile
    ((3, 3), 5, (4, 8, 8)),            # one interior point
])
def test_gs2d_all_schedules_bit_exact(gpu, shape, T, tile, sched):
    u0 = field("jacobi2d", shape, "f64", 21)
    want = oracle.gs2d(u0, T)
    got = _gs_run(u0, T, tile, sched)
    assert np.array_equal(got, want), (shape, T, tile, sched, np.abs(got - want).max())


@pytest.mark.parametrize("sched", ["naive"] + SCHEDS)
@pytest.mark.parametrize("shape,T,tile", [
    ((70, 200), 17, (4, 8, 64)),
    ((130, 90), 30, (8, 32, 32)),
    ((61, 77), 29, (7, 5, 13)),
    ((2, 2), 6, (4, 4, 4)),            # smallest grid
    ((1, 40), 5, (2, 2, 8)),           # one row: only ex changes
])
def test_fdtd2d_all_schedules_bit_exact(gpu, shape, T, tile, sched):
    f = _fdtd_fields(shape, 22)
    want = np.stack(oracle.fdtd2d(*f, T))
    got = _fdtd_run(f, T, tile, sched)
    assert np.array_equal(got, want), (shape, T, tile, sched, np.abs(got - want).max())


def test_front_kinds_reject_unsupported(gpu):
    import torch
    import paper_1802_00166_amd as pc
    x = torch.zeros((40, 40), dtype=torch.float32, device=gpu)
    with pytest.raises(pc.PcotError):
        pc.stencil_run("gs2d", "f32", x, 3, (4, 8, 8), "slt_wave")       # f64 only
    x = torch.zeros((40, 40), dtype=torch.float64, device=gpu)
    with pytest.raises(pc.PcotError):
        pc.stencil_run("gs2d", "f64", x, 3, None, "naive")               # sequential sweep
    with pytest.raises(pc.PcotError):
        pc.stencil_run("gs2d", "f64", x, 3, (64, 512, 512), "slt_wave")  # tile footprint above the LDS


@pytest.mark.slow
def test_gs2d_and_fdtd2d_full_size(gpu):
    """The paper's GS-2D and FDTD-2D shape (500 steps of 2000^2, Table 2) at
    the tiles the benchmark times, whole fields against the oracle."""
    import bench
    u0 = synth.jacobi2d_input(2000, 2000)
    want = oracle.gs2d(u0, 500)
    for tile, sched in [(bench.GS2D_TILE, "slt_wave"), (bench.GS2D_TILE, "cot_par")]:
        assert np.array_equal(_gs_run(u0, 500, tile, sched), want), (tile, sched)
    f = _fdtd_fields((2000, 2000), 23)
    want = np.stack(oracle.fdtd2d(*f, 500))
    for tile, sched in [(bench.FDTD2D_TILE, "slt_wave"), (None, "naive")]:
        assert np.array_equal(_fdtd_run(f, 500, tile, sched), want), (tile, sched)

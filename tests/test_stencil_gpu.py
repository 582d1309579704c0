"""GPU parity of the stencil path against the oracle, through the C ABI.

Every schedule and every tile shape must give the oracle's bits exactly
(f64, f32 and bf16 storage alike): the tiled and recursive schedules only
reorder the points of a fully permutable nest, and each point uses the fixed
operation order of its update rule without FMA contraction.
"""
import ctypes
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import field, run

pytestmark = pytest.mark.gpu

SCHEDS = ["naive", "slt_lex", "slt_wave", "cot_seq", "cot_par"]


@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("shape,T,tile", [
    ((70, 200), 17, (4, 8, 64)),
    ((130, 300), 40, (16, 32, 128)),
    ((45, 520), 33, (8, 16, 256)),
    ((100, 90), 64, (64, 4, 64)),
    ((61, 77), 29, (7, 5, 128)),       # odd leaf sizes, ragged everywhere
    ((40, 140), 12, (32, 16, 256)),    # T < b_t
    ((33, 70), 9, (1, 2, 64)),         # smallest leaf
])
def test_jacobi2d_f64_all_schedules_bit_exact(gpu, shape, T, tile, sched):
    u0 = field("jacobi2d", shape, "f64", 1)
    want = oracle.stencil("jacobi2d", "f64", u0, T)
    got = run("jacobi2d", "f64", u0, T, tile, sched)
    assert np.array_equal(got, want), np.abs(got - want).max()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("sched", ["naive", "slt_wave", "cot_par"])
@pytest.mark.parametrize("shape,T,tile", [
    ((70, 200), 17, (4, 8, 64)),
    ((130, 300), 40, (16, 32, 128)),
    ((61, 277), 29, (32, 5, 256)),
])
def test_jacobi2d_f32_bf16_bit_exact(gpu, shape, T, tile, sched, dtype):
    u0 = field("jacobi2d", shape, dtype, 2)
    want = oracle.stencil("jacobi2d", dtype, u0, T)
    got = run("jacobi2d", dtype, u0, T, tile, sched)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("T", [0, 1, 2, 3])
def test_jacobi2d_small_T_and_tiny_fields(gpu, T):
    for shape in [(3, 3), (3, 70), (70, 3), (4, 5)]:
        u0 = field("jacobi2d", shape, "f64", 3)
        want = oracle.stencil("jacobi2d", "f64", u0, T)
        for sched, tile in [("naive", None), ("slt_wave", (4, 8, 64)), ("cot_par", (2, 2, 64))]:
            assert np.array_equal(run("jacobi2d", "f64", u0, T, tile, sched), want), (shape, sched)


def test_jacobi2d_restart_and_constant_field_on_gpu(gpu):
    u0 = synth.jacobi2d_input(90, 150)
    a = run("jacobi2d", "f64", u0, 21, (8, 16, 64), "cot_seq")
    b = run("jacobi2d", "f64", a, 19, (8, 16, 64), "cot_seq")
    c = run("jacobi2d", "f64", u0, 40, (8, 16, 64), "cot_seq")
    assert np.array_equal(b, c)
    k = np.full((50, 140), float(np.float32(0.1)))
    assert np.array_equal(run("jacobi2d", "f64", k, 30, (16, 8, 128), "slt_wave"), k)


def test_jacobi2d_eigenmode_on_gpu(gpu):
    """Closed form independent of the oracle: a Fourier mode decays by lambda^T."""
    import math
    ny, nx, T = 33, 21, 200
    u0 = synth.jacobi2d_input(ny, nx, noise=0.0, modes=(1, 2))
    lam = (1 + 2 * math.cos(math.pi * 2 / (nx - 1)) + 2 * math.cos(math.pi / (ny - 1))) / 5
    got = run("jacobi2d", "f64", u0, T, (16, 8, 64), "cot_par")
    assert np.abs(got - lam ** T * u0).max() <= 8 * T * 2.0 ** -53


def test_workspace_status_and_errors(gpu):
    import paper_1802_00166_amd as pc
    import torch
    x = torch.zeros((20, 20), dtype=torch.float64, device="cuda:0")
    with pytest.raises(pc.PcotError) as e:
        pc.stencil_run("jacobi2d", "f64", x, 5, (4, 8, 100), "slt_wave")
    assert e.value.status == -2
    ws = pc.alloc_workspace(pc.workspace_bytes("jacobi2d", "f64", (20, 20), 5, (4, 8, 64), "slt_wave"))
    y = pc.stencil_run("jacobi2d", "f64", x, 5, (4, 8, 64), "slt_wave", workspace=ws)
    assert pc.stream_status(ws) == 0
    small = pc.alloc_workspace(256)
    tp = pc.make_tile(4, 8, 64)
    st = pc.pcot_stencil_run(pc.JACOBI2D, pc.F64, pc._dims((20, 20)), 5, ctypes.byref(tp), pc.SLT_WAVE,
                             ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                             ctypes.c_void_p(small.data_ptr()), 256, pc.stream_ptr())
    assert st == -5 and "workspace" in pc.last_error()
    with pytest.raises(pc.PcotError):
        pc.stencil_run("jacobi2d", "f64", x, 5, (4, 8, 64), "slt_wave", out=x)   # in == out


@pytest.mark.slow
def test_jacobi2d_full_size_f64_headline_tiles(gpu):
    """Jacobi-2D 4096^2, T=512, f64 at the launch configuration the benchmark
    times: whole field against the (threaded, bit-identical) oracle."""
    u0 = synth.jacobi2d_input(4096, 4096)
    threads = min(16, os.cpu_count() or 1)
    want = oracle.stencil("jacobi2d", "f64", u0, 512, threads=threads)
    import bench
    learned, _ = bench.pick_tiles()  # the tile and schedule the benchmark runs
    for tile, sched in [(tuple(learned["tile"]), learned["schedule"]), ((16, 64, 256), "cot_par"),
                        ((32, 128, 128), "slt_wave")]:
        got = run("jacobi2d", "f64", u0, 512, tile, sched)
        assert np.array_equal(got, want), (tile, sched)
    for (y, x) in [(1, 1), (2048, 2048), (4094, 4094), (1, 4094), (3000, 17)]:
        assert oracle.jacobi2d_point(u0, 512, y, x) == want[y, x]

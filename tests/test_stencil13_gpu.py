"""GPU parity of the Jacobi-1D and Heat-3D paths against the oracle, through
the C ABI.

As for Jacobi-2D, every schedule and tile shape reorders the points of a fully
permutable nest and keeps each point's fixed operation order with no FMA
contraction, so results must equal the oracle's bit for bit in every storage
type.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import field, run

pytestmark = pytest.mark.gpu

SCHEDS = ["naive", "slt_lex", "slt_wave", "cot_seq", "cot_par"]


# ------------------------------------------------------------- Jacobi-1D ---
@pytest.mark.parametrize("sched", SCHEDS)
def test_jacobi1d_headline_shape_bit_exact(gpu, sched):
    """N = 4096 points, T = 1000 steps, 64-step x 256-point leaves."""
    u0 = synth.jacobi1d_input(4096)
    want = oracle.stencil("jacobi1d", "f64", u0, 1000)
    got = run("jacobi1d", "f64", u0, 1000, (64, 256), sched)
    assert np.array_equal(got, want), np.abs(got - want).max()


@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("n,T,tile", [
    (70, 17, (4, 64)),
    (300, 130, (70, 128)),     # leaves of more than 64 levels
    (1000, 200, (200, 64)),    # T = b_t, three level groups per leaf
    (517, 77, (9, 256)),       # ragged
    (129, 300, (16, 128)),     # T >> n
    (66, 5, (1, 64)),          # one level per leaf
])
def test_jacobi1d_f64_all_schedules_bit_exact(gpu, n, T, tile, sched):
    u0 = field("jacobi1d", (n,), "f64", 11)
    want = oracle.stencil("jacobi1d", "f64", u0, T)
    got = run("jacobi1d", "f64", u0, T, tile, sched)
    assert np.array_equal(got, want), np.abs(got - want).max()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("sched", ["slt_lex", "cot_par"])
@pytest.mark.parametrize("n,T,tile", [(700, 90, (32, 128)), (4096, 300, (64, 256))])
def test_jacobi1d_f32_bf16_bit_exact(gpu, n, T, tile, sched, dtype):
    u0 = field("jacobi1d", (n,), dtype, 12)
    want = oracle.stencil("jacobi1d", dtype, u0, T)
    got = run("jacobi1d", dtype, u0, T, tile, sched)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n", [3, 1000, 4096, 10200, 10300, 20400])
def test_jacobi1d_naive_resident_block_bit_exact(gpu, n, dtype):
    """The untiled path keeps fields whose two levels fit one CU's LDS (up to
    10,224 f64 / 20,448 f32 or bf16 points) in one block for every step;
    larger ones take one kernel per step.  Both give the oracle's bits."""
    T = 157
    u0 = field("jacobi1d", (n,), dtype, 13)
    want = oracle.stencil("jacobi1d", dtype, u0, T)
    got = run("jacobi1d", dtype, u0, T, None, "naive")
    assert np.array_equal(got, want), (n, dtype)


def test_jacobi1d_tiny_fields_and_small_T(gpu):
    for n in [3, 4, 65, 66, 67]:
        for T in [0, 1, 2, 7]:
            u0 = field("jacobi1d", (n,), "f64", 13)
            want = oracle.stencil("jacobi1d", "f64", u0, T)
            for sched, tile in [("naive", None), ("slt_wave", (4, 64)), ("cot_seq", (3, 128))]:
                assert np.array_equal(run("jacobi1d", "f64", u0, T, tile, sched), want), (n, T, sched)


def test_jacobi1d_eigenmode_on_gpu(gpu):
    """Closed form independent of the oracle: sin(pi k x) decays by
    lambda = (1 + 2 cos(pi k / (n-1))) / 3 per step."""
    import math
    n, T, k = 257, 400, 3
    x = np.arange(n) / (n - 1)
    u0 = np.sin(math.pi * k * x)
    u0[0] = u0[-1] = 0.0
    lam = (1 + 2 * math.cos(math.pi * k / (n - 1))) / 3
    got = run("jacobi1d", "f64", u0, T, (32, 64), "cot_par")
    assert np.abs(got - lam ** T * u0).max() <= 4 * T * 2.0 ** -53


# --------------------------------------------------------------- Heat-3D ---
@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("shape,T,tile", [
    ((20, 18, 70), 9, (4, 8, 4, 64)),
    ((33, 13, 130), 13, (3, 16, 2, 64)),
    ((12, 30, 40), 5, (2, 5, 8, 64)),
    ((24, 20, 100), 20, (8, 6, 4, 64)),   # rings beyond 64 KiB of LDS
    ((9, 9, 9), 7, (1, 2, 2, 64)),        # smallest leaf
    ((20, 40, 70), 9, (2, 8, 16, 64)),    # 16 waves per leaf
])
def test_heat3d_f64_all_schedules_bit_exact(gpu, shape, T, tile, sched):
    u0 = field("heat3d", shape, "f64", 21)
    want = oracle.stencil("heat3d", "f64", u0, T)
    got = run("heat3d", "f64", u0, T, tile, sched)
    assert np.array_equal(got, want), np.abs(got - want).max()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("sched", ["slt_wave", "cot_par"])
def test_heat3d_f32_bf16_bit_exact(gpu, sched, dtype):
    u0 = field("heat3d", (30, 26, 140), dtype, 22)
    want = oracle.stencil("heat3d", dtype, u0, 12)
    got = run("heat3d", dtype, u0, 12, (4, 16, 4, 64), sched)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_heat3d_wide_leaves_f32_bf16_bit_exact(gpu, dtype):
    """b_y = 16 and b_t = 8 leaves, whose rings fit LDS only for 4-byte values."""
    u0 = field("heat3d", (26, 50, 90), dtype, 24)
    want = oracle.stencil("heat3d", dtype, u0, 13)
    for tile in [(4, 16, 16, 64), (8, 8, 8, 64)]:
        assert np.array_equal(run("heat3d", dtype, u0, 13, tile, "slt_wave"), want), tile


def test_heat3d_tiny_fields_and_small_T(gpu):
    for shape in [(3, 3, 3), (3, 4, 70), (5, 3, 3), (4, 66, 5)]:
        for T in [0, 1, 3]:
            u0 = field("heat3d", shape, "f64", 23)
            want = oracle.stencil("heat3d", "f64", u0, T)
            for sched, tile in [("naive", None), ("slt_lex", (2, 4, 2, 64)), ("cot_par", (4, 8, 4, 64))]:
                assert np.array_equal(run("heat3d", "f64", u0, T, tile, sched), want), (shape, T, sched)


def test_heat3d_constant_field_fixed_on_gpu(gpu):
    """(c - 2c) + c = 0 exactly, so every constant field is a fixed point."""
    k = np.full((14, 12, 80), 0.3)
    assert np.array_equal(run("heat3d", "f64", k, 11, (4, 8, 4, 64), "slt_wave"), k)


@pytest.mark.slow
def test_heat3d_full_size_bench_tiles(gpu):
    """Heat-3D 512^3, T = 128 in each storage type at the tile the benchmark
    times: the whole field against the (threaded, bit-identical) oracle."""
    import bench
    threads = min(16, os.cpu_count() or 1)
    u = synth.heat3d_input(512)
    for dtype in ["f64", "f32", "bf16"]:
        u0 = u if dtype == "f64" else (u.astype(np.float32) if dtype == "f32"
                                       else synth.to_bf16_bits(u.astype(np.float32)))
        want = oracle.stencil("heat3d", dtype, u0, 128, threads=threads)
        got = run("heat3d", dtype, u0, 128, bench.HEAT3D_TILES[dtype], "slt_wave")
        assert np.array_equal(got, want), dtype
        del want, got

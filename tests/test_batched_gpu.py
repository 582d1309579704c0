"""Batched uneven instances in one persistent launch (device tile queue),
HIP-graph capture of that launch, and the binary64 device error norms.

Every instance of a batch must equal the oracle bit for bit, exactly as when
it runs alone: the merged queue only interleaves independent instances.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import field, to_device, to_host

pytestmark = pytest.mark.gpu


def _uneven(kind, n, lo, hi, tlo, thi, seed):
    s = synth.test_rng(seed)
    d = {"jacobi1d": 1, "jacobi2d": 2, "heat3d": 3}[kind]
    ext = synth.randint(s, n * d, lo, hi)
    shapes = [tuple(int(v) for v in ext[i * d:(i + 1) * d]) for i in range(n)]
    Ts = [int(v) for v in synth.randint(s, n, tlo, thi, offset=n * d)]
    return shapes, Ts


@pytest.mark.parametrize("dtype", ["f32", "f64", "bf16"])
@pytest.mark.parametrize("sched", ["slt_wave", "cot_par"])
def test_batched_jacobi2d_uneven_bit_exact(gpu, dtype, sched):
    import paper_1802_00166_amd as pc
    shapes, Ts = _uneven("jacobi2d", 12, 20, 300, 1, 60, 31)
    tiles = [(8 * (1 + i % 3), 8 + 4 * (i % 5), 128) for i in range(12)]
    u0s = [field("jacobi2d", s, dtype, 40 + i) for i, s in enumerate(shapes)]
    outs = pc.stencil_run_batched("jacobi2d", dtype, [to_device(u, dtype) for u in u0s], Ts, tiles, sched)
    for i, (u, T) in enumerate(zip(u0s, Ts)):
        want = oracle.stencil("jacobi2d", dtype, u, T)
        assert np.array_equal(to_host(outs[i], dtype), want), (i, shapes[i], Ts[i], tiles[i])


def test_batched_jacobi1d_and_heat3d_bit_exact(gpu):
    import paper_1802_00166_amd as pc
    shapes, Ts = _uneven("jacobi1d", 9, 3, 900, 0, 150, 32)
    tiles = [(16 + 8 * (i % 4), 64) for i in range(9)]
    u0s = [field("jacobi1d", s, "f64", 50 + i) for i, s in enumerate(shapes)]
    outs = pc.stencil_run_batched("jacobi1d", "f64", [to_device(u, "f64") for u in u0s], Ts, tiles, "cot_par")
    for i, (u, T) in enumerate(zip(u0s, Ts)):
        assert np.array_equal(to_host(outs[i], "f64"), oracle.stencil("jacobi1d", "f64", u, T)), i
    shapes, Ts = _uneven("heat3d", 5, 3, 40, 1, 9, 33)
    tiles = [(1 + i % 2, 4 + 2 * i, 4, 64) for i in range(5)]
    u0s = [field("heat3d", s, "f64", 60 + i) for i, s in enumerate(shapes)]
    outs = pc.stencil_run_batched("heat3d", "f64", [to_device(u, "f64") for u in u0s], Ts, tiles, "slt_wave")
    for i, (u, T) in enumerate(zip(u0s, Ts)):
        assert np.array_equal(to_host(outs[i], "f64"), oracle.stencil("heat3d", "f64", u, T)), i


def test_batched_rejects_mixed_launch_shapes(gpu):
    import paper_1802_00166_amd as pc
    xs = [to_device(field("jacobi2d", (40, 40), "f32", 1), "f32") for _ in range(2)]
    with pytest.raises(pc.PcotError) as e:
        pc.stencil_run_batched("jacobi2d", "f32", xs, [5, 5], [(8, 8, 64), (8, 8, 128)], "slt_wave")
    assert "b_x differs" in str(e.value)
    with pytest.raises(pc.PcotError):
        pc.stencil_run_batched("jacobi2d", "f32", xs, [5, 5], [(8, 8, 64), (8, 8, 64)], "naive")


def test_batched_graph_capture_replays(gpu):
    """The batched launch recorded into a HIP graph: every replay, with eager
    work and new input contents in between, equals an eager run."""
    import torch
    import paper_1802_00166_amd as pc
    shapes, Ts = _uneven("jacobi2d", 16, 40, 260, 4, 48, 34)
    Ts[3] = 0                                  # a T = 0 instance is a plain copy
    tiles = [(16, 8 * (1 + i % 4), 64) for i in range(16)]
    u0s = [field("jacobi2d", s, "f32", 70 + i) for i, s in enumerate(shapes)]
    xs = [to_device(u, "f32") for u in u0s]
    outs = [torch.empty_like(x) for x in xs]
    ws = pc.alloc_workspace(pc.workspace_bytes_batched("jacobi2d", "f32", shapes, Ts, tiles, "cot_par"))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):               # eager run caches the plan (the only allocation)
        pc.stencil_run_batched("jacobi2d", "f32", xs, Ts, tiles, "cot_par", outs=outs, workspace=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pc.stencil_run_batched("jacobi2d", "f32", xs, Ts, tiles, "cot_par", outs=outs, workspace=ws)
    for rep in range(4):
        if rep == 2:                             # new contents, same buffers
            u0s = [u[::-1].copy() for u in u0s]
            for x, u in zip(xs, u0s):
                x.copy_(torch.from_numpy(u))
        for o in outs:
            o.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, (u, T) in enumerate(zip(u0s, Ts)):
            want = oracle.stencil("jacobi2d", "f32", u, T)
            assert np.array_equal(to_host(outs[i], "f32"), want), (rep, i)
        eager = pc.stencil_run_batched("jacobi2d", "f32", xs, Ts, tiles, "cot_par")
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert torch.equal(o, e)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("shape", [(1000,), (77, 130), (9, 21, 70)])
def test_error_norms_match_host_binary64(gpu, dtype, shape):
    import torch
    import paper_1802_00166_amd as pc
    r = field("jacobi2d", shape, "f64", 80)
    x = field("jacobi2d", shape, dtype, 81)
    xr = synth.from_bf16_bits(x).astype(np.float64) if dtype == "bf16" else x.astype(np.float64)
    inner = tuple(slice(1, -1) for _ in shape)
    e = (xr - r)[inner]
    got = pc.error_norms(dtype, to_device(x, dtype), torch.from_numpy(r).to("cuda:0"))
    assert got["max_abs"] == np.abs(e).max()
    assert got["max_ref"] == np.abs(r[inner]).max()
    assert got["sum_sq"] == pytest.approx(float((e * e).sum()), rel=1e-12)
    assert got["sum_ref_sq"] == pytest.approx(float((r[inner] ** 2).sum()), rel=1e-12)
    again = pc.error_norms(dtype, to_device(x, dtype), torch.from_numpy(r).to("cuda:0"))
    assert again == got                      # fixed reduction order: same bits every call

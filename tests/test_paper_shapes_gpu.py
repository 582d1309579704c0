"""Whole-field parity at the paper's own problem shapes (its Table 2, not
powers of two), in the launch configurations `bench.py --workload
paper_shapes` times: Jacobi-2D 3000^2 T=500, Heat-3D 350^3 T=50 (f64) and the
interval DP at N = 4000, against the threaded (bit-identical) oracle."""
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import run

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

THREADS = min(16, os.cpu_count() or 1)


def test_jacobi2d_paper_shape(gpu):
    import bench
    (ny, nx), T = bench.PAPER_SHAPES["jacobi2d"]
    tile, sched = bench.paper_jacobi2d_tile()
    u0 = synth.jacobi2d_input(ny, nx)
    want = oracle.stencil("jacobi2d", "f64", u0, T, threads=THREADS)
    assert np.array_equal(run("jacobi2d", "f64", u0, T, tuple(tile), sched), want)


def test_heat3d_paper_shape(gpu):
    import bench
    (n, _, _), T = bench.PAPER_SHAPES["heat3d"]
    u0 = synth.heat3d_input(n)
    want = oracle.stencil("heat3d", "f64", u0, T, threads=THREADS)
    assert np.array_equal(run("heat3d", "f64", u0, T, bench.PAPER_HEAT3D_TILE, "slt_wave"), want)


def test_matrix_chain_paper_shape(gpu):
    import torch
    import bench
    import paper_1802_00166_amd as pc
    N = bench.PAPER_SHAPES["matrix_chain"]
    p = synth.chain_dims(N)
    want = np.triu(oracle.matrix_chain(p, threads=THREADS))
    C = pc.dp_run(torch.from_numpy(p).to("cuda:0"), 100, bench.CHAIN_TILE, "slt_wave")
    torch.cuda.synchronize()
    assert np.array_equal(np.triu(C.cpu().numpy()), want)

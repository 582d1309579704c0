"""GPU parity of the interval DP (matrix chain) against the oracle, bit-exact.

Integer min and + are exact and associative, so every schedule, block size
and k-split must reproduce the oracle's triangle exactly (32-bit and 64-bit
arithmetic paths alike).
"""
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _run(p_np, pmax, tile, sched):
    import torch
    import paper_1802_00166_amd as pc
    p = torch.from_numpy(np.ascontiguousarray(p_np, dtype=np.int64)).to("cuda:0")
    C = pc.dp_run(p, pmax, tile, sched)
    torch.cuda.synchronize()
    return C.cpu().numpy()


def _upper(C):
    i, j = np.triu_indices(C.shape[0])
    return C[i, j]


@pytest.mark.parametrize("sched", ["slt_wave", "cot_par"])
@pytest.mark.parametrize("N,tile", [
    (1, (0, 32, 32, 16)), (2, (0, 32, 32, 16)), (3, (0, 64, 64, 64)), (10, (0, 32, 32, 16)),
    (33, (0, 32, 32, 16)), (64, (0, 64, 64, 64)), (65, (0, 32, 32, 32)), (130, (0, 64, 64, 16)),
    (257, (0, 32, 32, 256)), (300, (0, 64, 64, 128)),
])
def test_chain_u32_bit_exact(gpu, N, tile, sched):
    p = synth.randint(synth.test_rng(4000 + N), N + 1, 1, 100)
    want = oracle.matrix_chain(p)
    got = _run(p, 100, tile, sched)
    assert np.array_equal(_upper(got), _upper(want))
    assert np.all(np.tril(got, -1) == 0)


def test_chain_small_vs_enumeration(gpu):
    for n in range(1, 9):
        p = synth.randint(synth.test_rng(50 + n), n + 1, 1, 30)
        got = _run(p, 30, (0, 32, 32, 16), "slt_wave")
        assert got[0, n - 1] == oracle.chain_brute(p)


@pytest.mark.parametrize("sched", ["slt_wave", "cot_par"])
def test_chain_i64_path(gpu, sched):
    N = 150
    p = synth.randint(synth.test_rng(77), N + 1, 1, 100000)   # (N-1) pmax^3 >> 2^32
    want = oracle.matrix_chain(p)
    got = _run(p, 100000, (0, 64, 64, 64), sched)
    assert np.array_equal(_upper(got), _upper(want))


def test_chain_uniform_closed_form_at_u32_edge(gpu):
    N = 520
    got = _run(np.full(N + 1, 100), 100, (0, 64, 64, 256), "slt_wave")
    i, j = np.triu_indices(N)
    assert np.array_equal(got[i, j], (j - i) * 100 ** 3)


def test_chain_errors(gpu):
    import torch
    import paper_1802_00166_amd as pc
    p = torch.full((11,), 5, dtype=torch.int64, device="cuda:0")
    with pytest.raises(pc.PcotError) as e:
        pc.dp_run(p, 2 ** 30, (0, 64, 64, 64))
    assert e.value.status == -3          # (N-1) pmax^3 >= 2^62
    with pytest.raises(pc.PcotError):
        pc.dp_run(p, 100, (0, 48, 48, 64))  # unsupported block
    bad = torch.tensor([3, 0, 4, 5], dtype=torch.int64, device="cuda:0")
    ws = pc.alloc_workspace(pc.dp_workspace_bytes(3))
    pc.dp_run(bad, 100, workspace=ws)
    assert pc.stream_status(ws) == -7    # p = 0 is outside [1, pmax]


@pytest.mark.slow
def test_chain_full_size(gpu):
    """N = 4096, p uniform in [1, 100]: whole triangle against the (threaded,
    bit-identical) oracle, at the benchmark's tile and under both schedules."""
    p = synth.chain_dims(4096)
    want = _upper(oracle.matrix_chain(p, threads=min(16, os.cpu_count() or 1)))
    import bench
    for tile, sched in [(bench.CHAIN_TILE, "slt_wave"), ((0, 64, 64, 256), "slt_wave"),
                        ((0, 64, 64, 256), "cot_par")]:
        assert np.array_equal(_upper(_run(p, 100, tile, sched)), want), sched

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


def _split(p_np, pmax, tile, sched):
    import torch
    import paper_1802_00166_amd as pc
    p = torch.from_numpy(np.ascontiguousarray(p_np, dtype=np.int64)).to("cuda:0")
    C = pc.dp_run(p, pmax, tile, sched)
    S = pc.dp_split(p, C)
    torch.cuda.synchronize()
    return C.cpu().numpy(), S.cpu().numpy()


@pytest.mark.parametrize("N", [1, 2, 3, 7, 64, 300, 1000])
def test_chain_split_matches_oracle(gpu, N):
    """The parenthesization: smallest optimal k per cell (1-based, the
    oracle's sequential strict-minimum scan), zero on and below the diagonal."""
    p = synth.randint(synth.test_rng(90 + N), N + 1, 1, 100)
    C, S = _split(p, 100, (0, 32, 32, 32), "slt_wave")
    wC, wS = oracle.matrix_chain(p, want_split=True)
    assert np.array_equal(_upper(C), _upper(wC))
    assert np.array_equal(S, wS)


def test_chain_split_uniform_ties_take_smallest_k(gpu):
    """Uniform p: every split of a cell ties, so the split is the cell's
    first index (k = i)."""
    N = 200
    p = np.full(N + 1, 7, dtype=np.int64)
    C, S = _split(p, 7, (0, 32, 32, 32), "cot_par")
    i, j = np.triu_indices(N, 1)
    assert np.array_equal(S[i, j], i + 1)
    assert not S[np.tril_indices(N)].any()


def test_chain_split_reconstructs_cost(gpu):
    """Rebuilding the bracketing from split and summing its products gives
    C[1][N] (a property of any valid split table)."""
    N = 500
    p = synth.randint(synth.test_rng(95), N + 1, 1, 100)
    C, S = _split(p, 100, (0, 64, 64, 32), "slt_wave")

    def cost(i, j):   # 0-based cell (i, j)
        if i == j:
            return 0
        k = int(S[i, j])   # 1-based: A_k | A_{k+1}  ->  0-based split k - 1
        return cost(i, k - 1) + cost(k, j) + int(p[i]) * int(p[k]) * int(p[j + 1])
    import sys
    sys.setrecursionlimit(10000)
    assert cost(0, N - 1) == int(C[0, N - 1])


@pytest.mark.parametrize("sched", ["slt_wave", "cot_par"])
@pytest.mark.parametrize("N,pmax,kc", [(300, 100, 16), (517, 100, 48), (200, 1000, 32)])
def test_chain_block16_bit_exact(gpu, N, pmax, kc, sched):
    """16 x 16 tiles (32- and 64-bit paths)."""
    p = synth.randint(synth.test_rng(300 + N), N + 1, 1, pmax)
    want = _upper(oracle.matrix_chain(p))
    assert np.array_equal(_upper(_run(p, pmax, (0, 16, 16, kc), sched)), want)

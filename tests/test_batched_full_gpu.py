"""The 256-instance uneven batch exactly as the benchmark launches it: every
instance of the one persistent launch equals the oracle bit for bit, with the
best uniform tile, the cost model's tile for the batch and its per-instance
tiles, run eagerly and replayed from a HIP graph (with other work between
replays)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

_WANT = {}


def _batch():
    inst = synth.batched_instances(256)
    shapes = [(ny, nx) for (ny, nx, _) in inst]
    Ts = [TT for (_, _, TT) in inst]
    u0s = [synth.batched_field(i, ny, nx) for i, (ny, nx, _) in enumerate(inst)]
    return shapes, Ts, u0s


def _want(shapes, Ts, u0s):
    if not _WANT:
        for i, (u, T) in enumerate(zip(u0s, Ts)):
            _WANT[i] = oracle.stencil("jacobi2d", "f32", u, T, threads=16)
    return _WANT


def _tiles(name, shapes, Ts):
    from paper_1802_00166_amd import tune
    if name == "uniform":
        return [(16, 128, 256)] * len(shapes)
    model = tune.load_default_model()
    if model is None:
        pytest.skip("no trained cost model")
    if name == "model_batch":  # the benchmark's value: the model's one tile for the batch
        return [tune.batch_model_uniform(model, "jacobi2d", "f32", shapes, Ts)[0]] * len(shapes)
    return tune.batch_model_tiles(model, "jacobi2d", "f32", shapes, Ts)


@pytest.mark.parametrize("which", ["uniform", "model_batch", "model"])
def test_batched_256_benchmark_launch_bit_exact(gpu, which):
    import torch
    import paper_1802_00166_amd as pc
    shapes, Ts, u0s = _batch()
    tiles = _tiles(which, shapes, Ts)
    xs = [torch.from_numpy(u).to(gpu) for u in u0s]
    outs = [torch.empty_like(x) for x in xs]
    ws = pc.alloc_workspace(pc.workspace_bytes_batched("jacobi2d", "f32", shapes, Ts, tiles, "slt_wave"))
    pc.stencil_run_batched("jacobi2d", "f32", xs, Ts, tiles, "slt_wave", outs=outs, workspace=ws)
    torch.cuda.synchronize()
    assert pc.stream_status(ws) == 0, pc.last_error()
    want = _want(shapes, Ts, u0s)
    bad = [i for i in range(len(xs)) if not np.array_equal(outs[i].cpu().numpy(), want[i])]
    assert not bad, ("eager", which, bad[:8], [(shapes[i], Ts[i], tiles[i]) for i in bad[:4]])

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pc.stencil_run_batched("jacobi2d", "f32", xs, Ts, tiles, "slt_wave", outs=outs, workspace=ws)
    for rep in range(3):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert pc.stream_status(ws) == 0, pc.last_error()
        bad = [i for i in range(len(xs)) if not np.array_equal(outs[i].cpu().numpy(), want[i])]
        assert not bad, ("replay", rep, which, bad[:8])

"""Helpers for GPU parity tests: move seeded numpy fields to the device, run
through the C ABI, bring results back."""
import numpy as np


def to_device(a: np.ndarray, dtype: str):
    import torch
    if dtype == "bf16":
        t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint16).view(np.int16))
    else:
        t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda:0")


def to_host(t, dtype: str) -> np.ndarray:
    a = t.cpu().numpy()
    return a.view(np.uint16) if dtype == "bf16" else a


def run(kind, dtype, u0, T, tile=None, schedule="naive", out=None, workspace=None):
    import paper_1802_00166_amd as pc
    import torch
    x = to_device(u0, dtype)
    ws = workspace
    y = pc.stencil_run(kind, dtype, x, T, tile, schedule, out=out, workspace=ws)
    torch.cuda.synchronize()
    return to_host(y, dtype)


def field(kind, shape, dtype, stream_tag=0):
    import synth
    seed_stream = synth.STREAM_TESTS * 100 + stream_tag
    if dtype == "f64":
        return synth.uniform_field(shape, seed_stream, np.float64)
    u = synth.uniform_field(shape, seed_stream, np.float32)
    return synth.to_bf16_bits(u) if dtype == "bf16" else u

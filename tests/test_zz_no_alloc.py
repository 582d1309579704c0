"""The allocation-free norms entry point (static device scratch) against the
allocating one: identical bits on two calls in a row, the second smaller, and
replays from a HIP graph; the size limit is refused on the host."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _pair(gpu, shape, dtype, seed):
    import torch
    s = synth.test_rng(seed)
    n = int(np.prod(shape))
    r = synth.uniform_f64(s, n).reshape(shape)
    if dtype == "f64":
        x = r + 1e-9 * synth.uniform_f64(s + 1, n).reshape(shape)
        xt = torch.from_numpy(np.ascontiguousarray(x)).to(gpu)
    else:
        xt = torch.from_numpy(np.ascontiguousarray(r.astype(np.float32))).to(gpu)
    return xt, torch.from_numpy(np.ascontiguousarray(r)).to(gpu)


def test_static_norms_match_allocating_entry(gpu):
    import torch
    import paper_1802_00166_amd as pc
    out = torch.full((4,), -1.0, dtype=torch.float64, device=gpu)
    for shape, dtype, seed in [((300, 517), "f64", 1), ((37, 41), "f32", 2), ((19, 23, 29), "f64", 3)]:
        x, r = _pair(gpu, shape, dtype, seed)
        want = pc.error_norms(dtype, x, r)
        pc.error_norms_static(dtype, x, r, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = np.array([want["max_abs"], want["max_ref"], want["sum_sq"], want["sum_ref_sq"]])
        assert np.array_equal(got, ref), (shape, dtype, got, ref)


def test_static_norms_graph_replay(gpu):
    import torch
    import paper_1802_00166_amd as pc
    x, r = _pair(gpu, (257, 129), "f64", 4)
    out = torch.zeros(4, dtype=torch.float64, device=gpu)
    want = pc.error_norms("f64", x, r)
    ref = np.array([want["max_abs"], want["max_ref"], want["sum_sq"], want["sum_ref_sq"]])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pc.error_norms_static("f64", x, r, out, stream=side)   # first call on the device looks up the array
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pc.error_norms_static("f64", x, r, out)
    for rep in range(3):
        out.zero_()
        y, rr = _pair(gpu, (31, 33), "f64", 10 + rep)      # other use of the scratch between replays
        pc.error_norms_static("f64", y, rr, torch.zeros(4, dtype=torch.float64, device=gpu))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), rep


def test_static_norms_refuse_over_limit(gpu):
    import paper_1802_00166_amd as pc
    dims = (ctypes.c_int64 * 3)(1 << 13, 1 << 13, 1 << 12)   # > 2^36 interior points
    st = pc.pcot_error_norms_static(0, 3, dims, ctypes.c_void_p(16), ctypes.c_void_p(16),
                                    ctypes.c_void_p(16), None)
    assert st == -2  # PCOT_ERR_UNSUPPORTED
    assert "allocation-free limit" in pc.last_error()

"""Host-side checks of the autotuner and cost-model plumbing (no GPU):
candidate grids, features and the model file format."""
import ctypes
import math
import os

import numpy as np
import pytest


def _pc():
    import paper_1802_00166_amd as pc
    from paper_1802_00166_amd import tune
    return pc, tune


def test_candidate_grids_are_the_runnable_subset():
    pc, tune = _pc()
    for kind, dtype, shape, T, grid in [
        ("jacobi2d", "f64", (4096, 4096), 512,
         [(bt, by, bx) for bt in (4, 8, 16, 32, 64) for by in (16, 32, 64, 128, 256) for bx in (64, 128, 256)]),
        ("jacobi1d", "f64", (4096,), 1000, [(bt, bx) for bt in (16, 32, 64, 128, 256) for bx in (64, 128, 256)]),
        ("heat3d", "f32", (512, 512, 512), 128,
         [(bt, bz, by, 64) for bt in (2, 3, 4, 6, 8, 12) for bz in (16, 64, 256) for by in (2, 4, 8, 16)]),
    ]:
        prob = tune.problem(kind, dtype, shape, T)
        got = tune.candidates(prob)
        runnable = [t for t in grid if pc.tile_supported(kind, dtype, t)]
        want = [(t, s) for s in ("slt_lex", "slt_wave", "cot_seq", "cot_par") for t in runnable]
        assert got == want, kind
        assert tune.candidates(prob, ["cot_par"]) == [(t, "cot_par") for t in runnable]
    assert len(tune.candidates(tune.problem("jacobi2d", "f64", (64, 64), 8))) == 280
    dp = tune.candidates(tune.problem("matrix_chain", "", (4096,), 100))
    assert dp == [((0, b, b, k), s) for s in ("slt_wave", "cot_par") for b in (16, 32, 64)
                  for k in (16, 32, 64, 128, 256) if k >= b or b == 16]


def test_features_follow_their_definition():
    pc, tune = _pc()
    f = tune.features(tune.problem("jacobi2d", "f32", (1000, 300), 77), (16, 32, 128), "cot_par")
    want = [math.log2(1000), math.log2(300), math.log2(77), 4, 5, 7, 2, 4]
    assert np.allclose(f, want, rtol=1e-6)
    f = tune.features(tune.problem("jacobi1d", "f64", (4096,), 1000), (64, 256), "slt_lex")
    assert np.allclose(f, [12, 0, math.log2(1000), 6, 0, 8, 3, 1], rtol=1e-6)
    f = tune.features(tune.problem("heat3d", "bf16", (64, 32, 100), 10), (4, 16, 2, 64), "slt_wave")
    assert np.allclose(f, [11, math.log2(100), math.log2(10), 2, 5, 6, 1, 2], rtol=1e-6)
    f = tune.features(tune.problem("matrix_chain", "", (4096,), 100), (0, 64, 64, 128), "cot_par")
    assert np.allclose(f, [12, 6, 7, math.log2(100), 4, 0, 0, 0], rtol=1e-6)


def test_model_file_round_trip_and_rejection(tmp_path):
    pc, tune = _pc()
    rng = np.random.default_rng(5)
    params = rng.standard_normal(4801).astype(np.float32)
    p = tmp_path / "m.mlp"
    with open(p, "w") as f:
        f.write("pcot-mlp 1\n")
        f.write(" ".join("%.9g" % v for v in np.arange(8) * 0.5) + "\n")
        f.write(" ".join("%.9g" % v for v in np.arange(1, 9) * 0.25) + "\n")
        f.write("1.5 2.5\n")
        f.write("\n".join("%.9g" % v for v in params) + "\n")
    m = tune.Model.load(str(p))
    q = tmp_path / "m2.mlp"
    m.save(str(q))
    a = open(p).read().split()
    b = open(q).read().split()
    assert a[:2] == b[:2]
    assert np.array_equal(np.array(a[2:], dtype=np.float32), np.array(b[2:], dtype=np.float32))
    bad = tmp_path / "bad.mlp"
    bad.write_text("pcot-mlp 1\n1 2 3\n")
    with pytest.raises(pc.PcotError):
        tune.Model.load(str(bad))
    with pytest.raises(pc.PcotError):
        tune.Model.load(str(tmp_path / "missing.mlp"))


def test_train_and_tune_reject_bad_arguments_without_gpu():
    pc, tune = _pc()
    assert pc.pcot_tune_candidates(None, 0, None, None, 0) == -1
    recs = (pc.pcot_record * 1)()
    out = ctypes.c_void_p(0)
    assert pc.pcot_model_train(recs, 1, None, ctypes.byref(out), None, None) == -1   # n < 2
    recs2 = (pc.pcot_record * 2)()                                                  # ms = 0: invalid
    assert pc.pcot_model_train(recs2, 2, None, ctypes.byref(out), None, None) == -1
    order = (ctypes.c_int32 * 2)(0, 5)
    z = (ctypes.c_float * 4801)()
    assert pc.pcot_mlp_train(z, z, z, z, z, 2, order, 1, 2, 0, 1e-3, None, None) == -1   # row 5 of 2

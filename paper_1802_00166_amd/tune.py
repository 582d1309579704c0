"""Autotuner and learned cost model: Python wrappers over the C ABI.

Every step runs in the library: the sweep times candidates with HIP events,
the network trains and predicts in the device MLP kernels.  This module only
marshals arguments and keeps file paths.

    prob = tune.problem("jacobi2d", "f64", (4096, 4096), 512)
    best = tune.sweep(prob)                       # exhaustive timed sweep
    model = tune.Model.train(records)             # device training
    tile, sched, ms = model.predict(prob)         # argmin of predicted time
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

from . import (DTYPES, KINDS, MATRIX_CHAIN, MLP_PARAMS, SCHEDULES, TUNE_MODEL, TUNE_MODEL_VERIFY, TUNE_SWEEP,
               PcotError, check, last_error, make_tile, pcot_features, pcot_mlp_forward, pcot_mlp_grad,
               pcot_mlp_train, pcot_model_free, pcot_model_load, pcot_model_predict, pcot_model_predict_ms,
               pcot_model_save, pcot_model_train, pcot_problem, pcot_record, pcot_tile, pcot_train_opts,
               pcot_tune, pcot_tune_candidates, pcot_tune_opts, stream_ptr)

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL_DIR = os.path.join(HERE, "models")
SCHED_NAMES = {v: k for k, v in SCHEDULES.items()}
# schedules of the training sweeps of the stored stencil model
MODEL_SCHEDULES = ["slt_wave", "cot_par"]


def problem(kind: str, dtype: str, shape, T: int) -> pcot_problem:
    """A stencil problem, or kind="matrix_chain" with shape=(N,) and T=pmax."""
    p = pcot_problem()
    p.kind = MATRIX_CHAIN if kind == "matrix_chain" else KINDS[kind]
    p.dtype = DTYPES.get(dtype, 0)
    for i, v in enumerate(shape):
        p.dims[i] = int(v)
    p.T = int(T)
    return p


def mask_of(schedules) -> int:
    if not schedules:
        return 0
    m = 0
    for s in schedules:
        m |= 1 << SCHEDULES[s]
    return m


def tile_tuple(t: pcot_tile, kind: int):
    if kind == MATRIX_CHAIN:
        return (0, t.s[0], t.s[1], t.s[2])
    d = {1: 1, 2: 2, 3: 3}[kind]
    return (t.t,) + tuple(t.s[i] for i in range(d))


def _tile(t):
    return t if isinstance(t, pcot_tile) else make_tile(*t)


def candidates(prob: pcot_problem, schedules=None):
    n = pcot_tune_candidates(ctypes.byref(prob), mask_of(schedules), None, None, 0)
    if n < 0:
        raise PcotError(-1, last_error())
    tiles = (pcot_tile * n)()
    sch = (ctypes.c_int32 * n)()
    pcot_tune_candidates(ctypes.byref(prob), mask_of(schedules), tiles, sch, n)
    return [(tile_tuple(tiles[i], prob.kind), SCHED_NAMES[sch[i]]) for i in range(n)]


def features(prob: pcot_problem, tile, schedule: str) -> np.ndarray:
    f = (ctypes.c_float * 8)()
    tp = _tile(tile)
    check(pcot_features(ctypes.byref(prob), ctypes.byref(tp), SCHEDULES[schedule], f))
    return np.array(f, dtype=np.float32)


def _records_list(recs, n, kind):
    return [{"feat": [float(v) for v in recs[i].feat], "ms": float(recs[i].ms),
             "tile": list(tile_tuple(recs[i].tile, kind)), "schedule": SCHED_NAMES[recs[i].schedule]}
            for i in range(n)]


def tune(prob: pcot_problem, mode: int = TUNE_SWEEP, model=None, reps: int = 5, warmup: int = 2, topk: int = 3,
         schedules=None, stream=None):
    """Returns (best tile, best schedule, best ms, records)."""
    opts = pcot_tune_opts(mode, reps, warmup, topk, mask_of(schedules), model.ptr if model is not None else None)
    cap = max(1, len(candidates(prob, schedules)))
    recs = (pcot_record * cap)()
    best = pcot_tile()
    bs = ctypes.c_int32(0)
    bms = ctypes.c_double(0)
    nrec = ctypes.c_size_t(0)
    check(pcot_tune(ctypes.byref(prob), ctypes.byref(opts), ctypes.byref(best), ctypes.byref(bs), ctypes.byref(bms),
                    recs, cap, ctypes.byref(nrec), stream_ptr(stream)))
    return tile_tuple(best, prob.kind), SCHED_NAMES[bs.value], bms.value, _records_list(recs, nrec.value, prob.kind)


def sweep(prob, reps=5, warmup=2, schedules=None, stream=None):
    return tune(prob, TUNE_SWEEP, None, reps, warmup, 3, schedules, stream)


def _to_records(records):
    arr = (pcot_record * len(records))()
    for i, r in enumerate(records):
        for k in range(8):
            arr[i].feat[k] = float(r["feat"][k])
        arr[i].ms = float(r.get("ms", 1.0))
        t = r.get("tile")
        if t is not None:
            arr[i].tile = make_tile(*t)
        arr[i].schedule = SCHEDULES[r.get("schedule", "slt_wave")]
    return arr


class Model:
    """A trained cost model (owned pcot_model*)."""

    def __init__(self, ptr):
        self.ptr = ctypes.c_void_p(ptr)

    def __del__(self):
        # at interpreter exit the binding may already be torn down: then the
        # process frees everything anyway
        if getattr(self, "ptr", None) is not None and self.ptr.value and callable(pcot_model_free):
            pcot_model_free(self.ptr)
            self.ptr = None

    @classmethod
    def train(cls, records, epochs=300, batch=256, lr=1e-3, seed=1802, stream=None):
        arr = _to_records(records)
        opts = pcot_train_opts(int(epochs), int(batch), float(lr), int(seed))
        out = ctypes.c_void_p(0)
        loss = ctypes.c_float(0)
        check(pcot_model_train(arr, len(records), ctypes.byref(opts), ctypes.byref(out), ctypes.byref(loss),
                               stream_ptr(stream)))
        m = cls(out.value)
        m.final_loss = loss.value
        return m

    @classmethod
    def load(cls, path):
        out = ctypes.c_void_p(0)
        check(pcot_model_load(path.encode(), ctypes.byref(out)))
        return cls(out.value)

    def save(self, path):
        check(pcot_model_save(self.ptr, path.encode()))

    def predict_ms(self, records, stream=None) -> np.ndarray:
        arr = _to_records(records)
        out = (ctypes.c_float * len(records))()
        check(pcot_model_predict_ms(self.ptr, arr, len(records), out, stream_ptr(stream)))
        return np.array(out, dtype=np.float64)

    def predict(self, prob, schedules=None, stream=None):
        best = pcot_tile()
        bs = ctypes.c_int32(0)
        ms = ctypes.c_double(0)
        check(pcot_model_predict(self.ptr, ctypes.byref(prob), mask_of(schedules), ctypes.byref(best),
                                 ctypes.byref(bs), ctypes.byref(ms), stream_ptr(stream)))
        return tile_tuple(best, prob.kind), SCHED_NAMES[bs.value], ms.value


# ------------------------------------------------------ raw network access ---
def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def mlp_forward(params: np.ndarray, X: np.ndarray, stream=None) -> np.ndarray:
    params = np.ascontiguousarray(params, dtype=np.float32)
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.zeros(X.shape[0], dtype=np.float32)
    check(pcot_mlp_forward(_fptr(params), _fptr(X), X.shape[0], _fptr(y), stream_ptr(stream)))
    return y


def mlp_grad(params, X, y, stream=None):
    params = np.ascontiguousarray(params, dtype=np.float32)
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    g = np.zeros(MLP_PARAMS, dtype=np.float32)
    loss = ctypes.c_float(0)
    check(pcot_mlp_grad(_fptr(params), _fptr(X), _fptr(y), X.shape[0], _fptr(g), ctypes.byref(loss),
                        stream_ptr(stream)))
    return loss.value, g


def mlp_train(params, m, v, X, y, order, batch, step0=0, lr=1e-3, stream=None):
    """Adam epochs over `order` (epochs x n row indices); returns (params, m, v, epoch losses)."""
    params = np.array(params, dtype=np.float32)
    m = np.array(m, dtype=np.float32)
    v = np.array(v, dtype=np.float32)
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    order = np.ascontiguousarray(order, dtype=np.int32)
    epochs = order.shape[0]
    el = np.zeros(max(epochs, 1), dtype=np.float32)
    check(pcot_mlp_train(_fptr(params), _fptr(m), _fptr(v), _fptr(X), _fptr(y), X.shape[0],
                         order.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), epochs, int(batch), int(step0),
                         float(lr), _fptr(el), stream_ptr(stream)))
    return params, m, v, el[:epochs]


# ------------------------------------------------------ stored artefacts ---
def model_path(name: str = "stencil") -> str:
    return os.path.join(MODEL_DIR, name + ".mlp")


def load_default_model(name: str = "stencil"):
    p = model_path(name)
    return Model.load(p) if os.path.exists(p) else None


def predict_stencil(model: Model, kind: str, dtype: str, shape, T: int, schedules=None):
    tile, sched, _ = model.predict(problem(kind, dtype, shape, T), schedules)
    return tile, sched


def load_sweep_best(kind: str, dtype: str, shape, T: int):
    """Best (tile, schedule, ms) of a stored sweep of exactly this problem, if any."""
    p = os.path.join(MODEL_DIR, "sweeps.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        data = json.load(f)
    key = "%s/%s/%s/%d" % (kind, dtype, "x".join(str(int(v)) for v in shape), int(T))
    e = data.get(key)
    if not e:
        return None
    return tuple(e["best_tile"]), e["best_schedule"], e["best_ms"]


# Uniform tiles the batched launch is compared over (one tile for every
# instance); one executor instance runs a batch, so b_x is shared.
BATCH_UNIFORM_TILES = [(16, 64, 128), (32, 64, 128), (16, 64, 256), (32, 64, 256), (16, 32, 128),
                       (32, 32, 256), (16, 128, 256), (64, 64, 128)]


def batch_model_uniform(model: Model, kind: str, dtype: str, shapes, Ts, schedule: str = "slt_wave", topk: int = 1):
    """Tiles for a whole batch (one tile for every instance), ranked by the
    cost model; the `topk` best, best first.  The instances of a batch run
    together and fill the device, so what a tile costs there is its
    throughput on a full device, not an instance's stand-alone time (bound by
    its critical path, which favours small tiles).  The model ranks the
    candidates runnable for every instance on one problem that fills the
    device as the batch does: the batch's total extent as a cube of its
    dimension (each side capped at 4096, the largest trained extent), at the
    extent-weighted mean T."""
    d = len(shapes[0])
    vols = [float(np.prod(sh)) for sh in shapes]
    side = int(min(4096, round(sum(vols) ** (1.0 / d))))
    tw = max(1, int(round(sum(v * TT for v, TT in zip(vols, Ts)) / sum(vols))))
    rep = problem(kind, dtype, (side,) * d, tw)
    common = {tuple(c[0]) for c in candidates(rep, [schedule])}
    for sh, TT in zip(shapes, Ts):
        common &= {tuple(c[0]) for c in candidates(problem(kind, dtype, sh, TT), [schedule])}
    cand = sorted(common)
    ms = model.predict_ms([{"feat": list(features(rep, t, schedule)), "tile": list(t), "schedule": schedule}
                          for t in cand])
    order = np.argsort(np.asarray(ms), kind="stable")
    return [cand[int(i)] for i in order[:max(1, topk)]]


def batch_model_tiles(model: Model, kind: str, dtype: str, shapes, Ts, schedule: str = "slt_wave"):
    """Per-instance tiles of a batch from the cost model.  The batch runs one
    executor instance, so b_x is common: per instance the best predicted
    candidate of each b_x, then the b_x with the smallest predicted total."""
    per = []
    for sh, TT in zip(shapes, Ts):
        prob = problem(kind, dtype, sh, TT)
        cands = list(candidates(prob, [schedule]))
        ms = model.predict_ms([{"feat": list(features(prob, c[0], c[1])), "tile": list(c[0]),
                                "schedule": c[1]} for c in cands])
        best = {}
        for c, m in zip(cands, ms):
            bxc = c[0][-1]
            if bxc not in best or m < best[bxc][1]:
                best[bxc] = (tuple(c[0]), m)
        per.append(best)
    common = set(per[0])
    for p in per[1:]:
        common &= set(p)
    bx = min(sorted(common), key=lambda b: sum(p[b][1] for p in per))
    return [p[bx][0] for p in per]

"""Python binding of libpcot.so (the MI355X tiled / cache-oblivious loop-nest library).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/pcot.h.  PyTorch provides device
memory and streams.  There is no CPU fallback: importing this package raises
if the library has not been built (python -m paper_1802_00166_amd.build or
__graft_entry__.build()).
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcot.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libpcot.so is not built at %s; run __graft_entry__.build()" % LIB_PATH)

# torch first: its HIP runtime then serves the library too (both carry the
# soname libamdhip64.so.7), so device pointers and streams are shared.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

# enums (include/pcot.h)
JACOBI1D, JACOBI2D, HEAT3D = 1, 2, 3
F64, F32, BF16 = 0, 1, 2
NAIVE, SLT_LEX, SLT_WAVE, COT_SEQ, COT_PAR, TRAP, DIAMOND = 0, 1, 2, 3, 4, 5, 6
GS2D, FDTD2D, MOTIV1D = 4, 5, 6
KINDS = {"jacobi1d": JACOBI1D, "jacobi2d": JACOBI2D, "heat3d": HEAT3D, "gs2d": GS2D, "fdtd2d": FDTD2D,
         "motiv1d": MOTIV1D}
DTYPES = {"f64": F64, "f32": F32, "bf16": BF16}
SCHEDULES = {"naive": NAIVE, "slt_lex": SLT_LEX, "slt_wave": SLT_WAVE, "cot_seq": COT_SEQ, "cot_par": COT_PAR,
             "trap": TRAP, "diamond": DIAMOND}
STATUS = {0: "OK", -1: "INVALID", -2: "UNSUPPORTED", -3: "OVERFLOW", -4: "HIP", -5: "WORKSPACE",
          -6: "TIMEOUT", -7: "DEVICE", -8: "HOST"}


class pcot_tile(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int32), ("s", ctypes.c_int32 * 3)]


class pcot_problem(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dtype", ctypes.c_int32), ("dims", ctypes.c_int64 * 3),
                ("T", ctypes.c_int64)]


class pcot_record(ctypes.Structure):
    _fields_ = [("feat", ctypes.c_float * 8), ("ms", ctypes.c_float), ("tile", pcot_tile),
                ("schedule", ctypes.c_int32)]


class pcot_tune_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("reps", ctypes.c_int32), ("warmup", ctypes.c_int32),
                ("topk", ctypes.c_int32), ("sched_mask", ctypes.c_uint32), ("model", ctypes.c_void_p)]


class pcot_train_opts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


MATRIX_CHAIN = 4
TUNE_SWEEP, TUNE_MODEL, TUNE_MODEL_VERIFY = 0, 1, 2
MLP_PARAMS = 4801


class PcotError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, msg))
        self.status = status


_I32, _I64, _SZ, _P = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p
_I64P = ctypes.POINTER(ctypes.c_int64)
_TP = ctypes.POINTER(pcot_tile)

_SIGS = {
    "pcot_stencil_workspace": (_SZ, [_I32, _I32, _I64P, _I64, _TP, _I32]),
    "pcot_stencil_run": (_I32, [_I32, _I32, _I64P, _I64, _TP, _I32, _P, _P, _P, _SZ, _P]),
    "pcot_stencil_tile_supported": (_I32, [_I32, _I32, _TP]),
    "pcot_stencil_plan": (_I64, [_I32, _I64P, _I64, _TP, _I32, ctypes.POINTER(ctypes.c_int32), _I64]),
    "pcot_stencil_trap_plan": (_I64, [_I64P, _I64, _TP, _I32, ctypes.POINTER(ctypes.c_int32), _I64,
                                      ctypes.POINTER(ctypes.c_int32), _I64, _I64P, _I64P]),
    "pcot_stream_status": (_I32, [_P, _P]),
    "pcot_last_error": (ctypes.c_char_p, []),
    "pcot_version": (ctypes.c_char_p, []),
    "pcot_dp_workspace": (_SZ, [_I64, _TP, _I32]),
    "pcot_dp_run": (_I32, [_P, _I64, _I64, _TP, _I32, _P, _P, _SZ, _P]),
    "pcot_dp_split": (_I32, [_P, _I64, _P, _P, _P]),
    "pcot_stencil_workspace_batched": (_SZ, [_I32, _I32, _I32, _I64P, _I64P, _TP, _I32]),
    "pcot_stencil_run_batched": (_I32, [_I32, _I32, _I32, _I64P, _I64P, _TP, _I32, ctypes.POINTER(_P),
                                        ctypes.POINTER(_P), _P, _SZ, _P]),
    "pcot_error_norms": (_I32, [_I32, _I32, _I64P, _P, _P, ctypes.POINTER(ctypes.c_double), _P]),
    "pcot_error_norms_static": (_I32, [_I32, _I32, _I64P, _P, _P, _P, _P]),
    "pcot_tune_candidates": (_I64, [ctypes.POINTER(pcot_problem), ctypes.c_uint32, _TP,
                                    ctypes.POINTER(ctypes.c_int32), _I64]),
    "pcot_features": (_I32, [ctypes.POINTER(pcot_problem), _TP, _I32, ctypes.POINTER(ctypes.c_float)]),
    "pcot_tune": (_I32, [ctypes.POINTER(pcot_problem), ctypes.POINTER(pcot_tune_opts), _TP,
                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                         ctypes.POINTER(pcot_record), _SZ, ctypes.POINTER(ctypes.c_size_t), _P]),
    "pcot_model_train": (_I32, [ctypes.POINTER(pcot_record), _SZ, ctypes.POINTER(pcot_train_opts),
                                ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_float), _P]),
    "pcot_model_predict_ms": (_I32, [_P, ctypes.POINTER(pcot_record), _SZ, ctypes.POINTER(ctypes.c_float), _P]),
    "pcot_model_predict": (_I32, [_P, ctypes.POINTER(pcot_problem), ctypes.c_uint32, _TP,
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double), _P]),
    "pcot_model_save": (_I32, [_P, ctypes.c_char_p]),
    "pcot_model_load": (_I32, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]),
    "pcot_model_free": (None, [_P]),
    "pcot_mlp_forward": (_I32, [ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float), _I32,
                                ctypes.POINTER(ctypes.c_float), _P]),
    "pcot_mlp_grad": (_I32, [ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                             ctypes.POINTER(ctypes.c_float), _I32, ctypes.POINTER(ctypes.c_float),
                             ctypes.POINTER(ctypes.c_float), _P]),
    "pcot_mlp_train": (_I32, [ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                              ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                              ctypes.POINTER(ctypes.c_float), _I32, ctypes.POINTER(ctypes.c_int32), _I32, _I32,
                              _I32, ctypes.c_float, ctypes.POINTER(ctypes.c_float), _P]),
    "pcot_kernel_timing": (_I32, [_I32]),
    "pcot_kernel_timing_read": (_I32, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f


def optional_symbol(name, restype, argtypes):
    """Binds an entry point declared in include/pcot.h (None if not exported)."""
    f = getattr(_lib, name, None)
    if f is not None:
        f.restype = restype
        f.argtypes = argtypes
    return f


def last_error() -> str:
    return (_lib.pcot_last_error() or b"").decode()


def check(status: int) -> None:
    if status != 0:
        raise PcotError(status, last_error())


def make_tile(t: int, *s: int) -> pcot_tile:
    s = list(s) + [0] * (3 - len(s))
    return pcot_tile(int(t), (ctypes.c_int32 * 3)(*[int(v) for v in s]))


def _dims(shape):
    return (ctypes.c_int64 * 3)(*(list(int(v) for v in shape) + [0] * (3 - len(shape))))


# ------------------------------------------------------------ torch layer ---
def _torch():
    import torch
    return torch


def storage_dtype(dtype: str):
    torch = _torch()
    return {"f64": torch.float64, "f32": torch.float32, "bf16": torch.int16}[dtype]


def stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def workspace_bytes(kind: str, dtype: str, shape, T: int, tile, schedule: str) -> int:
    tp = tile if isinstance(tile, pcot_tile) else (make_tile(*tile) if tile is not None else None)
    n = pcot_stencil_workspace(KINDS[kind], DTYPES[dtype], _dims(shape), int(T),
                               ctypes.byref(tp) if tp is not None else None, SCHEDULES[schedule])
    if n == 0:
        raise PcotError(-1, last_error())
    return int(n)


def alloc_workspace(nbytes: int, device="cuda:0"):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def stencil_run(kind: str, dtype: str, x, T: int, tile=None, schedule: str = "naive", out=None,
                workspace=None, stream=None):
    """Runs T steps on device tensor x (shape = field extents incl. boundary;
    for fdtd2d a (3, ny, nx) tensor holding ex, ey, hz).

    bf16 fields are int16 tensors holding bfloat16 bit patterns.  Returns out.
    """
    torch = _torch()
    assert x.is_cuda and x.is_contiguous()
    if out is None:
        out = torch.empty_like(x)
    shape = tuple(x.shape[1:]) if kind == "fdtd2d" else tuple(x.shape)
    if kind == "fdtd2d":
        assert x.dim() == 3 and x.shape[0] == 3
    tp = tile if isinstance(tile, pcot_tile) else (make_tile(*tile) if tile is not None else None)
    nbytes = workspace_bytes(kind, dtype, shape, T, tp, schedule)
    if workspace is None or workspace.numel() < nbytes:
        workspace = alloc_workspace(nbytes, x.device)
    st = pcot_stencil_run(KINDS[kind], DTYPES[dtype], _dims(shape), int(T),
                          ctypes.byref(tp) if tp is not None else None, SCHEDULES[schedule],
                          ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                          ctypes.c_void_p(workspace.data_ptr()), ctypes.c_size_t(workspace.numel()),
                          stream_ptr(stream))
    check(st)
    return out


def _batch_args(shapes, Ts, tiles):
    n = len(shapes)
    if not (len(Ts) == n and len(tiles) == n):
        raise ValueError("shapes, Ts and tiles must have one entry per instance")
    dims = (ctypes.c_int64 * (3 * n))()
    for i, sh in enumerate(shapes):
        for j, v in enumerate(sh):
            dims[3 * i + j] = int(v)
    tarr = (ctypes.c_int64 * n)(*[int(t) for t in Ts])
    tl = (pcot_tile * n)(*[tp if isinstance(tp, pcot_tile) else make_tile(*tp) for tp in tiles])
    return n, dims, tarr, tl


def workspace_bytes_batched(kind: str, dtype: str, shapes, Ts, tiles, schedule: str) -> int:
    n, dims, tarr, tl = _batch_args(shapes, Ts, tiles)
    nb = pcot_stencil_workspace_batched(KINDS[kind], DTYPES[dtype], n, dims, tarr, tl, SCHEDULES[schedule])
    if nb == 0:
        raise PcotError(-1, last_error())
    return int(nb)


def stencil_run_batched(kind: str, dtype: str, xs, Ts, tiles, schedule: str = "slt_wave", outs=None,
                        workspace=None, stream=None):
    """Runs instance i for Ts[i] steps with tiles[i], all in one persistent launch.

    xs: list of contiguous device tensors (extents incl. boundary).  Returns outs."""
    torch = _torch()
    shapes = [tuple(x.shape) for x in xs]
    if outs is None:
        outs = [torch.empty_like(x) for x in xs]
    n, dims, tarr, tl = _batch_args(shapes, Ts, tiles)
    nb = workspace_bytes_batched(kind, dtype, shapes, Ts, tl, schedule)
    if workspace is None or workspace.numel() < nb:
        workspace = alloc_workspace(nb, xs[0].device)
    ins = (_P * n)(*[x.data_ptr() for x in xs])
    ous = (_P * n)(*[y.data_ptr() for y in outs])
    check(pcot_stencil_run_batched(KINDS[kind], DTYPES[dtype], n, dims, tarr, tl, SCHEDULES[schedule], ins, ous,
                                   ctypes.c_void_p(workspace.data_ptr()), ctypes.c_size_t(workspace.numel()),
                                   stream_ptr(stream)))
    return outs


def error_norms(dtype: str, x, r, stream=None) -> dict:
    """Binary64 device norms of x - r over the interior (r: float64 device tensor)."""
    torch = _torch()
    assert r.dtype == torch.float64 and r.shape == x.shape and r.is_contiguous() and x.is_contiguous()
    out = (ctypes.c_double * 4)()
    check(pcot_error_norms(DTYPES[dtype], x.dim(), _dims(x.shape), ctypes.c_void_p(x.data_ptr()),
                           ctypes.c_void_p(r.data_ptr()), out, stream_ptr(stream)))
    max_abs, max_ref, sse, ssr = list(out)
    return {"max_abs": max_abs, "max_ref": max_ref, "sum_sq": sse, "sum_ref_sq": ssr,
            "max_rel": max_abs / max_ref if max_ref > 0 else float("nan"),
            "l2_rel": (sse / ssr) ** 0.5 if ssr > 0 else float("nan")}


def error_norms_static(dtype: str, x, r, out, stream=None) -> None:
    """Allocation-free norms: enqueues the reduction, the four values land in
    `out` (a float64 device tensor of 4); no synchronisation."""
    torch = _torch()
    assert r.dtype == torch.float64 and r.shape == x.shape and r.is_contiguous() and x.is_contiguous()
    assert out.dtype == torch.float64 and out.numel() >= 4 and out.is_cuda
    check(pcot_error_norms_static(DTYPES[dtype], x.dim(), _dims(x.shape), ctypes.c_void_p(x.data_ptr()),
                                  ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  stream_ptr(stream)))


def stream_status(workspace, stream=None) -> int:
    return int(pcot_stream_status(ctypes.c_void_p(workspace.data_ptr()), stream_ptr(stream)))


def kernel_timing(enable: bool) -> None:
    check(pcot_kernel_timing(1 if enable else 0))


def kernel_timing_read():
    ms = ctypes.c_double(0)
    n = ctypes.c_int64(0)
    check(pcot_kernel_timing_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def tile_supported(kind: str, dtype: str, tile) -> bool:
    tp = tile if isinstance(tile, pcot_tile) else make_tile(*tile)
    return pcot_stencil_tile_supported(KINDS[kind], DTYPES[dtype], ctypes.byref(tp)) == 0


def dp_workspace_bytes(N: int, tile=(0, 64, 64, 256), schedule: str = "slt_wave") -> int:
    tp = tile if isinstance(tile, pcot_tile) else make_tile(*tile)
    n = pcot_dp_workspace(int(N), ctypes.byref(tp), SCHEDULES[schedule])
    if n == 0:
        raise PcotError(-1, last_error())
    return int(n)


def dp_run(p, pmax: int, tile=(0, 64, 64, 256), schedule: str = "slt_wave", out=None, workspace=None,
           stream=None):
    """Matrix-chain DP on device int64 tensor p (N+1 dims); returns the N x N int64 cost matrix.

    tile = (unused, b, b, k-chunk)."""
    torch = _torch()
    assert p.is_cuda and p.dtype == torch.int64 and p.is_contiguous()
    N = p.numel() - 1
    if out is None:
        out = torch.empty((N, N), dtype=torch.int64, device=p.device)
    tp = tile if isinstance(tile, pcot_tile) else make_tile(*tile)
    nbytes = dp_workspace_bytes(N, tp, schedule)
    if workspace is None or workspace.numel() < nbytes:
        workspace = alloc_workspace(nbytes, p.device)
    check(pcot_dp_run(ctypes.c_void_p(p.data_ptr()), int(N), int(pmax), ctypes.byref(tp), SCHEDULES[schedule],
                      ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(workspace.data_ptr()),
                      ctypes.c_size_t(workspace.numel()), stream_ptr(stream)))
    return out


def dp_split(p, C, out=None, stream=None):
    """Optimal split (1-based k of A_k | A_{k+1}, smallest on ties) of every
    cell from the final cost table C of dp_run; N x N int64 device tensor."""
    torch = _torch()
    assert p.is_cuda and C.is_cuda and p.dtype == torch.int64 and C.dtype == torch.int64
    N = p.numel() - 1
    assert C.shape == (N, N) and C.is_contiguous()
    if out is None:
        out = torch.empty((N, N), dtype=torch.int64, device=p.device)
    check(pcot_dp_split(ctypes.c_void_p(p.data_ptr()), int(N), ctypes.c_void_p(C.data_ptr()),
                        ctypes.c_void_p(out.data_ptr()), stream_ptr(stream)))
    return out


def plan(kind: str, shape, T: int, tile, schedule: str):
    """Leaf visiting order the planner emits (host only): list of tuples."""
    tp = tile if isinstance(tile, pcot_tile) else make_tile(*tile)
    d = len(shape)
    n = pcot_stencil_plan(KINDS[kind], _dims(shape), int(T), ctypes.byref(tp), SCHEDULES[schedule], None, 0)
    if n < 0:
        raise PcotError(-1, last_error())
    buf = (ctypes.c_int32 * (4 * max(n, 1)))()
    pcot_stencil_plan(KINDS[kind], _dims(shape), int(T), ctypes.byref(tp), SCHEDULES[schedule], buf, n)
    return [tuple(buf[4 * i: 4 * i + d + 1]) for i in range(n)]


def trap_plan(shape, T: int, tile, schedule: str = "trap"):
    """Tiles of a trapezoid plan of the 2D stencil (host only).

    Returns (tiles, edges, traffic): tiles an int32 array (n, 12) of
    lo_y, hi_y, slo_y, shi_y, fo_y, lo_x, hi_x, slo_x, shi_x, fo_x, t0, nt in
    queue order; edges an int32 array (m, 2) of (predecessor, successor);
    traffic (elements loaded, elements stored) by the executor."""
    import numpy as np
    tp = tile if isinstance(tile, pcot_tile) else make_tile(*tile)
    ne = ctypes.c_int64(0)
    tr = (ctypes.c_int64 * 2)()
    n = pcot_stencil_trap_plan(_dims(shape), int(T), ctypes.byref(tp), SCHEDULES[schedule], None, 0, None, 0,
                               ctypes.byref(ne), tr)
    if n < 0:
        raise PcotError(-1, last_error())
    tiles = np.zeros((max(n, 1), 12), dtype=np.int32)
    edges = np.zeros((max(ne.value, 1), 2), dtype=np.int32)
    pcot_stencil_trap_plan(_dims(shape), int(T), ctypes.byref(tp), SCHEDULES[schedule],
                           tiles.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n,
                           edges.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ne.value, ctypes.byref(ne), tr)
    return tiles[:n], edges[:ne.value], (int(tr[0]), int(tr[1]))

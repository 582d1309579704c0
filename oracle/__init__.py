"""Oracle: slow, plain CPU definitions of what the hot path computes.

TEST INFRASTRUCTURE ONLY.  Imported by `tests/`, `__graft_entry__.smoke()` and
the CPU-baseline leg of `bench.py`; never by the product package, which must
fail loudly when its HIP library is missing instead of falling back here.

Contents
  * stencils (Jacobi-1D/2D, Heat-3D; f64, f32, bf16 storage), matrix-chain DP
    and single-point stencil evaluation: plain C in oracle.c, called via ctypes;
  * gs2d (in-place Gauss-Seidel, lexicographic order) and fdtd2d (the
    three-statement 2D Yee update in program order): plain C in oracle.c;
  * chain_brute: enumerates every full bracketing (no DP table);
  * cot_leaves / slt_leaves: the paper's leaf enumerations written from its
    description (bounding box, padding to b*2^k, recursive halving into
    orthants, zero- and empty-orthant early exits);
  * check_plan: brute-force coverage and dependence-order check of a tile list;
  * check_trap_plan: the same for concurrent-start trapezoid plans (coverage
    of every step, transitive predecessors of every input, footprints);
  * mlp_*: the 8-64-64-1 ReLU cost model (forward, backward, Adam) in float64.

Parity pins for each function live in tests/test_oracle_pins.py.  The cost
model and the plan checker have no printed values in the paper; their pins
are mathematical (finite differences, closed forms, brute force).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from itertools import product

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")
_lib = None


CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (IEEE doubles via SSE2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc"] + CFLAGS + ["-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        I = ctypes.c_int64
        for name, argt in [
            ("oracle_jacobi1d_f64", [P, P, I, I]), ("oracle_jacobi1d_f32", [P, P, I, I]),
            ("oracle_jacobi1d_bf16", [P, P, I, I]),
            ("oracle_jacobi2d_f64", [P, P, I, I, I]), ("oracle_jacobi2d_f32", [P, P, I, I, I]),
            ("oracle_jacobi2d_bf16", [P, P, I, I, I]),
            ("oracle_heat3d_f64", [P, P, I, I, I, I]), ("oracle_heat3d_f32", [P, P, I, I, I, I]),
            ("oracle_heat3d_bf16", [P, P, I, I, I, I]),
            ("oracle_matrix_chain", [P, I, P, P]),
            ("oracle_gs2d_f64", [P, P, I, I, I]), ("oracle_fdtd2d_f64", [P, P, P, I, I, I]),
            ("oracle_motiv_f64", [P, P, I, I]),
        ]:
            f = getattr(lib, name)
            f.argtypes = argt
            f.restype = ctypes.c_int
        lib.oracle_jacobi2d_point_f64.argtypes = [P, I, I, I, I, I]
        lib.oracle_jacobi2d_point_f64.restype = ctypes.c_double
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


_DT = {"f64": np.float64, "f32": np.float32, "bf16": np.uint16}


def stencil(kind: str, dtype: str, u0: np.ndarray, T: int, threads: int = 1) -> np.ndarray:
    """u_T from u_0 for kind in {jacobi1d, jacobi2d, heat3d}, dtype in {f64, f32, bf16}.

    bf16 arrays are uint16 bit patterns.  `threads` > 1 splits the outer
    spatial loop (identical bits).
    """
    lib = _load()
    a = np.ascontiguousarray(u0, dtype=_DT[dtype])
    out = np.empty_like(a)
    set_threads(threads)
    fn = getattr(lib, "oracle_%s_%s" % (kind, dtype))
    if kind == "jacobi1d":
        assert a.ndim == 1
        rc = fn(_ptr(a), _ptr(out), a.shape[0], int(T))
    elif kind == "jacobi2d":
        assert a.ndim == 2
        rc = fn(_ptr(a), _ptr(out), a.shape[0], a.shape[1], int(T))
    elif kind == "heat3d":
        assert a.ndim == 3
        rc = fn(_ptr(a), _ptr(out), a.shape[0], a.shape[1], a.shape[2], int(T))
    else:
        raise ValueError(kind)
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return out


def gs2d(u0: np.ndarray, T: int) -> np.ndarray:
    """T in-place Gauss-Seidel sweeps (lexicographic order) of the 5-point
    average, f64, boundary fixed (oracle.c: oracle_gs2d_f64)."""
    a = np.ascontiguousarray(u0, dtype=np.float64)
    out = np.empty_like(a)
    assert a.ndim == 2
    _load().oracle_gs2d_f64(_ptr(a), _ptr(out), a.shape[0], a.shape[1], int(T))
    return out


FDTD_CE, FDTD_CH = 0.25, 0.5


def fdtd2d(ex: np.ndarray, ey: np.ndarray, hz: np.ndarray, T: int):
    """T steps of the three-statement 2D Yee update (oracle.c:
    oracle_fdtd2d_f64); returns new (ex, ey, hz), inputs untouched."""
    e1, e2, h = (np.array(v, dtype=np.float64, order="C", copy=True) for v in (ex, ey, hz))
    assert e1.shape == e2.shape == h.shape and e1.ndim == 2
    _load().oracle_fdtd2d_f64(_ptr(e1), _ptr(e2), _ptr(h), e1.shape[0], e1.shape[1], int(T))
    return e1, e2, h


def motiv(a: np.ndarray, T: int) -> np.ndarray:
    """The appendix's motivating 1D program run as written, with its
    two-buffer allocation X[t mod 2] (oracle.c: oracle_motiv_f64): T steps of
    S1 (interior, reading the left boundary value of the previous step) then
    S2 / S3 (both boundaries through g).  Returns X after T steps."""
    x = np.ascontiguousarray(a, dtype=np.float64)
    assert x.ndim == 1 and x.shape[0] >= 3
    out = np.empty_like(x)
    _load().oracle_motiv_f64(_ptr(x), _ptr(out), x.shape[0], int(T))
    return out


def motiv_tiled_order(a: np.ndarray, T: int, bt: int, bx: int, aux: bool = True) -> np.ndarray:
    """The same program executed tile by tile in a different order: the
    skewed iteration space (t, j = i + t) cut into bt x bx boxes, visited
    band by band, left to right; every box runs its points level by level.
    With aux=True the values of S2 and S3 go to single-assignment arrays
    Y[t], Z[t] (the appendix's affine split; S1 reads Y[t-1] instead of
    X[(t-1)%2][0]) and X keeps the two-buffer allocation for S1 only.  With
    aux=False the original allocation is kept, whose memory-based
    dependences such an order violates.  Pure Python; small sizes."""
    N = len(a)
    X = [np.array(a, dtype=np.float64), np.array(a, dtype=np.float64)]
    Y = [float(a[0])] + [0.0] * T
    Z = [float(a[N - 1])] + [0.0] * T
    f = lambda p, q, r, s: 0.25 * (((p + q) + r) + s)
    g = lambda y: 0.5 * y + 0.25
    if aux:
        for t in range(1, T + 1):  # S2, S3 depend only on themselves
            Y[t] = g(Y[t - 1])
            Z[t] = g(Z[t - 1])
    for t0 in range(1, T + 1, bt):
        for j0 in range(1 + t0, N - 2 + T + 1, bx):
            for t in range(t0, min(t0 + bt, T + 1)):
                cur, old = X[t % 2], X[(t - 1) % 2]
                for j in range(j0, j0 + bx):
                    i = j - t
                    if 1 <= i <= N - 2:
                        if aux:
                            left = Y[t - 1] if i == 1 else old[i - 1]
                            right = Z[t - 1] if i == N - 2 else old[i + 1]
                            cur[i] = f(left, old[i], right, Y[t - 1])
                        else:
                            cur[i] = f(old[i - 1], old[i], old[i + 1], old[0])
                if not aux and j0 == 1 + t0:   # boundaries updated with the first box of a level
                    cur[0] = g(old[0])
                    cur[N - 1] = g(old[N - 1])
    out = X[T % 2].copy()
    if aux:
        out[0], out[N - 1] = Y[T], Z[T]
    return out


def jacobi2d_point(u0: np.ndarray, T: int, y: int, x: int) -> float:
    a = np.ascontiguousarray(u0, dtype=np.float64)
    return float(_load().oracle_jacobi2d_point_f64(_ptr(a), a.shape[0], a.shape[1], int(T), int(y), int(x)))


def matrix_chain(p: np.ndarray, threads: int = 1, want_split: bool = False):
    """Returns C (N x N int64, upper triangle incl. diagonal), and split if asked."""
    lib = _load()
    p = np.ascontiguousarray(p, dtype=np.int64)
    N = p.shape[0] - 1
    C = np.empty((N, N), dtype=np.int64)
    S = np.empty((N, N), dtype=np.int64) if want_split else None
    set_threads(threads)
    rc = lib.oracle_matrix_chain(_ptr(p), N, _ptr(C), _ptr(S) if S is not None else None)
    if rc != 0:
        raise ValueError("bad chain")
    return (C, S) if want_split else C


def chain_brute(p) -> int:
    """Minimum cost over every full binary bracketing of A_1..A_N (no DP table).

    Each bracketing is built as an explicit tree; its cost is the sum, over
    internal nodes joining A_i..A_k with A_{k+1}..A_j, of p[i-1]*p[k]*p[j].
    """
    p = [int(v) for v in p]
    N = len(p) - 1

    def trees(i, j):
        if i == j:
            return [("leaf", i)]
        out = []
        for k in range(i, j):
            for L in trees(i, k):
                for R in trees(k + 1, j):
                    out.append(("node", i, k, j, L, R))
        return out

    def cost(t):
        if t[0] == "leaf":
            return 0
        _, i, k, j, L, R = t
        return p[i - 1] * p[k] * p[j] + cost(L) + cost(R)

    return min(cost(t) for t in trees(1, N)) if N >= 1 else 0


# ------------------------------------------------------------- planning ---
# Domain of a d-dimensional radius-1 stencil over T steps, after the skew
# (t, i_1..i_d) -> (t, i_1 + t, ..., i_d + t) that makes every dependence
# non-negative (Section 4, the Heat-2D skewing example; appendix, the
# (t,i) -> (t, i+t) schedule of the 1D-Jacobi example):
#   0 <= t < T,  1 + t <= j_k <= n_k - 2 + t.
# Its bounding box is t in [0, T), j_k in [1, n_k - 2 + T - 1].


def skewed_bbox(dims, T):
    lo = [0] + [1 for _ in dims]
    hi = [T - 1] + [n - 2 + T - 1 for n in dims]  # inclusive
    return lo, hi


def in_domain(pt, dims, T):
    t = pt[0]
    if not (0 <= t < T):
        return False
    return all(1 + t <= j <= n - 2 + t for j, n in zip(pt[1:], dims))


def box_has_domain_point(lo, size, dims, T):
    """Brute force: does the box [lo, lo+size) contain a domain point?"""
    ranges = [range(l, l + s) for l, s in zip(lo, size)]
    for pt in product(*ranges):
        if in_domain(pt, dims, T):
            return True
    return False


def padded_extent(n, b):
    """Smallest b * 2^k >= n (Section 4, computing the bounding box)."""
    e = b
    while e < n:
        e *= 2
    return e


def cot_leaves(dims, T, tile, parallel_groups=False):
    """Leaves of the recursive decomposition in visiting order.

    tile = (b_t, b_1, ..., b_d).  The bounding box is padded per dimension to
    b*2^k; an orthant of size > b in some dimension is halved in every such
    dimension (the others are already at leaf size, so halving them would
    give zero-width orthants, which are skipped); orthants containing no
    domain point are skipped; leaves are visited in lexicographic orthant
    order (time bit most significant).

    parallel_groups: the parallel version runs the orthants of one split as
    tasks grouped by their number of upper halves, with a taskwait between
    groups; the orthants of a group run concurrently.  Their leaf sequences
    are therefore merged round-robin (one leaf of each member in turn), and
    groups follow each other.  Returns leaf origins as tile-grid indices.
    """
    lo, hi = skewed_bbox(dims, T)
    size = [padded_extent(h - l + 1, b) for l, h, b in zip(lo, hi, tile)]

    def rec(org, sz):
        if any(s <= 0 for s in sz):
            return []
        if not box_has_domain_point(org, sz, dims, T):
            return []
        if all(s <= b for s, b in zip(sz, tile)):
            return [tuple((o - l) // b for o, l, b in zip(org, lo, tile))]
        halves = []
        for o, s, b in zip(org, sz, tile):
            if s > b:
                h = s // 2
                halves.append([(o, h), (o + h, s - h)])
            else:
                halves.append([(o, s), (o + s, 0)])
        children = list(product(*[range(2)] * len(sz)))

        def child(bits):
            return rec([halves[d][bits[d]][0] for d in range(len(sz))],
                       [halves[d][bits[d]][1] for d in range(len(sz))])

        out = []
        if not parallel_groups:
            for bits in children:
                out += child(bits)
            return out
        for g in range(len(sz) + 1):
            seqs = [child(bits) for bits in children if sum(bits) == g]
            for i in range(max([len(q) for q in seqs] + [0])):
                for q in seqs:
                    if i < len(q):
                        out.append(q[i])
        return out

    return rec(lo, size)


def slt_leaves(dims, T, tile, wavefront=False):
    """Single-level tiles aligned at the bounding box's low corner, non-empty only.

    Lexicographic order of tile indices, or (wavefront) sorted by the sum of
    tile indices first.
    """
    lo, hi = skewed_bbox(dims, T)
    counts = [(h - l + 1 + b - 1) // b for l, h, b in zip(lo, hi, tile)]
    out = []
    for idx in product(*[range(c) for c in counts]):
        org = [l + i * b for l, i, b in zip(lo, idx, tile)]
        if box_has_domain_point(org, tile, dims, T):
            out.append(tuple(idx))
    if wavefront:
        out.sort(key=lambda k: (sum(k), k))
    return out


def check_plan(order, dims, T, tile):
    """Brute-force check of a tile visiting order.

    Every domain point must lie in exactly one listed tile, no listed tile
    may be empty or repeated, and for every dependence (t-1, j - delta) ->
    (t, j) with delta_k in {0, 1, 2} along one axis and 1 along the others
    (the skewed radius-1 stencil), the source's tile must not come after the
    sink's.  Returns a list of problems (empty when the plan is legal).
    """
    problems = []
    pos = {}
    for i, k in enumerate(order):
        k = tuple(k)
        if k in pos:
            problems.append(("duplicate", k))
        pos[k] = i
    lo, hi = skewed_bbox(dims, T)
    d = len(dims)

    def tile_of(pt):
        return tuple((c - l) // b for c, l, b in zip(pt, lo, tile))

    seen = set()
    deltas = []
    for axis in range(d):
        for dl in (0, 2):
            v = [1] * d
            v[axis] = dl
            deltas.append(tuple(v))
    deltas.append(tuple([1] * d))
    for pt in product(*[range(l, h + 1) for l, h in zip(lo, hi)]):
        if not in_domain(pt, dims, T):
            continue
        k = tile_of(pt)
        seen.add(k)
        if k not in pos:
            problems.append(("uncovered", pt))
            continue
        if pt[0] == 0:
            continue
        for dv in deltas:
            src = (pt[0] - 1,) + tuple(j - dd for j, dd in zip(pt[1:], dv))
            if in_domain(src, dims, T):
                ks = tile_of(src)
                if ks in pos and pos[ks] > pos[k]:
                    problems.append(("order", src, pt))
    for k in pos:
        if k not in seen:
            problems.append(("empty", k))
    return problems


def check_trap_plan(dims, T, tiles, edges, footprint):
    """Brute-force legality check of a concurrent-start (trapezoid) plan of
    the 2D radius-1 stencil, from the definition of a legal tiled execution.

    `tiles`: rows (lo_y, hi_y, slo_y, shi_y, fo_y, lo_x, hi_x, slo_x, shi_x,
    fo_x, t0, nt) in queue order; level l of a tile computes time step t0 + l
    over [lo + slo*l, hi + shi*l) per axis, cut to the interior.  `edges`:
    (predecessor, successor) pairs.  Checks, over every point of the
    iteration space: each interior point of each step is computed by exactly
    one tile; every edge goes forward in the queue; every input of a point
    (the point itself and its four neighbours one step earlier, interior
    only: boundary cells never change) is computed by the same tile or by a
    transitive predecessor; and each tile's inputs lie inside its register
    footprint [fo, fo + F).  Returns a list of problems (empty when legal).
    """
    ny, nx = dims
    problems = []
    owner = np.full((T, ny, nx), -1, dtype=np.int64)
    for i, t in enumerate(tiles):
        lo_y, hi_y, slo_y, shi_y, fo_y, lo_x, hi_x, slo_x, shi_x, fo_x, t0, nt = (int(v) for v in t)
        for l in range(nt):
            ya, yb = max(lo_y + slo_y * l, 1), min(hi_y + shi_y * l, ny - 1)
            xa, xb = max(lo_x + slo_x * l, 1), min(hi_x + shi_x * l, nx - 1)
            if ya >= yb or xa >= xb:
                continue
            if ya - 1 < fo_y or yb + 1 > fo_y + footprint[0] or xa - 1 < fo_x or xb + 1 > fo_x + footprint[1]:
                problems.append(("footprint", i, l))
            blk = owner[t0 + l, ya:yb, xa:xb]
            if (blk >= 0).any():
                problems.append(("overlap", i, l))
            blk[...] = i
    if (owner[:, 1:ny - 1, 1:nx - 1] < 0).any():
        problems.append(("uncovered", int((owner[:, 1:ny - 1, 1:nx - 1] < 0).sum())))
        return problems
    n = len(tiles)
    preds = [[] for _ in range(n)]
    for a, b in edges:
        if not a < b:
            problems.append(("edge order", int(a), int(b)))
        preds[int(b)].append(int(a))
    reach = [0] * n  # bitset of transitive predecessors (queue order is topological)
    for i in range(n):
        r = 0
        for a in preds[i]:
            r |= reach[a] | (1 << a)
        reach[i] = r
    sink = owner[1:, 1:ny - 1, 1:nx - 1]
    pairs = set()
    for dy, dx in ((0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)):
        src = owner[:-1, 1 + dy:ny - 1 + dy, 1 + dx:nx - 1 + dx]
        # boundary cells (never computed) carry -1 and need no producer
        m = (src >= 0) & (src != sink)
        if m.any():
            pairs.update(zip(src[m].tolist(), sink[m].tolist()))
    for a, b in pairs:
        if not (reach[b] >> a) & 1:
            problems.append(("dependence", a, b))
    return problems


# ------------------------------------------------------------ cost model ---
# 8 features -> 64 ReLU -> 64 ReLU -> 1 (log time), mean squared error,
# Adam(beta1, beta2, eps).  float64 throughout.

MLP_SHAPES = [("W1", (64, 8)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
              ("W3", (1, 64)), ("b3", (1,))]


def mlp_forward(params, X):
    W1, b1, W2, b2, W3, b3 = [np.asarray(params[k], dtype=np.float64) for k, _ in MLP_SHAPES]
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    yhat = (h2 @ W3.T + b3)[:, 0]
    return yhat, (X, z1, h1, z2, h2)


def mlp_loss(params, X, y):
    yhat, _ = mlp_forward(params, X)
    r = yhat - np.asarray(y, dtype=np.float64)
    return float(np.mean(r * r))


def mlp_backward(params, X, y):
    """Gradients of the mean squared error with respect to every parameter."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(params[k], dtype=np.float64) for k, _ in MLP_SHAPES]
    yhat, (X, z1, h1, z2, h2) = mlp_forward(params, X)
    n = X.shape[0]
    g_y = 2.0 * (yhat - np.asarray(y, dtype=np.float64)) / n        # dL/dyhat
    g = {}
    g["W3"] = g_y[None, :] @ h2                                     # (1, 64)
    g["b3"] = np.array([g_y.sum()])
    g_h2 = g_y[:, None] @ W3                                        # (n, 64)
    g_z2 = g_h2 * (z2 > 0.0)
    g["W2"] = g_z2.T @ h1
    g["b2"] = g_z2.sum(axis=0)
    g_h1 = g_z2 @ W2
    g_z1 = g_h1 * (z1 > 0.0)
    g["W1"] = g_z1.T @ X
    g["b1"] = g_z1.sum(axis=0)
    return g


def adam_step(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015) with bias correction; step counts from 1."""
    newp, newm, newv = {}, {}, {}
    for k, _ in MLP_SHAPES:
        g = np.asarray(grads[k], dtype=np.float64)
        mk = beta1 * np.asarray(m[k], dtype=np.float64) + (1.0 - beta1) * g
        vk = beta2 * np.asarray(v[k], dtype=np.float64) + (1.0 - beta2) * g * g
        mhat = mk / (1.0 - beta1 ** step)
        vhat = vk / (1.0 - beta2 ** step)
        newp[k] = np.asarray(params[k], dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
        newm[k], newv[k] = mk, vk
    return newp, newm, newv

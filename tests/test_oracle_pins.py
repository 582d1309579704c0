"""Pins of the oracle against facts fixed by the mathematics, not by the oracle itself.

Each test is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign or index, a transposed operand, a different summation order, a
wrong rounding mode, a wrong time parity) fails at least one of them:

* Fourier modes of the discrete operators (closed-form decay factors), on
  non-square grids with different modes per axis;
* constant fields stay exactly constant; zero stays zero;
* restart: T1 steps then T2 steps equal T1+T2 steps bit for bit;
* hand-derived order- and rounding-sensitive single steps (tests/golden);
* the DP against explicit enumeration of every bracketing, closed forms for
  N = 1, 2, 3, uniform dimensions and exact cubic scaling;
* the plan enumerations against hand-enumerated leaves and a brute-force
  coverage and dependence check;
* the cost model against finite differences and closed forms.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
EPS64 = 2.0 ** -53
EPS32 = 2.0 ** -24


def _mode(shape, modes):
    """prod_k sin(pi m_k i_k / (n_k - 1)), boundary exactly 0."""
    a = np.ones(shape)
    for ax, (n, m) in enumerate(zip(shape, modes)):
        v = np.sin(m * math.pi * np.arange(n) / (n - 1))
        v[0] = 0.0
        v[-1] = 0.0
        sh = [1] * len(shape)
        sh[ax] = n
        a = a * v.reshape(sh)
    return a


def _lam(kind, shape, modes):
    c = [math.cos(math.pi * m / (n - 1)) for n, m in zip(shape, modes)]
    if kind == "jacobi1d":
        return (1.0 + 2.0 * c[0]) / 3.0
    if kind == "jacobi2d":
        return (1.0 + 2.0 * c[0] + 2.0 * c[1]) / 5.0
    if kind == "heat3d":
        return 1.0 - 0.25 * sum(1.0 - ci for ci in c)
    raise ValueError(kind)


@pytest.mark.parametrize("kind,shape,modes,T", [
    ("jacobi1d", (65,), (1,), 300),
    ("jacobi1d", (65,), (63,), 41),          # negative decay factor
    ("jacobi1d", (4096,), (3,), 1000),
    ("jacobi2d", (33, 21), (1, 2), 200),     # non-square, different modes per axis
    ("jacobi2d", (17, 40), (15, 1), 60),
    ("heat3d", (11, 9, 14), (1, 2, 3), 50),
    ("heat3d", (12, 10, 8), (10, 1, 6), 30),
])
def test_fourier_mode_decay_f64(kind, shape, modes, T):
    phi = _mode(shape, modes)
    lam = _lam(kind, shape, modes)
    got = oracle.stencil(kind, "f64", phi, T)
    want = (lam ** T) * phi
    tol = 8 * T * EPS64 * np.abs(phi).max() + 1e-300
    assert np.abs(got - want).max() <= tol, (np.abs(got - want).max(), tol, lam)


@pytest.mark.parametrize("kind,shape,modes,T", [
    ("jacobi1d", (33,), (2,), 40),
    ("jacobi2d", (19, 23), (2, 1), 40),
    ("heat3d", (9, 10, 11), (1, 1, 2), 20),
])
def test_fourier_mode_decay_f32(kind, shape, modes, T):
    phi = _mode(shape, modes).astype(np.float32)
    lam = _lam(kind, shape, modes)
    got = oracle.stencil(kind, "f32", phi, T).astype(np.float64)
    want = (lam ** T) * phi.astype(np.float64)
    tol = 8 * T * EPS32 * np.abs(phi).max()
    assert np.abs(got - want).max() <= tol


def test_fourier_mode_with_noise_is_a_contraction():
    """With noise of amplitude a, ||u_T - lam^T phi||_inf <= a (+ rounding): the
    Jacobi-2D operator has non-negative weights summing to one."""
    u0 = synth.jacobi2d_input(40, 36, noise=1e-3)
    phi = synth.jacobi2d_input(40, 36, noise=0.0)
    lam = _lam("jacobi2d", (40, 36), (1, 1))
    got = oracle.stencil("jacobi2d", "f64", u0, 30)
    assert np.abs(got - lam ** 30 * phi).max() <= 1e-3 + 1e-13


@pytest.mark.parametrize("c", [1.0, 0.5, float(np.float32(0.1)), 0.0, -3.25])
@pytest.mark.parametrize("kind,shape", [("jacobi1d", (37,)), ("jacobi2d", (13, 17)), ("heat3d", (7, 8, 9))])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_constant_field_is_fixed(kind, shape, c, dtype):
    a = np.full(shape, c, dtype=np.float64 if dtype == "f64" else np.float32)
    got = oracle.stencil(kind, dtype, a, 25)
    assert np.array_equal(got, a)


def test_constant_field_heat3d_any_double():
    rng = np.random.default_rng(5)
    for c in rng.uniform(-10, 10, size=20):
        a = np.full((5, 6, 7), c)
        assert np.array_equal(oracle.stencil("heat3d", "f64", a, 4), a)


@pytest.mark.parametrize("kind,shape", [("jacobi1d", (37,)), ("jacobi2d", (13, 17)), ("heat3d", (7, 8, 9))])
def test_constant_field_bf16(kind, shape):
    for c in [1.0, 0.5, 0.1015625, 3.0]:
        h = synth.to_bf16_bits(np.full(shape, c, dtype=np.float32))
        got = oracle.stencil(kind, "bf16", h, 9)
        assert np.array_equal(got, h)


@pytest.mark.parametrize("kind,shape", [("jacobi1d", (50,)), ("jacobi2d", (20, 31)), ("heat3d", (9, 11, 10))])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_restart_is_bit_exact(kind, shape, dtype):
    u = synth.uniform_field(shape, synth.STREAM_TESTS, np.float32 if dtype != "f64" else np.float64)
    if dtype == "bf16":
        u = synth.to_bf16_bits(u)
    a = oracle.stencil(kind, dtype, u, 7)
    b = oracle.stencil(kind, dtype, a, 6)
    c = oracle.stencil(kind, dtype, u, 13)
    assert np.array_equal(b, c)
    # a different step count must differ (guards against a no-op oracle)
    assert not np.array_equal(a, c)


def test_zero_steps_is_identity_and_zero_stays_zero():
    u = synth.uniform_field((10, 12), synth.STREAM_TESTS)
    assert np.array_equal(oracle.stencil("jacobi2d", "f64", u, 0), u)
    z = np.zeros((6, 7, 8))
    assert np.array_equal(oracle.stencil("heat3d", "f64", z, 5), z)


def test_boundary_cells_never_change():
    u = synth.uniform_field((15, 16), synth.STREAM_TESTS, zero_boundary=False)
    got = oracle.stencil("jacobi2d", "f64", u, 9)
    m = np.ones_like(u, dtype=bool)
    m[1:-1, 1:-1] = False
    assert np.array_equal(got[m], u[m])
    assert not np.array_equal(got[~m], u[~m])


def _golden_cases():
    with open(os.path.join(GOLD, "order_pins.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c["name"])
def test_hand_derived_order_and_rounding(case):
    shape = tuple(case["shape"])
    a = np.zeros(shape)
    for k, v in case["cells"].items():
        a[tuple(int(s) for s in k.split(","))] = v
    dt = case["dtype"]
    if dt == "f64":
        u = a
    elif dt == "f32":
        u = a.astype(np.float32)
    else:
        u = synth.to_bf16_bits(a.astype(np.float32))
    out = oracle.stencil(case["kind"], dt, u, 1)
    if dt == "bf16":
        out = synth.from_bf16_bits(out)
    got = float(out[tuple(case["point"])])
    assert got == case["expected"], (got, case["expected"])
    assert got != case["wrong_order"]


def test_bf16_storage_roundtrip_and_rounding():
    f = np.array([1.0, 1.00390625, 1.01171875, -2.5, 3.0e38, 1e-40], dtype=np.float32)
    h = synth.to_bf16_bits(f)
    back = synth.from_bf16_bits(h)
    assert back[0] == 1.0 and back[1] == 1.0 and back[2] == 1.015625 and back[3] == -2.5
    assert np.array_equal(synth.to_bf16_bits(back), h)


def test_point_evaluation_matches_full_oracle():
    u0 = synth.jacobi2d_input(48, 40)
    full = oracle.stencil("jacobi2d", "f64", u0, 17)
    for (y, x) in [(1, 1), (24, 20), (46, 38), (5, 33), (30, 2)]:
        assert oracle.jacobi2d_point(u0, 17, y, x) == full[y, x]


def test_threaded_oracle_is_bit_identical():
    u0 = synth.jacobi2d_input(64, 70)
    a = oracle.stencil("jacobi2d", "f64", u0, 11, threads=1)
    b = oracle.stencil("jacobi2d", "f64", u0, 11, threads=4)
    assert np.array_equal(a, b)
    p = synth.chain_dims(60)
    assert np.array_equal(oracle.matrix_chain(p, threads=1), oracle.matrix_chain(p, threads=4))


# -------------------------------------------------------------------- DP ---

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8])
def test_chain_vs_enumeration_of_all_bracketings(n):
    for seed in range(4):
        p = synth.randint(synth.test_rng(100 * n + seed), n + 1, 1, 30)
        C = oracle.matrix_chain(p)
        assert C[0, n - 1] == oracle.chain_brute(p)
        # every sub-chain too
        for i in range(n):
            for j in range(i, n):
                assert C[i, j] == oracle.chain_brute(p[i:j + 2])


def test_chain_brute_n10():
    p = synth.randint(synth.test_rng(999), 11, 1, 100)
    assert oracle.matrix_chain(p)[0, 9] == oracle.chain_brute(p)


def test_chain_closed_forms():
    assert oracle.matrix_chain(np.array([7, 9]))[0, 0] == 0
    assert oracle.matrix_chain(np.array([2, 3, 4]))[0, 1] == 2 * 3 * 4
    p0, p1, p2, p3 = 10, 30, 5, 60
    want = min(p0 * p1 * p2 + p0 * p2 * p3, p1 * p2 * p3 + p0 * p1 * p3)
    assert oracle.matrix_chain(np.array([p0, p1, p2, p3]))[0, 2] == want == 4500


def test_chain_uniform_dims_and_split_tiebreak():
    c, n = 7, 50
    C, S = oracle.matrix_chain(np.full(n + 1, c), want_split=True)
    i, j = np.triu_indices(n)
    assert np.array_equal(C[i, j], (j - i) * c ** 3)
    # all k tie; the smallest k (1-based k = i+1) is reported
    off = j > i
    assert np.array_equal(S[i[off], j[off]], i[off] + 1)


def test_chain_uniform_100_at_u32_edge():
    n = 4096
    # C[0][n-1] = (n-1)*100^3 = 4.095e9, just under 2^32; verify on a short prefix
    # with the closed form, and the exact bound formula.
    C = oracle.matrix_chain(np.full(65, 100))
    assert C[0, 63] == 63 * 100 ** 3
    assert (n - 1) * 100 ** 3 < 2 ** 32


def test_chain_cubic_scaling_and_bounds():
    p = synth.randint(synth.test_rng(7), 41, 1, 20)
    C = oracle.matrix_chain(p)
    C3 = oracle.matrix_chain(3 * p)
    assert np.array_equal(C3, 27 * C)
    i, j = np.triu_indices(40)
    pm = int(p.max())
    assert np.all(C[i, j] >= 0) and np.all(C[i, j] <= (j - i) * pm ** 3)


# ------------------------------------------------------------------ plans ---

def test_plan_enumerations_hand_example():
    with open(os.path.join(GOLD, "plan_1d_small.json")) as f:
        g = json.load(f)
    assert [list(k) for k in oracle.slt_leaves(g["dims"], g["T"], g["tile"])] == g["slt_lex"]
    assert [list(k) for k in oracle.cot_leaves(g["dims"], g["T"], g["tile"])] == g["cot_seq"]


def test_padding_is_minimal():
    for n in range(1, 200):
        for b in (1, 2, 3, 5, 16):
            e = oracle.padded_extent(n, b)
            k = int(round(math.log2(e // b)))
            assert e == b * 2 ** k and e >= n and (k == 0 or b * 2 ** (k - 1) < n)


@pytest.mark.parametrize("dims,T,tile", [
    ((10,), 7, (3, 4)),
    ((12, 9), 5, (2, 3, 4)),
    ((9, 8), 6, (4, 2, 2)),
    ((6, 7, 5), 3, (2, 2, 3, 2)),
])
def test_plan_enumerations_are_legal_and_complete(dims, T, tile):
    for order in (oracle.slt_leaves(dims, T, tile), oracle.slt_leaves(dims, T, tile, wavefront=True),
                  oracle.cot_leaves(dims, T, tile), oracle.cot_leaves(dims, T, tile, parallel_groups=True)):
        assert oracle.check_plan(order, dims, T, tile) == []
    assert sorted(oracle.slt_leaves(dims, T, tile)) == sorted(oracle.cot_leaves(dims, T, tile))


def test_plan_checker_catches_bad_orders():
    dims, T, tile = (12, 9), 5, (2, 3, 4)
    good = oracle.slt_leaves(dims, T, tile)
    assert oracle.check_plan(list(reversed(good)), dims, T, tile) != []
    assert oracle.check_plan(good[:-1], dims, T, tile) != []
    assert oracle.check_plan(good + [good[0]], dims, T, tile) != []


def test_cot_order_differs_from_lex_when_box_is_deep():
    dims, T, tile = (18, 18), 8, (2, 4, 4)
    a = oracle.slt_leaves(dims, T, tile)
    b = oracle.cot_leaves(dims, T, tile)
    assert sorted(a) == sorted(b) and a != b


# ------------------------------------------------------------- cost model ---

def _rand_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return {k: rng.uniform(-scale, scale, size=s) for k, s in oracle.MLP_SHAPES}


def test_mlp_gradients_vs_central_differences():
    rng = np.random.default_rng(11)
    P = _rand_params(3)
    X = rng.normal(size=(17, 8))
    y = rng.normal(size=17)
    g = oracle.mlp_backward(P, X, y)
    h = 1e-6
    for k, shape in oracle.MLP_SHAPES:
        flat = P[k].reshape(-1)
        idxs = rng.choice(flat.size, size=min(flat.size, 12), replace=False)
        for i in idxs:
            Pp = {kk: vv.copy() for kk, vv in P.items()}
            Pm = {kk: vv.copy() for kk, vv in P.items()}
            Pp[k].reshape(-1)[i] += h
            Pm[k].reshape(-1)[i] -= h
            fd = (oracle.mlp_loss(Pp, X, y) - oracle.mlp_loss(Pm, X, y)) / (2 * h)
            an = g[k].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (k, i, fd, an)


def test_mlp_zero_weights_closed_form():
    P = {k: np.zeros(s) for k, s in oracle.MLP_SHAPES}
    P["b3"] = np.array([0.75])
    X = np.random.default_rng(1).normal(size=(9, 8))
    y = np.linspace(-1, 2, 9)
    yhat, _ = oracle.mlp_forward(P, X)
    assert np.all(yhat == 0.75)
    g = oracle.mlp_backward(P, X, y)
    assert abs(g["b3"][0] - 2.0 * np.mean(0.75 - y)) < 1e-15
    for k in ("W1", "b1", "W2", "b2", "W3"):
        assert np.all(g[k] == 0.0)


def test_adam_first_step_closed_form():
    P = _rand_params(4)
    G = _rand_params(5, scale=2.0)
    zeros = {k: np.zeros(s) for k, s in oracle.MLP_SHAPES}
    newp, m, v = oracle.adam_step(P, G, zeros, zeros, 1, lr=1e-2, eps=1e-8)
    for k, _ in oracle.MLP_SHAPES:
        # bias-corrected moments equal g and g^2 after one step
        want = P[k] - 1e-2 * G[k] / (np.abs(G[k]) + 1e-8)
        assert np.allclose(newp[k], want, rtol=0, atol=1e-12)
        assert np.allclose(m[k], 0.1 * G[k]) and np.allclose(v[k], 0.001 * G[k] ** 2)


# Hand-enumerated 2D orders (tests/golden/cot_order_2d.json): a problem in
# which the recursive order differs from the lexicographic one, the parallel
# grouping differs from the sequential one, and both wrong bit orders (and a
# concatenating merge) give other sequences, so each of those mistakes in the
# oracle fails here.
def _cot2d():
    with open(os.path.join(GOLD, "cot_order_2d.json")) as f:
        return json.load(f)


def test_cot_order_2d_hand_enumeration():
    g = _cot2d()
    pr = g["problem"]
    dims, T, tile = tuple(pr["dims"]), pr["T"], tuple(pr["tile"])
    got = {
        "slt_lex": oracle.slt_leaves(dims, T, tile),
        "slt_wave": oracle.slt_leaves(dims, T, tile, wavefront=True),
        "cot_seq": oracle.cot_leaves(dims, T, tile),
        "cot_par": oracle.cot_leaves(dims, T, tile, parallel_groups=True),
    }
    for name, order in got.items():
        assert [list(k) for k in order] == g[name], name
        assert oracle.check_plan(order, dims, T, tile) == [], name


def test_cot_order_2d_golden_discriminates():
    g = _cot2d()
    seqs = [g["slt_lex"], g["slt_wave"], g["cot_seq"], g["cot_par"]]
    assert len({json.dumps(s) for s in seqs}) == 4
    for name, w in g["wrong"].items():
        assert sorted(map(tuple, w)) == sorted(map(tuple, g["cot_seq"])), name
        if name.startswith("cot_seq"):
            assert w != g["cot_seq"], name
        else:
            assert w != g["cot_par"], name
    # the wrong orders are still legal visiting orders: only the golden tells them apart
    pr = g["problem"]
    for name, w in g["wrong"].items():
        assert oracle.check_plan([tuple(k) for k in w], tuple(pr["dims"]), pr["T"], tuple(pr["tile"])) == [], name


def _mlp_golden_params(g):
    P = {k: np.zeros(s) for k, s in oracle.MLP_SHAPES}
    for name in ("W1", "W2"):
        for key, v in g[name].items():
            i, j = (int(t) for t in key.split(","))
            P[name][i, j] = v
    for name in ("b1", "b2"):
        for key, v in g[name].items():
            P[name][int(key)] = v
    for key, v in g["W3"].items():
        P["W3"][0, int(key)] = v
    P["b3"][0] = g["b3"]
    return P


def test_mlp_forward_hand_computed_value():
    with open(os.path.join(GOLD, "mlp_forward.json")) as f:
        g = json.load(f)
    P = _mlp_golden_params(g)
    yhat, _ = oracle.mlp_forward(P, np.array(g["X"], dtype=np.float64))
    assert list(yhat) == g["expected"]
    for name, w in g["wrong"].items():
        assert w != g["expected"], name


# ------------------------------------------------------- Gauss-Seidel-2D ---
def _gs_single_assignment(u0, T):
    """Time-expanded form: v[t][i][j] from v[t-1] (c, s, e) and v[t] (n, w),
    one array per step, no in-place update (pure Python, small sizes)."""
    ny, nx = u0.shape
    v = [u0.astype(np.float64).copy()]
    for t in range(1, T + 1):
        cur = v[t - 1].copy()
        for i in range(1, ny - 1):
            for j in range(1, nx - 1):
                c, n = v[t - 1][i, j], cur[i - 1, j]
                s, e, w = v[t - 1][i + 1, j], v[t - 1][i, j + 1], cur[i, j - 1]
                cur[i, j] = 0.2 * ((((c + n) + s) + e) + w)
        v.append(cur)
    return v[T]


def test_gs2d_equals_single_assignment_form():
    rng = np.random.default_rng(5)
    u0 = rng.random((7, 9))
    assert np.array_equal(oracle.gs2d(u0, 3), _gs_single_assignment(u0, 3))


def test_gs2d_linear_integer_field_is_fixed():
    """A linear field (boundary included) is discrete-harmonic: n + s = e + w
    = 2c, so 0.2 * 5c = c exactly for integer c; a wrong neighbour breaks it."""
    i, j = np.mgrid[0:9, 0:11]
    u0 = (3 + 2 * i + 5 * j).astype(np.float64)
    assert np.array_equal(oracle.gs2d(u0, 6), u0)


def test_gs2d_one_interior_point_is_jacobi():
    rng = np.random.default_rng(6)
    u0 = rng.random((3, 3))
    assert np.array_equal(oracle.gs2d(u0, 4), oracle.stencil("jacobi2d", "f64", u0, 4))


def test_gs2d_one_sweep_exact_rationals():
    """One sweep on a 4x5 grid in exact rational arithmetic (lexicographic,
    new north and west values): the oracle is within rounding of it, and it
    is not the Jacobi result."""
    from fractions import Fraction as Fr
    vals = [[0, 1, 2, 3, 4], [5, 7, 11, 13, 6], [8, 17, 19, 23, 9], [10, 12, 14, 15, 16]]
    u = [[Fr(v) for v in row] for row in vals]
    for i in range(1, 3):
        for j in range(1, 4):
            u[i][j] = Fr(1, 5) * (u[i][j] + u[i - 1][j] + u[i + 1][j] + u[i][j + 1] + u[i][j - 1])
    got = oracle.gs2d(np.array(vals, dtype=np.float64), 1)
    exact = np.array([[float(v) for v in row] for row in u])
    assert np.allclose(got, exact, rtol=4e-16, atol=0)
    jac = oracle.stencil("jacobi2d", "f64", np.array(vals, dtype=np.float64), 1)
    assert not np.allclose(got[1:3, 1:4], jac[1:3, 1:4])


def test_gs2d_restart():
    rng = np.random.default_rng(7)
    u0 = rng.random((12, 17))
    assert np.array_equal(oracle.gs2d(oracle.gs2d(u0, 3), 4), oracle.gs2d(u0, 7))


# --------------------------------------------------------------- FDTD-2D ---
def _fdtd_single_assignment(ex, ey, hz, T):
    """Time-expanded Yee update: E^t from E^{t-1} and H^{t-1}, then H^t from
    H^{t-1} and E^t (pure Python loops, one array per field and step)."""
    ny, nx = hz.shape
    E1, E2, H = [ex.copy()], [ey.copy()], [hz.copy()]
    for t in range(1, T + 1):
        a, b, h = E1[-1].copy(), E2[-1].copy(), H[-1].copy()
        for i in range(1, ny):
            for j in range(nx):
                b[i, j] = E2[-1][i, j] - 0.25 * (H[-1][i, j] - H[-1][i - 1, j])
        for i in range(ny):
            for j in range(1, nx):
                a[i, j] = E1[-1][i, j] + 0.25 * (H[-1][i, j] - H[-1][i, j - 1])
        for i in range(ny - 1):
            for j in range(nx - 1):
                h[i, j] = H[-1][i, j] - 0.5 * ((b[i + 1, j] - b[i, j]) - (a[i, j + 1] - a[i, j]))
        E1.append(a)
        E2.append(b)
        H.append(h)
    return E1[-1], E2[-1], H[-1]


def test_fdtd2d_impulse_golden():
    with open(os.path.join(os.path.dirname(__file__), "golden", "fdtd_impulse.json")) as f:
        g = json.load(f)
    shape = tuple(g["shape"])
    hz = np.zeros(shape)
    hz[tuple(g["impulse"])] = 1.0
    ex, ey, h = oracle.fdtd2d(np.zeros(shape), np.zeros(shape), hz, 1)
    for name, arr in (("hz", h), ("ey", ey), ("ex", ex)):
        want = np.zeros(shape)
        for i, j, v in g[name]:
            want[i, j] = v
        assert np.array_equal(arr, want), name


def test_fdtd2d_equals_single_assignment_form():
    rng = np.random.default_rng(8)
    f = [rng.random((6, 8)) - 0.5 for _ in range(3)]
    got = oracle.fdtd2d(*f, 3)
    want = _fdtd_single_assignment(*f, 3)
    for g_, w_ in zip(got, want):
        assert np.array_equal(g_, w_)


def test_fdtd2d_constant_fields_and_restart():
    c = [np.full((9, 10), v) for v in (0.75, -1.5, 3.0)]
    for g_, w_ in zip(oracle.fdtd2d(*c, 5), c):
        assert np.array_equal(g_, w_)
    rng = np.random.default_rng(9)
    f = [rng.random((13, 11)) for _ in range(3)]
    a = oracle.fdtd2d(*oracle.fdtd2d(*f, 2), 3)
    b = oracle.fdtd2d(*f, 5)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


# ------------------------------------- motivating example (appendix, Fig. motiv) ---
def _motiv_single_assignment(a, T):
    """Full expansion: one array per time step (no reuse of memory), S1 on
    the interior from step t-1, S2 / S3 on the two boundaries."""
    N = len(a)
    X = [np.array(a, dtype=np.float64)]
    for t in range(1, T + 1):
        p = X[-1]
        cur = np.empty(N)
        for i in range(1, N - 1):
            cur[i] = 0.25 * (((p[i - 1] + p[i]) + p[i + 1]) + p[0])
        cur[0] = 0.5 * p[0] + 0.25
        cur[N - 1] = 0.5 * p[N - 1] + 0.25
        X.append(cur)
    return X[T]


def test_motiv_equals_single_assignment_form():
    a = np.random.default_rng(11).random(23)
    assert np.array_equal(oracle.motiv(a, 46), _motiv_single_assignment(a, 46))


def test_motiv_fixed_point_and_boundary_closed_form():
    assert np.array_equal(oracle.motiv(np.full(17, 0.5), 34), np.full(17, 0.5))
    a = np.zeros(9)
    for T in (1, 2, 5, 30):
        out = oracle.motiv(a, T)
        assert out[0] == out[-1] == 0.5 - 0.5 * 2.0 ** -T      # g(y) = y/2 + 1/4 from 0, exact


@pytest.mark.parametrize("bt,bx", [(1, 4), (4, 8), (8, 16), (16, 5), (50, 100)])
def test_motiv_tiled_order_needs_the_auxiliary_arrays(bt, bx):
    """Tiles of the skewed space in band / left-to-right order give the
    program's result when S2 and S3 write single-assignment arrays (the
    appendix's split); with the original allocation the same order breaks the
    memory-based dependences whenever a band holds more than one level and a
    level more than one tile."""
    a = np.random.default_rng(12).random(31)
    T = 62
    want = oracle.motiv(a, T)
    assert np.array_equal(oracle.motiv_tiled_order(a, T, bt, bx, aux=True), want)
    if bt > 1 and bx + bt < len(a):
        assert not np.array_equal(oracle.motiv_tiled_order(a, T, bt, bx, aux=False), want)

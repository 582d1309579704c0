"""The cost model's network on the device against the binary64 CPU oracle:
forward, loss gradient, one Adam step, and training that learns."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def to_dict(flat):
    d, o = {}, 0
    for k, shp in oracle.MLP_SHAPES:
        n = int(np.prod(shp))
        d[k] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    assert o == 4801
    return d


def to_flat(d):
    return np.concatenate([np.asarray(d[k], dtype=np.float64).ravel() for k, _ in oracle.MLP_SHAPES])


def he_params(seed):
    rng = np.random.default_rng(seed)
    p = np.zeros(4801, dtype=np.float32)
    p[0:512] = rng.uniform(-1, 1, 512) * np.sqrt(6 / 8)
    p[512:576] = rng.uniform(-0.1, 0.1, 64)
    p[576:4672] = rng.uniform(-1, 1, 4096) * np.sqrt(6 / 64)
    p[4672:4736] = rng.uniform(-0.1, 0.1, 64)
    p[4736:4800] = rng.uniform(-1, 1, 64) * np.sqrt(6 / 64)
    p[4800] = 0.3
    return p


def batch(seed, n):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 8)).astype(np.float32)
    y = (np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2] - 0.3 * X[:, 7]).astype(np.float32)
    return X, y


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("n", [1, 37, 256, 1000])
def test_forward_matches_oracle(gpu, n):
    from paper_1802_00166_amd import tune
    p = he_params(1)
    X, _ = batch(2, n)
    got = tune.mlp_forward(p, X)
    want, _ = oracle.mlp_forward(to_dict(p), X)
    assert rel(got, want) <= 1e-5


@pytest.mark.parametrize("n", [1, 64, 200, 256])
def test_gradient_matches_oracle_per_tensor(gpu, n):
    from paper_1802_00166_amd import tune
    p = he_params(3)
    X, y = batch(4, n)
    loss, g = tune.mlp_grad(p, X, y)
    want = oracle.mlp_backward(to_dict(p), X, y)
    assert abs(loss - oracle.mlp_loss(to_dict(p), X, y)) <= 1e-5 * abs(oracle.mlp_loss(to_dict(p), X, y))
    gd = to_dict(g)
    for k, _ in oracle.MLP_SHAPES:
        assert rel(gd[k], want[k]) <= 1e-5, k


def test_gradient_closed_form_at_zero_weights(gpu):
    """All weights zero: yhat = b3 everywhere, so dL/db3 = 2 mean(b3 - y) and
    every other gradient is 0 (ReLU of 0 passes nothing back)."""
    from paper_1802_00166_amd import tune
    p = np.zeros(4801, dtype=np.float32)
    p[4800] = 0.75
    X, y = batch(5, 128)
    loss, g = tune.mlp_grad(p, X, y)
    assert np.all(g[:4800] == 0)
    assert g[4800] == pytest.approx(2 * np.mean(0.75 - y.astype(np.float64)), rel=1e-6)
    assert loss == pytest.approx(np.mean((0.75 - y.astype(np.float64)) ** 2), rel=1e-6)


def test_one_adam_step_matches_oracle(gpu):
    from paper_1802_00166_amd import tune
    p = he_params(6)
    X, y = batch(7, 96)
    order = np.arange(96, dtype=np.int32)[None, :]
    z = np.zeros(4801, dtype=np.float32)
    p1, m1, v1, el = tune.mlp_train(p, z, z, X, y, order, batch=96, step0=0, lr=1e-3)
    g = oracle.mlp_backward(to_dict(p), X, y)
    zero = {k: np.zeros(s) for k, s in oracle.MLP_SHAPES}
    wp, wm, wv = oracle.adam_step(to_dict(p), g, zero, zero, 1, lr=1e-3)
    assert el[0] == pytest.approx(oracle.mlp_loss(to_dict(p), X, y), rel=1e-5)
    assert np.abs(p1 - to_flat(wp)).max() <= 1e-3 * 1e-3 + 1e-6
    assert rel(m1, to_flat(wm)) <= 1e-5
    assert rel(v1, to_flat(wv)) <= 1e-4


def test_two_steps_continue_the_step_count(gpu):
    """Two batches of one epoch equal two oracle Adam steps (t = 1, 2)."""
    from paper_1802_00166_amd import tune
    p = he_params(8)
    X, y = batch(9, 80)
    order = np.arange(80, dtype=np.int32)[None, :]
    z = np.zeros(4801, dtype=np.float32)
    p2, _, _, _ = tune.mlp_train(p, z, z, X, y, order, batch=40, lr=1e-3)
    d = to_dict(p)
    m = {k: np.zeros(s) for k, s in oracle.MLP_SHAPES}
    v = {k: np.zeros(s) for k, s in oracle.MLP_SHAPES}
    for t, rows in [(1, slice(0, 40)), (2, slice(40, 80))]:
        g = oracle.mlp_backward(d, X[rows], y[rows])
        d, m, v = oracle.adam_step(d, g, m, v, t, lr=1e-3)
    assert np.abs(p2 - to_flat(d)).max() <= 2e-6


def test_training_learns_a_smooth_target(gpu):
    from paper_1802_00166_amd import tune
    X, y = batch(10, 2048)
    rng = np.random.default_rng(11)
    order = np.stack([rng.permutation(2048) for _ in range(60)]).astype(np.int32)
    z = np.zeros(4801, dtype=np.float32)
    p, _, _, el = tune.mlp_train(he_params(12), z, z, X, y, order, batch=256, lr=1e-3)
    assert el[-1] < 0.1 * el[0]
    want, _ = oracle.mlp_forward(to_dict(p), X)
    assert np.mean((want - y) ** 2) < 0.1 * np.var(y)

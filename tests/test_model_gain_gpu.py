"""The stored cost model on held-out problems: its tile choices against the
exhaustive sweep and against one fixed tile for every shape (the method
without the model: the sweep best of the 4096^2 f64 problem), all timed here.
The model's own top-1 pick must be within 10% of the sweep's best as a
geometric mean, and beat the fixed tile.

Held-out problems: 16 instances of the uneven batch (their shapes come from
the batch's own seeded stream, which the training sweeps never used), the
4096^2 f64 headline problem and a Heat-3D problem (256 x 192 x 320, T = 48,
f32).
"""
import math

import pytest

import synth

pytestmark = pytest.mark.gpu

FIXED = ((16, 64, 256), "slt_wave")


def _compare(tune, model, prob, schedules):
    _, _, best_ms, recs = tune.sweep(prob, reps=5, warmup=1, schedules=schedules)
    # the model's own pick (top 1 of the predictions), re-timed beside the sweep
    _, _, pick_ms, _ = tune.tune(prob, tune.TUNE_MODEL_VERIFY, model, reps=5, warmup=1, topk=1,
                                 schedules=schedules)
    fixed_ms = {(tuple(r["tile"]), r["schedule"]): r["ms"] for r in recs}.get(FIXED)
    return best_ms, pick_ms, fixed_ms


def test_model_picks_within_ten_percent_of_sweep_and_beat_a_fixed_tile(gpu):
    from paper_1802_00166_amd import tune
    model = tune.load_default_model()
    if model is None:
        pytest.skip("no stored model (paper_1802_00166_amd/models/stencil.mlp)")
    probs = [("jacobi2d", "f32", (ny, nx), T) for ny, nx, T in synth.batched_instances(256)[3::16][:16]]
    probs.append(("jacobi2d", "f64", (4096, 4096), 512))
    # a Heat-3D problem held out of the training sweeps
    probs.append(("heat3d", "f32", (256, 192, 320), 48))
    ratios, gains = [], []
    for kind, dtype, shape, T in probs:
        prob = tune.problem(kind, dtype, shape, T)
        best_ms, pick_ms, fixed_ms = _compare(tune, model, prob, ["slt_wave"])
        ratios.append(pick_ms / best_ms)
        if fixed_ms is not None:
            gains.append(fixed_ms / pick_ms)
        print("%s %s T=%d: sweep %.3f ms, model %.3f ms (x%.3f), fixed %s ms"
              % (dtype, "x".join(map(str, shape)), T, best_ms, pick_ms, pick_ms / best_ms,
                 "%.3f" % fixed_ms if fixed_ms is not None else "n/a"))
    gm = math.exp(sum(math.log(r) for r in ratios) / len(ratios))
    gg = math.exp(sum(math.log(g) for g in gains) / len(gains))
    print("geomean model/sweep %.4f over %d problems (worst %.3f); geomean gain over the fixed tile %.4f"
          % (gm, len(ratios), max(ratios), gg))
    assert gm <= 1.10
    assert gg > 1.0


def test_chain_model_pick_within_ten_percent_of_sweep(gpu):
    """The interval-DP model at N = 4096, pmax = 100 (held out of its
    training sweeps): its pick, re-timed, within 10% of the exhaustive sweep."""
    from paper_1802_00166_amd import tune
    model = tune.load_default_model("chain")
    if model is None:
        pytest.skip("no stored model (paper_1802_00166_amd/models/chain.mlp)")
    prob = tune.problem("matrix_chain", "f64", (4096,), 100)
    two = ["slt_wave", "cot_par"]
    _, _, best_ms, _ = tune.sweep(prob, reps=5, warmup=1, schedules=two)
    _, _, pick_ms, _ = tune.tune(prob, tune.TUNE_MODEL_VERIFY, model, reps=5, warmup=1, topk=1, schedules=two)
    print("chain N=4096: sweep %.3f ms, model %.3f ms (x%.3f)" % (best_ms, pick_ms, pick_ms / best_ms))
    assert pick_ms <= 1.10 * best_ms

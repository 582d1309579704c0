"""Autotuner sweeps and the learned cost model on the GPU."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_sweep_best_is_the_fastest_record(gpu):
    from paper_1802_00166_amd import tune
    prob = tune.problem("jacobi2d", "f32", (300, 420), 48)
    tile, sched, ms, recs = tune.sweep(prob, reps=3, warmup=1, schedules=["slt_wave", "cot_par"])
    assert len(recs) == len(tune.candidates(prob, ["slt_wave", "cot_par"]))
    fastest = min(recs, key=lambda r: r["ms"])
    assert ms == pytest.approx(fastest["ms"]) and tuple(fastest["tile"]) == tile and fastest["schedule"] == sched
    for r in recs:
        assert np.allclose(r["feat"], tune.features(prob, r["tile"], r["schedule"]))


def test_dp_and_3d_sweeps(gpu):
    from paper_1802_00166_amd import tune
    tile, sched, ms, recs = tune.sweep(tune.problem("matrix_chain", "", (700,), 100), reps=2, warmup=1)
    assert len(recs) == 24 and ms == min(r["ms"] for r in recs) and tile[1] in (16, 32, 64)
    tile, sched, ms, recs = tune.sweep(tune.problem("heat3d", "f32", (40, 50, 70), 10), reps=2, warmup=1,
                                       schedules=["slt_wave"])
    assert len(recs) >= 10 and ms == min(r["ms"] for r in recs)


def test_model_modes_pick_from_the_grid(gpu):
    from paper_1802_00166_amd import tune
    prob = tune.problem("jacobi2d", "f32", (260, 300), 40)
    _, _, _, recs = tune.sweep(prob, reps=2, warmup=1, schedules=["slt_wave", "cot_par"])
    model = tune.Model.train(recs, epochs=200, batch=64, seed=3)
    assert model.final_loss < 0.5
    pred = model.predict_ms(recs)
    # ranks learnt on its own training shape: the predicted best is among the measured top quarter
    ms = np.array([r["ms"] for r in recs])
    best_pred = int(np.argmin(pred))
    assert (ms < ms[best_pred]).sum() <= len(recs) // 4
    tile, sched, pms = model.predict(prob, ["slt_wave", "cot_par"])
    assert (tile, sched) in tune.candidates(prob, ["slt_wave", "cot_par"])
    assert pms == pytest.approx(pred.min(), rel=1e-5)
    t2, s2, ms2, r2 = tune.tune(prob, tune.TUNE_MODEL_VERIFY, model, reps=2, warmup=1, topk=4,
                                schedules=["slt_wave", "cot_par"])
    assert len(r2) == 4 and ms2 == min(r["ms"] for r in r2)

"""Trains the stencil cost model from timed sweeps and evaluates it.

    python -m paper_1802_00166_amd.train_model --out DIR [--shapes 64]

1. Training set: timed sweeps (pcot_tune, every runnable tile of the grid,
   schedules SLT_WAVE and COT_PAR) of Jacobi-2D shapes drawn like the uneven
   batch (extents uniform in [128, 2048] per axis, T uniform in [32, 512],
   f32 and f64 alternating) and a few Jacobi-1D shapes, from a seed of their
   own so the evaluated problems stay held out.
2. The MLP is trained on the device (pcot_model_train) and saved.
3. Held-out evaluation: the 4096^2 f64 T = 512 Jacobi-2D problem (all four
   tiled schedules) and instances of the uneven batch.  For each, the
   model's pick (no timing) is re-timed and compared with the exhaustive
   sweep's best, and with one fixed tile (the sweep-best of the 4096^2
   problem applied to every shape: the method without the model).

Writes DIR/stencil.mlp, DIR/sweeps.json (best of every evaluated sweep) and
DIR/report.json; the training records go to DIR/records.jsonl.

    python -m paper_1802_00166_amd.train_model --out DIR --chain

trains the interval-DP model instead: sweeps (both schedules, every
supported (b, k-chunk)) of chains with N uniform in [256, 4096] and pmax in
{10, 100, 1000} (the 1000 ones take the 64-bit path), then evaluates held-out
chains, among them N = 4096 with pmax = 100.  Writes DIR/chain.mlp and
DIR/report_chain.json.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np


def log(*a):
    print(*a, flush=True)


def sample_shapes(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        ny, nx = (int(v) for v in rng.integers(128, 2049, size=2))
        T = int(rng.integers(32, 513))
        out.append(("jacobi2d", "f32" if i % 2 == 0 else "f64", (ny, nx), T))
    return out


# The headline problem's neighbourhood, kept out of the training sweeps: both
# extents within 1/8 of 4096 and T within 1/8 of 512.
def near_headline(ny, nx, T):
    return ny >= 3584 and nx >= 3584 and T >= 448


def sample_large(n, seed):
    """Large training shapes, so that 4096-class problems are interpolated
    rather than extrapolated; shapes near the 4096^2, T = 512 problem are
    redrawn, so its whole neighbourhood stays held out."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        ny, nx = (int(v) for v in rng.integers(2048, 4097, size=2))
        T = int(rng.integers(128, 513))
        if near_headline(ny, nx, T):
            continue
        out.append(("jacobi2d", "f64" if len(out) % 2 == 0 else "f32", (ny, nx), T))
    return out


def sample_heat3d(n, seed):
    """Heat-3D training shapes, extents in [64, 400] (the 512^3 benchmark
    problem and its neighbourhood stay out), T in [16, 128], the three
    storage types in turn."""
    rng = np.random.default_rng(seed)
    dts = ["f64", "f32", "bf16"]
    return [("heat3d", dts[i % 3], tuple(int(v) for v in rng.integers(64, 401, size=3)), int(rng.integers(16, 129)))
            for i in range(n)]


def batch_instances(count=256, seed_stream=4):
    """Shapes of the uneven batch, from the shared seeded generator when the
    repository's input module is present, else from numpy (documented)."""
    try:
        import synth
        return synth.batched_instances(count)
    except ImportError:
        rng = np.random.default_rng(1802 + seed_stream)
        return [(int(rng.integers(128, 2049)), int(rng.integers(128, 2049)), int(rng.integers(32, 513)))
                for _ in range(count)]


def chain_shapes(n, seed):
    rng = np.random.default_rng(seed)
    return [(int(rng.integers(256, 4097)), int(rng.choice([10, 100, 1000]))) for _ in range(n)]


def train_chain(args, tune):
    """Interval-DP cost model: training sweeps, device training, held-out picks."""
    two = ["slt_wave", "cot_par"]
    t_start = time.time()
    records = []
    for i, (N, pmax) in enumerate(chain_shapes(args.shapes, args.seed + 11)):
        t0 = time.time()
        tile, sched, ms, recs = tune.sweep(tune.problem("matrix_chain", "f64", (N,), pmax), reps=args.reps, warmup=1,
                                           schedules=two)
        records += recs
        log("chain sweep %d/%d N=%d pmax=%d: %d candidates, best %s %s %.3f ms (%.1f s)"
            % (i + 1, args.shapes, N, pmax, len(recs), tile, sched, ms, time.time() - t0))
    t0 = time.time()
    model = tune.Model.train(records, epochs=args.epochs, batch=64, lr=1e-3, seed=args.seed)
    train_s = time.time() - t0
    model.save(os.path.join(args.out, "chain.mlp"))
    pred = model.predict_ms(records)
    rmse = float(np.sqrt(np.mean((np.log(pred) - np.log([r["ms"] for r in records])) ** 2)))
    log("trained on %d records in %.2f s, train RMSE(ln ms) %.3f" % (len(records), train_s, rmse))
    evals, held_sq = [], []
    for N, pmax in [(4096, 100)] + chain_shapes(6, args.seed + 12):
        prob = tune.problem("matrix_chain", "f64", (N,), pmax)
        _, _, _, recs = tune.sweep(prob, reps=args.reps + 2, warmup=1, schedules=two)
        best = min(recs, key=lambda r: r["ms"])
        pr = model.predict_ms(recs)
        held_sq += [float(np.log(pv) - np.log(r["ms"])) ** 2 for pv, r in zip(pr, recs)]
        _, _, pick_ms, again = tune.tune(prob, tune.TUNE_MODEL_VERIFY, model, reps=args.reps + 2, warmup=1, topk=1,
                                         schedules=two)
        e = {"problem": "matrix_chain/N=%d/pmax=%d" % (N, pmax), "sweep_best": [best["tile"], best["schedule"],
             best["ms"]], "model_pick": [again[0]["tile"], again[0]["schedule"], pick_ms],
             "pick_over_best": pick_ms / best["ms"]}
        evals.append(e)
        log("eval %s: sweep %s %s %.3f ms | model %s %s %.3f ms (x%.3f)" %
            (e["problem"], best["tile"], best["schedule"], best["ms"], again[0]["tile"], again[0]["schedule"],
             pick_ms, pick_ms / best["ms"]))
    ratios = [e["pick_over_best"] for e in evals]
    rep = {"records": len(records), "train_shapes": args.shapes, "train_seconds": train_s, "train_rmse_ln_ms": rmse,
           "heldout_rmse_ln_ms": float(np.sqrt(np.mean(held_sq))), "heldout_candidates": len(held_sq),
           "geomean_pick_over_best": float(math.exp(np.mean(np.log(ratios)))), "max_pick_over_best": max(ratios),
           "evaluations": evals, "wall_seconds": time.time() - t_start}
    with open(os.path.join(args.out, "report_chain.json"), "w") as f:
        json.dump(rep, f, indent=1)
    log("chain model: geomean model/sweep %.4f (max %.4f), held-out RMSE(ln ms) %.3f" %
        (rep["geomean_pick_over_best"], rep["max_pick_over_best"], rep["heldout_rmse_ln_ms"]))
    return 0


def key_of(kind, dtype, shape, T):
    return "%s/%s/%s/%d" % (kind, dtype, "x".join(str(int(v)) for v in shape), int(T))


def main():
    from . import tune
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--shapes", type=int, default=64)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--eval-batch", type=int, default=16, help="held-out uneven-batch instances evaluated")
    ap.add_argument("--epochs", type=int, default=1500)
    ap.add_argument("--seed", type=int, default=77)
    ap.add_argument("--large-shapes", type=int, default=8,
                    help="extra training shapes with extents in [2048, 4096] (T in [128, 512])")
    ap.add_argument("--heat3d-shapes", type=int, default=9, help="Heat-3D training sweeps")
    ap.add_argument("--extra-records", default=None,
                    help="JSON-lines records of earlier training sweeps to train on as well")
    ap.add_argument("--skip-small", action="store_true",
                    help="do not sweep the --shapes set (use with --extra-records holding it)")
    ap.add_argument("--eval-only", metavar="MODEL", default=None,
                    help="skip the training sweeps and training; evaluate this saved model")
    ap.add_argument("--chain", action="store_true", help="train and evaluate the interval-DP model instead")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    if args.chain:
        return train_chain(args, tune)
    two = ["slt_wave", "cot_par"]
    t_start = time.time()

    if args.eval_only:
        model = tune.Model.load(args.eval_only)
        model.final_loss = None
        records, train, sweep_s, train_s, rmse = [], [], 0.0, 0.0, None
        return evaluate_all(args, tune, model, records, train, sweep_s, train_s, rmse, t_start)

    # ---- 1. training sweeps
    train = [] if args.skip_small else sample_shapes(args.shapes, args.seed)
    if not args.skip_small:
        train += [("jacobi1d", "f64", (n,), T) for n, T in [(1024, 256), (4096, 1000), (16384, 512), (65536, 256)]]
    train += sample_large(args.large_shapes, args.seed + 1)
    train += sample_heat3d(args.heat3d_shapes, args.seed + 2)
    records = []
    if args.extra_records:
        with open(args.extra_records) as f:
            records = [json.loads(l) for l in f if l.strip()]
        log("loaded %d earlier records" % len(records))
    sweep_s = 0.0
    with open(os.path.join(args.out, "records.jsonl"), "w") as rf:
        for r in records:
            rf.write(json.dumps(r) + "\n")
        for i, (kind, dtype, shape, T) in enumerate(train):
            t0 = time.time()
            tile, sched, ms, recs = tune.sweep(tune.problem(kind, dtype, shape, T), reps=args.reps, warmup=1,
                                               schedules=two)
            sweep_s += time.time() - t0
            for r in recs:
                r["problem"] = key_of(kind, dtype, shape, T)
                rf.write(json.dumps(r) + "\n")
            records += recs
            log("train sweep %d/%d %s: %d candidates, best %s %s %.3f ms (%.1f s)"
                % (i + 1, len(train), key_of(kind, dtype, shape, T), len(recs), tile, sched, ms, time.time() - t0))

    # ---- 2. device training
    t0 = time.time()
    model = tune.Model.train(records, epochs=args.epochs, batch=256, lr=1e-3, seed=args.seed)
    train_s = time.time() - t0
    path = os.path.join(args.out, "stencil.mlp")
    model.save(path)
    pred = model.predict_ms(records)
    ms = np.array([r["ms"] for r in records])
    rmse = float(np.sqrt(np.mean((np.log(pred) - np.log(ms)) ** 2)))
    log("trained on %d records in %.2f s: final loss %.4f, train RMSE(ln ms) %.3f" %
        (len(records), train_s, model.final_loss, rmse))
    return evaluate_all(args, tune, model, records, train, sweep_s, train_s, rmse, t_start)


# Heat-3D problems held out of the training sweeps
HELD_OUT_HEAT3D = [("heat3d", "f32", (256, 192, 320), 48), ("heat3d", "f64", (300, 300, 300), 60)]


def evaluate_all(args, tune, model, records, train, sweep_s, train_s, rmse, t_start):
    """Held-out evaluation: sweep, model pick re-timed, fixed tile."""
    two = ["slt_wave", "cot_par"]
    sweeps, evals = {}, []
    held_sq = []  # squared ln-time prediction errors over every timed held-out candidate of the model's schedules

    def evaluate(kind, dtype, shape, T, schedules, fixed):
        prob = tune.problem(kind, dtype, shape, T)
        t0 = time.time()
        recs = []
        for sch in (schedules or ["slt_lex", "slt_wave", "cot_seq", "cot_par"]):
            _, _, _, rs = tune.sweep(prob, reps=args.reps + 2, warmup=1, schedules=[sch])
            recs += rs
            log("  %s %s: %d candidates (%.1f s)" % (key_of(kind, dtype, shape, T), sch, len(rs), time.time() - t0))
        best = min(recs, key=lambda r: r["ms"])
        bt, bs, bms = tuple(best["tile"]), best["schedule"], best["ms"]
        sw_s = time.time() - t0
        mt, msch, pms = model.predict(prob, two)
        mine = [r for r in recs if r["schedule"] in two]
        if mine:
            pred = model.predict_ms(mine)
            held_sq.extend(float(np.log(pv) - np.log(r["ms"])) ** 2 for pv, r in zip(pred, mine))
        times = {(tuple(r["tile"]), r["schedule"]): r["ms"] for r in recs}
        # the pick and the fixed tile re-timed in one more session, beside the sweep's best
        t0 = time.time()
        _, _, _, again = tune.tune(prob, tune.TUNE_MODEL_VERIFY, model, reps=args.reps + 2, warmup=1, topk=1,
                                   schedules=two)
        pick_ms = again[0]["ms"]
        model_s = time.time() - t0
        fixed_ms = times.get((tuple(fixed[0]), fixed[1])) if fixed else None
        e = {"problem": key_of(kind, dtype, shape, T), "sweep_best": [list(bt), bs, bms],
             "model_pick": [list(mt), msch, pick_ms, pms], "pick_over_best": pick_ms / bms,
             "fixed": [list(fixed[0]), fixed[1], fixed_ms] if fixed else None,
             "gain_over_fixed": (fixed_ms / pick_ms) if fixed_ms else None,
             "sweep_s": sw_s, "model_s": model_s, "candidates": len(recs)}
        sweeps[e["problem"]] = {"best_tile": list(bt), "best_schedule": bs, "best_ms": bms}
        evals.append(e)
        log("eval %s: sweep %s %s %.3f ms | model %s %s %.3f ms (x%.3f) | fixed %s" %
            (e["problem"], bt, bs, bms, mt, msch, pick_ms, pick_ms / bms,
             ("%.3f ms" % fixed_ms) if fixed_ms else "-"))
        return bt, bs

    head = evaluate("jacobi2d", "f64", (4096, 4096), 512, None, None)
    fixed = (head[0], head[1])
    inst = batch_instances(256)
    step = max(1, len(inst) // max(1, args.eval_batch))
    for (ny, nx, T) in inst[::step][:args.eval_batch]:
        evaluate("jacobi2d", "f32", (ny, nx), T, two, fixed if fixed[1] in two else (fixed[0], "cot_par"))
    for kind, dtype, shape, T in HELD_OUT_HEAT3D:
        evaluate(kind, dtype, shape, T, two, None)

    ratios = [e["pick_over_best"] for e in evals]
    gains = [e["gain_over_fixed"] for e in evals if e["gain_over_fixed"]]
    rep = {
        "records": len(records), "train_shapes": len(train), "sweep_seconds": sweep_s, "train_seconds": train_s,
        "final_loss": getattr(model, "final_loss", None), "train_rmse_ln_ms": rmse,
        "heldout_rmse_ln_ms": float(np.sqrt(np.mean(held_sq))) if held_sq else None,
        "heldout_candidates": len(held_sq),
        "geomean_pick_over_best": float(math.exp(np.mean(np.log(ratios)))),
        "max_pick_over_best": float(max(ratios)),
        "geomean_gain_over_fixed": float(math.exp(np.mean(np.log(gains)))) if gains else None,
        "evaluations": evals, "wall_seconds": time.time() - t_start,
    }
    with open(os.path.join(args.out, "sweeps.json"), "w") as f:
        json.dump(sweeps, f, indent=1)
    with open(os.path.join(args.out, "report.json"), "w") as f:
        json.dump(rep, f, indent=1)
    log("geomean model/sweep %.4f (max %.4f), geomean gain over fixed tile %s, held-out RMSE(ln ms) %s" %
        (rep["geomean_pick_over_best"], rep["max_pick_over_best"], rep["geomean_gain_over_fixed"],
         rep["heldout_rmse_ln_ms"]))
    return 0


if __name__ == "__main__":
    sys.exit(main())

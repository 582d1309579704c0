#!/usr/bin/env python3
"""Benchmark: Jacobi-2D 5-point, 4096 x 4096 f64, T = 512 time steps, on one MI355X.

One "step" of this benchmark is one whole run of the hot path: T = 512 time
steps of the stencil over the 4096^2 field (4094^2 * 512 = 8,581,548,032
point updates), time-skewed tiles executed by the persistent HIP executor in
the chosen schedule.  The input field (sin(pi x) sin(pi y) plus seeded noise
of amplitude 1e-3, zero boundary) is resident in HBM before timing starts.

Prints ONE JSON line.  `value` is GUpdates/s of the whole job.  Extra keys:
  roofline      the dominant kernel (the tiled executor) against its binding
                roof, from HIP-event kernel times taken inside the timed loop;
  cpu_baseline  the oracle (plain C loop nest) on the host cores, on a bounded
                sample of the same workload;
  tiles         the tile/schedule the cost model picked ("learned") and the
                best of the exhaustive sweep re-timed here ("swept").
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NY = NX = 4096
T = 512
UPDATES = (NY - 2) * (NX - 2) * T
DEFAULT_TILE = (16, 64, 256)
DEFAULT_SCHED = "slt_wave"

HBM_PEAK_GBS = 8000.0
# FP64 vector: 256 CUs x 64 lanes x 2.4 GHz = 39.3e12 non-fused FP64 ops/s
# (the 78.6 TFLOP/s headline counts an FMA as two; the update rule has no FMA).
FP64_OPS_PEAK = 256 * 64 * 2.4e9
OPS_PER_UPDATE = 5  # 4 adds + 1 multiply


def alg_bytes_per_update(tile, elem=8):
    """Algorithmic HBM bytes per update of a b_t x b_y x b_x skewed tile: read
    and write of the bottom/top plane once per tile, plus two-wide low faces
    read and high faces written at every level."""
    bt, by, bx = tile
    return elem * (2.0 / bt + 4.0 / bx + 4.0 / by)


def roofline(tile, kernel_s, traffic=None):
    B = alg_bytes_per_update(tile)
    rate = UPDATES / kernel_s
    hbm_roof = HBM_PEAK_GBS * 1e9 / B
    alu_roof = FP64_OPS_PEAK / OPS_PER_UPDATE
    if hbm_roof <= alu_roof:
        ach = UPDATES * B / kernel_s / 1e9
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                "alg_bytes_per_update": round(B, 4), "updates_per_s_roof": hbm_roof}
    ach = OPS_PER_UPDATE * UPDATES / kernel_s / 1e12
    peak = FP64_OPS_PEAK / 1e12
    return {"bound": "alu", "achieved": round(ach, 3), "peak": round(peak, 2), "unit": "TFLOP/s",
            "frac": round(ach / peak, 4), "traffic": traffic,
            "alg_bytes_per_update": round(B, 4), "updates_per_s_roof": alu_roof}


def kernel_sources_digest():
    """Digest of the sources of the Jacobi-2D executor; stored HBM-traffic
    counters are reported only while it matches (else traffic is null)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("tiled2d.hip", "common.hpp", "bufio.hpp", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_1802_00166_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(tile, sched):
    """HBM bytes per launch from the committed rocprofv3 counter summary, when
    it was taken on this tile, schedule and kernel source."""
    p = os.path.join(ROOT, "profiles", "traffic_jacobi2d_4096_T512_f64.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("digest") != kernel_sources_digest() or list(d.get("tile", [])) != list(tile) \
            or d.get("schedule") != sched:
        return None
    return d.get("hbm_bytes_per_launch")


def calibrate_copy(reps=5):
    """A plain device copy of known size (512 MiB read + 512 MiB written), for
    scaling FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    n = 64 << 20
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": reps}), flush=True)


def cpu_baseline(u0, sample_T=T):
    """Oracle on the host: the full 4096^2 field for `sample_T` steps (by
    default the whole job), on up to 16 host threads (the threaded oracle
    gives the single-thread oracle's bits)."""
    import oracle
    threads = min(16, os.cpu_count() or 1)
    oracle.stencil("jacobi2d", "f64", u0[:64, :64], 1, threads=threads)  # load/build
    t0 = time.perf_counter()
    oracle.stencil("jacobi2d", "f64", u0, sample_T, threads=threads)
    dt = time.perf_counter() - t0
    upd = (NY - 2) * (NX - 2) * sample_T
    return {"value": round(upd / dt / 1e9, 4), "unit": "GUpdates/s", "cores": threads, "kind": "oracle",
            "sample": "Jacobi-2D 4096^2 f64, %d of the 512 steps, plain C loop nest, %d OpenMP threads, %.2f s"
                      % (sample_T, threads, dt)}


def pick_tiles():
    """Tile choice of the learned cost model when a trained model file is
    present, else the default; plus the sweep's best if a sweep was recorded."""
    learned = {"tile": list(DEFAULT_TILE), "schedule": DEFAULT_SCHED, "source": "default"}
    swept = None
    try:
        from paper_1802_00166_amd import tune
        m = tune.load_default_model()
        if m is not None:
            # the model ranks the schedules it was trained on
            tile, sched = tune.predict_stencil(m, "jacobi2d", "f64", (NY, NX), T, tune.MODEL_SCHEDULES)
            learned = {"tile": list(tile), "schedule": sched, "source": "mlp"}
        sw = tune.load_sweep_best("jacobi2d", "f64", (NY, NX), T)
        if sw is not None:
            swept = {"tile": list(sw[0]), "schedule": sw[1], "source": "sweep"}
    except ImportError:
        pass
    return learned, swept


def time_runs(pc, torch, x, out, ws, tile, sched, steps, warmup):
    for _ in range(warmup):
        pc.stencil_run("jacobi2d", "f64", x, T, tile, sched, out=out, workspace=ws)
    torch.cuda.synchronize()
    pc.kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pc.stencil_run("jacobi2d", "f64", x, T, tile, sched, out=out, workspace=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kms, kn = pc.kernel_timing_read()
    pc.kernel_timing(False)
    st = pc.stream_status(ws)
    if st != 0:
        raise RuntimeError("device error %d: %s" % (st, pc.last_error()))
    return dt, kms / max(kn, 1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tile", type=str, default=None, help="bt,by,bx")
    ap.add_argument("--schedule", type=str, default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-swept", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run the plain copy used to scale the HBM traffic counters")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(multi-GPU sharding is described in DESIGN.md, not built)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1802_00166_amd as pc
    import synth

    u0 = synth.jacobi2d_input(NY, NX)
    x = torch.from_numpy(u0).to("cuda:0")
    out = torch.empty_like(x)

    learned, swept = pick_tiles()
    if args.tile:
        learned = {"tile": [int(v) for v in args.tile.split(",")], "schedule": args.schedule or DEFAULT_SCHED,
                   "source": "cli"}
    elif args.schedule:
        learned["schedule"] = args.schedule
    tile = tuple(learned["tile"])
    sched = learned["schedule"]
    ws = pc.alloc_workspace(pc.workspace_bytes("jacobi2d", "f64", (NY, NX), T, tile, sched))

    dt, kern_ms = time_runs(pc, torch, x, out, ws, tile, sched, args.steps, args.warmup)
    ms_per_step = dt / args.steps * 1e3
    value = UPDATES / (dt / args.steps) / 1e9

    tiles = {"learned": dict(learned, gupd_s=round(value, 2))}
    if swept is not None and not args.no_swept:
        st = tuple(swept["tile"])
        ws2 = pc.alloc_workspace(pc.workspace_bytes("jacobi2d", "f64", (NY, NX), T, st, swept["schedule"]))
        dt2, _ = time_runs(pc, torch, x, out, ws2, st, swept["schedule"], max(3, args.steps // 2), 1)
        v2 = UPDATES / (dt2 / max(3, args.steps // 2)) / 1e9
        tiles["swept"] = dict(swept, gupd_s=round(v2, 2))
        tiles["learned_over_swept"] = round(value / v2, 4)

    rec = {
        "metric": "GUpdates/s, Jacobi-2D 4096^2 FP64, T=512 (time-skewed tiles, learned tile choice)",
        "value": round(value, 2),
        "unit": "GUpdates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: sin(pi x)sin(pi y) + 1e-3*(2U-1) noise (SplitMix64 stream 2), zero boundary",
        "config": {"workload": "jacobi2d_5pt_4096x4096_T512_f64", "updates_per_step": UPDATES,
                   "tile_bt_by_bx": list(tile), "schedule": sched},
        "roofline": dict(roofline(tile, kern_ms / 1e3, stored_traffic(tile, sched)), kernel_ms=round(kern_ms, 4)),
        "alg_bytes_per_update": round(alg_bytes_per_update(tile), 4),
        "streaming_roof_gupd_s": HBM_PEAK_GBS / 16.0,
        "tiles": tiles,
    }
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(u0)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()

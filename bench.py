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
# matrix chain N = 4096: (unused, b, b, k-chunk)
CHAIN_TILE = (0, 32, 32, 64)
# Gauss-Seidel-2D and FDTD-2D at the paper's shape (500 steps of 2000^2)
GS2D_TILE = (16, 32, 64)
FDTD2D_TILE = (16, 32, 32)
# the appendix's motivating 1D program, N = 4096, T = 2N
MOTIV_TILE = (64, 256)
# concurrent-start schedules of the headline problem: (b_t, F_y, F_x), schedule
TRAP_CANDIDATES = [((16, 64, 128), "trap"), ((8, 64, 128), "trap"), ((8, 64, 128), "diamond"),
                   ((8, 32, 128), "trap")]
# Heat-3D 512^3, T = 128: the tile each storage type is benchmarked with
HEAT3D_TILES = {"f64": (3, 64, 16, 64), "f32": (4, 64, 8, 64), "bf16": (4, 64, 8, 64)}

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


def measure_copy_gbs(torch, reps=5):
    """Achieved bandwidth of a plain 1 GiB device-to-device copy (read +
    written bytes over HIP-event time): the practical ceiling the executor's
    HBM rate is also compared with."""
    n = 128 << 20
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * n * 8 / (ms * 1e-3) / 1e9


def host_info():
    """Host CPU model, logical CPU count and the oracle's compiler and flags."""
    import platform
    import subprocess
    import oracle
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cc = subprocess.run(["gcc", "--version"], stdout=subprocess.PIPE, text=True).stdout.splitlines()[0]
    except (OSError, IndexError):
        cc = "gcc"
    return {"nproc": os.cpu_count(), "cpu_model": model, "compiler": cc, "flags": " ".join(oracle.CFLAGS)}


def cpu_baseline(u0, sample_T=T):
    """Oracle on the host: the full 4096^2 field for `sample_T` steps (by
    default the whole job).  `value` is the single-thread oracle (the binding
    one); `all_cores` is the same source on up to 16 OpenMP threads (same bits:
    the threads split the outer loop of each step)."""
    import oracle
    threads = min(16, os.cpu_count() or 1)
    oracle.stencil("jacobi2d", "f64", u0[:64, :64], 1)  # load/build
    upd = (NY - 2) * (NX - 2) * sample_T
    t0 = time.perf_counter()
    oracle.stencil("jacobi2d", "f64", u0, sample_T, threads=1)
    dt1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.stencil("jacobi2d", "f64", u0, sample_T, threads=threads)
    dtn = time.perf_counter() - t0
    rec = {"value": round(upd / dt1 / 1e9, 4), "unit": "GUpdates/s", "cores": 1, "kind": "oracle",
           "sample": "Jacobi-2D 4096^2 f64, %d of the 512 steps, plain C loop nest, 1 thread, %.2f s"
                     % (sample_T, dt1),
           "all_cores": {"value": round(upd / dtn / 1e9, 4), "cores": threads, "seconds": round(dtn, 3)}}
    rec.update(host_info())
    return rec


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


# --------------------------------------------------------------- workloads ---
# The other configurations of the hot path, selected with --workload (the
# default is the Jacobi-2D headline above).  Same JSON contract; the
# roofline object describes each one's dominant kernel.
VALU_OPS_PEAK = 256 * 64 * 2.4e9  # non-fused vector ops/s (f64, and f32 without packed math)


def _timed(pc, torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    pc.kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    kms, kn = pc.kernel_timing_read()
    pc.kernel_timing(False)
    return dt, (kms / kn if kn else dt * 1e3)


def _roof(updates, kernel_s, bytes_per_update, ops_per_update, ops_peak=VALU_OPS_PEAK, note=None):
    hbm_roof = HBM_PEAK_GBS * 1e9 / bytes_per_update if bytes_per_update > 0 else float("inf")
    alu_roof = ops_peak / ops_per_update
    if hbm_roof <= alu_roof:
        ach = updates * bytes_per_update / kernel_s / 1e9
        r = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(ach / HBM_PEAK_GBS, 4)}
    else:
        ach = updates * ops_per_update / kernel_s / 1e12
        r = {"bound": "alu", "achieved": round(ach, 3), "peak": round(ops_peak / 1e12, 2), "unit": "TFLOP/s",
             "frac": round(ach / (ops_peak / 1e12), 4)}
    r.update({"traffic": None, "alg_bytes_per_update": round(bytes_per_update, 4),
              "ops_per_update": ops_per_update, "kernel_ms": round(kernel_s * 1e3, 4)})
    if note:
        r["note"] = note
    return r


def _record(metric, value, unit, steps, warmup, dt, dtype, data, config, roofline, cpu, higher=True):
    rec = {"metric": metric, "value": round(value, 3), "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": round(dt * 1e3, 4), "higher_is_better": higher, "scaling": "weak", "vs_baseline": None,
           "dtype": dtype, "data": data, "config": config, "roofline": roofline}
    if cpu is not None:
        rec["cpu_baseline"] = cpu
    return rec


def workload_jacobi1d(args, pc, torch):
    import synth
    n, TT, tile, sched = 4096, 1000, (64, 256), "slt_lex"
    upd = (n - 2) * TT
    u0 = synth.jacobi1d_input(n)
    x = torch.from_numpy(u0).to("cuda:0")
    y = torch.empty_like(x)
    ws = pc.alloc_workspace(pc.workspace_bytes("jacobi1d", "f64", (n,), TT, tile, sched))
    dt, kms = _timed(pc, torch, lambda: pc.stencil_run("jacobi1d", "f64", x, TT, tile, sched, out=y, workspace=ws),
                     args.steps, args.warmup)
    wsn = pc.alloc_workspace(pc.workspace_bytes("jacobi1d", "f64", (n,), TT, None, "naive"))
    dtn, _ = _timed(pc, torch, lambda: pc.stencil_run("jacobi1d", "f64", x, TT, None, "naive", out=y, workspace=wsn),
                    args.steps, args.warmup)
    cpu = None
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        reps = 20
        for _ in range(reps):
            oracle.stencil("jacobi1d", "f64", u0, TT)
        c = (time.perf_counter() - t0) / reps
        cpu = {"value": round(upd / c / 1e9, 4), "unit": "GUpdates/s", "cores": 1, "kind": "oracle",
               "sample": "the whole job (N=4096, T=1000), single-thread plain C loop nest, mean of %d runs" % reps}
    return _record("GUpdates/s, Jacobi-1D N=4096 FP64, T=1000 (64-step x 256-point time-skewed tiles, lexicographic)",
                   upd / dt / 1e9, "GUpdates/s", args.steps, args.warmup, dt, "f64",
                   "synthetic: interior U[0,1) (SplitMix64 stream 1), zero boundary",
                   {"workload": "jacobi1d_3pt_4096_T1000_f64", "tile_bt_bx": list(tile), "schedule": sched},
                   _roof(upd, kms / 1e3, 8 * (2.0 / tile[0] + 4.0 / tile[1]), 3,
                         note="the 32 KiB field stays on chip: bound by latency, not by either roof"), cpu) | {
        "resident_block_untiled": {"ms": round(dtn * 1e3, 4), "gupd_s": round(upd / dtn / 1e9, 3),
                                   "note": "both levels of the field in one CU's LDS, all steps in one launch"}}


def workload_gs2d(args, pc, torch):
    """In-place Gauss-Seidel-2D at the paper's GS-2D shape (500 sweeps of
    2000^2, Table 2), front executor in skewed tiles, wavefront tile order."""
    import synth
    n, TT, tile, sched = 2000, 500, GS2D_TILE, "slt_wave"
    upd = (n - 2) * (n - 2) * TT
    u0 = synth.jacobi2d_input(n, n)
    x = torch.from_numpy(u0).to("cuda:0")
    y = torch.empty_like(x)
    ws = pc.alloc_workspace(pc.workspace_bytes("gs2d", "f64", (n, n), TT, tile, sched))
    dt, kms = _timed(pc, torch, lambda: pc.stencil_run("gs2d", "f64", x, TT, tile, sched, out=y, workspace=ws),
                     args.steps, args.warmup)
    cpu = None
    if not args.no_cpu:
        import oracle
        s = 50
        t0 = time.perf_counter()
        oracle.gs2d(u0, s)
        c = time.perf_counter() - t0
        cpu = {"value": round((n - 2) ** 2 * s / c / 1e9, 4), "unit": "GUpdates/s", "cores": 1, "kind": "oracle",
               "sample": "%d of the 500 sweeps, single-thread plain C in-place loop nest, %.2f s" % (s, c)}
    bt, by, bx = tile
    # each tile reads and writes its footprint once: ~ 2 * 8 * (by + bt)(bx + bt) bytes per bt*by*bx updates
    bpu = 16.0 * (by + bt) * (bx + bt) / (bt * by * bx)
    return _record("GUpdates/s, Gauss-Seidel-2D 2000^2 FP64, 500 in-place sweeps (skewed tiles, wavefront order)",
                   upd / dt / 1e9, "GUpdates/s", args.steps, args.warmup, dt, "f64",
                   "synthetic: sin(pi x)sin(pi y) + 1e-3*(2U-1) noise (SplitMix64 stream 2), zero boundary",
                   {"workload": "gs2d_5pt_2000x2000_T500_f64", "tile_bt_by_bx": list(tile), "schedule": sched},
                   _roof(upd, kms / 1e3, bpu, 5), cpu)


def workload_fdtd2d(args, pc, torch):
    """FDTD-2D (three statements per step, embedded) at the paper's shape
    (500 steps of 2000^2, Table 2); the untiled three-kernel step beside it."""
    import numpy as np
    import synth
    n, TT, tile, sched = 2000, 500, FDTD2D_TILE, "slt_wave"
    upd = n * n * TT  # iterations of the embedded nest (three statements each)
    s = synth.test_rng(23)
    f = np.stack([synth.uniform_f64(s, n * n, offset=k * n * n).reshape(n, n) - 0.5 for k in range(3)])
    x = torch.from_numpy(np.ascontiguousarray(f)).to("cuda:0")
    y = torch.empty_like(x)
    ws = pc.alloc_workspace(pc.workspace_bytes("fdtd2d", "f64", (n, n), TT, tile, sched))
    dt, kms = _timed(pc, torch, lambda: pc.stencil_run("fdtd2d", "f64", x, TT, tile, sched, out=y, workspace=ws),
                     args.steps, args.warmup)
    wsn = pc.alloc_workspace(pc.workspace_bytes("fdtd2d", "f64", (n, n), TT, None, "naive"))
    dtn, _ = _timed(pc, torch, lambda: pc.stencil_run("fdtd2d", "f64", x, TT, None, "naive", out=y, workspace=wsn),
                    max(2, args.steps // 2), 1)
    cpu = None
    if not args.no_cpu:
        import oracle
        st = 20
        t0 = time.perf_counter()
        oracle.fdtd2d(f[0], f[1], f[2], st)
        c = time.perf_counter() - t0
        cpu = {"value": round(n * n * st / c / 1e9, 4), "unit": "GIterations/s", "cores": 1, "kind": "oracle",
               "sample": "%d of the 500 steps, single-thread plain C three loop nests, %.2f s" % (st, c)}
    bt, by, bx = tile
    bpu = 3 * 16.0 * (by + bt) * (bx + bt) / (bt * by * bx)
    rec = _record("GIterations/s, FDTD-2D 2000^2 FP64, 500 steps (three statements per iteration, embedded nest "
                  "in skewed tiles, wavefront order)", upd / dt / 1e9, "GIterations/s", args.steps, args.warmup, dt,
                  "f64", "synthetic: ex, ey, hz uniform[-0.5, 0.5) (SplitMix64 test stream 23)",
                  {"workload": "fdtd2d_2000x2000_T500_f64", "tile_bt_by_bx": list(tile), "schedule": sched},
                  _roof(upd, kms / 1e3, bpu, 11), cpu)
    rec["untiled_three_kernel_step"] = {"ms": round(dtn * 1e3, 3), "giter_s": round(upd / dtn / 1e9, 2)}
    return rec


def workload_motiv1d(args, pc, torch):
    """The appendix's motivating 1D program, N = 4096, T = 2N, with the
    schedule-independent allocation (two interior buffers, single-assignment
    boundary arrays), skewed tiles in wavefront order."""
    import synth
    n, TT, tile, sched = 4096, 8192, MOTIV_TILE, "slt_wave"
    upd = (n - 2) * TT
    a = synth.uniform_f64(synth.test_rng(77), n)
    x = torch.from_numpy(a).to("cuda:0")
    y = torch.empty_like(x)
    ws = pc.alloc_workspace(pc.workspace_bytes("motiv1d", "f64", (n,), TT, tile, sched))
    dt, kms = _timed(pc, torch, lambda: pc.stencil_run("motiv1d", "f64", x, TT, tile, sched, out=y, workspace=ws),
                     args.steps, args.warmup)
    cpu = None
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        oracle.motiv(a, TT)
        c = time.perf_counter() - t0
        cpu = {"value": round(upd / c / 1e9, 4), "unit": "GUpdates/s", "cores": 1, "kind": "oracle",
               "sample": "the whole job, single-thread plain C with the program's own allocation, %.3f s" % c}
    bt, bx = tile
    rec = _record("GUpdates/s, motivating 1D program (appendix) N=4096 FP64, T=8192, single-assignment boundary "
                  "arrays", upd / dt / 1e9, "GUpdates/s", args.steps, args.warmup, dt, "f64",
                  "synthetic: uniform[0,1) (SplitMix64 test stream 77)",
                  {"workload": "motiv1d_4096_T8192_f64", "tile_bt_bx": list(tile), "schedule": sched},
                  _roof(upd, kms / 1e3, 8 * (2.0 / bt + 4.0 / bx), 4,
                        note="a 32 KiB field over 8192 dependent steps: latency-bound"), cpu)
    rec["workspace_bytes"] = int(pc.workspace_bytes("motiv1d", "f64", (n,), TT, tile, sched))
    rec["full_expansion_bytes"] = 8 * n * (TT + 1)
    return rec


def workload_trap(args, pc, torch):
    """The headline problem under the concurrent-start schedules (trapezoid
    hyperspace cut, and the diamond shift of it) beside the box tiles."""
    import synth
    u0 = synth.jacobi2d_input(NY, NX)
    x = torch.from_numpy(u0).to("cuda:0")
    out = torch.empty_like(x)
    res = {}
    best = None
    for tile, sched in TRAP_CANDIDATES:
        ws = pc.alloc_workspace(pc.workspace_bytes("jacobi2d", "f64", (NY, NX), T, tile, sched))
        dt, kms = time_runs(pc, torch, x, out, ws, tile, sched, args.steps, args.warmup)
        _, _, tr = pc.trap_plan((NY, NX), T, tile, sched)
        bpu = 8.0 * (tr[0] + tr[1]) / UPDATES
        key = "%s_%d_%d_%d" % ((sched,) + tuple(tile))
        res[key] = {"gupd_s": round(UPDATES / (dt / args.steps) / 1e9, 2), "kernel_ms": round(kms, 3),
                    "alg_bytes_per_update": round(bpu, 4)}
        if best is None or dt < best[0]:
            best = (dt, kms, tile, sched, bpu)
    dt, kms, tile, sched, bpu = best
    rec = _record("GUpdates/s, Jacobi-2D 4096^2 FP64, T=512, concurrent-start schedules (trapezoid / diamond tiles)",
                  UPDATES / (dt / args.steps) / 1e9, "GUpdates/s", args.steps, args.warmup, dt / args.steps, "f64",
                  "synthetic: sin(pi x)sin(pi y) + 1e-3*(2U-1) noise (SplitMix64 stream 2), zero boundary",
                  {"workload": "jacobi2d_5pt_4096x4096_T512_f64_trap", "tile_bt_fy_fx": list(tile), "schedule": sched},
                  _roof(UPDATES, kms / 1e3, bpu, 5), None)
    rec["candidates"] = res
    return rec


def heat3d_alg_bytes(tile, e):
    """Algorithmic HBM bytes per update of a Heat-3D tile: the input planes
    read and the top level written once per tile (2/b_t), and the two-wide
    faces of every level but the top one written by the tile and read by its
    neighbour (the top level's outputs feed no level of the tile)."""
    bt, bz, by, bx = tile
    return e * (2.0 / bt + (bt - 1.0) / bt * 4.0 * (1.0 / bx + 1.0 / by + 1.0 / bz))


def workload_heat3d(args, pc, torch, dtype):
    import numpy as np
    import synth
    n, TT = 512, 128
    tile = HEAT3D_TILES[dtype]
    sched = "slt_wave"
    upd = (n - 2) ** 3 * TT
    u = synth.heat3d_input(n)
    if dtype == "f64":
        x = torch.from_numpy(u).to("cuda:0")
    elif dtype == "f32":
        x = torch.from_numpy(u.astype(np.float32)).to("cuda:0")
    else:
        x = torch.from_numpy(synth.to_bf16_bits(u.astype(np.float32)).view(np.int16)).to("cuda:0")
    y = torch.empty_like(x)
    ws = pc.alloc_workspace(x.numel() * x.element_size() + (64 << 20))
    dt, kms = _timed(pc, torch, lambda: pc.stencil_run("heat3d", dtype, x, TT, tile, sched, out=y, workspace=ws),
                     args.steps, args.warmup)
    dtn, _ = _timed(pc, torch, lambda: pc.stencil_run("heat3d", dtype, x, TT, None, "naive", out=y, workspace=ws),
                    1, 1)
    pc.stencil_run("heat3d", dtype, x, TT, tile, sched, out=y, workspace=ws)
    torch.cuda.synchronize()
    err = None
    if dtype != "f64":
        # reference: the f64 path on the f64 input (bit-identical to the f64 oracle)
        x64 = torch.from_numpy(u).to("cuda:0")
        r64 = torch.empty_like(x64)
        ws64 = pc.alloc_workspace(x64.numel() * 8 + (64 << 20))
        pc.stencil_run("heat3d", "f64", x64, TT, (2, 32, 8, 64), sched, out=r64, workspace=ws64)
        nm = pc.error_norms(dtype, y, r64)
        err = {"max_rel": nm["max_rel"], "l2_rel": nm["l2_rel"], "reference": "FP64 path (bit-identical to the FP64 oracle)"}
        del x64, r64, ws64
    e = {"f64": 8, "f32": 4, "bf16": 2}[dtype]
    bt, bz, by, bx = tile
    cpu = None
    if not args.no_cpu and dtype == "f64":
        import oracle
        threads = min(16, os.cpu_count() or 1)
        ts = 8
        t0 = time.perf_counter()
        oracle.stencil("heat3d", "f64", u, ts, threads=threads)
        c = time.perf_counter() - t0
        cpu = {"value": round((n - 2) ** 3 * ts / c / 1e9, 4), "unit": "GUpdates/s", "cores": threads, "kind": "oracle",
               "sample": "Heat-3D 512^3 f64, %d of the 128 steps, plain C loop nest, %d OpenMP threads, %.2f s"
                         % (ts, threads, c)}
    rec = _record("GUpdates/s, Heat-3D 512^3 %s, T=128 (time-skewed tiles)" % dtype.upper(), upd / dt / 1e9,
                  "GUpdates/s", args.steps, args.warmup, dt, dtype,
                  "synthetic: interior U[0,1) (SplitMix64 stream 3), zero boundary",
                  {"workload": "heat3d_7pt_512_T128_%s" % dtype, "tile_bt_bz_by_bx": list(tile), "schedule": sched},
                  _roof(upd, kms / 1e3, heat3d_alg_bytes(tile, e), 11), cpu)
    rec["naive_gupd_s"] = round(upd / dtn / 1e9, 2)
    rec["streaming_roof_gupd_s"] = HBM_PEAK_GBS / (2 * e)
    if err:
        rec["error_vs_fp64"] = err
    return rec


def workload_matrix_chain(args, pc, torch):
    import synth
    N, pmax, tile, sched = 4096, 100, CHAIN_TILE, "slt_wave"
    upd = (N ** 3 - N) // 6
    p = torch.from_numpy(synth.chain_dims(N)).to("cuda:0")
    C = torch.empty((N, N), dtype=torch.int64, device="cuda:0")
    ws = pc.alloc_workspace(pc.dp_workspace_bytes(N, tile, sched))
    dt, kms = _timed(pc, torch, lambda: pc.dp_run(p, pmax, tile, sched, out=C, workspace=ws), args.steps, args.warmup)
    cpu = None
    if not args.no_cpu:
        import oracle
        Ns = 1024
        ps = synth.chain_dims(Ns)
        t0 = time.perf_counter()
        oracle.matrix_chain(ps)
        c = time.perf_counter() - t0
        cpu = {"value": round((Ns ** 3 - Ns) / 6 / c / 1e9, 4), "unit": "GUpdates/s", "cores": 1, "kind": "oracle",
               "sample": "matrix chain N=%d (same generator), single-thread plain C DP, %.2f s" % (Ns, c)}
    # the interval-DP cost model's pick for this problem, re-timed beside the fixed tile
    learned = None
    try:
        from paper_1802_00166_amd import tune
        m = tune.load_default_model("chain")
        if m is not None:
            lt, ls, _ = m.predict(tune.problem("matrix_chain", "f64", (N,), pmax), ["slt_wave", "cot_par"])
            wsl = pc.alloc_workspace(pc.dp_workspace_bytes(N, lt, ls))
            dtl, _ = _timed(pc, torch, lambda: pc.dp_run(p, pmax, lt, ls, out=C, workspace=wsl),
                            max(3, args.steps // 2), 1)
            learned = {"tile_b_b_kchunk": list(lt[1:]), "schedule": ls, "gupd_s": round(upd / dtl / 1e9, 2),
                       "learned_over_fixed_time": round(dtl / dt, 4)}
    except ImportError:
        pass
    # u32 path: v_mul_u32_u24, v_add3_u32, v_min3_u32 per pair of candidate splits -> 2.5 VALU ops/update
    rec = _record("GUpdates/s, matrix-chain interval DP N=4096 (exact), tile diagonals", upd / dt / 1e9,
                   "GUpdates/s", args.steps, args.warmup, dt, "u32 (exact; int64 API)",
                   "synthetic: p_i ~ U{1..100} (SplitMix64 stream 5)",
                   {"workload": "matrix_chain_4096_pmax100", "tile_b_b_kchunk": list(tile[1:]), "schedule": sched},
                   _roof(upd, kms / 1e3, 2 * 4 / 32, 2.5), cpu)
    if learned is not None:
        rec["model_pick"] = learned
    return rec


def _batch_bytes(tiles, inst):
    """Update-weighted algorithmic bytes per update of a batch (f32)."""
    tot = w = 0.0
    for (bt, by, bx), (ny, nx, TT) in zip(tiles, inst):
        u = (ny - 2) * (nx - 2) * TT
        tot += u * 4 * (2.0 / bt + 4.0 / bx + 4.0 / by)
        w += u
    return tot / w


def workload_batched(args, pc, torch):
    """The uneven batch: 256 f32 instances in one persistent launch, replayed
    from a HIP graph.  The value is the cost model's batch choice: one tile
    for every instance, the fastest on the batch of the model's three best
    for one problem that fills the device as the batch does
    (tune.batch_model_uniform, three timings: the tuner's verify mode).
    Beside it, for context: the model's top-1 alone, a sweep over eight
    uniform tiles, and the model's per-instance picks (one b_x for the
    batch), which follow each instance's stand-alone critical path rather
    than the batch's throughput."""
    import numpy as np
    import synth
    from paper_1802_00166_amd import tune
    inst = synth.batched_instances(256)
    xs = [torch.from_numpy(synth.batched_field(i, ny, nx)).to("cuda:0") for i, (ny, nx, _) in enumerate(inst)]
    Ts = [TT for (_, _, TT) in inst]
    shapes = [(ny, nx) for (ny, nx, _) in inst]
    upd = sum((ny - 2) * (nx - 2) * TT for (ny, nx, TT) in inst)
    model = tune.load_default_model()
    choice = {"uniform_%d_%d_%d" % t: [t] * len(inst) for t in tune.BATCH_UNIFORM_TILES}
    if model is None:
        raise RuntimeError("the batched workload needs the stored cost model (paper_1802_00166_amd/models/stencil.mlp)")
    top = tune.batch_model_uniform(model, "jacobi2d", "f32", shapes, Ts, topk=3)
    for i, t in enumerate(top):
        choice["model_batch_%d" % (i + 1)] = [t] * len(inst)
    choice["model"] = tune.batch_model_tiles(model, "jacobi2d", "f32", shapes, Ts)
    results = {}
    for name, tiles in choice.items():
        outs = [torch.empty_like(x) for x in xs]
        ws = pc.alloc_workspace(pc.workspace_bytes_batched("jacobi2d", "f32", shapes, Ts, tiles, "slt_wave"))
        pc.stencil_run_batched("jacobi2d", "f32", xs, Ts, tiles, "slt_wave", outs=outs, workspace=ws)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            pc.stencil_run_batched("jacobi2d", "f32", xs, Ts, tiles, "slt_wave", outs=outs, workspace=ws)
        for _ in range(args.warmup):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
        torch.cuda.synchronize()
        results[name] = (time.perf_counter() - t0) / args.steps
        if pc.stream_status(ws) != 0:
            raise RuntimeError("device error in the batched run: %s" % pc.last_error())
    # the model's three best batch tiles, each timed on the batch (the
    # tuner's verify mode): the value is the fastest of them
    best = min((k for k in results if k.startswith("model_batch_")), key=results.get)
    mt = top[int(best.rsplit("_", 1)[1]) - 1]
    dt = results[best]
    rec = _record("GUpdates/s, 256 uneven Jacobi-2D FP32 instances, one persistent launch replayed from a HIP graph",
                  upd / dt / 1e9, "GUpdates/s", args.steps, args.warmup, dt, "f32",
                  "synthetic: 256 shapes n_y, n_x ~ U{128..2048}, T ~ U{32..512}, every cell U[0,1) (SplitMix64 stream 4)",
                  {"workload": "batched_jacobi2d_256_f32", "instances": len(inst), "updates_per_step": upd,
                   "tiles": "model_top3_verified", "tile_bt_by_bx": list(mt), "schedule": "slt_wave"},
                  _roof(upd, dt, _batch_bytes(choice[best], inst), 5, note="graph-replay wall time per launch"), None)
    rec["graph_replay_ms"] = {k: round(v * 1e3, 3) for k, v in results.items()}
    unif = min((k for k in results if k.startswith("uniform")), key=results.get)
    rec["best_uniform"] = unif
    rec["model_top1_tile"] = list(top[0])
    rec["model_top1_over_best_uniform_time"] = round(results["model_batch_1"] / results[unif], 4)
    rec["model_top3_verified_over_best_uniform_time"] = round(dt / results[unif], 4)
    rec["per_instance_picks_over_best_uniform_time"] = round(results["model"] / results[unif], 4)
    return rec


def workload_tile_variability(args, pc, torch):
    """Run-time spread over the tile space of the Jacobi-2D headline problem,
    per schedule: every feasible candidate of the tuner's grid (b_t, b_y, b_x)
    timed under SLT_LEX, SLT_WAVE, COT_SEQ and COT_PAR (median of `steps`
    runs after one warm-up each).  The paper's robustness claim is about this
    spread (how much the choice of tile sizes matters under each schedule), so
    the record carries mean, standard deviation and relative standard
    deviation of the times; the value is the best candidate's rate."""
    import numpy as np
    from paper_1802_00166_amd import tune
    prob = tune.problem("jacobi2d", "f64", (NY, NX), T)
    per, best = {}, None
    for sch in ["slt_lex", "slt_wave", "cot_seq", "cot_par"]:
        t0 = time.perf_counter()
        _, _, _, recs = tune.sweep(prob, reps=max(3, args.steps // 2), warmup=1, schedules=[sch])
        ms = np.array([r["ms"] for r in recs])
        g = UPDATES / (ms * 1e-3) / 1e9
        b = int(np.argmin(ms))
        per[sch] = {"candidates": int(len(ms)), "best_tile": list(recs[b]["tile"]), "best_ms": round(float(ms[b]), 4),
                    "best_gupd_s": round(float(g[b]), 2), "median_ms": round(float(np.median(ms)), 4),
                    "mean_ms": round(float(ms.mean()), 4), "std_ms": round(float(ms.std()), 4),
                    "rsd": round(float(ms.std() / ms.mean()), 4), "worst_over_best": round(float(ms.max() / ms[b]), 3),
                    "mean_gupd_s": round(float(g.mean()), 2), "sweep_s": round(time.perf_counter() - t0, 1)}
        print("# %s: %d candidates, best %s %.3f ms, RSD %.3f" % (sch, len(ms), per[sch]["best_tile"], ms[b],
                                                                  per[sch]["rsd"]), file=sys.stderr, flush=True)
        if best is None or ms[b] < best[2]:
            best = (sch, tuple(recs[b]["tile"]), float(ms[b]))
    sch, tile, bms = best
    rec = _record("GUpdates/s, Jacobi-2D 4096^2 FP64, T=512: best of the full tile sweep; run-time spread per schedule",
                  UPDATES / (bms * 1e-3) / 1e9, "GUpdates/s", max(3, args.steps // 2), 1, bms * 1e-3, "f64",
                  "synthetic: sin(pi x)sin(pi y) + 1e-3*(2U-1) noise (SplitMix64 stream 2), zero boundary",
                  {"workload": "jacobi2d_5pt_4096x4096_T512_f64_tile_sweep", "tile_bt_by_bx": list(tile),
                   "schedule": sch},
                  _roof(UPDATES, bms * 1e-3, 8 * (2.0 / tile[0] + 4.0 / tile[1] + 4.0 / tile[2]), 5), None)
    rec["variability"] = per
    return rec


# The paper's own problem shapes (its Table 2), deliberately not powers of
# two: the Jacobi-2D rule at the Heat-2D shape, Heat-3D, and the interval DP
# at N = 4000.  The paper's figures are single CPU cores running other code:
# context, not a target.
PAPER_SHAPES = {"jacobi2d": ((3000, 3000), 500), "heat3d": ((350, 350, 350), 50), "matrix_chain": 4000}
PAPER_HEAT3D_TILE = (3, 64, 16, 64)


def paper_jacobi2d_tile():
    """The cost model's tile for the paper's Heat-2D shape (else the default)."""
    try:
        from paper_1802_00166_amd import tune
        m = tune.load_default_model()
        if m is not None:
            (ny, nx), TT = PAPER_SHAPES["jacobi2d"]
            return tune.predict_stencil(m, "jacobi2d", "f64", (ny, nx), TT, tune.MODEL_SCHEDULES)
    except ImportError:
        pass
    return DEFAULT_TILE, DEFAULT_SCHED


def workload_paper_shapes(args, pc, torch):
    import numpy as np
    import synth
    rows = {}
    (ny, nx), TT = PAPER_SHAPES["jacobi2d"]
    tile, sched = paper_jacobi2d_tile()
    u = synth.jacobi2d_input(ny, nx)
    x = torch.from_numpy(u).to("cuda:0")
    y = torch.empty_like(x)
    ws = pc.alloc_workspace(pc.workspace_bytes("jacobi2d", "f64", (ny, nx), TT, tuple(tile), sched))
    upd2 = (ny - 2) * (nx - 2) * TT
    dt2, k2 = _timed(pc, torch, lambda: pc.stencil_run("jacobi2d", "f64", x, TT, tuple(tile), sched, out=y,
                                                       workspace=ws), args.steps, args.warmup)
    del x, y, ws
    (nz, n1, n2), T3 = PAPER_SHAPES["heat3d"]
    u3 = synth.heat3d_input(nz)
    x = torch.from_numpy(u3).to("cuda:0")
    y = torch.empty_like(x)
    ws = pc.alloc_workspace(x.numel() * 8 + (64 << 20))
    upd3 = (nz - 2) * (n1 - 2) * (n2 - 2) * T3
    dt3, _ = _timed(pc, torch, lambda: pc.stencil_run("heat3d", "f64", x, T3, PAPER_HEAT3D_TILE, "slt_wave", out=y,
                                                      workspace=ws), args.steps, args.warmup)
    del x, y, ws
    N = PAPER_SHAPES["matrix_chain"]
    p = torch.from_numpy(synth.chain_dims(N)).to("cuda:0")
    C = torch.empty((N, N), dtype=torch.int64, device="cuda:0")
    ws = pc.alloc_workspace(pc.dp_workspace_bytes(N, CHAIN_TILE, "slt_wave"))
    updc = (N ** 3 - N) // 6
    dtc, _ = _timed(pc, torch, lambda: pc.dp_run(p, 100, CHAIN_TILE, "slt_wave", out=C, workspace=ws),
                    args.steps, args.warmup)
    rows["heat3d_7pt_350_T50_f64"] = {"gupd_s": round(upd3 / dt3 / 1e9, 2), "ms": round(dt3 * 1e3, 3),
                                      "tile_bt_bz_by_bx": list(PAPER_HEAT3D_TILE), "schedule": "slt_wave",
                                      "paper_cpu_1core_gupd_s": "about 1.1-1.2 (its Heat-3D, SLT sequential)"}
    rows["matrix_chain_4000"] = {"gupd_s": round(updc / dtc / 1e9, 2), "ms": round(dtc * 1e3, 3),
                                 "tile_b_b_kchunk": list(CHAIN_TILE[1:]), "schedule": "slt_wave",
                                 "paper_cpu_1core_gupd_s": "21.0-22.8 (its OSP, SLT sequential)"}
    rec = _record("GUpdates/s, Jacobi-2D 3000^2 FP64, T=500 (the paper's Heat-2D shape; learned tile)",
                  upd2 / dt2 / 1e9, "GUpdates/s", args.steps, args.warmup, dt2, "f64",
                  "synthetic: the headline's recipes at the paper's shapes (Jacobi-2D stream 2, Heat-3D stream 3, "
                  "chain stream 5)",
                  {"workload": "paper_shapes_jacobi2d_3000_T500_f64", "tile_bt_by_bx": list(tile), "schedule": sched},
                  _roof(upd2, k2 / 1e3, alg_bytes_per_update(tuple(tile)), 5), None)
    rec["paper_cpu_1core_gupd_s"] = "about 2.05 (its Heat-2D, SLT sequential; another update rule)"
    rec["context_rows"] = rows
    return rec


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
    ap.add_argument("--workload", default="jacobi2d",
                    choices=["jacobi2d", "jacobi1d", "heat3d_f64", "heat3d_f32", "heat3d_bf16", "matrix_chain",
                             "batched", "tile_variability", "paper_shapes", "gs2d", "fdtd2d", "motiv1d",
                             "trap"])
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; --gpus %d is not supported "
              "(sharding across GPUs is not implemented)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.workload != "jacobi2d":
        import torch
        import paper_1802_00166_amd as pc
        if args.workload == "jacobi1d":
            rec = workload_jacobi1d(args, pc, torch)
        elif args.workload.startswith("heat3d_"):
            rec = workload_heat3d(args, pc, torch, args.workload.split("_")[1])
        elif args.workload == "matrix_chain":
            rec = workload_matrix_chain(args, pc, torch)
        elif args.workload == "tile_variability":
            rec = workload_tile_variability(args, pc, torch)
        elif args.workload == "paper_shapes":
            rec = workload_paper_shapes(args, pc, torch)
        elif args.workload == "gs2d":
            rec = workload_gs2d(args, pc, torch)
        elif args.workload == "fdtd2d":
            rec = workload_fdtd2d(args, pc, torch)
        elif args.workload == "motiv1d":
            rec = workload_motiv1d(args, pc, torch)
        elif args.workload == "trap":
            rec = workload_trap(args, pc, torch)
        else:
            rec = workload_batched(args, pc, torch)
        print(json.dumps(rec), flush=True)
        return

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
        cg = measure_copy_gbs(torch)
        r = rec["roofline"]
        r["copy_gbs"] = round(cg, 1)
        if r.get("unit") == "GB/s":
            r["frac_of_copy"] = round(r["achieved"] / cg, 4)
        rec["cpu_baseline"] = cpu_baseline(u0)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()

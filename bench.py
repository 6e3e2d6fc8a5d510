"""Benchmark of the spectral hot path on one MI355X.

One "step" is one tau-step of the whole workload: the fused xi-march carrying the four
Runge-Kutta stages, the tau-push, the field outputs and the renormalization, for every mode.
Default workload: the 3D spectral run -- 205,859 modes of the 512 x 512 (k_x, k_y) grid
with |k| <= 6, 4096 xi cells, electron beam n_b = 0.01 n_p, gamma = 1000, length 100,
d_tau = 10, random-phase seed 1e-6, FP32 state with FP64 oscillator carry; outputs: the
per-step max over xi of ln A for every mode and full ln|E|, ln|B| snapshots every 500 steps.

Prints one JSON line (see the field list at the bottom).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("mode·ξ·τ cell-updates/s at 1 GPU; surrogate vs solver speed at "
          "≤1e-2 log-amp err")
HBM_PEAK_GBS = 8000.0
# VALU peak of MI355X without packed FP32 (which this library does not use): 256 CUs x 4 SIMDs
# x 16 lanes x 2.4 GHz, one wave64 instruction per SIMD every 4 cycles; an FMA counts as two
# flops, so FP32 and FP64 FMAs both peak at 78.6 TFLOP/s
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4          # wave64 VALU instructions per second
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# the march's arithmetic per cell-update (one mode, one cell, one tau-step; per column of the
# mode's two real columns): RK4 stage inputs 3 x 3 FMA (18 flops), the exact propagator of each
# of the 4 stages (difference, 2 FMA for n_p at the centre, 2 for n_p at the face, a product
# and an FMA for d_xi n_p: 12 flops, 48), d_xi n_p at the centre for the fields (3), the stage
# derivatives (difference and sum for rho, one product each for the two currents: 4 per
# stage, 16), the field energies and their sum over the columns (12), the update (3 FMA, 6):
# 103 flops per column
FLOP_PER_CELL_UPDATE = 2 * 103


def kernel_source_hash():
    p = os.path.join(ROOT, "paper_2607_24234_amd", "csrc", "qs_spectral.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def _counter_entry(path, precision_name, steps_per_launch):
    """The counter summary entry for this precision taken on launches of this many steps, if
    it was taken on the current kernel source (else None)."""
    try:
        d = json.load(open(path))
    except Exception:
        return None
    for key, e in d.items():
        if key.split("_")[0] != precision_name or not isinstance(e, dict):
            continue
        if e.get("kernel_sha256_16") == kernel_source_hash() and int(e.get("steps_per_dispatch", 0)) == int(steps_per_launch):
            return e
    return None


def read_traffic(precision_name, steps_per_launch):
    """HBM bytes of one launch (FETCH_SIZE + WRITE_SIZE, calibrated against a plain copy) from
    the rocprofv3 counter summary taken on launches of the same length and the current kernel
    source (else None)."""
    e = _counter_entry(os.path.join(ROOT, "profiles", "march_spectral3d_traffic.json"), precision_name,
                       steps_per_launch)
    try:
        return None if e is None else float(e["bytes_per_step"]) * steps_per_launch
    except Exception:
        return None


def read_valu(precision_name, steps_per_launch):
    """Wave64 VALU instructions per cell-update of the stepping launch (SQ_INSTS_VALU over
    the launch's cell-updates) from the rocprofv3 counter summary taken on launches of the
    same length and the current kernel source (else None)."""
    e = _counter_entry(os.path.join(ROOT, "profiles", "march_spectral3d_valu.json"), precision_name,
                       steps_per_launch)
    try:
        return None if e is None else float(e["wave_instructions_per_cell_update"])
    except Exception:
        return None


def read_workload_traffic(workload, amount):
    """Calibrated HBM bytes (FETCH_SIZE + WRITE_SIZE against a plain copy) of one launch, or of
    one tau-step for the finite-width pass sequence, from the rocprofv3 counter summary -- only
    if the counters were taken on the current source of the kernels (else None)."""
    p = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        e = json.load(open(p))[workload]
        src = os.path.join(ROOT, e["source"])
        if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != e["source_sha256_16"]:
            return None
        return float(e[amount])
    except Exception:
        return None


def launch_plan(args, insts, precision, steps_per_call):
    """The march's launch plan: the library's autotuner (qs_tune: candidate column counts and
    segment lengths timed on the device for calls of this length) or its built-in heuristic."""
    from paper_2607_24234_amd import qs
    if args.plan == "auto":
        return {}, "heuristic"
    t = time.perf_counter()
    tuned = qs.tune(insts, precision=precision, steps_per_call=max(1, int(steps_per_call)))
    print("[plan] autotuner: %s (%.1f s)" % (tuned, time.perf_counter() - t), file=sys.stderr, flush=True)
    return ({"columns_per_lane": tuned["columns_per_lane"], "segment_cells": tuned["segment_cells"]},
            "autotuner (qs_tune, calls of %d steps)" % steps_per_call)


def _scaled(v, f):
    return None if v is None else v * f


def host_cpu():
    """The host's CPU model and the cores this process may use."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, avail


def cpu_baseline(inst, seconds=15.0):
    """The FP64 oracle timed on the host cores on a bounded sample of the same workload:
    modes spread evenly over the mode list, all 4096 cells, a fixed number of tau-steps;
    the mode count is sized from a short probe so that each of three timed runs takes about
    seconds/3, and the median run is reported."""
    import numpy as np
    import oracle as O
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from helpers import mode_k, oracle_beam
    O.build()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    beam = oracle_beam(inst)
    k_all = mode_k(inst)
    steps = 10

    def timed(n_modes, n_steps):
        sel = np.linspace(0, len(k_all) - 1, n_modes).astype(int)
        st = O.seed(beam, k_all[sel], O.SEED_NOISE, inst["seed_amp"], rng_seed=inst["rng_seed"])
        t = time.perf_counter()
        O.run(beam, k_all[sel], inst["d_tau"], n_steps, st, want_fields=False, want_max=True,
              n_threads=threads)
        return time.perf_counter() - t

    probe_modes = 2 * threads
    rate = probe_modes * inst["n_xi"] * 2 / timed(probe_modes, 2)
    n_modes = int(max(threads, min(len(k_all), seconds / 3 * rate / (inst["n_xi"] * steps))))
    n_modes = max(threads, n_modes // threads * threads)
    runs = sorted(timed(n_modes, steps) for _ in range(3))
    dt = runs[1]
    cells = n_modes * inst["n_xi"] * steps
    model, avail = host_cpu()
    return {"value": cells / dt, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "cpu_model": model, "cpus_available": avail,
            "runs_s": runs,
            "sample": "%d modes evenly spread over the 205,859-mode list x %d cells x %d steps "
                      "(FP64, per-step max ln A output); median of 3 runs, %.1f s wall each"
                      % (n_modes, inst["n_xi"], steps, dt)}


def _line(metric, value, unit, K, W, ms, dtype, config, roofline, cpu, **extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": K, "warmup": W,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": dtype, "data": "synthetic", "config": config, "roofline": roofline, "cpu_baseline": cpu}
    out.update(extra)
    print(json.dumps(out), flush=True)


def bench_batched(args):
    """The 256-instance parameter sweep (128 modes each, 128..8192 cells, 200 steps) as one
    library call of 200 steps (one persistent launch) with per-step max ln A."""
    import numpy as np
    import torch
    from paper_2607_24234_amd import inputs, qs
    insts = inputs.batched()
    K = insts[0]["n_steps"]
    plan, plan_src = launch_plan(args, insts, qs.QS_FP32, K)
    s = qs.Solver(insts, precision=qs.QS_FP32, **plan)
    buf = torch.empty((K, s.total_modes), dtype=torch.float32, device="cuda")
    L = qs.lib()
    qs._check(L.qs_step_tau(s.ctx, 5, 1, None, None, buf.data_ptr()))
    torch.cuda.synchronize()
    s2 = qs.Solver(insts, precision=qs.QS_FP32, **plan)       # timed from the initial state
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(s2.stream)
    qs._check(L.qs_step_tau(s2.ctx, K, 1, None, None, buf.data_ptr()))
    e1.record(s2.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s2.sync_check()
    cells = sum(len(d["kx"]) * d["n_xi"] for d in insts)
    launch = e0.elapsed_time(e1) * 1e-3
    rate = cells * K / launch
    flops = FLOP_PER_CELL_UPDATE * rate / 1e12
    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from helpers import oracle_run
        O.build()
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
        pick = [0, 64, 128, 192]
        t = time.perf_counter()
        done = 0
        for i in pick:
            oracle_run(insts[i], 20, instance=i, n_threads=threads)
            done += len(insts[i]["kx"]) * insts[i]["n_xi"] * 20
        dt = time.perf_counter() - t
        cpu = {"value": done / dt, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
               "sample": "instances 0, 64, 128, 192 (all 128 modes, all cells) x 20 steps, FP64, "
                         "per-step max ln A; %.1f s wall" % dt}
    _line(METRIC, cells * K / wall, "cell-updates/s", K, 0, wall / K * 1e3, "f32",
          {"workload": "batched sweep: 256 instances x 128 modes, log-uniform n_b in [1e-3, 1e-1], "
                       "gamma in [10, 1e4], L in [5, 200], 128..8192 cells, 200 steps, noise seed 1e-6",
           "cells_per_step": cells, "plan": dict(s2.plan(), source=plan_src)},
          {"bound": "alu", "achieved": flops, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
           "frac": flops / VALU_PEAK_TFLOPS, "traffic": read_workload_traffic("batched", "bytes_per_launch"),
           "kernel": "march_kernel (persistent, xi-segmented), one launch = 200 steps of all instances, two per sweep",
           "algorithmic_flop_per_cell_update": FLOP_PER_CELL_UPDATE,
           "algorithmic_flop_per_launch": FLOP_PER_CELL_UPDATE * cells * K, "avg_launch_ms": launch * 1e3,
           "hbm": {"algorithmic_bytes_per_cell_update": 24, "achieved_GBs": 24 * rate / 1e9,
                   "frac": 24 * rate / 1e9 / HBM_PEAK_GBS}}, cpu)


GRID_FLOPS_PER_CELL = 1330.0   # four 2D FFTs per slice per stage (5 N log2 N each) x 4 stages
# HBM bytes per cell-update of the 256 x 256 pass structure: per stage the march (4 read,
# 8 written), the row transform (16 + 16), the column pass (16 + 16) and the inverse rows with
# the update (36 read, 16 written) = 128 B, four stages, plus the per-step field pass (march
# 4 + 8, rows 12 + 16, columns 16 + 24, inverse rows 24) = 104 B
GRID_BYTES_PER_CELL = 4 * 128.0 + 104.0


def bench_finite_width(args):
    """The finite-width narrow beam: 256 x 256 transverse grid over 16 c/w_p, 8192 cells,
    Gaussian sigma_r = 0.5, n_b = 0.05, gamma = 2000, centroid seed; K steps with per-step
    max ln A over the grid."""
    import numpy as np
    import torch
    from paper_2607_24234_amd import inputs, qs
    K = 10 if args.steps == 2000 else args.steps
    W = 1
    d = inputs.finite_width()
    s = qs.GridSolver(d)
    s.step(W, max_ln_a=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s.stream)
    out = s.step(K, max_ln_a=True)
    e1.record(s.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.sync_check()
    cells = s.cells
    step_s = e0.elapsed_time(e1) * 1e-3 / K
    achieved = GRID_BYTES_PER_CELL * cells / step_s / 1e9
    flops = GRID_FLOPS_PER_CELL * cells / step_s / 1e12
    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        O.build()
        n = 8
        x = (np.arange(256) - 128) * 16 / 256
        g = np.exp(-(x[None, :] ** 2 + x[:, None] ** 2) / (2 * 0.5 ** 2))
        G = O.Grid(256, 256, n, 16.0, 16.0, 200.0 / 8192, 2000.0, np.broadcast_to(0.05 * g, (n, 256, 256)).copy())
        st = O.grid_seed(G, 3, 1e-6, offset=5e-4, sigma_r=0.5)
        t = time.perf_counter()
        O.grid_run(G, 2.0, 1, st, want_fields=False, want_max=True)
        dt = time.perf_counter() - t
        cpu = {"value": 256 * 256 * n / dt, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
               "sample": "256 x 256 grid x %d cells x 1 step with the field evaluation, FP64, "
                         "single thread; %.1f s wall" % (n, dt)}
    _line(METRIC, cells * K / wall, "cell-updates/s", K, W, wall / K * 1e3, "f32",
          {"workload": "finite width: 256x256 grid over 16 c/w_p, 8192 xi cells (L = 200), Gaussian "
                       "sigma_r = 0.5, n_b/n_p = 0.05, gamma_b = 2000, d_tau = 2, centroid 1e-3 sigma_r "
                       "+ 1e-6 noise", "cells_per_step": cells,
           "max_ln_a_last": float(out["max_ln_a"][-1].item())},
          {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": read_workload_traffic("finite_width", "bytes_per_step"),
           "kernel": "one tau-step of launches (4 stage evaluations: march, row FFT, column FFT + spectral "
                     "operators, inverse row FFT + update; plus the field pass for the per-step maximum)",
           "bytes_per_cell_update": GRID_BYTES_PER_CELL, "algorithmic_flops_per_cell": GRID_FLOPS_PER_CELL,
           "tflops": flops, "valu_frac": flops / 157.3, "gpu_ms_per_step": step_s * 1e3}, cpu)


def bench_svea(args):
    """The envelope-approximation variant on the 3D spectral mode set (205,859 modes of the
    512^2 grid within |k| <= 6, 4096 cells over L = 100, n_b = 0.01, gamma = 1000, d_tau = 10),
    front-impulse seed, FP64: one library call of K steps (one launch)."""
    import numpy as np
    import torch
    from paper_2607_24234_amd import inputs, qs
    K = 20 if args.steps == 2000 else args.steps
    d = inputs.spectral3d()
    k = np.hypot(d["kx"], d["ky"])
    sv = qs.SVEASolver(d["species"], d["gamma"], k, d["length"], d["n_xi"], d["d_tau"])
    sv.step(2)
    sv.seed_impulse()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(sv.stream)
    sv.step(K)
    e1.record(sv.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cells = len(k) * d["n_xi"]
    launch = e0.elapsed_time(e1) * 1e-3
    # the state (n, m complex, FP64: 32 B) is read and written once per sweep of four steps
    achieved = 16.0 * cells * K / launch / 1e9
    ln = sv.ln_envelope()
    torch.cuda.synchronize()
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import svea as OS
        sel = np.linspace(0, len(k) - 1, 256).astype(np.int64)
        a = OS.svea_coefficient(d["species"], d["gamma"], k[sel])
        t = time.perf_counter()
        OS.run(a, d["n_xi"], d["length"] / d["n_xi"], d["d_tau"], 4, out_every=10 ** 9)
        dt = time.perf_counter() - t
        cpu = {"value": len(sel) * d["n_xi"] * 4 / dt, "unit": "cell-updates/s", "cores": torch.get_num_threads(),
               "kind": "oracle", "sample": "256 modes spread over the mode list x 4096 cells x 4 steps, FP64 numpy; "
                                           "%.1f s wall" % dt}
    _line(METRIC, cells * K / wall, "cell-updates/s", K, 2, wall / K * 1e3, "f64",
          {"workload": "envelope-approximation variant, 205,859 modes (512^2 grid, |k| <= 6) x 4096 cells, L = 100, "
                       "n_b/n_p = 0.01, gamma_b = 1000, d_tau = 10, front impulse", "cells_per_step": cells,
           "max_ln_envelope": float(ln.max().item())},
          {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
           "traffic": _scaled(read_workload_traffic("svea", "bytes_per_launch"), K / 20.0),
           "kernel": "svea_step (one lane per mode, all K steps in one launch, four steps per sweep)",
           "algorithmic_bytes_per_cell_update": 16.0,
           "algorithmic_bytes_per_launch": 16.0 * cells * K, "avg_launch_ms": launch * 1e3}, cpu)


def bench_regime(args):
    """The E/B regime diagnostic on a snapshot of the 3D run: the spectral solver (FP32, the
    3D workload) run 500 steps, its ln|E|, ln|B| snapshot (205,859 modes x 4096 cells), and the
    map with the one-skin-depth window (40 cells either side), K calls timed."""
    import numpy as np
    import torch
    from paper_2607_24234_amd import inputs, qs
    K = 20 if args.steps == 2000 else args.steps
    inst = inputs.spectral3d()
    s = qs.Solver([inst], precision=qs.QS_FP32)
    s.step(500)
    f = s.step(0, snapshots=True)
    s.sync_check()
    te = s.snapshot_view(f["ln_e"])[0]
    tb = s.snapshot_view(f["ln_b"])[0]
    n_xi, n_modes = te.shape
    w = qs.half_window_cells(1.0, inst["length"] / n_xi)
    R = torch.empty_like(te)
    F = torch.empty(n_modes, dtype=torch.int32, device="cuda")
    L = qs.lib()
    stream = torch.cuda.current_stream()
    sp = qs._stream_ptr(stream)

    def call():
        qs._check(L.qs_regime_map(qs._vp(te), qs._vp(tb), n_modes, n_xi, w, qs.QS_FP32, qs._vp(R), qs._vp(F), sp))

    for _ in range(2):
        call()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(K):
        call()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch = e0.elapsed_time(e1) * 1e-3 / K
    cells = n_modes * n_xi
    achieved = 12.0 * cells / launch / 1e9
    fr = F.cpu().numpy()
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import regime as RG
        cols = torch.as_tensor(np.linspace(0, n_modes - 1, 512).astype(np.int64), device="cuda")
        es = te[:, cols].cpu().numpy().astype(np.float64)
        bs = tb[:, cols].cpu().numpy().astype(np.float64)
        t = time.perf_counter()
        RG.first_e_cell(RG.log_ratio_map(es, bs, w))
        dt = time.perf_counter() - t
        cpu = {"value": 512 * n_xi / dt, "unit": "map cells/s", "cores": torch.get_num_threads(), "kind": "oracle",
               "sample": "512 modes spread over the mode list x 4096 cells, FP64 numpy; %.1f s wall" % dt}
    _line(METRIC, cells * K / wall, "map cells/s", K, 2, wall / K * 1e3, "f32",
          {"workload": "E/B regime map of one ln|E|, ln|B| snapshot of the 3D run after 500 steps: 205,859 modes "
                       "x 4096 cells, window of 2 x 40 + 1 cells (one skin depth either side)",
           "cells": cells, "half_window_cells": w, "modes_with_electric_region": int((fr >= 0).sum())},
          {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
           "traffic": read_workload_traffic("regime", "bytes_per_launch"),
           "kernel": "regime_stream<float> (a 64-mode block per 16-wave workgroup walks xi through LDS; "
                     "head/middle/tail window sums, no subtraction)",
           "algorithmic_bytes_per_launch": 12.0 * cells, "avg_launch_ms": launch * 1e3}, cpu)


def surrogate_vs_solver(n_cmp, cfg=None, log=None, n_stream=10_000_000):
    """The growth-map surrogate end to end: trained by the library (qs_surrogate_train, its
    default configuration unless `cfg`), then n_cmp scattered box queries answered by the
    solver alone and by AUTO at tolerance 1e-2 (network where the held-out error table
    trusts it, solver elsewhere), each timed with its own fallback and device
    synchronization; the errors are AUTO's and the network's against the solver's answers.
    The per-query comparison: the solver's time per query on that batch (its batched
    throughput) against AUTO's per query on a stream of n_stream scattered queries, error
    estimation and fallback included (on n_cmp alone AUTO's time is mostly the latency of its
    one fallback run, which does not shrink with the number of queries it answers).
    Returns (the figures, the loaded surrogate)."""
    import tempfile
    import numpy as np
    import torch
    from paper_2607_24234_amd import inputs, qs, surrogate as S

    log = log or (lambda m: None)
    path = os.path.join(tempfile.mkdtemp(prefix="qs_surrogate_"), "surrogate.bin")
    t = time.perf_counter()
    st = S.train(path, cfg)
    train_wall = time.perf_counter() - t
    log("trained in %.1f s: %s" % (train_wall, st))
    sur = S.load(path)
    q = torch.as_tensor(inputs.growth_queries(n_cmp, 3 + n_cmp), device="cuda")
    auto = torch.empty(n_cmp, device="cuda")
    used = torch.zeros(n_cmp, dtype=torch.uint8, device="cuda")
    sol = torch.empty(n_cmp, device="cuda")
    net = torch.empty(n_cmp, device="cuda")
    # warm both paths on a few queries (kernel loads, network weight packing)
    qs.growth_map(sur.net, sur.table, 1e-2, q[:64], qs.GROWTH_AUTO, auto[:64], used[:64])
    qs.growth_map(None, None, 0.0, q[:8], qs.GROWTH_SOLVER, sol[:8])
    torch.cuda.synchronize()
    t = time.perf_counter()
    qs.growth_map(sur.net, sur.table, 1e-2, q, qs.GROWTH_AUTO, auto, used)
    torch.cuda.synchronize()
    auto_s = time.perf_counter() - t
    t = time.perf_counter()
    qs.growth_map(None, None, 0.0, q, qs.GROWTH_SOLVER, sol)
    torch.cuda.synchronize()
    sol_s = time.perf_counter() - t
    qs.growth_map(sur.net, None, 0.0, q, qs.GROWTH_SURROGATE, net)
    torch.cuda.synchronize()
    da = (auto - sol).abs().cpu().numpy().astype(np.float64)
    dn = (net - sol).abs().cpu().numpy().astype(np.float64)
    n_sol = int(used.sum().item())
    log("AUTO %.4f s (%d to the solver), SOLVER %.3f s on the same %d: %.1fx" % (auto_s, n_sol, sol_s, n_cmp,
                                                                               sol_s / auto_s))
    del q, auto, used
    qb = torch.as_tensor(inputs.growth_queries(n_stream, 4 + n_stream), device="cuda")
    ob = torch.empty(n_stream, device="cuda")
    ub = torch.zeros(n_stream, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    t = time.perf_counter()
    qs.growth_map(sur.net, sur.table, 1e-2, qb, qs.GROWTH_AUTO, ob, ub)
    torch.cuda.synchronize()
    stream_s = time.perf_counter() - t
    n_fb = int(ub.sum().item())
    del qb, ob, ub
    dense = dense_map_vs_surrogate(sur, log)
    per_sol, per_auto = sol_s / n_cmp, stream_s / n_stream
    log("AUTO on a stream of %d: %.4f s (%d to the solver), %.2f ns per query against the solver's %.2f us: %.0fx"
        % (n_stream, stream_s, n_fb, per_auto * 1e9, per_sol * 1e6, per_sol / per_auto))
    fig = {"queries": n_cmp, "tol": 1e-2,
           "solver_s": sol_s, "solver_s_per_query": per_sol,
           "auto_s": auto_s, "auto_speedup_same_batch": sol_s / auto_s,
           "auto_stream": {"queries": n_stream, "s": stream_s, "to_solver": n_fb, "s_per_query": per_auto},
           "auto_speedup_per_query": per_sol / per_auto,
           "dense_map": dense,
           "auto_fraction_to_solver": n_sol / n_cmp,
           "auto_err_vs_solver": {"rms": float(np.sqrt(np.mean(da * da))), "p99": float(np.percentile(da, 99)),
                                  "max": float(da.max()), "within_tol": float(np.mean(da <= 1e-2))},
           "network_err_vs_solver": {"rms": float(np.sqrt(np.mean(dn * dn))), "p99": float(np.percentile(dn, 99)),
                                     "max": float(dn.max()), "within_tol": float(np.mean(dn <= 1e-2))},
           "heldout": st, "train_wall_s": train_wall,
           "queries_recipe": "uniform over log10 n_b in [-3, -1], log10 gamma in [1, 4], k in [0.05, 4], "
                             "xi in [0, 200], tau in [0, tau_f]"}
    return fig, sur


def dense_map_vs_surrogate(sur, log):
    """Dense growth maps of 8 beams (n_b in {0.003, 0.03} x gamma in {20, 100, 500, 2500}, the
    uniform seed S = 1e-6), each 128 modes k in [0.05, 4] x 8192 cells of width h0 = 200/8192 x
    the 201 steps 0..200 of its tau_f/200: 1.7e9 outputs.  The solver marches the 8 beams in one
    context, writing the fields of every step, and takes the windowed growth of every output
    (qs_growth_targets): about one cell-update per output.  The network (surrogate mode, no
    fallback) answers the same points as queries at the cell centres and steps, beam by beam
    (the queries of a beam are made before its timed calls).  Both timed on the device with
    their buffers allocated before."""
    import numpy as np
    import torch
    from paper_2607_24234_amd import inputs, qs

    n_k, n_xi, n_steps = 128, 8192, 200
    ks = np.linspace(0.05, 4.0, n_k)
    beams = [(nb, g) for nb in (0.003, 0.03) for g in (20.0, 100.0, 500.0, 2500.0)]
    insts = [dict(species=[inputs.ELECTRON + (nb,)], gamma=g, length=200.0, n_xi=n_xi, kx=ks, ky=None,
                  d_tau=10.0 * math.sqrt(g / nb) / n_steps, seed_kind=inputs.SEED_UNIFORM, seed_amp=1e-6, rng_seed=0)
             for nb, g in beams]
    s = qs.Solver(insts, precision=qs.QS_FP32)
    n_snap = n_steps + 1
    le = torch.empty((n_snap, s.snap_elems), dtype=torch.float32, device="cuda")
    lb = torch.empty_like(le)
    G = torch.empty_like(le)
    gi = qs.GrowthInstances(insts)
    torch.cuda.synchronize()
    t = time.perf_counter()
    s.step(n_steps, out_every=1, snapshots=True, out={"ln_e": le[:n_steps], "ln_b": lb[:n_steps]})
    s.step(0, snapshots=True, out={"ln_e": le[n_steps:], "ln_b": lb[n_steps:]})
    qs.growth_targets(gi, le, lb, G, stream=s.stream)
    torch.cuda.synchronize()
    solver_s = time.perf_counter() - t
    s.sync_check()
    del le, lb
    # beam b's block of a snapshot row: [cell][mode] at offset b * n_xi * n_k
    per = n_snap * n_xi * n_k
    h0 = 200.0 / n_xi
    kt = torch.as_tensor(ks, device="cuda")
    chunk = 10_000_000
    net_s, sq, mx, within, p99s = 0.0, 0.0, 0.0, 0.0, []
    y = torch.empty(per, dtype=torch.float32, device="cuda")
    for b, (nb, g) in enumerate(beams):
        dt = insts[b]["d_tau"]
        idx = torch.arange(per, device="cuda", dtype=torch.int64)
        m, j, st = idx % n_k, (idx // n_k) % n_xi, idx // (n_k * n_xi)
        q = torch.stack([torch.full((per,), math.log(nb), device="cuda", dtype=torch.float64),
                         torch.full((per,), math.log(g), device="cuda", dtype=torch.float64),
                         kt[m], (j.double() + 0.5) * h0, st.double() * dt], 1).float()
        del idx, m, j, st
        if b == 0:
            qs.growth_map(sur.net, None, 0.0, q[:1024], qs.GROWTH_SURROGATE, y[:1024], stream=sur.net.stream)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for a in range(0, per, chunk):
            qs.growth_map(sur.net, None, 0.0, q[a:a + chunk], qs.GROWTH_SURROGATE, y[a:a + chunk],
                          stream=sur.net.stream)
        torch.cuda.synchronize()
        net_s += time.perf_counter() - t
        del q
        ref = G.view(n_snap, len(beams), n_xi * n_k)[:, b].reshape(-1)
        fin = torch.isfinite(ref)
        d = (y - ref)[fin].double().abs()
        sq += float(d.pow(2).sum())
        mx = max(mx, float(d.max()))
        within += float((d <= 1e-2).double().sum())
        p99s.append(float(torch.quantile(d[::97].float(), 0.99)))
    n = per * len(beams)
    err = {"rms": math.sqrt(sq / n), "p99_worst_beam": max(p99s), "max": mx, "within_1e-2": within / n}
    log("dense maps (%d beams x %d modes x %d cells x %d steps = %.2e outputs): solver %.4f s, network %.3f s "
        "(solver %.0fx faster); network against the solver's maps: %s" % (len(beams), n_k, n_xi, n_snap, n, solver_s,
                                                                         net_s, net_s / solver_s, err))
    s.close()
    return {"outputs": n, "beams": [{"nb_over_np": nb, "gamma_b": g} for nb, g in beams], "modes": n_k,
            "cells": n_xi, "steps": n_snap, "solver_s": solver_s, "network_s": net_s,
            "solver_speedup": net_s / solver_s, "network_err_vs_solver": err}


def bench_surrogate(args):
    """Growth-map queries: the network's throughput on 1e8 scattered queries (the timed
    region), and AUTO against the solver on 1e5 of them."""
    import numpy as np
    import torch
    from paper_2607_24234_amd import inputs, qs

    def log(msg):
        print("[surrogate] %s" % msg, file=sys.stderr, flush=True)

    if args.surrogate_file:
        # a trained network from a file: the inference alone (no training, no solver runs)
        from paper_2607_24234_amd import surrogate as S
        fig, sur = None, S.load(args.surrogate_file)
    else:
        cfg = {"epochs": args.epochs} if args.epochs else None
        fig, sur = surrogate_vs_solver(100000, cfg, log)
    n_q = int(1e8)
    chunk = int(1e7)
    q = torch.as_tensor(inputs.growth_queries(chunk, 3), device="cuda")
    out = torch.empty(chunk, device="cuda")
    stream = sur.net.stream
    qs.growth_map(sur.net, None, 0.0, q[:1024], qs.GROWTH_SURROGATE, out[:1024], stream=stream)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n_q // chunk):
            qs.growth_map(sur.net, None, 0.0, q, qs.GROWTH_SURROGATE, out, stream=stream)
        e1.record()
    torch.cuda.synchronize()
    sur_s = e0.elapsed_time(e1) * 1e-3
    log("network %.3f s for %d queries" % (sur_s, n_q))
    qps = n_q / sur_s
    tf = 1.58e6 * qps / 1e12
    cpu = None
    if not args.no_cpu_baseline:
        # the FP64 oracle (numpy) on a sample of the same queries: inputs, baseline, network
        import oracle.growth as OG
        import oracle.mlp as OM
        P = qs.unpack_params(sur.net.get_params())
        P = [(np.asarray(W, np.float64), np.asarray(b, np.float64)) for W, b in P]
        qh = q[:20000].cpu().numpy().astype(np.float64)
        t = time.perf_counter()
        OM.forward(P, OG.features(qh))
        OG.baseline(qh)
        dt = time.perf_counter() - t
        cpu = {"value": len(qh) / dt, "unit": "queries/s", "cores": torch.get_num_threads(), "kind": "oracle",
               "sample": "%d of the same queries through the FP64 oracle (numpy: inputs, baseline, network); "
                         "%.1f s wall" % (len(qh), dt)}
    _line(METRIC, qps, "queries/s", n_q // chunk, 1, sur_s / (n_q // chunk) * 1e3, "bf16",
          {"workload": "growth-map queries uniform over log n_b in [-3, -1], log gamma in [1, 4], k in "
                       "[0.05, 4], xi in [0, 200], tau in [0, tau_f]; network 5-512x4-1 trained by the library "
                       "on the batched uniform-seed sweep (1e7 examples), held out: a second sweep (4e6)",
           "queries": n_q},
          {"bound": "mfma", "achieved": tf, "peak": 2500.0, "unit": "TFLOP/s", "frac": tf / 2500.0,
           "traffic": None, "kernel": "fused network forward (one persistent kernel, activations in LDS; "
                                      "3 bf16 512x512 layers on the matrix cores, fp32 first/last "
                                      "layers), 1.58 MFLOP per query"},
          cpu, surrogate=fig, network_s_per_query=sur_s / n_q,
          network_speedup_vs_solver=None if fig is None else (fig["solver_s"] / fig["queries"]) / (sur_s / n_q))


def bench_growth_solver(args):
    """The growth map's solver alone on args.queries scattered box queries (the method without
    the surrogate): every query marched to its own xi and tau, 32 of any beams per wavefront,
    timed around one qs_growth_map call with its host preparation and synchronization."""
    import torch
    from paper_2607_24234_amd import inputs, qs

    n = args.queries
    q = torch.as_tensor(inputs.growth_queries(n, 3 + n), device="cuda")
    out = torch.empty(n, device="cuda")
    qs.growth_map(None, None, 0.0, q[:8], qs.GROWTH_SOLVER, out[:8])
    torch.cuda.synchronize()
    t = time.perf_counter()
    qs.growth_map(None, None, 0.0, q, qs.GROWTH_SOLVER, out)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t
    assert bool(torch.isfinite(out).all())
    _line("growth-map queries answered by the solver", n / sec, "queries/s", 1, 1, sec * 1e3, "f32",
          {"workload": "growth-map queries uniform over log n_b in [-3, -1], log gamma in [1, 4], k in "
                       "[0.05, 4], xi in [0, 200], tau in [0, tau_f]; the solver alone", "queries": n},
          None, None, s_per_query=sec / n)


def bench_mlp_train(args):
    """The surrogate network's training step alone (forward, backward and AdamW on random data,
    no surrogate build) at batches of 8192, 32,768 and 65,536 examples; the line reports the
    largest."""
    import numpy as np
    import torch
    from paper_2607_24234_amd import qs

    net = qs.MLP(max_batch=65536)
    rng = np.random.default_rng(0)
    net.set_params((0.02 * rng.standard_normal(net.n_params)).astype(np.float32))
    x = torch.rand((65536 * 8, 5), device="cuda") * 2 - 1
    t = torch.randn(65536 * 8, device="cuda")
    res = {}
    for B, n in ((8192, 400), (32768, 100), (65536, 50)):
        for _ in range(5):
            net.train_step(x[:B], t[:B], 1e-4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n):
            o = (i * B) % (65536 * 8 - B)
            net.train_step(x[o:o + B], t[o:o + B], 1e-4)
        torch.cuda.synchronize()
        per = (time.perf_counter() - t0) / n
        res[B] = per
        print("[mlp_train] batch %d: %.1f us per step, %.1f TFLOP/s" % (B, per * 1e6, 4.7e6 * B / per / 1e12),
              file=sys.stderr, flush=True)
    B = 65536
    tf = 4.7e6 * B / res[B] / 1e12
    _line("surrogate training examples/s", B / res[B], "examples/s", 50, 5, res[B] * 1e3, "bf16",
          {"workload": "network 5-512x4-1 AdamW steps on random data", "batch": B},
          {"bound": "mfma", "achieved": tf, "peak": 2500.0, "unit": "TFLOP/s", "frac": tf / 2500.0, "traffic": None,
           "kernel": "one training step (forward, backward, AdamW: ~25 kernels), 4.7 MFLOP per example"},
          None, us_per_step={str(k): v * 1e6 for k, v in res.items()})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--snapshot-every", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plan", choices=["tuned", "auto"], default="tuned",
                    help="march launch plan of the spectral and batched workloads: the autotuner's "
                         "(timed candidates, a few seconds) or the built-in heuristic")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--workload", choices=["spectral3d", "batched", "finite_width", "surrogate", "svea", "regime",
                                           "growth_solver", "mlp_train"],
                    default="spectral3d",
                    help="spectral3d (default, the headline line); batched: 256-instance sweep in "
                         "one persistent launch; finite_width: 256^2 transverse grid x 8192 cells; "
                         "surrogate: growth-map queries, network against solver; svea: the envelope-"
                         "approximation variant on the 3D mode set; regime: the E/B regime map of a "
                         "3D snapshot; growth_solver: the growth map's solver alone on --queries "
                         "scattered queries; mlp_train: the network's training step alone")
    ap.add_argument("--queries", type=int, default=1_000_000,
                    help="growth_solver workload: number of scattered queries")
    ap.add_argument("--epochs", type=int, default=0,
                    help="surrogate training epochs (0: the library's default)")
    ap.add_argument("--surrogate-file", default=None, metavar="PATH",
                    help="surrogate workload: load this trained surrogate (qs_surrogate_train's file) and "
                         "time its inference only, with no training and no solver comparison")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="leave the surrogate-against-solver figures out of the default line")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (x3) and exit: "
                         "the reference reading for HBM traffic counters")
    args = ap.parse_args()

    if args.copy_calibration > 0:
        import torch
        n = args.copy_calibration
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n, "copies": 3}), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the spectral modes are independent, so a "
              "multi-GPU run is G independent shards of the mode list (see the design notes); "
              "run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2607_24234_amd import inputs, qs

    torch.cuda.set_device(0)
    if args.workload != "spectral3d":
        {"batched": bench_batched, "finite_width": bench_finite_width,
         "surrogate": bench_surrogate, "svea": bench_svea, "regime": bench_regime,
         "growth_solver": bench_growth_solver, "mlp_train": bench_mlp_train}[args.workload](args)
        return
    inst = inputs.spectral3d()
    prec = qs.QS_FP32 if args.precision == "fp32" else qs.QS_FP64
    plan, plan_src = launch_plan(args, [inst], prec, min(args.steps, args.snapshot_every) if args.snapshot_every > 0 else args.steps)
    solver = qs.Solver([inst], precision=prec, **plan)
    # snapshot rows padded to whole wavefront pieces (32 modes): every snapshot store then
    # fills whole cache lines
    solver.set_snapshot_align(32)
    n_modes, n_xi = solver.total_modes, inst["n_xi"]
    dtype = solver.dtype
    K, W = args.steps, args.warmup

    # output buffers, allocated before timing
    every = args.snapshot_every
    n_snap = -(-K // every) if every > 0 else 0
    max_buf = torch.empty((max(K, W, 1), n_modes), dtype=dtype, device="cuda")
    snap_e = torch.empty((max(n_snap, 1), solver.snap_elems), dtype=dtype, device="cuda")
    snap_b = torch.empty_like(snap_e)
    stream = solver.stream
    L = qs.lib()

    # The K steps as library calls, one per snapshot interval: the call writes ln|E|, ln|B| of
    # every cell at its first step and advances `every` steps (one persistent launch; the
    # stepping kernel writes the snapshot during its first sweep).
    chunks = []
    s = 0
    while s < K:
        e = min(K, s + every) if every > 0 else K
        chunks.append((s, e - s, every > 0))
        s = e

    def run_chunk(s0, n, snap):
        pe = snap_e[s0 // every].data_ptr() if snap else None
        pb = snap_b[s0 // every].data_ptr() if snap else None
        qs._check(L.qs_step_tau(solver.ctx, n, max(n, 1), pe, pb, max_buf[s0].data_ptr()))

    if W > 0:
        qs._check(L.qs_step_tau(solver.ctx, W, 1, None, None, max_buf[0].data_ptr()))
    torch.cuda.synchronize()
    solver.sync_check()

    # HIP events on the solver's stream around every call
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in chunks]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (s0, n, snap), (ea, eb) in zip(chunks, ev):
        ea.record(stream)
        run_chunk(s0, n, snap)
        eb.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    solver.sync_check()

    wall = t1 - t0
    dur = [ea.elapsed_time(eb) * 1e-3 for ea, eb in ev]
    cells = n_modes * n_xi
    value = cells * K / wall
    # dominant kernel: the persistent launch of one snapshot interval (its first step also
    # writes the snapshot); timed by HIP events on the solver's stream around each call
    run_steps = sum(n for (s0, n, snap) in chunks)
    run_time = sum(dur)
    avg_launch = run_time / len(chunks)
    steps_per_launch = run_steps / len(chunks)
    rate = cells * run_steps / run_time          # cell-updates/s inside the launches
    flops = FLOP_PER_CELL_UPDATE * rate / 1e12   # TFLOP/s of the method's arithmetic
    bpc = 24 if prec == qs.QS_FP32 else 48       # state bytes per cell-update, two steps per sweep
    traffic = read_traffic(args.precision, steps_per_launch)
    valu = read_valu(args.precision, steps_per_launch)
    growth = float((max_buf[K - 1].max() - max_buf[0].max()).item()) if K > 1 else 0.0
    plan = solver.plan()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": wall / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == qs.QS_FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": "spectral3d: 512x512 (k_x,k_y) grid |k|<=6 (205,859 modes), 4096 xi cells, "
                               "n_b/n_p=0.01, gamma_b=1000, length 100, d_tau=10, noise seed 1e-6",
                   "modes": n_modes, "n_xi": n_xi, "d_tau": inst["d_tau"],
                   "state": args.precision, "oscillator_carry": "f64",
                   "outputs": "per-step max ln A per mode; ln|E|,ln|B| snapshots every %d steps (rows aligned to "
                              "32 modes)" % args.snapshot_every,
                   "growth_nepers_over_run": growth,
                   "plan": dict(plan, source=plan_src)},
        "roofline": {"bound": "alu", "achieved": flops, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": flops / VALU_PEAK_TFLOPS,
                     "traffic": traffic,
                     "kernel": "march_kernel (fields; the interval's first step also writes the snapshot): one "
                               "persistent launch = one snapshot interval, all modes, two tau-steps per sweep",
                     "algorithmic_flop_per_cell_update": FLOP_PER_CELL_UPDATE,
                     "steps_per_launch": steps_per_launch,
                     "algorithmic_flop_per_launch": FLOP_PER_CELL_UPDATE * cells * steps_per_launch,
                     "avg_launch_ms": avg_launch * 1e3,
                     "gpu_ms_per_step": sum(dur) / K * 1e3,
                     "valu_issue": (None if valu is None else
                                    {"instructions_per_cell_update": valu,
                                     "frac_of_issue_peak": valu * rate / VALU_ISSUE_PEAK,
                                     "source": "rocprofv3 SQ_INSTS_VALU on the same kernel source"}),
                     "hbm": {"algorithmic_bytes_per_cell_update": bpc,
                             "achieved_GBs": bpc * rate / 1e9, "frac": bpc * rate / 1e9 / HBM_PEAK_GBS}},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_seconds)
    if not args.no_surrogate:
        # the metric's second half: the growth-map surrogate against the solver at 1e-2
        del snap_e, snap_b, max_buf
        solver.close()
        torch.cuda.empty_cache()
        out["surrogate"], _ = surrogate_vs_solver(
            100000, None, lambda m: print("[surrogate] %s" % m, file=sys.stderr, flush=True))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

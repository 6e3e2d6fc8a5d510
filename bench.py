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


def kernel_source_hash():
    p = os.path.join(ROOT, "paper_2607_24234_amd", "csrc", "qs_spectral.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def read_traffic(precision_name, steps_per_launch):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated against a plain copy) from
    the rocprofv3 counter summary, per tau-step, times the steps of one launch -- only if the
    counters were taken on the current kernel source (else None)."""
    p = os.path.join(ROOT, "profiles", "march_spectral3d_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        e = d.get(precision_name)
        if not e or e.get("kernel_sha256_16") != kernel_source_hash():
            return None
        return float(e["bytes_per_step"]) * steps_per_launch
    except Exception:
        return None


def cpu_baseline(inst, seconds=15.0):
    """The FP64 oracle timed on the host cores on a bounded sample of the same workload:
    modes spread evenly over the mode list, all 4096 cells, a fixed number of tau-steps;
    the mode count is sized from a short probe so that the timed run takes ~`seconds`."""
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
    n_modes = int(max(threads, min(len(k_all), seconds * rate / (inst["n_xi"] * steps))))
    n_modes = max(threads, n_modes // threads * threads)
    dt = timed(n_modes, steps)
    cells = n_modes * inst["n_xi"] * steps
    return {"value": cells / dt, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": "%d modes evenly spread over the 205,859-mode list x %d cells x %d steps "
                      "(FP64, per-step max ln A output), %.1f s wall" % (n_modes, inst["n_xi"], steps, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--snapshot-every", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
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
    inst = inputs.spectral3d()
    prec = qs.QS_FP32 if args.precision == "fp32" else qs.QS_FP64
    solver = qs.Solver([inst], precision=prec)
    n_modes, n_xi = solver.total_modes, inst["n_xi"]
    dtype = solver.dtype
    K, W = args.steps, args.warmup

    # output buffers, allocated before timing
    every = args.snapshot_every
    n_snap = -(-K // every) if every > 0 else 0
    max_buf = torch.empty((max(K, W, 1), n_modes), dtype=dtype, device="cuda")
    snap_e = torch.empty((max(n_snap, 1), n_modes * n_xi), dtype=dtype, device="cuda")
    snap_b = torch.empty_like(snap_e)
    stream = solver.stream
    L = qs.lib()

    # The K steps as library calls: each snapshot step alone (it also writes ln|E|, ln|B| of
    # every cell), the steps between two snapshots as one call (one persistent launch).
    chunks = []
    s = 0
    while s < K:
        if every > 0 and s % every == 0:
            chunks.append((s, 1, True))
            s += 1
        else:
            e = min(K, (s // every + 1) * every) if every > 0 else K
            chunks.append((s, e - s, False))
            s = e

    def run_chunk(s0, n, snap):
        pe = snap_e[s0 // every].data_ptr() if snap else None
        pb = snap_b[s0 // every].data_ptr() if snap else None
        qs._check(L.qs_step_tau(solver.ctx, n, 1, pe, pb, max_buf[s0].data_ptr()))

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
    bpc = 48 if prec == qs.QS_FP32 else 96
    # dominant kernel: the persistent launches that advance the steps between snapshots
    runs = [(n, d) for (s0, n, snap), d in zip(chunks, dur) if not snap]
    if not runs:
        runs = [(n, d) for (s0, n, snap), d in zip(chunks, dur)]
    run_steps = sum(n for n, _ in runs)
    run_time = sum(d for _, d in runs)
    avg_launch = run_time / len(runs)
    steps_per_launch = run_steps / len(runs)
    achieved = bpc * cells * run_steps / run_time / 1e9
    traffic = read_traffic(args.precision, steps_per_launch)
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
                   "outputs": "per-step max ln A per mode; ln|E|,ln|B| snapshots every %d steps" % args.snapshot_every,
                   "growth_nepers_over_run": growth,
                   "plan": plan},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "march_kernel (fields, no snapshot): one persistent launch = "
                               "the tau-steps between two snapshots, all modes",
                     "steps_per_launch": steps_per_launch,
                     "algorithmic_bytes_per_launch": bpc * cells * steps_per_launch,
                     "avg_launch_ms": avg_launch * 1e3,
                     "gpu_ms_per_step": sum(dur) / K * 1e3},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark of the particle hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload (the headline configuration): a 4096^2 doubly periodic grid with two
FP32 velocity snapshots from the k0 = 20 random-phase spectrum (ping-pong time
levels, dt = 1e-3), 2^24 passive tracers in split form (int cell + FP32
offset, FP64 displacement), bilinear interpolation.  One step = one RK4 step
of every particle (cell location, 4 stages of spatial + temporal
interpolation, combine, wrap, FP64 displacement), plus the cell-order re-sort
every 20 steps and the FP64 MSD/dispersion reduction every 100 steps, all
inside the timed region.  Inputs are resident in HBM before timing starts.

Prints one JSON line.  The roofline object reports the step kernel's
algorithmic bytes per launch over its average duration, measured with HIP
events on the stream it runs on, against the 8 TB/s HBM peak.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (RK4+interp) at 2^24 particles, 4096² grid; HBM GB/s fraction"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step32_spec4096_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2607_17836_amd", "csrc", "step.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def state_bytes(precision: str, kind: str) -> int:
    """Bytes of one particle's state read (and again written) per step."""
    if precision == "fp32_split":   # packed cell u32 + float2 offset + double2 displacement
        return 4 + 8 + 16 + (8 if kind == "inertial" else 0)
    return 16 + 16 + (16 if kind == "inertial" else 0)   # double2 pos + double2 disp


def field_pair_bytes(n: int, precision: str) -> int:
    return n * n * (16 if precision == "fp32_split" else 32)


def kernel_source_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def run_gpu(w, steps, warmup, lpt, **over):
    import torch
    tr = None
    try:
        from paper_2607_17836_amd import workloads
        t0 = time.perf_counter()
        tr = workloads.build_tracker(w, lpt, time_kernels=True, **over)
        tr.synchronize()
        log(f"[bench] setup of {w.name}: {time.perf_counter() - t0:.1f} s")
        tr.step(warmup, w.dt, w.stats_every)
        tr.synchronize()
        tr.get_timing(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr.step(steps, w.dt, w.stats_every)
        tr.synchronize()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        timing = tr.get_timing(reset=True)
        nstats = len(tr.get_stats(0))
        return elapsed, timing, nstats
    finally:
        if tr is not None:
            tr.close()


def cpu_baseline(w, budget_s=15.0):
    """The FP64 oracle (single thread, as written) on a bounded sample of the
    same workload: the same fields in FP64, a prefix of the same particles."""
    import oracle
    a, b, _ = w.snapshots()
    fl = oracle.grid_flow(a[0], a[1], b[0], b[1], scheme="bilinear", time_mode=oracle.PINGPONG)
    x0, y0 = oracle.init_uniform(w.species[0][4], 1 << 20)
    # calibrate on a small batch, then size the sample to ~budget_s
    sp = oracle.Species(x0[:4096], y0[:4096])
    t0 = time.perf_counter()
    oracle.run(fl, sp, 5, w.dt)
    per = (time.perf_counter() - t0) / (4096 * 5)
    count = int(min(1 << 20, max(4096, budget_s / per / 20)))
    nsteps = 20
    sp = oracle.Species(x0[:count], y0[:count])
    t0 = time.perf_counter()
    oracle.run(fl, sp, nsteps, w.dt, stats_every=10)
    el = time.perf_counter() - t0
    return {"value": count * nsteps / el, "unit": "particle-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{count} of the 2^24 tracers x {nsteps} steps on the same 4096^2 fields "
                      f"(FP64), {el:.1f} s, single-threaded C oracle"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--tile-records", type=int, default=0,
                    help="LDS tile capacity of the step kernel (0 default, -1 off)")
    ap.add_argument("--block-size", type=int, default=0, help="step-kernel block size (0 default)")
    ap.add_argument("--sort-interval", type=int, default=None,
                    help="steps between cell-order re-sorts (default: the workload's)")
    ap.add_argument("--bw-probe", action="store_true",
                    help="only run the copy/triad bandwidth probe and print its JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); this build has no "
              f"multi-GPU path", file=sys.stderr)
        sys.exit(2)

    from paper_2607_17836_amd import lpt, workloads
    lpt.load()
    probe = lpt.Tracker(16, "fp64")
    copy_gbs, triad_gbs = probe.bw_probe(1 << 30, 10)
    probe.close()
    log(f"[bench] achievable bandwidth: copy {copy_gbs:.0f} GB/s, triad {triad_gbs:.0f} GB/s")
    if args.bw_probe:
        print(json.dumps({"copy_gbps": copy_gbs, "triad_gbps": triad_gbs,
                          "bytes_per_buffer": 1 << 30, "iters": 10}), flush=True)
        return
    w = workloads.C3_SPLIT
    if args.sort_interval is not None:
        w = dataclasses.replace(w, sort_interval=args.sort_interval)
    over = dict(tile_records=args.tile_records, block_size=args.block_size)
    npart = w.particles
    elapsed, timing, nstats = run_gpu(w, args.steps, args.warmup, lpt, **over)
    value = npart * args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    kern_ms = timing["step_kernel_ms"] / max(1, timing["step_launches"])
    b_alg = 2 * state_bytes(w.precision, "tracer") + field_pair_bytes(w.n, w.precision) / npart
    bytes_per_launch = b_alg * npart
    achieved = bytes_per_launch / (kern_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tf = json.load(open(TRAFFIC_FILE))
        if tf.get("kernel_source_sha256_16") == kernel_source_hash():
            traffic = tf.get("hbm_bytes_per_launch")
    log(f"[bench] {args.steps} steps in {elapsed:.3f} s; step kernel {kern_ms * 1e3:.1f} us avg "
        f"over {timing['step_launches']} launches; sort {timing['sort_ms']:.2f} ms over "
        f"{timing['sorts']} sorts; {nstats} stats records")

    extra = {}
    if not args.no_fp64:
        w64 = workloads.Workload(w.name.replace("fp32split", "fp64"), w.n, "fp64", w.field, w.k0,
                                 w.field_seed, w.dt, w.time_mode, w.steps, w.stats_every,
                                 w.sort_interval, w.sort_tile, w.species)
        k64 = max(100, args.steps // 4)
        e64, t64, _ = run_gpu(w64, k64, min(args.warmup, 20), lpt, **over)
        extra["fp64_same_workload"] = {
            "value": npart * k64 / e64, "unit": "particle-steps/s", "steps": k64,
            "step_kernel_us": 1e3 * t64["step_kernel_ms"] / max(1, t64["step_launches"])}
        log(f"[bench] FP64 path on the same workload: {npart * k64 / e64:.3e} particle-steps/s")

    out = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": w.n, "particles": npart, "precision": w.precision,
                   "scheme": "bilinear", "dt": w.dt, "time_mode": w.time_mode,
                   "sort_interval": w.sort_interval, "sort_tile": w.sort_tile,
                   "stats_every": w.stats_every, "tile_records": args.tile_records,
                   "block_size": args.block_size, "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "step32_kernel<bilinear, tracer>",
                     "kernel_avg_us": kern_ms * 1e3, "alg_bytes_per_particle_step": b_alg,
                     "alg_bytes_per_launch": bytes_per_launch,
                     "achievable_copy_gbps": copy_gbs, "achievable_triad_gbps": triad_gbs,
                     "frac_of_copy": achieved / copy_gbs},
    }
    out.update(extra)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Launch-shape autotuner of the step path.

Picks block size and particles per thread, LDS tile capacity, re-sort
interval and key, persistent launches, fused or per-species step launches and
hipGraph chunk length for one
workload by timing candidates with HIP events on a throwaway context of that workload (``lpt_time_steps``), by
coordinate descent from the library defaults.  None of these choices changes
a per-particle result (see ``lpt_set_tuning``), only the time per step.
Results are cached in a JSON file keyed by the device, the grid, the
precision and the species mix.  The package ships a table of tunings taken
on MI355X (``tuned_mi355x.json``, written by ``python -m
paper_2607_17836_amd.autotune <workload> --out <file>``); an entry there is
used before the user cache and before tuning.
"""
from __future__ import annotations

import json
import os

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "lpt_tuning.json")
SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_mi355x.json")

# Coordinates of the descent; a tuple of names is one coordinate whose values
# set them together (two rows per thread pay only with the larger block).
SPACE = {
    ("block_size", "rows"): ((256, 1), (128, 1), (512, 1), (512, 2), (256, 2)),
    "tile_records": (0, -1, 800, 1600, 2400),
    "sort_interval": (20, 10, 12, 16, 40, 5),
    "persistent": (0, 1),
    "graph_chunk": (0, 100),
    "halo_scale": (0.125, 0.25, 0.5, 1.0),
    "fused": (1, 0, 2),
    "sort_cells": (2, 0, 1),
}


def device_key(index: int = 0) -> str:
    """The device part of a tuning key: the gfx architecture and the compute
    unit count (stable, unlike the marketing name, which depends on the
    driver's name table)."""
    import torch
    p = torch.cuda.get_device_properties(index)
    return f"{p.gcnArchName.split(':')[0]}/{p.multi_processor_count}cu"


def workload_key(w, device_name: str) -> str:
    mix = ";".join(f"{k}:{st}:{sch}:{cnt}" for k, st, sch, cnt, _ in w.species)
    return f"{device_name}|n={w.n}|{w.precision}|{w.time_mode}|dt={w.dt}|K={w.stats_every}|{mix}"


def _rows_apply(w):
    """Two rows per thread exist for FP32-split bilinear tracer bodies only
    (an inertial species of St = 0 steps as a tracer); elsewhere `rows` has
    no effect, and trying it would only let noise pick it."""
    return w.precision == "fp32_split" and any(
        sch == "bilinear" and (kind == "tracer" or st == 0.0) for kind, st, sch, _, _ in w.species)


def _valid(t, precision, rows_apply=True):
    if t.get("rows", 1) != 1 and not rows_apply:
        return False
    rec = 32 if precision == "fp64" else 16
    if t["tile_records"] > 0 and t["tile_records"] * rec > 61440:
        return False
    if t["graph_chunk"] and t["graph_chunk"] % max(1, t["sort_interval"]):
        return False
    return True


def tune(w, lpt_mod, workloads_mod, trial_steps=80, rounds=2, log=None, warm_steps=200):
    """Coordinate descent over SPACE, after `warm_steps` steps of the workload
    (so that the trials see a developed particle distribution, not the
    initial one); a candidate replaces the incumbent only if it is 1% faster
    in a second measurement of both.  Returns (best tuning dict, ms per
    step)."""
    tr = workloads_mod.build_tracker(w, lpt_mod)
    try:
        if warm_steps:
            tr.step(warm_steps, w.dt, w.stats_every)
        best = tr.get_tuning()
        best.update(sort_interval=w.sort_interval or 20, graph_chunk=0, persistent=0,
                    tile_records=0, block_size=256, halo_scale=0.125, fused=1,
                    max_workgroups=0, sort_cells=2, rows=1)

        def measure(t):
            tr.set_tuning(**t)
            tr.time_steps(max(10, trial_steps // 4), w.dt, w.stats_every)   # warm (captures graphs)
            return tr.time_steps(trial_steps, w.dt, w.stats_every) / trial_steps

        best_ms = measure(best)
        for _ in range(rounds):
            improved = False
            for name, values in SPACE.items():
                names = name if isinstance(name, tuple) else (name,)
                for v in values:
                    setting = dict(zip(names, v if isinstance(name, tuple) else (v,)))
                    if all(best[k] == x for k, x in setting.items()):
                        continue
                    cand = dict(best, **setting)
                    if not _valid(cand, w.precision, _rows_apply(w)):
                        continue
                    ms = measure(cand)
                    if log:
                        log(f"[autotune] {cand} -> {ms * 1e3:.1f} us/step")
                    if ms < best_ms * 0.99:
                        # confirm against a fresh measurement of the incumbent,
                        # so that one noisy trial does not move the choice
                        inc = measure(best)
                        again = measure(cand)
                        if log:
                            log(f"[autotune]   recheck: {again * 1e3:.1f} against "
                                f"{inc * 1e3:.1f} us/step")
                        if again < inc * 0.99:
                            best, best_ms, improved = cand, again, True
                        else:
                            best_ms = min(inc, best_ms)
            if not improved:
                break
        return best, best_ms
    finally:
        tr.close()


def load_cache(path=None):
    path = path or os.environ.get("LPT_TUNE_CACHE", DEFAULT_CACHE)
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def cached_or_tune(w, lpt_mod, workloads_mod, device_name, path=None, log=None, **kw):
    """The shipped or cached tuning of a workload on this device, tuning it
    first if neither has an entry."""
    key = workload_key(w, device_name)
    shipped = load_cache(SHIPPED)
    if key in shipped:
        return shipped[key]["tuning"], shipped[key]["ms_per_step"], True
    path = path or os.environ.get("LPT_TUNE_CACHE", DEFAULT_CACHE)
    cache = load_cache(path)
    if key in cache:
        return cache[key]["tuning"], cache[key]["ms_per_step"], True
    best, ms = tune(w, lpt_mod, workloads_mod, log=log, **kw)
    cache[key] = {"tuning": best, "ms_per_step": ms}
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass
    return best, ms, False


if __name__ == "__main__":
    import argparse
    import sys

    ap = argparse.ArgumentParser(description="tune one workload of the workloads module on GPU 0 "
                                 "and add its entry to a tuning table")
    ap.add_argument("workload", help="name of a Workload in paper_2607_17836_amd.workloads, "
                    "e.g. C4_BATCH, or a workload function and its argument, e.g. "
                    "c2_spectrum:catmull_rom")
    ap.add_argument("--out", required=True, help="JSON table to add the entry to")
    a = ap.parse_args()
    import torch

    from paper_2607_17836_amd import lpt, workloads
    name, _, arg = a.workload.partition(":")
    wl = getattr(workloads, name)(arg) if arg else getattr(workloads, name)
    dev = device_key(0)
    best, ms = tune(wl, lpt, workloads, log=lambda m: print(m, flush=True))
    table = load_cache(a.out)
    table[workload_key(wl, dev)] = {"tuning": best, "ms_per_step": ms}
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print(f"{a.workload}: {best} -> {ms * 1e3:.1f} us/step", file=sys.stderr)

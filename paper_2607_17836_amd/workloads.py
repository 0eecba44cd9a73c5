"""Named synthetic workloads (sizes, seeds, time steps, schedules).

Holds no arithmetic of the method: only the recipes that the benchmark and the
GPU tests share.  Every field comes from :mod:`paper_2607_17836_amd.synth`.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

from . import synth


@dataclass(frozen=True)
class Workload:
    name: str
    n: int                       # grid points per side
    precision: str               # "fp64" | "fp32_split"
    field: str                   # "taylor_green" | "spectrum"
    k0: float = 10.0             # spectrum peak scale
    field_seed: int = 0
    dt: float = 1e-3
    time_mode: str = "pingpong"  # "bracket" for steady fields
    steps: int = 100
    stats_every: int = 10
    sort_interval: int = 0
    sort_tile: int = 16
    # species: (kind, St, scheme, count, init seed)
    species: tuple = field(default_factory=tuple)

    def snapshots(self):
        """((ua, va), (ub, vb)) float64 arrays [n, n] and their times."""
        if self.field == "taylor_green":
            u, v, _ = synth.taylor_green(self.n)
            t_end = self.dt * self.steps
            return (u, v), (u, v), (0.0, t_end)
        a, b = synth.spectrum_snapshots(self.n, self.k0, self.field_seed, self.dt)
        return a, b, (0.0, self.dt)

    @property
    def particles(self):
        return sum(s[3] for s in self.species)


# Steady Taylor-Green on 64^2, 4096 uniform tracers, bilinear, dt = 0.01,
# 1000 steps, statistics every 10 steps.
C1_TG = Workload("tg64_fp64_bilinear_4096", 64, "fp64", "taylor_green", dt=0.01,
                 time_mode="bracket", steps=1000, stats_every=10,
                 species=(("tracer", 0.0, "bilinear", 4096, 1),))


def c2_spectrum(scheme: str, per_species: int = 1 << 20, n: int = 1024, steps: int = 500):
    """1024^2 random-phase spectrum (k0 = 10, two snapshots 0.005 apart,
    ping-pong), 2^20 tracers + 2^20 inertial particles at St = 0.1 with
    v0 = u(x0), one scheme, 500 steps of dt = 0.005."""
    return Workload(f"spec{n}_fp64_{scheme}", n, "fp64", "spectrum", k0=10.0, field_seed=2,
                    dt=0.005, steps=steps, stats_every=10, sort_interval=20,
                    species=(("tracer", 0.0, scheme, per_species, 21),
                             ("inertial", 0.1, scheme, per_species, 22)))


# The headline workload: 4096^2 FP32 fields from the k0 = 20 spectrum, 2^24
# tracers in split (int cell + FP32 offset) form, bilinear, dt = 1e-3,
# ping-pong time levels, FP64 MSD every 100 steps, cell-order re-sort every
# 16 steps (the measured optimum of re-sort cost against tile locality).
C3_SPLIT = Workload("spec4096_fp32split_bilinear_2p24", 4096, "fp32_split", "spectrum", k0=20.0,
                    field_seed=3, dt=1e-3, steps=10000, stats_every=100, sort_interval=16,
                    sort_tile=16, species=(("tracer", 0.0, "bilinear", 1 << 24, 31),))

# One GPU's share of the headline on eight: 2^21 tracers on the same full
# 4096^2 field (the field is replicated, the particles are split).
# The headline's particles and fields in FP64 positions and FP64 node records:
# the plain FP64 path on the same workload.
C3_FP64 = dataclasses.replace(C3_SPLIT, name="spec4096_fp64_bilinear_2p24", precision="fp64")

C3_SHARE8 = dataclasses.replace(C3_SPLIT, name="spec4096_fp32split_bilinear_2p21_share8",
                                species=(("tracer", 0.0, "bilinear", 1 << 21, 31),))

# Batching: 2048^2 FP32, 8 Stokes-number species, counts 2^16..2^23, scheme
# k mod 3, inertial velocities from the field.
C4_STS = (0.0, 0.01, 0.05, 0.1, 0.5, 1.0, 5.0, 10.0)
C4_BATCH = Workload("spec2048_fp32split_8species", 2048, "fp32_split", "spectrum", k0=10.0,
                    field_seed=4, dt=1e-3, steps=1000, stats_every=100, sort_interval=20,
                    species=tuple(("inertial" if st > 0 else "tracer", st,
                                   ("bilinear", "catmull_rom", "bspline")[k % 3], 1 << (16 + k),
                                   40 + k) for k, st in enumerate(C4_STS)))


def build_tracker(w: Workload, lpt_mod, **over):
    """Create a Tracker for a workload, set its snapshots and species."""
    kw = dict(precision=w.precision, sort_interval=w.sort_interval, sort_tile=w.sort_tile)
    kw.update(over)
    tr = lpt_mod.Tracker(w.n, **kw)
    a, b, (ta, tb) = w.snapshots()
    tr.set_time_mode(w.time_mode)
    tr.set_snapshot(0, ta, *a)
    tr.set_snapshot(1, tb, *b)
    for kind, st, scheme, count, seed in w.species:
        zeros = np.zeros(count)
        sid = tr.add_species(kind, st, scheme, zeros, zeros)
        tr.init_uniform(sid, seed)
    return tr

"""Host-side parts of bench.py's contract (no GPU): the algorithmic bytes and
flops per particle-step that the roofline divides, and the refusal of
multi-GPU runs."""
import dataclasses
import os
import subprocess
import sys

import bench
from paper_2607_17836_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_per_particle_step():
    # 2 x 32 B of split state (int32 cell pair 8, binary32 offsets 8, FP64
    # displacement 16) plus the 4096^2 x 16 B field pair read once, shared by
    # the particles: 80 B; the library's state (unwrapped cells and offsets,
    # no stored displacement) moves 2 x 16 + 16 = 48 B
    w = workloads.C3_SPLIT
    assert bench.alg_bytes_per_step(w) / w.particles == 2 * 32 + 4096 ** 2 * 16 / 2 ** 24 == 80.0
    assert bench.alg_bytes_per_step(w, layout=True) / w.particles == 48.0
    s = workloads.C3_SHARE8
    assert bench.alg_bytes_per_step(s) / s.particles == 2 * 32 + 4096 ** 2 * 16 / 2 ** 21 == 192.0
    d = dataclasses.replace(w, precision="fp64")
    assert bench.alg_bytes_per_step(d) / d.particles == 2 * 32 + 4096 ** 2 * 32 / 2 ** 24 == 96.0
    # the batching mix: tracers 32 B, inertial 40 B of state, 2048^2 x 16 B field
    c = workloads.C4_BATCH
    exp = sum(cnt * 2 * (40 if kind == "inertial" else 32) for kind, _, _, cnt, _ in c.species)
    assert bench.alg_bytes_per_step(c) == exp + 2048 ** 2 * 16


def test_multi_gpu_request_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_field_step_algorithmic_bytes():
    """One field step at n = 2048 moves 4 + 4 grid fields (8 n^2 bytes each)
    and 14 spectral arrays of n x 683 complex doubles (the columns inside
    the 2/3 band: 3 * 682 < 2048 <= 3 * 683)."""
    import bench
    n = 2048
    assert bench.ns_alg_bytes_per_step(n) == 8 * n * n * 8 + 14 * n * 683 * 16


def test_coupled_step_algorithmic_bytes():
    """A coupled step adds to the field step the ingest of the new level
    (u, v read once and half of each 32-byte record written: 32 n^2 bytes)
    and the FP64 tracer step (64 B per tracer, both levels of the 32-byte
    node records read once)."""
    import bench
    n, m = 2048, 1 << 20
    assert bench.coupled_alg_bytes_per_step(n, m) == (bench.ns_alg_bytes_per_step(n) + 32 * n * n
                                                       + 64 * m + 32 * n * n)


def test_flops_per_particle_step_counts():
    """The arithmetic side of the roofline: an FMA counts 2 flops.  Per stage
    a bilinear tracer takes 2 (weights) + 4 (2D products) + 32 (two
    components at two levels, 4 nodes) + 6 (blend) + 4 (stage position); a
    bicubic one 48 + 16 + 128 + 6 + 4; then the RK4 combine (14) and the
    displacement (2).  An inertial particle adds 32 per step for the drag
    and stage velocities and 14 for its velocity combine."""
    b = bench
    assert b.flops_per_particle("bilinear", False) == 4 * 48 + 16 == 208
    assert b.flops_per_particle("catmull_rom", False) == 4 * 202 + 16 == 824
    assert b.flops_per_particle("bspline", False) == 824
    assert b.flops_per_particle("bilinear", True) - 208 == 32 + 14
    w = workloads.C4_BATCH
    tot = sum(cnt * b.flops_per_particle(sch, kind == "inertial" and st > 0)
              for kind, st, sch, cnt, _ in w.species)
    assert b.alg_flops_per_step(w) == tot

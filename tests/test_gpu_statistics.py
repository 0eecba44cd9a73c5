"""GPU statistics records (Sec. 3.2 and 5.5 quantities) against closed forms
and exact sums, through the C ABI.

The per-wave partials carry M2, the sum of squared deviations of
r2 = dx^2 + dy^2 about each wave's own mean, merged pairwise (Chan, Golub &
LeVeque) in a fixed order, so a record's SEM holds its accuracy where the
spread of r2 is tiny against its mean -- uniform flow, where every particle
moves alike and the SEM is zero up to rounding.
"""
import math

import numpy as np
import pytest

from paper_2607_17836_amd import lpt

pytestmark = pytest.mark.gpu

L = 2 * np.pi


def say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("precision", ["fp64", "fp32_split"])
@pytest.mark.parametrize("block", [64, 256])
def test_uniform_flow_msd_is_ballistic_and_sem_vanishes(precision, block):
    """u = (U, V) everywhere: every tracer and every inertial particle of
    St = 0 moves by (U, V) t, so MSD_x = U^2 t^2, MSD_y = V^2 t^2, D_x =
    U^2 t / 2 and the SEM is zero; species of 1, 63, 3000 and 70001
    particles (one wave, a partial wave, several merge chunks) and re-sorts
    every 3 steps.  FP64: the SEM stays below 1e-13 of the MSD (where the
    one-pass variance (sum r2^2 - N m^2)/(N - 1) is left with cancellation
    error alone).
    FP32 split: the displacement per step is a binary32 number of cells, so
    the MSD holds to 1e-6 and the SEM equals the exact two-pass SEM of the
    downloaded displacements to 1e-6."""
    say(f"uniform-flow statistics {precision} block={block}")
    n, dt, U, V = 64, 0.01, 0.7, -0.4
    tr = lpt.Tracker(n, precision, sort_interval=3, block_size=block)
    tr.set_snapshot(0, 0.0, np.full((n, n), U), np.full((n, n), V))
    tr.set_snapshot(1, 10.0, np.full((n, n), U), np.full((n, n), V))
    counts = (1, 63, 3000, 70001)
    rng = np.random.default_rng(17)
    x0s = []
    for k, cnt in enumerate(counts):
        x0, y0 = rng.uniform(0, L, cnt), rng.uniform(0, L, cnt)
        x0s.append((x0, y0))
        if k == 1:
            tr.add_species("inertial", 0.0, "catmull_rom", x0, y0)
        else:
            tr.add_species("tracer", 0.0, ("bilinear", "bspline")[k % 2], x0, y0)
    tr.step(20, dt, stats_every=5)
    for sid, cnt in enumerate(counts):
        st = tr.get_stats(sid)
        assert len(st) == 4 and np.all(st["n"] == cnt)
        t = st["t"]
        np.testing.assert_allclose(t, [0.05, 0.1, 0.15, 0.2], rtol=1e-13)
        tol = 1e-12 if precision == "fp64" else 1e-6
        np.testing.assert_allclose(st["msd_x"], U * U * t * t, rtol=tol)
        np.testing.assert_allclose(st["msd_y"], V * V * t * t, rtol=tol)
        np.testing.assert_allclose(st["msd"], (U * U + V * V) * t * t, rtol=tol)
        np.testing.assert_allclose(st["d_x"], U * U * t / 2, rtol=tol)
        assert np.all(st["sem"] >= 0.0)
        if cnt == 1:
            assert np.all(st["sem"] == 0.0)
        if precision == "fp64":
            assert np.all(st["sem"] <= 1e-13 * st["msd"]), (sid, st["sem"] / st["msd"])
        elif cnt > 1:
            _, _, xu, yu = tr.get_positions(sid)
            x0, y0 = x0s[sid]
            dx, dy = xu - x0, yu - y0
            r2 = dx * dx + dy * dy
            m = math.fsum(r2) / cnt
            sem = math.sqrt(math.fsum((r2 - m) ** 2) / (cnt - 1) / cnt)
            assert abs(st["sem"][-1] - sem) <= 1e-6 * sem, (st["sem"][-1], sem)
    tr.close()


def test_statistics_do_not_depend_on_block_size_or_launch_shape():
    """The partials are per wave and merged in a fixed order over the wave
    index, which is the particle's slot divided by 64 whatever the block
    size, so statistics records are the same bits for 64-, 256- and
    512-thread blocks, persistent launches and fused or per-species
    launches."""
    say("statistics invariance")
    from paper_2607_17836_amd import synth
    n, dt = 128, 0.002
    (ua, va), (ub, vb) = synth.spectrum_snapshots(n, 8, 12, dt)
    outs = []
    for block, persistent, fused in ((256, 0, 1), (64, 0, 1), (512, 1, 0), (128, 1, 2)):
        tr = lpt.Tracker(n, "fp32_split", sort_interval=4, block_size=block)
        tr.set_tuning(persistent=persistent, fused=fused, max_workgroups=16 * persistent)
        tr.set_time_mode("pingpong")
        tr.set_snapshot(0, 0.0, ua, va)
        tr.set_snapshot(1, dt, ub, vb)
        for k, (kind, st, sch, cnt) in enumerate((("tracer", 0.0, "bilinear", 9000),
                                                  ("inertial", 0.1, "catmull_rom", 4097))):
            z = np.zeros(cnt)
            tr.init_uniform(tr.add_species(kind, st, sch, z, z), 50 + k)
        tr.step(12, dt, stats_every=4)
        outs.append([tr.get_stats(s) for s in (0, 1)])
        tr.close()
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            for f in ("t", "msd_x", "msd_y", "msd", "d_x", "d_y", "sem", "n"):
                np.testing.assert_array_equal(a[f], b[f], err_msg=f)

"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP64 positions within 1e-10 absolute after 10 steps (periodic
distance for wrapped coordinates), long-run MSD within 1e-3 relative; the
sort is bit-exact against a stable argsort; the FP32-split path is held to
bounds derived from binary32 rounding (see each test).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2607_17836_amd import lpt, synth, workloads

pytestmark = pytest.mark.gpu

L = 2 * np.pi
SCHEMES = ["bilinear", "catmull_rom", "bspline"]


def pdist(a, b):
    d = np.abs(np.asarray(a) - np.asarray(b)) % L
    return np.minimum(d, L - d)


def say(msg):
    print(msg, flush=True)


def bench_tracker(w):
    """A tracker of workload w in the launch configuration bench.py times:
    the shipped MI355X tuning table's entry for the workload on this device,
    if it has one (the library defaults otherwise)."""
    from paper_2607_17836_amd import autotune
    tr = workloads.build_tracker(w, lpt)
    ent = autotune.load_cache(autotune.SHIPPED).get(
        autotune.workload_key(w, autotune.device_key(0)))
    if ent:
        tr.set_tuning(**ent["tuning"])
        say(f"  launch shape of the benchmark: {ent['tuning']}")
    return tr


# --------------------------------------------------------------------------
# a3 + a4 + a5: cell location, spatial and temporal interpolation
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [37, 64])
@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("compat", [False, True])
def test_interp_fp64_matches_oracle(n, scheme, compat):
    say(f"interp fp64 n={n} scheme={scheme} compat={compat}")
    rng = np.random.default_rng(n)
    ua, va, ub, vb = (rng.standard_normal((n, n)) for _ in range(4))
    h = L / n
    x, y = rng.uniform(-2 * L, 3 * L, 3000), rng.uniform(-2 * L, 3 * L, 3000)
    if not compat:   # nodes, the seam and far images (the compatibility
        # fallback is discontinuous across its cell set, so skip them there)
        x = np.concatenate([x, np.arange(n) * h, [0.0, L, -h, L - 1e-14]])
        y = np.concatenate([y, np.arange(n)[::-1] * h, [L, 0.0, 2 * L, -1e-14]])
    tr = lpt.Tracker(n, "fp64", compat_edge=compat)
    tr.set_snapshot(0, 0.0, ua, va)
    tr.set_snapshot(1, 1.0, ub, vb)
    gu, gv = tr.interp(scheme, x, y, 0.3, 0.7)
    tr.close()
    ce = 1 if compat else 0
    eu = 0.3 * oracle.interp(ua, x, y, scheme, compat_edge=ce) + 0.7 * oracle.interp(ub, x, y, scheme, compat_edge=ce)
    ev = 0.3 * oracle.interp(va, x, y, scheme, compat_edge=ce) + 0.7 * oracle.interp(vb, x, y, scheme, compat_edge=ce)
    assert np.max(np.abs(gu - eu)) < 1e-12 and np.max(np.abs(gv - ev)) < 1e-12


@pytest.mark.parametrize("scheme", SCHEMES)
def test_interp_fp32_split_within_binary32_rounding(scheme):
    """FP32 path: fields rounded to binary32 (in cells per unit time), weights
    and sums in binary32.  Against the FP64 oracle on the binary32-rounded
    fields the error is a few binary32 ulps of sum |w| |f|: bound 2e-6 * max|f|."""
    say(f"interp fp32 scheme={scheme}")
    n = 64
    rng = np.random.default_rng(7)
    ua, va, ub, vb = (rng.standard_normal((n, n)) for _ in range(4))
    x, y = rng.uniform(0, L, 4000), rng.uniform(0, L, 4000)
    tr = lpt.Tracker(n, "fp32_split")
    tr.set_snapshot(0, 0.0, ua, va)
    tr.set_snapshot(1, 1.0, ub, vb)
    gu, gv = tr.interp(scheme, x, y, 0.25, 0.75)
    tr.close()
    r = lambda f: f.astype(np.float32).astype(np.float64)
    eu = 0.25 * oracle.interp(r(ua), x, y, scheme) + 0.75 * oracle.interp(r(ub), x, y, scheme)
    ev = 0.25 * oracle.interp(r(va), x, y, scheme) + 0.75 * oracle.interp(r(vb), x, y, scheme)
    fmax = max(np.abs(ua).max(), np.abs(ub).max())
    assert np.max(np.abs(gu - eu)) < 2e-6 * fmax
    assert np.max(np.abs(gv - ev)) < 2e-6 * fmax


# --------------------------------------------------------------------------
# a2: initial positions (SplitMix64) bit-exact
# --------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "fp32_split"])
def test_init_uniform_bit_exact(precision):
    say(f"init_uniform {precision}")
    tr = lpt.Tracker(64, precision)
    u, v, _ = synth.taylor_green(64)
    tr.set_snapshot(0, 0.0, u, v)
    tr.set_snapshot(1, 1.0, u, v)
    sid = tr.add_species("tracer", 0.0, "bilinear", np.zeros(5000), np.zeros(5000))
    tr.init_uniform(sid, 123456789)
    xw, yw, xu, yu = tr.get_positions(sid)
    tr.close()
    ex, ey = oracle.init_uniform(123456789, 5000)
    np.testing.assert_array_equal(xu, ex)
    np.testing.assert_array_equal(yu, ey)
    if precision == "fp64":
        np.testing.assert_array_equal(xw, ex)
    else:   # split form: (cell + offset) * h, offset rounded to binary32
        assert np.max(pdist(xw, ex)) < 1e-7 * (L / 64)


# --------------------------------------------------------------------------
# C1: steady Taylor-Green, 64^2, 4096 tracers, bilinear, dt 0.01
# --------------------------------------------------------------------------
def test_c1_taylor_green_parity():
    w = workloads.C1_TG
    say(f"C1 {w.name}")
    tr = workloads.build_tracker(w, lpt)
    (u, v), _, (ta, tb) = w.snapshots()
    fl = oracle.grid_flow(u, v, scheme="bilinear", t_slot=(ta, tb))
    x0, y0 = oracle.init_uniform(1, 4096)
    sp = oracle.Species(x0, y0)
    # 10 steps: positions within 1e-10
    tr.step(10, w.dt, w.stats_every)
    rec_o = oracle.run(fl, sp, 10, w.dt, stats_every=w.stats_every)
    xw, yw, xu, yu = tr.get_positions(0)
    assert np.max(pdist(xw, sp.xw)) < 1e-10 and np.max(pdist(yw, sp.yw)) < 1e-10
    assert np.max(np.abs(xu - (x0 + sp.dx))) < 1e-10 and np.max(np.abs(yu - (y0 + sp.dy))) < 1e-10
    # the remaining 990 steps: MSD series within 1e-3 relative
    tr.step(w.steps - 10, w.dt, w.stats_every)
    rec_o = np.vstack([rec_o, oracle.run(fl, sp, w.steps - 10, w.dt, t_start=10 * w.dt, step0=10,
                                         stats_every=w.stats_every)])
    st = tr.get_stats(0)
    tr.close()
    assert len(st) == w.steps // w.stats_every == len(rec_o)
    np.testing.assert_allclose(st["t"], rec_o[:, 0], rtol=1e-12)
    np.testing.assert_allclose(st["msd"], rec_o[:, 3], rtol=1e-3)
    np.testing.assert_allclose(st["msd_x"], rec_o[:, 1], rtol=1e-3)
    np.testing.assert_allclose(st["d_y"], rec_o[:, 5], rtol=1e-3)
    np.testing.assert_allclose(st["sem"], rec_o[:, 6], rtol=1e-3)
    assert np.all(st["n"] == 4096)


# --------------------------------------------------------------------------
# C2 shape: spectrum, ping-pong, tracers + inertial St = 0.1, all schemes
# --------------------------------------------------------------------------
def _spectrum_oracle_pair(w, scheme, ids=None):
    a, b, _ = w.snapshots()
    fl = oracle.grid_flow(a[0], a[1], b[0], b[1], scheme=scheme, time_mode=oracle.PINGPONG)
    sps = []
    for kind, st, _, count, seed in w.species:
        x0, y0 = oracle.init_uniform(seed, count)
        if ids is not None:
            x0, y0 = x0[ids], y0[ids]
        if kind == "inertial":
            u0, v0 = oracle.velocity(fl, x0, y0, 0.0, step=0, t_n=0.0, dt=w.dt)
            sps.append(oracle.Species(x0, y0, kind=oracle.INERTIAL, st=st, vx0=u0, vy0=v0))
        else:
            sps.append(oracle.Species(x0, y0))
    return fl, sps


@pytest.mark.parametrize("scheme", SCHEMES)
def test_c2_shape_parity_and_msd(scheme):
    """1024^2 spectrum at reduced particle count: 10-step positions within
    1e-10, particle velocities within 1e-9, and the 500-step MSD series of
    both species within 1e-3 relative."""
    w = workloads.c2_spectrum(scheme, per_species=1 << 12, n=1024, steps=500)
    say(f"C2 shape {w.name} particles={w.particles}")
    tr = workloads.build_tracker(w, lpt)
    fl, sps = _spectrum_oracle_pair(w, scheme)
    tr.step(10, w.dt, w.stats_every)
    recs = [[oracle.run(fl, sp, 10, w.dt, stats_every=w.stats_every)] for sp in sps]
    for sid, sp in enumerate(sps):
        xw, yw, xu, yu = tr.get_positions(sid)
        assert np.max(pdist(xw, sp.xw)) < 1e-10 and np.max(pdist(yw, sp.yw)) < 1e-10
        assert np.max(np.abs(xu - (sp.x0 + sp.dx))) < 1e-10
        assert np.max(np.abs(yu - (sp.y0 + sp.dy))) < 1e-10
    vx, vy = tr.get_velocities(1)
    assert np.max(np.abs(vx - sps[1].vx)) < 1e-9 and np.max(np.abs(vy - sps[1].vy)) < 1e-9
    tr.step(w.steps - 10, w.dt, w.stats_every)
    for sid, sp in enumerate(sps):
        recs[sid].append(oracle.run(fl, sp, w.steps - 10, w.dt, t_start=10 * w.dt, step0=10,
                                    stats_every=w.stats_every))
        ro = np.vstack(recs[sid])
        st = tr.get_stats(sid)
        assert len(st) == len(ro) == w.steps // w.stats_every
        np.testing.assert_allclose(st["msd"], ro[:, 3], rtol=1e-3)
        np.testing.assert_allclose(st["d_x"], ro[:, 4], rtol=1e-3)
    tr.close()


@pytest.mark.parametrize("scheme", SCHEMES)
def test_c2_full_size_sampled(scheme):
    """The full 1024^2, 2^20 + 2^20 configuration, in the benchmark's launch
    shape: 10-step positions of 512 sampled particles per species
    within 1e-10 of the oracle run on those particles alone, and the GPU
    statistics equal to exact sums of the downloaded displacements."""
    w = workloads.c2_spectrum(scheme)
    say(f"C2 full {w.name} particles={w.particles}")
    tr = bench_tracker(w)
    tr.step(10, w.dt, 10)
    ids = np.random.default_rng(99).choice(1 << 20, 512, replace=False)
    fl, sps = _spectrum_oracle_pair(w, scheme, ids)
    for sid, sp in enumerate(sps):
        oracle.run(fl, sp, 10, w.dt)
        xw, yw, xu, yu = tr.get_positions(sid)
        assert np.max(pdist(xw[ids], sp.xw)) < 1e-10 and np.max(pdist(yw[ids], sp.yw)) < 1e-10
        x0, y0 = oracle.init_uniform(w.species[sid][4], 1 << 20)
        dx, dy = xu - x0, yu - y0
        st = tr.get_stats(sid)[-1]
        mx = math.fsum(dx * dx) / dx.size
        my = math.fsum(dy * dy) / dy.size
        assert abs(st["msd_x"] - mx) <= 1e-12 * mx and abs(st["msd_y"] - my) <= 1e-12 * my
        r2 = dx * dx + dy * dy
        sem = math.sqrt(np.var(r2, ddof=1) / r2.size)
        assert abs(st["sem"] - sem) <= 1e-6 * sem
    tr.close()


@pytest.mark.parametrize("scheme", SCHEMES)
def test_c2_full_size_500_steps_sampled(scheme):
    """The full 1024^2, 2^20 + 2^20 configuration over its whole 500 steps
    in the benchmark's launch shape (a record every 10): the 512 sampled
    particles per
    species within 1e-6 of the oracle run on those particles alone, and the
    last record equal to exact sums of the downloaded displacements of the
    whole population.  The tolerance follows from the flow's sensitivity:
    perturbing the oracle's own start positions by 1e-15 (relative) moves
    its 500-step positions by up to 9e-9 (Catmull-Rom tracers), so rounding
    differences of a few ulps per step stay well inside 1e-6."""
    w = workloads.c2_spectrum(scheme)
    say(f"C2 full 500 steps {w.name} particles={w.particles}")
    tr = bench_tracker(w)
    tr.step(w.steps, w.dt, w.stats_every)
    ids = np.random.default_rng(98).choice(1 << 20, 512, replace=False)
    fl, sps = _spectrum_oracle_pair(w, scheme, ids)
    for sid, sp in enumerate(sps):
        oracle.run(fl, sp, w.steps, w.dt)
        xw, yw, xu, yu = tr.get_positions(sid)
        assert np.max(pdist(xw[ids], sp.xw)) < 1e-6 and np.max(pdist(yw[ids], sp.yw)) < 1e-6
        x0, y0 = oracle.init_uniform(w.species[sid][4], 1 << 20)
        dx, dy = xu - x0, yu - y0
        st = tr.get_stats(sid)
        assert len(st) == w.steps // w.stats_every
        mx = math.fsum(dx * dx) / dx.size
        my = math.fsum(dy * dy) / dy.size
        assert abs(st[-1]["msd_x"] - mx) <= 1e-12 * mx and abs(st[-1]["msd_y"] - my) <= 1e-12 * my
        r2 = dx * dx + dy * dy
        sem = math.sqrt(np.var(r2, ddof=1) / r2.size)
        assert abs(st[-1]["sem"] - sem) <= 1e-6 * sem
    tr.close()


# --------------------------------------------------------------------------
# Inertial closed forms on the GPU (Sec. 5.3)
# --------------------------------------------------------------------------
def test_gpu_uniform_flow_inertial_closed_form_and_table1():
    """u = (1, 0): the GPU reproduces the RK4 closed form of the linear Stokes
    drag system and the printed transit times 0.25 -> 0.5 (Table
    uniform_validation) to three decimals; St = 0 is the tracer."""
    say("uniform flow / Table 1")
    import os
    from closed_forms import rk4_linear_closed_form as _rk4_linear_closed_form
    n = 16
    tr = lpt.Tracker(n, "fp64")
    one, zero = np.ones((n, n)), np.zeros((n, n))
    tr.set_snapshot(0, 0.0, one, zero)
    tr.set_snapshot(1, 100.0, one, zero)
    rows = [l.split() for l in open(os.path.join(os.path.dirname(__file__), "golden", "table1_transit.txt"))
            if l.strip() and not l.startswith("#")]
    sts = [float(r[0]) for r in rows]
    for st in sts:
        tr.add_species("inertial", st, "bilinear", [0.25], [0.25], [0.0], [0.0])
    dt = 1e-3
    prev = np.full(len(sts), 0.25)
    found = [None] * len(sts)
    k = 0
    while any(f is None for f in found):
        tr.step(1, dt)
        k += 1
        for s in range(len(sts)):
            if found[s] is None:
                x = tr.get_positions(s)[2][0]
                if x >= 0.5:
                    found[s] = (k - 1) * dt + dt * (0.5 - prev[s]) / (x - prev[s])
                prev[s] = x
    for (st_s, t_s), t in zip(rows, found):
        assert abs(t - float(t_s)) <= 0.0005 + 1e-9, (st_s, t, t_s)
    # discrete closed form after all k steps for St = 0.1
    s = sts.index(0.1)
    xe, ve = _rk4_linear_closed_form(0.1, dt, k, 0.0, 0.0, 1.0)
    assert abs(tr.get_positions(s)[2][0] - 0.25 - xe) < 1e-12
    assert abs(tr.get_velocities(s)[0][0] - ve) < 1e-13
    tr.close()


def test_st_zero_inertial_is_bitwise_tracer():
    say("St = 0")
    n = 64
    (ua, va), (ub, vb) = synth.spectrum_snapshots(n, 10, 5, 0.01)
    x0, y0 = synth.random_points(2000, 3)
    tr = lpt.Tracker(n, "fp64")
    tr.set_time_mode("pingpong")
    tr.set_snapshot(0, 0.0, ua, va)
    tr.set_snapshot(1, 0.01, ub, vb)
    a = tr.add_species("tracer", 0.0, "catmull_rom", x0, y0)
    b = tr.add_species("inertial", 0.0, "catmull_rom", x0, y0)
    tr.step(50, 0.01)
    pa, pb = tr.get_positions(a), tr.get_positions(b)
    tr.close()
    for qa, qb in zip(pa, pb):
        np.testing.assert_array_equal(qa, qb)


# --------------------------------------------------------------------------
# a9: radix sort and sort invariance
# --------------------------------------------------------------------------
@pytest.mark.parametrize("count", [1, 63, 4097, 100003, (1 << 20) + 7])
@pytest.mark.parametrize("bits", [5, 8, 16, 24, 32])
def test_radix_sort_bit_exact(count, bits):
    say(f"radix sort count={count} bits={bits}")
    rng = np.random.default_rng(count + bits)
    keys = rng.integers(0, 1 << bits, count, dtype=np.uint64).astype(np.uint32)
    if count > 100:   # heavy ties
        keys[: count // 3] = keys[0]
    tr = lpt.Tracker(16, "fp64")
    dk = torch.from_numpy(keys.view(np.int32)).cuda()
    sk, perm = tr.radix_sort(dk, bits)
    torch.cuda.synchronize()
    tr.close()
    expect = oracle.sort_permutation(keys)
    np.testing.assert_array_equal(perm.cpu().numpy().view(np.uint32), expect.astype(np.uint32))
    np.testing.assert_array_equal(sk.cpu().numpy().view(np.uint32), keys[expect])


@pytest.mark.parametrize("precision", ["fp64", "fp32_split"])
def test_sorting_never_changes_results(precision):
    """Per-particle results are bit-identical with and without cell-order
    re-sorting, by tiles or by tiles and cells (each particle's arithmetic
    does not depend on its slot)."""
    say(f"sort invariance {precision}")
    n = 256
    (ua, va), (ub, vb) = synth.spectrum_snapshots(n, 10, 8, 0.002)
    outs = []
    for interval, cells in ((0, 0), (3, 0), (3, 1), (3, 2)):
        tr = lpt.Tracker(n, precision, sort_interval=interval, sort_tile=8)
        tr.set_tuning(sort_cells=cells)
        tr.set_time_mode("pingpong")
        tr.set_snapshot(0, 0.0, ua, va)
        tr.set_snapshot(1, 0.002, ub, vb)
        z = np.zeros(20000)
        s0 = tr.add_species("tracer", 0.0, "bilinear", z, z)
        s1 = tr.add_species("inertial", 0.3, "bspline", z[:7777], z[:7777])
        tr.init_uniform(s0, 11)
        tr.init_uniform(s1, 12)
        tr.step(25, 0.002, stats_every=5)
        outs.append((tr.get_positions(s0), tr.get_positions(s1), tr.get_velocities(s1)))
        tr.close()
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            for qa, qb in zip(a, b):
                np.testing.assert_array_equal(qa, qb)


@pytest.mark.parametrize("precision", ["fp64", "fp32_split"])
def test_lds_tiles_never_change_results(precision):
    """The step kernel's LDS field tiles are copies of the node records, so
    per-particle results are bit-identical with tiles off, with the default
    tile and with a tile too small to hold most blocks' boxes.  One inertial
    species starts ten times faster than any node, so its stage positions
    leave the tile halo and exercise the per-lane fallback to global
    gathers; halo scales from 0.125 (one cell) to 4 (the 16-cell clamp)
    change every block's box; an even-sized grid and an odd one cover both index wraps; block
    sizes of 64 to 512 threads change the tile fill's work split."""
    for n in (256, 200):
        say(f"lds tiles {precision} n={n}")
        (ua, va), (ub, vb) = synth.spectrum_snapshots(n, 10, 8, 0.002)
        outs = []
        # (tile records, halo scale, block size): the tile fill's chunks per
        # wave depend on the block's wave count, so blocks of 1, 2 and 8 waves
        # are covered too (their statistics sum in another tree: positions
        # and velocities only)
        cases = ((-1, 1.0, 0), (0, 1.0, 0), (64, 1.0, 0), (0, 0.3, 0), (0, 0.125, 0),
                 (0, 4.0, 0), (0, 1.0, 64), (0, 1.0, 128), (0, 1.0, 512))
        for tile, halo, block in cases:
            tr = lpt.Tracker(n, precision, sort_interval=4, sort_tile=8 if n == 256 else 0,
                             tile_records=tile, block_size=block)
            tr.set_tuning(halo_scale=halo)
            tr.set_time_mode("pingpong")
            tr.set_snapshot(0, 0.0, ua, va)
            tr.set_snapshot(1, 0.002, ub, vb)
            z = np.zeros(30000)
            fast = np.full(5000, 40.0)
            sids = [tr.add_species("tracer", 0.0, sch, z, z) for sch in SCHEMES]
            sids.append(tr.add_species("inertial", 0.3, "catmull_rom", z[:9000], z[:9000]))
            sids.append(tr.add_species("inertial", 0.05, "bilinear", z[:5000], z[:5000],
                                       fast, -fast))
            for k, sid in enumerate(sids):
                tr.init_uniform(sid, 100 + k)
            tr.step(13, 0.002, stats_every=13)
            outs.append([tr.get_positions(s) for s in sids] +
                        [tr.get_velocities(s) for s in sids[3:]] +
                        ([tr.get_stats(s)["msd"] for s in sids] if block == 0 else []))
            tr.close()
        for other in outs[1:]:
            for a, b in zip(outs[0], other):
                for qa, qb in zip(a, b):
                    np.testing.assert_array_equal(qa, qb)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_tile_escapees_match_oracle(scheme):
    """FP64 inertial particles launched far faster than the flow leave the
    LDS tile during their stages; their trajectories still match the oracle
    within 1e-10 after 10 steps."""
    say(f"tile escapees {scheme}")
    n, dt, count = 128, 0.002, 6000
    (ua, va), (ub, vb) = synth.spectrum_snapshots(n, 6, 9, dt)
    x0, y0 = oracle.init_uniform(77, count)
    rng = np.random.default_rng(5)
    vx0 = rng.normal(0.0, 30.0, count)
    vy0 = rng.normal(0.0, 30.0, count)
    tr = lpt.Tracker(n, "fp64", sort_interval=2, sort_tile=8)
    tr.set_time_mode("pingpong")
    tr.set_snapshot(0, 0.0, ua, va)
    tr.set_snapshot(1, dt, ub, vb)
    sid = tr.add_species("inertial", 0.02, scheme, x0, y0, vx0, vy0)
    tr.step(10, dt)
    xw, yw, xu, yu = tr.get_positions(sid)
    vx, vy = tr.get_velocities(sid)
    tr.close()
    fl = oracle.grid_flow(ua, va, ub, vb, scheme=scheme, time_mode=oracle.PINGPONG)
    sp = oracle.Species(x0, y0, kind=oracle.INERTIAL, st=0.02, vx0=vx0, vy0=vy0)
    oracle.run(fl, sp, 10, dt)
    assert np.max(pdist(xw, sp.xw)) < 1e-10 and np.max(pdist(yw, sp.yw)) < 1e-10
    assert np.max(np.abs(xu - (x0 + sp.dx))) < 1e-10
    assert np.max(np.abs(vx - sp.vx)) < 1e-8 and np.max(np.abs(vy - sp.vy)) < 1e-8


@pytest.mark.parametrize("cells", [0, 1, 2])
@pytest.mark.parametrize("precision", ["fp64", "fp32_split"])
def test_sort_produces_stable_tile_order(precision, cells):
    """Right after initialisation (slots in original order), lpt_sort leaves
    the slots in the stable argsort order of the cell-tile keys of the
    stored cells, species by species: tiles alone (sort_cells 0), or tiles
    and then the cells row-major inside each tile (1, and 2, whose first
    re-sort after placement uses that key)."""
    say(f"sort order {precision} cells={cells}")
    n = 128
    u, v, _ = synth.taylor_green(n)
    tr = lpt.Tracker(n, precision, sort_tile=8)
    tr.set_tuning(sort_cells=cells)
    tr.set_snapshot(0, 0.0, u, v)
    tr.set_snapshot(1, 1.0, u, v)
    z = np.zeros(30000)
    s0 = tr.add_species("tracer", 0.0, "bilinear", z, z)
    s1 = tr.add_species("tracer", 0.0, "bilinear", z[:5000], z[:5000])
    tr.init_uniform(s0, 5)
    tr.init_uniform(s1, 6)
    tr.sort()
    orders = [tr.get_order(s0), tr.get_order(s1)]
    tr.close()
    for seed, count, order in ((5, 30000, orders[0]), (6, 5000, orders[1])):
        x0, y0 = oracle.init_uniform(seed, count)
        if precision == "fp64":
            ci, cj = oracle.cells_of(n, x0), oracle.cells_of(n, y0)
        else:   # the split path stores floor(x * n / L)
            ci = np.floor(x0 * (n / L)).astype(np.int32)
            cj = np.floor(y0 * (n / L)).astype(np.int32)
        keys = oracle.cell_keys(n, 8, ci, cj, coarse=cells == 0)
        np.testing.assert_array_equal(order, oracle.sort_permutation(keys))


# --------------------------------------------------------------------------
# a8: statistics against exact sums
# --------------------------------------------------------------------------
def test_stats_match_exact_sums_of_displacements():
    say("stats vs fsum")
    n = 128
    (ua, va), (ub, vb) = synth.spectrum_snapshots(n, 10, 9, 0.01)
    tr = lpt.Tracker(n, "fp32_split", sort_interval=7)
    tr.set_time_mode("pingpong")
    tr.set_snapshot(0, 0.0, ua, va)
    tr.set_snapshot(1, 0.01, ub, vb)
    z = np.zeros(99999)
    sid = tr.add_species("tracer", 0.0, "catmull_rom", z, z)
    tr.init_uniform(sid, 77)
    tr.step(40, 0.01, stats_every=20)
    st = tr.get_stats(sid)
    _, _, xu, yu = tr.get_positions(sid)
    tr.close()
    x0, y0 = oracle.init_uniform(77, 99999)
    dx, dy = xu - x0, yu - y0
    mx, my = math.fsum(dx * dx) / dx.size, math.fsum(dy * dy) / dy.size
    last = st[-1]
    assert len(st) == 2 and abs(last["t"] - 0.4) < 1e-14
    assert abs(last["msd_x"] - mx) <= 1e-12 * mx and abs(last["msd_y"] - my) <= 1e-12 * my
    assert abs(last["d_x"] - mx / 0.8) <= 1e-12 * mx
    r2 = dx * dx + dy * dy
    assert abs(last["sem"] - math.sqrt(np.var(r2, ddof=1) / r2.size)) <= 1e-6 * last["sem"]


# --------------------------------------------------------------------------
# NEXT: stream-function snapshots (eq. particle_velocity_reconstruction)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("scheme", SCHEMES)
def test_psi_snapshot_matches_psi_interpolation_with_fd(scheme):
    """Tracers driven by psi snapshots follow the paper's production path
    (psi interpolated at x +- dx, y +- dy, then centred differences): the GPU
    forms the grid differences once per snapshot, the oracle interpolates psi
    four times per stage; positions agree within 1e-10 after 10 steps."""
    say(f"psi snapshots {scheme}")
    n = 128
    _, _, (pa, pb) = synth.spectrum_snapshots(n, 8, 13, 0.01, with_psi=True)
    x0, y0 = synth.random_points(3000, 14)
    tr = lpt.Tracker(n, "fp64")
    tr.set_time_mode("pingpong")
    tr.set_snapshot_psi(0, 0.0, pa)
    tr.set_snapshot_psi(1, 0.01, pb)
    sid = tr.add_species("tracer", 0.0, scheme, x0, y0)
    tr.step(10, 0.01)
    xw, yw, xu, yu = tr.get_positions(sid)
    tr.close()
    fl = oracle.psi_flow(pa, pb, scheme=scheme, time_mode=oracle.PINGPONG)
    sp = oracle.Species(x0, y0)
    oracle.run(fl, sp, 10, 0.01)
    assert np.max(pdist(xw, sp.xw)) < 1e-10 and np.max(pdist(yw, sp.yw)) < 1e-10


# --------------------------------------------------------------------------
# FP32 split precision (reported error, sanity bound)
# --------------------------------------------------------------------------
def test_fp32_split_tracks_fp64_oracle():
    """256^2 spectrum (k0 = 20), 4096 tracers, 100 steps of 1e-3.  Against the
    oracle on the binary32-rounded fields, the split path's error comes from
    binary32 velocities (relative 2^-24 per stage, ~100 steps): bound
    1e-6 absolute on positions; MSD within 1e-4 relative."""
    say("fp32 split vs oracle")
    n = 256
    (ua, va), (ub, vb) = synth.spectrum_snapshots(n, 20, 3, 1e-3)
    r = lambda f: f.astype(np.float32).astype(np.float64)
    tr = lpt.Tracker(n, "fp32_split", sort_interval=10)
    tr.set_time_mode("pingpong")
    tr.set_snapshot(0, 0.0, ua, va)
    tr.set_snapshot(1, 1e-3, ub, vb)
    z = np.zeros(4096)
    sid = tr.add_species("tracer", 0.0, "bilinear", z, z)
    sin = tr.add_species("inertial", 0.05, "catmull_rom", z, z)
    tr.init_uniform(sid, 31)
    tr.init_uniform(sin, 32)
    tr.step(100, 1e-3, stats_every=50)
    xw, yw, xu, yu = tr.get_positions(sid)
    st = tr.get_stats(sid)
    iw = tr.get_positions(sin)
    ivx, ivy = tr.get_velocities(sin)
    tr.close()
    fl = oracle.grid_flow(r(ua), r(va), r(ub), r(vb), time_mode=oracle.PINGPONG)
    x0, y0 = oracle.init_uniform(31, 4096)
    sp = oracle.Species(x0, y0)
    rec = oracle.run(fl, sp, 100, 1e-3, stats_every=50)
    err = max(np.max(pdist(xw, sp.xw)), np.max(pdist(yw, sp.yw)))
    say(f"fp32 split tracer max position error after 100 steps: {err:.3e}")
    assert err < 1e-6
    assert np.max(np.abs(xu - (x0 + sp.dx))) < 1e-6
    np.testing.assert_allclose(st["msd"], rec[:, 3], rtol=1e-4)
    flc = oracle.grid_flow(r(ua), r(va), r(ub), r(vb), scheme="catmull_rom", time_mode=oracle.PINGPONG)
    x1, y1 = oracle.init_uniform(32, 4096)
    u0, v0 = oracle.velocity(flc, x1, y1, 0.0, step=0, t_n=0.0, dt=1e-3)
    si = oracle.Species(x1, y1, kind=oracle.INERTIAL, st=0.05, vx0=u0, vy0=v0)
    oracle.run(flc, si, 100, 1e-3)
    erri = max(np.max(pdist(iw[0], si.xw)), np.max(pdist(iw[1], si.yw)))
    errv = max(np.max(np.abs(ivx - si.vx)), np.max(np.abs(ivy - si.vy)))
    say(f"fp32 split inertial errors: position {erri:.3e}, velocity {errv:.3e}")
    assert erri < 1e-6 and errv < 1e-5


def test_c3_full_size_sampled():
    """The headline configuration as the benchmark runs it (4096^2 FP32
    fields, 2^24 split tracers, the benchmark's launch shape: 512-slot blocks
    of two rows per thread, re-sorted every 16 steps, so the run includes two
    permuting steps): after 20 steps, 1024 sampled particles lie within 1e-6
    of the FP64 oracle on the binary32-rounded fields."""
    w = workloads.C3_SPLIT
    say(f"C3 full {w.name}")
    tr = bench_tracker(w)
    tr.step(20, w.dt, w.stats_every)
    xw, yw, xu, yu = tr.get_positions(0)
    tr.close()
    a, b, _ = w.snapshots()
    r = lambda f: f.astype(np.float32).astype(np.float64)
    fl = oracle.grid_flow(r(a[0]), r(a[1]), r(b[0]), r(b[1]), time_mode=oracle.PINGPONG)
    ids = np.random.default_rng(5).choice(1 << 24, 1024, replace=False)
    x0, y0 = oracle.init_uniform(31, 1 << 24)
    sp = oracle.Species(x0[ids], y0[ids])
    oracle.run(fl, sp, 20, w.dt)
    err = max(np.max(pdist(xw[ids], sp.xw)), np.max(pdist(yw[ids], sp.yw)))
    say(f"C3 sampled max position error after 20 steps: {err:.3e}")
    assert err < 1e-6


def test_c3_fp64_full_size_sampled():
    """The headline configuration on the FP64 path (4096^2 FP64 node
    records, 2^24 FP64 tracers), in its own benchmark launch shape (an
    800-record tile, re-sorts every 10 steps, so the run includes a permuting
    step): after 10 steps, 1024 sampled particles within 1e-10 of the FP64
    oracle, wrapped and unwrapped."""
    w = workloads.C3_FP64
    say(f"C3 FP64 full {w.name}")
    tr = bench_tracker(w)
    tr.step(10, w.dt, w.stats_every)
    xw, yw, xu, yu = tr.get_positions(0)
    tr.close()
    a, b, _ = w.snapshots()
    fl = oracle.grid_flow(a[0], a[1], b[0], b[1], time_mode=oracle.PINGPONG)
    ids = np.random.default_rng(7).choice(1 << 24, 1024, replace=False)
    x0, y0 = oracle.init_uniform(31, 1 << 24)
    sp = oracle.Species(x0[ids], y0[ids])
    oracle.run(fl, sp, 10, w.dt)
    ox, oy = sp.unwrapped()
    err = max(np.max(pdist(xw[ids], sp.xw)), np.max(pdist(yw[ids], sp.yw)))
    erru = max(np.max(np.abs(xu[ids] - ox)), np.max(np.abs(yu[ids] - oy)))
    say(f"C3 FP64 sampled max position error after 10 steps: {err:.3e} (unwrapped {erru:.3e})")
    assert err < 1e-10 and erru < 1e-10


def test_c4_full_size_sampled():
    """The batching configuration at full size (2048^2 FP32 fields, 8 species
    of 2^16 .. 2^23 particles, Stokes numbers 0 .. 10, scheme k mod 3; in the
    benchmark's launch shape, re-sorted at the first step): after 10
    steps, 64 sampled particles of every species match the FP64 oracle on the
    binary32-rounded fields within the binary32 bounds of the split path
    (positions 1e-6; velocities 1e-5, whose initial values the GPU forms in
    binary32)."""
    w = workloads.C4_BATCH
    say(f"C4 full {w.name}")
    nsteps = 10
    tr = bench_tracker(w)
    tr.step(nsteps, w.dt, w.stats_every)
    got = []
    for k, (kind, st, scheme, cnt, seed) in enumerate(w.species):
        pos = tr.get_positions(k)
        vel = tr.get_velocities(k) if kind == "inertial" else None
        got.append((pos, vel))
    tr.close()
    a, b, _ = w.snapshots()
    r = lambda f: f.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(6)
    for k, (kind, st, scheme, cnt, seed) in enumerate(w.species):
        fl = oracle.grid_flow(r(a[0]), r(a[1]), r(b[0]), r(b[1]), scheme=scheme,
                              time_mode=oracle.PINGPONG)
        ids = rng.choice(cnt, 64, replace=False)
        x0, y0 = oracle.init_uniform(seed, cnt)
        x0, y0 = x0[ids], y0[ids]
        if kind == "inertial":
            u0, v0 = oracle.velocity(fl, x0, y0, 0.0, step=0, t_n=0.0, dt=w.dt)
            sp = oracle.Species(x0, y0, kind=oracle.INERTIAL, st=st, vx0=u0, vy0=v0)
        else:
            sp = oracle.Species(x0, y0)
        oracle.run(fl, sp, nsteps, w.dt)
        (xw, yw, xu, yu), vel = got[k]
        err = max(np.max(pdist(xw[ids], sp.xw)), np.max(pdist(yw[ids], sp.yw)))
        say(f"C4 species {k} ({kind}, St {st}, {scheme}): position error {err:.3e}")
        assert err < 1e-6, (k, err)
        if vel is not None:
            errv = max(np.max(np.abs(vel[0][ids] - sp.vx)), np.max(np.abs(vel[1][ids] - sp.vy)))
            assert errv < 1e-5, (k, errv)


# --------------------------------------------------------------------------
# Error conventions: status codes, state unchanged
# --------------------------------------------------------------------------
def test_error_paths_leave_state_unchanged():
    say("error paths")
    n = 32
    u, v, _ = synth.taylor_green(n)
    tr = lpt.Tracker(n, "fp64")
    x0, y0 = synth.random_points(100, 1)
    with pytest.raises(lpt.LptError) as e:
        tr.add_species("inertial", 0.5, "bilinear", x0, y0)   # v0 from field, no snapshots
    assert e.value.status == lpt.E_STATE
    tr.set_snapshot(0, 0.0, u, v)
    with pytest.raises(lpt.LptError) as e:
        tr.step(1, 0.01)
    assert e.value.status == lpt.E_STATE                       # no species
    tr.set_snapshot(1, 0.1, u, v)
    sid = tr.add_species("tracer", 0.0, "bilinear", x0, y0)
    for bad in [(-1, 0.01, 0), (1, 0.0, 0), (1, float("nan"), 0), (1, 0.01, -1)]:
        with pytest.raises(lpt.LptError) as e:
            tr.step(*bad)
        assert e.value.status == lpt.E_ARG
    with pytest.raises(lpt.LptError) as e:
        tr.add_species("tracer", -1.0, "bilinear", x0, y0)
    assert e.value.status == lpt.E_ARG
    tr.step(5, 0.01)
    before = tr.get_positions(sid)
    with pytest.raises(lpt.LptError) as e:
        tr.step(10, 0.01)                                      # would leave [0, 0.1]
    assert e.value.status == lpt.E_RANGE
    assert tr.get_time()[0] == 5
    for a, b in zip(before, tr.get_positions(sid)):
        np.testing.assert_array_equal(a, b)
    with pytest.raises(lpt.LptError) as e:
        tr.add_species("tracer", 0.0, "bilinear", x0, y0)      # after the first step
    assert e.value.status == lpt.E_STATE
    tr.set_time_mode("pingpong")
    with pytest.raises(lpt.LptError) as e:
        tr.step(1, 0.05)                                       # dt != snapshot spacing
    assert e.value.status == lpt.E_ARG
    with pytest.raises(lpt.LptError) as e:
        tr.get_velocities(sid)                                 # tracer: no velocity
    assert e.value.status == lpt.E_STATE
    tr.close()

"""GPU derivatives of the FP64 tracer map (through the C ABI) against the
oracle's independent forward tangent and full-tape reverse sweep.

Tolerances: dL/dx0 and F within 1e-9 relative to their scale (both sides
differentiate the same FP64 map; they differ only in rounding order), grid
gradients within 1e-10 of their largest entry (FP64 atomics sum in
scheduling order)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2607_17836_amd import lpt, synth

pytestmark = pytest.mark.gpu

L = 2 * np.pi
SCHEMES = ["bilinear", "catmull_rom", "bspline"]


def say(msg):
    print(msg, flush=True)


def _setup(n, scheme, time_mode, x0, y0, fields, t_slot, block=0):
    (ua, va), (ub, vb) = fields
    tr = lpt.Tracker(n, "fp64", block_size=block)
    tr.set_time_mode(time_mode)
    tr.set_snapshot(0, t_slot[0], ua, va)
    tr.set_snapshot(1, t_slot[1], ub, vb)
    tr.add_species("tracer", 0.0, scheme, x0, y0)
    return tr


def _scale(a):
    return max(1.0, float(np.max(np.abs(a))))


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("time_mode", ["pingpong", "bracket"])
def test_adjoint_and_grid_gradient_match_oracle(scheme, time_mode):
    n, dt, nsteps, count = 48, 0.01, 37, 3000
    say(f"adjoint {scheme} {time_mode}")
    fields = synth.spectrum_snapshots(n, 5, 4, dt)
    t_slot = (0.0, dt) if time_mode == "pingpong" else (0.0, nsteps * dt)
    x0, y0 = oracle.init_uniform(21, count)
    rng = np.random.default_rng(8)
    a, b = rng.normal(size=count), rng.normal(size=count)
    tr = _setup(n, scheme, time_mode, x0, y0, fields, t_slot)
    tr.forward_checkpointed(nsteps, dt, 10)
    gx, gy, gU = tr.adjoint(a, b)
    tr.close()
    (ua, va), (ub, vb) = fields
    tm = oracle.PINGPONG if time_mode == "pingpong" else oracle.BRACKET
    fl = oracle.grid_flow(ua, va, ub, vb, scheme=scheme, time_mode=tm, t_slot=t_slot)
    ox, oy, oU = oracle.adjoint(fl, x0, y0, a, b, nsteps, dt)
    assert np.max(np.abs(gx - ox)) < 1e-9 * _scale(ox)
    assert np.max(np.abs(gy - oy)) < 1e-9 * _scale(oy)
    assert np.max(np.abs(gU - oU)) < 1e-10 * _scale(oU)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_jacobian_matches_oracle_forward_tangent(scheme):
    n, dt, nsteps, count = 64, 0.01, 50, 4000
    say(f"jacobian {scheme}")
    fields = synth.spectrum_snapshots(n, 6, 5, dt)
    x0, y0 = oracle.init_uniform(31, count)
    tr = _setup(n, scheme, "pingpong", x0, y0, fields, (0.0, dt))
    tr.forward_checkpointed(nsteps, dt, 16)
    F = tr.jacobian()
    xw, yw, xu, yu = tr.get_positions(0)
    tr.close()
    (ua, va), (ub, vb) = fields
    fl = oracle.grid_flow(ua, va, ub, vb, scheme=scheme, time_mode=oracle.PINGPONG)
    sp = oracle.Species(x0, y0)
    Fo = oracle.tangent(fl, sp, nsteps, dt)
    assert np.max(np.abs(F - Fo)) < 1e-9 * _scale(Fo)
    # the checkpointed forward is an ordinary run
    assert np.max(np.abs(xu - (x0 + sp.dx))) < 1e-10


def test_checkpoint_spacing_and_block_size_do_not_change_results():
    """Recomputed segments repeat the forward trajectory bit for bit, so the
    adjoint of the particles does not depend on the checkpoint spacing or the
    block size; the grid gradient agrees to atomic-summation rounding."""
    n, dt, nsteps, count = 32, 0.01, 24, 5000
    fields = synth.spectrum_snapshots(n, 4, 6, dt)
    x0, y0 = oracle.init_uniform(41, count)
    rng = np.random.default_rng(9)
    a, b = rng.normal(size=count), rng.normal(size=count)
    outs = []
    for every, block in ((1, 0), (5, 128), (24, 512), (100, 0)):
        say(f"ckpt every {every} block {block}")
        tr = _setup(n, "catmull_rom", "pingpong", x0, y0, fields, (0.0, dt), block)
        tr.forward_checkpointed(nsteps, dt, every)
        outs.append(tr.adjoint(a, b))
        tr.close()
    for gx, gy, gU in outs[1:]:
        np.testing.assert_array_equal(gx, outs[0][0])
        np.testing.assert_array_equal(gy, outs[0][1])
        assert np.max(np.abs(gU - outs[0][2])) < 1e-12 * _scale(outs[0][2])


@pytest.mark.parametrize("scheme", ["bilinear", "catmull_rom"])
def test_cell_ordered_run_matches_oracle_and_unsorted(scheme):
    """With re-sorting enabled every checkpoint segment (three here) starts
    from cell order, so each block's grid gradient is summed in an LDS box
    of its tile, and the sweep carries the adjoint vectors back through each
    segment's permutation: per-particle adjoints and Jacobians stay
    bit-identical to the unsorted run, the grid gradient agrees with it to
    atomic-summation rounding and with the oracle to the usual bound."""
    n, dt, nsteps = 128, 0.01, 30
    say(f"cell-ordered adjoint {scheme}")
    fields = synth.spectrum_snapshots(n, 6, 12, dt)
    x0, y0 = synth.lattice_points(n, 128)
    count = x0.size
    rng = np.random.default_rng(12)
    a, b = rng.normal(size=count), rng.normal(size=count)
    outs = []
    for interval in (0, 5):
        (ua, va), (ub, vb) = fields
        tr = lpt.Tracker(n, "fp64", sort_interval=interval, sort_tile=16)
        tr.set_time_mode("pingpong")
        tr.set_snapshot(0, 0.0, ua, va)
        tr.set_snapshot(1, dt, ub, vb)
        tr.add_species("tracer", 0.0, scheme, x0, y0)
        tr.forward_checkpointed(nsteps, dt, 10)
        outs.append(tr.adjoint(a, b) + (tr.jacobian(),))
        tr.close()
    np.testing.assert_array_equal(outs[1][0], outs[0][0])
    np.testing.assert_array_equal(outs[1][1], outs[0][1])
    np.testing.assert_array_equal(outs[1][3], outs[0][3])
    assert np.max(np.abs(outs[1][2] - outs[0][2])) < 1e-12 * _scale(outs[0][2])
    (ua, va), (ub, vb) = fields
    fl = oracle.grid_flow(ua, va, ub, vb, scheme=scheme, time_mode=oracle.PINGPONG)
    ox, oy, oU = oracle.adjoint(fl, x0, y0, a, b, nsteps, dt)
    assert np.max(np.abs(outs[1][0] - ox)) < 1e-9 * _scale(ox)
    assert np.max(np.abs(outs[1][2] - oU)) < 1e-10 * _scale(oU)


def test_autograd_function_matches_central_differences():
    """torch.autograd through LptTrajectory: gradients for the initial
    positions and both snapshots against central differences of the
    library's own forward map (Catmull-Rom: smooth in space)."""
    n, dt, nsteps, count = 32, 0.01, 20, 64
    say("autograd")
    dev = "cuda"
    (ua, va), (ub, vb) = synth.spectrum_snapshots(n, 4, 7, dt)
    Ua = torch.tensor(np.stack([ua, va]), device=dev, requires_grad=True)
    Ub = torch.tensor(np.stack([ub, vb]), device=dev, requires_grad=True)
    x0n, y0n = oracle.init_uniform(51, count)
    x0 = torch.tensor(x0n, device=dev, requires_grad=True)
    y0 = torch.tensor(y0n, device=dev, requires_grad=True)
    w = torch.tensor(np.random.default_rng(3).normal(size=(2, count)), device=dev)
    args = (nsteps, dt, "catmull_rom", 6, "pingpong", (0.0, dt))
    xT, yT = lpt.LptTrajectory.apply(x0, y0, Ua, Ub, *args)
    loss = (w[0] * xT + w[1] * yT).sum()
    loss.backward()

    def L(x0_, y0_, Ua_, Ub_):
        with torch.no_grad():
            a, b = lpt.LptTrajectory.apply(x0_, y0_, Ua_, Ub_, *args)
            return float((w[0] * a + w[1] * b).sum())

    eps = 1e-6
    for k in (0, 17, 63):
        e = torch.zeros(count, dtype=torch.float64, device=dev)
        e[k] = eps
        fd = (L(x0.detach() + e, y0.detach(), Ua.detach(), Ub.detach()) -
              L(x0.detach() - e, y0.detach(), Ua.detach(), Ub.detach())) / (2 * eps)
        assert abs(fd - float(x0.grad[k])) < 1e-6 * max(1.0, abs(fd))
    gUa = Ua.grad.cpu().numpy()
    for idx in np.argsort(np.abs(gUa).ravel())[-3:]:
        c, j, i = np.unravel_index(idx, gUa.shape)
        e = torch.zeros_like(Ua)
        e[c, j, i] = eps
        fd = (L(x0.detach(), y0.detach(), Ua.detach() + e, Ub.detach()) -
              L(x0.detach(), y0.detach(), Ua.detach() - e, Ub.detach())) / (2 * eps)
        assert abs(fd - gUa[c, j, i]) < 1e-6 * max(1.0, abs(fd))


def test_ftle_field_on_a_lattice_matches_oracle():
    """C5-shaped (reduced): a Taylor-Green field plus a 0.1-amplitude
    spectral perturbation, tracers on the cell-centre lattice, steady
    snapshots; FTLE from the GPU Jacobian equals the oracle's on a sample."""
    n, dt, nsteps = 256, 0.01, 200
    say("ftle lattice")
    u, v, _ = synth.taylor_green(n)
    (pu, pv), _ = synth.spectrum_snapshots(n, 10, 5, dt)
    u, v = u + 0.1 * pu, v + 0.1 * pv
    x0, y0 = synth.lattice_points(n, 128)
    tr = _setup(n, "bilinear", "bracket", x0, y0, ((u, v), (u, v)), (0.0, nsteps * dt))
    tr.forward_checkpointed(nsteps, dt, 20)
    F = tr.jacobian()
    sig, F2 = tr.ftle(with_jacobian=True)   # the library's FTLE (lpt_ftle)
    tr.close()
    np.testing.assert_array_equal(F2, F)
    ids = np.random.default_rng(4).choice(x0.size, 96, replace=False)
    fl = oracle.grid_flow(u, v, scheme="bilinear", t_slot=(0.0, nsteps * dt))
    Fo = oracle.tangent(fl, oracle.Species(x0[ids], y0[ids]), nsteps, dt)
    assert np.max(np.abs(F[ids] - Fo)) < 1e-9 * _scale(Fo)
    np.testing.assert_allclose(sig[ids], oracle.ftle(Fo, nsteps * dt), rtol=1e-9, atol=1e-12)
    assert np.all(np.isfinite(sig))


def test_derivative_error_paths():
    n = 16
    u, v, _ = synth.taylor_green(n)
    x0, y0 = oracle.init_uniform(1, 100)
    tr = lpt.Tracker(n, "fp32_split")
    tr.set_snapshot(0, 0.0, u, v)
    tr.set_snapshot(1, 1.0, u, v)
    tr.add_species("tracer", 0.0, "bilinear", x0, y0)
    with pytest.raises(lpt.LptError) as e:
        tr.forward_checkpointed(5, 0.01, 2)
    assert e.value.status == lpt.E_STATE
    tr.close()
    tr = lpt.Tracker(n, "fp64")
    tr.set_snapshot(0, 0.0, u, v)
    tr.set_snapshot(1, 1.0, u, v)
    tr.add_species("tracer", 0.0, "bilinear", x0, y0)
    with pytest.raises(lpt.LptError) as e:
        tr.jacobian()
    assert e.value.status == lpt.E_STATE
    tr.forward_checkpointed(5, 0.01, 2)
    tr.step(1, 0.01)
    with pytest.raises(lpt.LptError) as e:
        tr.adjoint(np.ones(100), np.ones(100))
    assert e.value.status == lpt.E_STATE
    with pytest.raises(lpt.LptError) as e:
        tr.forward_checkpointed(5, 0.01, 0)
    assert e.value.status == lpt.E_ARG
    tr.close()
    tr = lpt.Tracker(n, "fp64")
    tr.set_snapshot(0, 0.0, u, v)
    tr.set_snapshot(1, 1.0, u, v)
    tr.add_species("inertial", 0.5, "bilinear", x0, y0)
    with pytest.raises(lpt.LptError) as e:
        tr.forward_checkpointed(5, 0.01, 2)
    assert e.value.status == lpt.E_STATE
    tr.close()


def test_full_size_adjoint_sampled():
    """The 2048^2 FP64 adjoint configuration at full size (steady TG + 0.1 x
    spectrum, 2^22 tracers on the cell-centre lattice, bilinear, 200 steps of
    0.01, checkpoints every 20, re-sorted once before the run):
    - F and dL/dx0 of 256 sampled particles against the oracle's forward
      tangent (F^T (a, b)), within 1e-9 of their scale;
    - the grid gradient at 6 nodes of slot 0 (the 3 largest |dL/du| and 3
      random ones) against central differences of L over the whole run on
      the GPU, an independent algorithm.  The map is only piecewise smooth
      (a stage point crossing a cell edge changes its interpolation
      weights), so the difference quotient carries kink errors that shrink
      with h, erratically; particles the node does not influence give
      bit-identical terms, which cancel exactly, so h can be tiny.  Measured
      at the largest entry (adjoint 25.8833757): 25.8257 at h = 1e-4,
      25.8647 at 1e-5, 25.8819 at 1e-6, 25.88336 at 1e-7, 25.88331 at 1e-8.
      With h = 1e-8 the bound is 2e-5 of the largest entry."""
    n, nsteps, dt, every = 2048, 200, 0.01, 20
    u, v, _ = synth.taylor_green(n)
    (pu, pv), _ = synth.spectrum_snapshots(n, 10, 5, dt)
    u, v = u + 0.1 * pu, v + 0.1 * pv
    x0, y0 = synth.lattice_points(n, 2048)
    npart = x0.size
    rng = np.random.default_rng(51)
    a, b = rng.normal(size=npart), rng.normal(size=npart)

    def tracker(uu):
        tr = lpt.Tracker(n, "fp64", sort_interval=20)
        tr.set_snapshot(0, 0.0, uu, v)
        tr.set_snapshot(1, nsteps * dt, u, v)
        tr.add_species("tracer", 0.0, "bilinear", x0, y0)
        return tr

    say("full-size adjoint: checkpointed run, reverse sweeps")
    tr = tracker(u)
    tr.forward_checkpointed(nsteps, dt, every)
    gx, gy, gU = tr.adjoint(a, b)
    F = tr.jacobian()
    tr.close()

    ids = np.random.default_rng(7).choice(npart, 256, replace=False)
    fl = oracle.grid_flow(u, v, u, v, t_slot=(0.0, nsteps * dt))
    Fo = oracle.tangent(fl, oracle.Species(x0[ids], y0[ids]), nsteps, dt)
    assert np.max(np.abs(F[ids] - Fo)) < 1e-9 * _scale(Fo)
    ex = Fo[:, 0, 0] * a[ids] + Fo[:, 1, 0] * b[ids]
    ey = Fo[:, 0, 1] * a[ids] + Fo[:, 1, 1] * b[ids]
    assert np.max(np.abs(gx[ids] - ex)) < 1e-9 * _scale(ex)
    assert np.max(np.abs(gy[ids] - ey)) < 1e-9 * _scale(ey)

    g0 = gU[0, 0]
    flat = np.argsort(np.abs(g0).ravel())
    nodes = list(flat[-3:]) + list(np.random.default_rng(8).choice(n * n, 3, replace=False))
    h = 1e-8
    gmax = np.max(np.abs(g0))
    for node in nodes:
        j, i = divmod(int(node), n)
        Ls = []
        for sgn in (1.0, -1.0):
            say(f"full-size adjoint: central difference at node ({i}, {j}), {sgn:+.0f}h")
            up = u.copy()
            up[j, i] += sgn * h
            trf = tracker(up)
            trf.step(nsteps, dt)
            _, _, xu, yu = trf.get_positions(0)
            trf.close()
            Ls.append(np.dot(a, xu) + np.dot(b, yu))
        fd = (Ls[0] - Ls[1]) / (2 * h)
        say(f"  node ({i}, {j}): adjoint {g0[j, i]:.9g}, central difference {fd:.9g}")
        assert abs(fd - g0[j, i]) < 2e-5 * gmax, (i, j, fd, g0[j, i])


@pytest.mark.parametrize("scheme", ["bilinear", "catmull_rom"])
def test_deterministic_grid_gradient_is_bit_reproducible(scheme):
    """LPT_FLAG_DETERMINISTIC_GRAD sums the grid gradient as exact
    fixed-point integers: two runs, and runs with 64- and 512-thread blocks
    (other LDS boxes, other atomic orders), give the same bits; the result
    matches the oracle's reverse sweep within 1e-10 of its largest entry and
    the default FP64-atomic gradient within 1e-12; dL/dx0 is unchanged."""
    n, dt, nsteps, count = 64, 0.01, 30, 5000
    say(f"deterministic grid gradient {scheme}")
    fields = synth.spectrum_snapshots(n, 6, 14, dt)
    x0, y0 = oracle.init_uniform(33, count)
    rng = np.random.default_rng(34)
    a, b = rng.normal(size=count), rng.normal(size=count)

    def run(det, block):
        (ua, va), (ub, vb) = fields
        tr = lpt.Tracker(n, "fp64", block_size=block, sort_interval=1, deterministic_grad=det)
        tr.set_time_mode("pingpong")
        tr.set_snapshot(0, 0.0, ua, va)
        tr.set_snapshot(1, dt, ub, vb)
        tr.add_species("tracer", 0.0, scheme, x0, y0)
        tr.forward_checkpointed(nsteps, dt, 10)
        out = tr.adjoint(a, b)
        tr.close()
        return out

    d1, d2, d64, d512 = run(True, 0), run(True, 0), run(True, 64), run(True, 512)
    for other in (d2, d64, d512):
        np.testing.assert_array_equal(d1[2], other[2])
        np.testing.assert_array_equal(d1[0], other[0])
    f = run(False, 0)
    (ua, va), (ub, vb) = fields
    fl = oracle.grid_flow(ua, va, ub, vb, scheme=scheme, time_mode=oracle.PINGPONG)
    ox, oy, oU = oracle.adjoint(fl, x0, y0, a, b, nsteps, dt)
    assert np.max(np.abs(d1[2] - oU)) < 1e-10 * _scale(oU)
    assert np.max(np.abs(d1[2] - f[2])) < 1e-12 * _scale(oU)
    np.testing.assert_array_equal(d1[0], f[0])
    assert np.max(np.abs(d1[0] - ox)) < 1e-9 * _scale(ox)

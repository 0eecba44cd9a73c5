"""GPU parity of the Eulerian field producer (libns2d.so, Sec. 3.1) with the
FP64 oracle (oracle/ns2d.py), and of the coupled loop in which its velocity
feeds the particle library in stream order (Alg. coupled_EL: fluid step,
then the particle step between the two retained levels).

Tolerance: the two sides differ only in the rounding of the transforms
(rocFFT against numpy's pocketfft) and of the pointwise products, about
1e-16 relative per transform and step.  Measured on MI355X, of each
field's maximum: hipFFT at most 4.9e-16 (n = 8), 1.1e-15 (n = 64),
1.5e-15 (n = 96), 5.2e-15 (n = 512), 1.5e-15 (n = 2048), 2.2e-15
(n = 4096); the library's own transforms at most
3.9e-15 (n = 512), 3.2e-15 (n = 1024), 9.4e-16 (n = 2048).  The bound is
1e-13; at n = 4096 both paths are compared after 2 steps."""
import numpy as np
import pytest

import oracle
from oracle.ns2d import NS2D
from paper_2607_17836_amd import lpt, ns2d, synth

pytestmark = pytest.mark.gpu

REL = 1e-13


def say(msg):
    print(f"[ns2d] {msg}", flush=True)


def _compare(gpu_fields, ora_fields, rel=REL, what=""):
    for name, g, o in zip(("u", "v", "omega", "psi"), gpu_fields, ora_fields):
        scale = np.abs(o).max()
        err = np.abs(g - o).max()
        assert err <= rel * scale, f"{what} {name}: max |GPU - oracle| = {err:.3e}, scale {scale:.3e}"
    return max(np.abs(g - o).max() / np.abs(o).max() for g, o in zip(gpu_fields, ora_fields))


@pytest.mark.parametrize("n,length,transforms", [
    (64, 2 * np.pi, "auto"), (128, 3.0, "auto"), (256, 2 * np.pi, "builtin"),
    (512, 2 * np.pi, "builtin"), (1024, 3.0, "auto"),
    (8, 2 * np.pi, "hipfft"), (96, 3.0, "hipfft"), (512, 2 * np.pi, "hipfft")])
def test_matches_oracle_step_by_step(n, length, transforms):
    """Step 0 (band truncation), step 1 (forward Euler), step 2 (first AB2
    step) and step 30: the library's own transforms (the default) at every
    radix pattern below 2048 -- 64 (8 8), 128 (8 8 2), 256 (8 8 4), 512
    (8 8 8), 1024 (8 8 8 2) -- with L != 2 pi on some; hipFFT, on request,
    on the smallest grid (n = 8, band |m| <= 2), on n = 96 (divisible by 3:
    the edge of the 2/3 rule; radix-3 transforms; L != 2 pi) and at 512."""
    say(f"n={n} L={length} transforms={transforms}")
    # nu k_max^2 dt <= 0.2 at every size: the explicit viscous term stays stable
    nu, dt = 2e-4, 2e-3
    w0 = synth.random_vorticity(n, min(n / 10, 40.0), 21, omega_rms=5.0)
    g = ns2d.Ns2d(n, nu, dt, length=length, transforms=transforms)
    assert g.builtin == (transforms != "hipfft")
    o = NS2D(n, nu, dt, length=length)
    g.set_vorticity(w0)
    o.set_vorticity(w0)
    worst = _compare(g.get_fields(), o.fields(), what="step 0")
    for upto in (1, 2, 30):
        g.step(upto - g.steps)
        o.step(upto - o.steps)
        assert g.steps == upto
        worst = max(worst, _compare(g.get_fields(), o.fields(), what=f"step {upto}"))
    say(f"n={n}: worst relative difference {worst:.2e}")
    g.close()


@pytest.mark.parametrize("transforms", ["auto", "hipfft"])
def test_largest_grid_matches_oracle(transforms):
    """4096^2, the largest grid here (the particle headline's grid; 1.5 GB of
    fields), 2 steps, every grid value compared: the library's own transforms
    (radix 8 8 8 8, 512 threads a transform, the default) and hipFFT."""
    n = 4096
    say(f"n={n} transforms={transforms}")
    w0 = synth.random_vorticity(n, 20.0, 26, omega_rms=3.0)
    g = ns2d.Ns2d(n, 2e-5, 5e-4, transforms=transforms)
    assert g.builtin == (transforms == "auto")
    o = NS2D(n, 2e-5, 5e-4)
    g.set_vorticity(w0)
    o.set_vorticity(w0)
    g.step(2)
    o.step(2)
    worst = _compare(g.get_fields(), o.fields(), what="n=4096 step 2")
    say(f"n={n}: worst relative difference {worst:.2e}")
    g.close()


@pytest.mark.parametrize("transforms", ["auto", "hipfft"])
def test_full_size_matches_oracle(transforms):
    """2048^2 (the benchmark's grid), 3 steps, every grid value compared,
    with the library's own transforms and with hipFFT."""
    n, nu, dt = 2048, 1e-4, 1e-3
    say(f"full size n={n} transforms={transforms}")
    w0 = synth.random_vorticity(n, 10.0, 22, omega_rms=3.0)
    g = ns2d.Ns2d(n, nu, dt, transforms=transforms)
    assert g.builtin == (transforms == "auto")
    o = NS2D(n, nu, dt)
    g.set_vorticity(w0)
    o.set_vorticity(w0)
    g.step(3)
    o.step(3)
    worst = _compare(g.get_fields(), o.fields(), what="n=2048 step 3")
    say(f"n={n}: worst relative difference {worst:.2e}")
    g.close()


@pytest.mark.parametrize("n,nu", [(64, 0.05), (512, 0.005)])
def test_taylor_green_vortex_decay_on_the_gpu(n, nu):
    """psi = sin x sin y decays as exp(-2 nu t) in every field (no advection
    for a Laplacian eigenfunction); AB2 error below 1e-8 at nu dt <= 5e-5;
    the library's own transforms at n = 64 and 512.  nu keeps
    nu k_max^2 dt below 1 (0.29 at n = 512): the explicit viscous term would
    otherwise amplify the transforms' rounding in the highest modes."""
    dt, steps = 1e-3, 200
    x = np.arange(n) * (2 * np.pi / n)
    X, Y = x[None, :], x[:, None]
    g = ns2d.Ns2d(n, nu, dt)
    assert g.builtin
    g.set_vorticity(2 * np.sin(X) * np.sin(Y))
    g.step(steps)
    u, v, w, psi = g.get_fields()
    a = np.exp(-2 * nu * dt * steps)
    np.testing.assert_allclose(u, a * np.sin(X) * np.cos(Y), atol=1e-8)
    np.testing.assert_allclose(v, -a * np.cos(X) * np.sin(Y), atol=1e-8)
    np.testing.assert_allclose(w, 2 * a * np.sin(X) * np.sin(Y), atol=2e-8)
    np.testing.assert_allclose(psi, a * np.sin(X) * np.sin(Y), atol=1e-8)
    g.close()


def test_device_vorticity_input_and_velocity_pointers():
    """A device vorticity array gives the same state as a host one, and the
    velocity pointers hold the grid velocity that get_fields returns."""
    import torch
    n = 64
    w0 = synth.random_vorticity(n, 6.0, 23)
    a = ns2d.Ns2d(n, 1e-3, 1e-3)
    b = ns2d.Ns2d(n, 1e-3, 1e-3)
    a.set_vorticity(w0)
    b.set_vorticity(torch.from_numpy(w0).cuda())
    a.step(4)
    b.step(4)
    fa, fb = a.get_fields(), b.get_fields()
    for x, y in zip(fa, fb):
        np.testing.assert_array_equal(x, y)

    class View:   # a torch view of n*n device doubles at a raw address
        def __init__(self, ptr):
            self.__cuda_array_interface__ = dict(shape=(n, n), typestr="<f8", data=(ptr, False),
                                                 version=3, strides=None)

    # the fields read into device buffers equal the host read-back
    dev = [torch.empty(n * n, dtype=torch.float64, device="cuda") for _ in range(4)]
    assert ns2d.load().ns2d_get_fields(b._h, *[d.data_ptr() for d in dev], 1) == ns2d.OK
    b.synchronize()
    for d, h in zip(dev, fb):
        np.testing.assert_array_equal(d.cpu().numpy().reshape(n, n), h)

    pu, pv = b.velocity_ptrs()
    b.synchronize()
    np.testing.assert_array_equal(torch.as_tensor(View(pu), device="cuda").cpu().numpy(), fb[0])
    np.testing.assert_array_equal(torch.as_tensor(View(pv), device="cuda").cpu().numpy(), fb[1])
    a.close()
    b.close()


def test_errors():
    g = ns2d.Ns2d(64, 1e-3, 1e-3)
    with pytest.raises(ns2d.Ns2dError) as e:
        g.step(1)
    assert e.value.status == ns2d.E_STATE
    g.set_vorticity(np.zeros((64, 64)))
    with pytest.raises(ns2d.Ns2dError) as e:
        g.step(-1)
    assert e.value.status == ns2d.E_ARG
    g.step(0)
    u, v, w, psi = g.get_fields()
    assert not np.any(u) and not np.any(psi)
    g.close()


@pytest.mark.parametrize("n,length", [(128, 2 * np.pi), (512, 2 * np.pi), (512, 3.0)])
def test_coupled_loop_matches_the_oracles(n, length):
    """The producer's velocity streamed into the particle library each step
    (ping-pong slots, device pointers, same stream), tracers and inertial
    particles, against the field oracle feeding the particle oracle the same
    levels: positions within 1e-10 after 10 steps (the library's own
    transforms at n = 128 and 512; a domain of side 3 as well as 2 pi)."""
    nu, dt, nsteps = 1e-3, 2e-3, 10
    L = length
    say(f"coupled loop n={n} L={L}")
    w0 = synth.random_vorticity(n, 8.0, 24, omega_rms=5.0)
    g = ns2d.Ns2d(n, nu, dt, length=L)
    g.set_vorticity(w0)
    tr = lpt.Tracker(n, "fp64", length=L)
    tr.set_time_mode("pingpong")
    tr.set_snapshot_device(0, 0.0, *g.velocity_ptrs())
    g.step(1)
    tr.set_snapshot_device(1, dt, *g.velocity_ptrs())
    x0, y0 = oracle.init_uniform(81, 2000, L)
    rng = np.random.default_rng(82)
    vx0, vy0 = rng.normal(size=500), rng.normal(size=500)
    st = tr.add_species("tracer", 0.0, "bilinear", x0, y0)
    si = tr.add_species("inertial", 0.2, "catmull_rom", x0[:500], y0[:500], vx0, vy0)
    for s in range(nsteps):
        tr.step(1, dt)
        g.step(1)
        tr.set_snapshot_device(s % 2, (s + 2) * dt, *g.velocity_ptrs())
    xt = tr.get_positions(st)
    xi = tr.get_positions(si)
    tr.close()
    g.close()

    o = NS2D(n, nu, dt, length=L)
    o.set_vorticity(w0)
    levels = [o.fields()[:2]]
    for _ in range(nsteps):
        o.step(1)
        levels.append(o.fields()[:2])
    sp_t = oracle.Species(x0, y0, length=L)
    sp_i = oracle.Species(x0[:500], y0[:500], kind=oracle.INERTIAL, st=0.2, vx0=vx0, vy0=vy0,
                          length=L)
    for k in range(nsteps):
        (ua, va), (ub, vb) = levels[k], levels[k + 1]
        for sp, scheme in ((sp_t, oracle.BILINEAR), (sp_i, oracle.CATMULL_ROM)):
            fl = oracle.grid_flow(ua, va, ub, vb, scheme=scheme, t_slot=(k * dt, (k + 1) * dt),
                                  length=L)
            oracle.run(fl, sp, 1, dt, t_start=k * dt, step0=k)

    def pdist(a, b):
        d = np.abs(np.asarray(a) - np.asarray(b)) % L
        return np.minimum(d, L - d)

    for got, sp in ((xt, sp_t), (xi, sp_i)):
        assert np.max(pdist(got[0], sp.xw)) < 1e-10 and np.max(pdist(got[1], sp.yw)) < 1e-10


def test_own_transforms_match_hipfft():
    """The library's own transforms and hipFFT give the same fields to
    rounding (1e-13 of each field's maximum) after 20 steps at n = 1024."""
    n = 1024
    w0 = synth.random_vorticity(n, 20.0, 25, omega_rms=8.0)
    out = []
    for tf in ("auto", "hipfft"):
        g = ns2d.Ns2d(n, 5e-4, 1e-3, transforms=tf)
        g.set_vorticity(w0)
        g.step(20)
        out.append(g.get_fields())
        g.close()
    worst = _compare(out[0], out[1], what="own vs hipFFT")
    say(f"own vs hipFFT: worst relative difference {worst:.2e}")


def test_coupled_loop_on_two_streams_equals_one_stream():
    """The coupled loop with the field producer and the particles on two
    HIP streams (ordered by two events) gives bit-identical particles to the
    same loop on one stream: 12 steps with re-sorts every 4, tracers and
    inertial particles, n = 512 (own transforms)."""
    from paper_2607_17836_amd import coupled
    n, nu, dt = 512, 1e-3, 2e-3
    w0 = synth.random_vorticity(n, 8.0, 27, omega_rms=3.0)
    x0, y0 = oracle.init_uniform(83, 20000)
    out = []
    for streams in (1, 2):
        loop = coupled.CoupledLoop(n, nu, dt, w0, streams=streams, sort_interval=4)
        st = loop.tracker.add_species("tracer", 0.0, "bilinear", x0, y0)
        si = loop.tracker.add_species("inertial", 0.3, "catmull_rom", x0[:5000], y0[:5000])
        loop.step(12, stats_every=6)
        out.append([loop.tracker.get_positions(st), loop.tracker.get_positions(si),
                    loop.tracker.get_stats(st)["msd"], loop.field.get_fields()])
        loop.close()
    for a, b in zip(out[0][:2], out[1][:2]):
        for qa, qb in zip(a, b):
            np.testing.assert_array_equal(qa, qb)
    np.testing.assert_array_equal(out[0][2], out[1][2])
    for qa, qb in zip(out[0][3], out[1][3]):
        np.testing.assert_array_equal(qa, qb)


def test_coupled_loop_fp32_split_tracers_match_the_oracles():
    """The producer's FP64 levels streamed into an FP32-split tracker (the
    FP32 ingest from device pointers): 8 coupled steps against the field
    oracle's levels rounded to binary32 and stepped by the particle oracle;
    binary32 velocities bound the position error by 1e-6 (as in the FP32
    parity tests)."""
    from paper_2607_17836_amd import coupled
    n, nu, dt, nsteps = 512, 1e-3, 2e-3, 8
    say("coupled loop fp32_split")
    w0 = synth.random_vorticity(n, 8.0, 28, omega_rms=3.0)
    x0, y0 = oracle.init_uniform(84, 4000)
    loop = coupled.CoupledLoop(n, nu, dt, w0, precision="fp32_split", sort_interval=4)
    sid = loop.tracker.add_species("tracer", 0.0, "bilinear", x0, y0)
    loop.step(nsteps)
    xw, yw, _, _ = loop.tracker.get_positions(sid)
    loop.close()

    o = NS2D(n, nu, dt)
    o.set_vorticity(w0)
    r32 = lambda f: f.astype(np.float32).astype(np.float64)
    levels = [tuple(r32(f) for f in o.fields()[:2])]
    for _ in range(nsteps):
        o.step(1)
        levels.append(tuple(r32(f) for f in o.fields()[:2]))
    sp = oracle.Species(x0, y0)
    for k in range(nsteps):
        (ua, va), (ub, vb) = levels[k], levels[k + 1]
        fl = oracle.grid_flow(ua, va, ub, vb, t_slot=(k * dt, (k + 1) * dt))
        oracle.run(fl, sp, 1, dt, t_start=k * dt, step0=k)
    d = np.abs(np.concatenate([xw - sp.xw, yw - sp.yw])) % (2 * np.pi)
    err = np.minimum(d, 2 * np.pi - d).max()
    say(f"coupled fp32_split: max position error {err:.2e}")
    assert err < 1e-6

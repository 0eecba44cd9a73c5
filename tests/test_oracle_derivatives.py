"""Pins of the oracle's derivatives of the discrete tracer map: the forward
tangent F = dx_T/dx_0 (for finite-time Lyapunov exponents) and the reverse
sweep for L = sum(a x_T + b y_T) with its gradient on the velocity grid.

The paper has no adjoint.  Each pin below is fixed by the mathematics rather
than by re-typing the oracle: exact invariants of the flow map and of the
interpolation weights, central differences of the separately pinned forward
oracle, and the duality between forward and reverse mode (two different
algorithms)."""
import numpy as np
import pytest

import oracle
from paper_2607_17836_amd import synth

L = 2 * np.pi


def _spectrum_flow(scheme, n=32, k0=4.0, seed=3, dt=0.01):
    (ua, va), (ub, vb) = synth.spectrum_snapshots(n, k0, seed, dt)
    return (ua, va, ub, vb), oracle.grid_flow(ua, va, ub, vb, scheme=scheme,
                                              time_mode=oracle.PINGPONG)


def _final_unwrapped(fl, x0, y0, nsteps, dt):
    sp = oracle.Species(x0, y0)
    oracle.run(fl, sp, nsteps, dt)
    return sp.unwrapped()


def test_interp_gradient_matches_central_differences():
    """The spatial gradient of each interpolant equals central differences of
    the (separately pinned) interpolant itself, away from cell edges, where
    bilinear is only piecewise smooth."""
    rng = np.random.default_rng(0)
    n = 24
    f = rng.normal(size=(n, n))
    h = L / n
    eps = 1e-6
    for scheme in ("bilinear", "catmull_rom", "bspline"):
        for _ in range(40):
            ci, cj = rng.integers(0, n, 2)
            x = (ci + rng.uniform(0.1, 0.9)) * h
            y = (cj + rng.uniform(0.1, 0.9)) * h
            _, gx, gy = oracle.interp_grad(f, x, y, scheme)
            fx = (oracle.interp(f, x + eps, y, scheme) - oracle.interp(f, x - eps, y, scheme)) / (2 * eps)
            fy = (oracle.interp(f, x, y + eps, scheme) - oracle.interp(f, x, y - eps, scheme)) / (2 * eps)
            assert abs(gx - fx[0]) < 1e-6 * (1 + abs(gx)), (scheme, gx, fx)
            assert abs(gy - fy[0]) < 1e-6 * (1 + abs(gy)), (scheme, gy, fy)


def test_tangent_is_identity_in_uniform_flow():
    """A uniform flow translates every particle: F = I exactly (analytic
    source), and to rounding for a gridded uniform field (the weights'
    derivatives sum to zero)."""
    x0, y0 = oracle.init_uniform(3, 50)
    sp = oracle.Species(x0, y0)
    F = oracle.tangent(oracle.uniform_flow(0.7, -0.3), sp, 100, 0.01)
    assert np.all(F == np.eye(2)[None])
    u = np.full((16, 16), 0.7)
    v = np.full((16, 16), -0.3)
    for scheme in ("bilinear", "catmull_rom", "bspline"):
        sp = oracle.Species(x0, y0)
        F = oracle.tangent(oracle.grid_flow(u, v, scheme=scheme), sp, 50, 0.01)
        assert np.max(np.abs(F - np.eye(2)[None])) < 1e-13, scheme


@pytest.mark.parametrize("eps,omega", [(0.0, 0.0), (0.3, 1.8)])
def test_tangent_preserves_area_in_taylor_green(eps, omega):
    """The (oscillating) Taylor-Green flow of eq. kinematic_flow is
    divergence-free, so its flow map preserves area: det F = 1.  RK4's map
    does so to O(dt^4) per unit time; a dropped stage term in the tangent
    breaks it at O(dt)."""
    x0, y0 = oracle.init_uniform(11, 64)
    sp = oracle.Species(x0, y0)
    F = oracle.tangent(oracle.tg_flow(eps=eps, omega=omega), sp, 400, 0.005)
    det = F[:, 0, 0] * F[:, 1, 1] - F[:, 0, 1] * F[:, 1, 0]
    assert np.max(np.abs(det - 1.0)) < 1e-8, np.max(np.abs(det - 1.0))
    assert np.max(np.abs(F)) > 1.5   # the map does stretch


@pytest.mark.parametrize("scheme", ["catmull_rom", "bspline"])
def test_tangent_matches_central_differences_of_the_map(scheme):
    """F agrees with central differences of the forward oracle's final
    unwrapped positions (C1 interpolants, so the map is smooth)."""
    _, fl = _spectrum_flow(scheme)
    dt, nsteps = 0.01, 30
    x0, y0 = oracle.init_uniform(7, 12)
    F = oracle.tangent(fl, oracle.Species(x0, y0), nsteps, dt)
    e = 1e-6
    xp, yp = _final_unwrapped(fl, x0 + e, y0, nsteps, dt)
    xm, ym = _final_unwrapped(fl, x0 - e, y0, nsteps, dt)
    col0 = np.stack([(xp - xm) / (2 * e), (yp - ym) / (2 * e)], 1)
    xp, yp = _final_unwrapped(fl, x0, y0 + e, nsteps, dt)
    xm, ym = _final_unwrapped(fl, x0, y0 - e, nsteps, dt)
    col1 = np.stack([(xp - xm) / (2 * e), (yp - ym) / (2 * e)], 1)
    fd = np.stack([col0, col1], 2)
    assert np.max(np.abs(F - fd)) < 1e-6 * max(1.0, np.max(np.abs(F)))


@pytest.mark.parametrize("scheme", ["bilinear", "catmull_rom", "bspline"])
def test_reverse_sweep_is_the_transposed_tangent(scheme):
    """dL/dx0 from the reverse sweep equals F^T (a, b) from the forward
    tangent: two different algorithms for the same derivative."""
    _, fl = _spectrum_flow(scheme)
    x0, y0 = oracle.init_uniform(9, 40)
    rng = np.random.default_rng(1)
    a, b = rng.normal(size=40), rng.normal(size=40)
    F = oracle.tangent(fl, oracle.Species(x0, y0), 25, 0.01)
    gx, gy, _ = oracle.adjoint(fl, x0, y0, a, b, 25, 0.01)
    ref = np.einsum("pki,pk->pi", F, np.stack([a, b], 1))
    assert np.max(np.abs(ref[:, 0] - gx)) < 1e-12 * max(1, np.max(np.abs(gx)))
    assert np.max(np.abs(ref[:, 1] - gy)) < 1e-12 * max(1, np.max(np.abs(gy)))


@pytest.mark.parametrize("scheme", ["bilinear", "catmull_rom", "bspline"])
def test_grid_gradient_uniform_shift_invariant(scheme):
    """In a uniform gridded flow, adding delta to every u node of both time
    levels adds delta to the interpolated velocity everywhere (partition of
    unity) and leaves its gradient zero, so every tracer moves by exactly
    delta*T: the u-part of the grid gradient sums to sum(a)*T and the v-part
    to sum(b)*T.  (In a non-uniform flow the shifted stage points see other
    velocities, so the invariant needs the uniform base flow.)"""
    n = 16
    u = np.full((n, n), 0.6)
    v = np.full((n, n), -0.45)
    fl = oracle.grid_flow(u, v, u, v, scheme=scheme, time_mode=oracle.PINGPONG)
    x0, y0 = oracle.init_uniform(13, 30)
    rng = np.random.default_rng(2)
    a, b = rng.normal(size=30), rng.normal(size=30)
    nsteps, dt = 20, 0.01
    gx, gy, gU = oracle.adjoint(fl, x0, y0, a, b, nsteps, dt)
    T = nsteps * dt
    assert abs(gU[:, 0].sum() - a.sum() * T) < 1e-12 * max(1, abs(a.sum() * T))
    assert abs(gU[:, 1].sum() - b.sum() * T) < 1e-12 * max(1, abs(b.sum() * T))
    # each time level carries half of it: ping-pong alternates the roles
    assert abs(gU[0, 0].sum() - gU[1, 0].sum()) < 1e-12
    np.testing.assert_allclose(gx, a, rtol=0, atol=1e-13)
    np.testing.assert_allclose(gy, b, rtol=0, atol=1e-13)


@pytest.mark.parametrize("scheme", ["bilinear", "catmull_rom", "bspline"])
def test_grid_gradient_matches_central_differences(scheme):
    """Perturbing one grid value of one time level changes L as the grid
    gradient says (nodes chosen where the gradient is largest)."""
    (ua, va, ub, vb), fl = _spectrum_flow(scheme, n=16)
    x0, y0 = oracle.init_uniform(17, 6)
    rng = np.random.default_rng(3)
    a, b = rng.normal(size=6), rng.normal(size=6)
    nsteps, dt = 8, 0.01
    _, _, gU = oracle.adjoint(fl, x0, y0, a, b, nsteps, dt)
    flat = np.argsort(np.abs(gU).ravel())[-6:]
    eps = 1e-6
    for idx in flat:
        s, c, j, i = np.unravel_index(idx, gU.shape)

        def loss(sign):
            f = [ua.copy(), va.copy(), ub.copy(), vb.copy()]
            f[2 * s + c][j, i] += sign * eps
            flp = oracle.grid_flow(*f, scheme=scheme, time_mode=oracle.PINGPONG)
            xt, yt = _final_unwrapped(flp, x0, y0, nsteps, dt)
            return float(np.sum(a * xt + b * yt))

        fd = (loss(1) - loss(-1)) / (2 * eps)
        assert abs(fd - gU[s, c, j, i]) < 1e-6 * max(1.0, abs(fd)), (scheme, idx, fd, gU[s, c, j, i])


def test_ftle_of_a_translation_is_zero_and_of_a_stretch_is_its_rate():
    """FTLE = (1/T) ln sqrt(lambda_max(F^T F)): zero for F = I, and the
    stretch rate s for F = diag(e^{sT}, e^{-sT})."""
    T, s = 2.0, 0.8
    F = np.stack([np.eye(2), np.diag([np.exp(s * T), np.exp(-s * T)])])
    out = oracle.ftle(F, T)
    assert abs(out[0]) < 1e-15 and abs(out[1] - s) < 1e-14

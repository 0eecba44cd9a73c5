"""Pins of the Eulerian field-producer oracle (oracle/ns2d.py) to facts the
oracle does not compute itself: closed-form solutions, a brute-force
convolution, conservation laws of the truncated system and the order of the
time integrator (Sec. 3.1, eqs. spectral_vorticity_derivatives to
ab2_fluid)."""
import itertools

import numpy as np

from oracle.ns2d import NS2D, band_mask
from paper_2607_17836_amd import synth


def _grid(n, length=2 * np.pi):
    x = np.arange(n) * (length / n)
    return x[None, :], x[:, None]


def _band_field(n, seed, kmax):
    """Real field sum_m c(m) exp(i m.x) over |m_x|, |m_y| <= kmax with
    Hermitian c, summed mode by mode on the grid (no FFT).  Returns the grid
    values and the coefficient dictionary."""
    rng = np.random.default_rng(seed)
    X, Y = _grid(n)
    coef = {}
    for mx, my in itertools.product(range(-kmax, kmax + 1), repeat=2):
        if (mx, my) == (0, 0) or (mx, my) in coef:
            continue
        c = complex(rng.normal(), rng.normal())
        coef[(mx, my)] = c
        coef[(-mx, -my)] = c.conjugate()
    f = np.zeros((n, n))
    for (mx, my), c in coef.items():
        f += (c * np.exp(1j * (mx * X + my * Y))).real
    return f, coef


def test_taylor_green_vortex_decays_as_exp_minus_2_nu_t():
    """psi = sin x sin y is a Laplacian eigenfunction (omega = 2 psi), so the
    advection term vanishes and every field decays as exp(-2 nu t); the
    velocity is (sin x cos y, -cos x sin y) by u = dpsi/dy, v = -dpsi/dx.
    The AB2 error of this linear decay is below 1e-8 of the amplitude at
    nu dt = 5e-5 (first step: forward Euler, error (2 nu dt)^2 / 2)."""
    n, nu, dt, steps = 32, 0.05, 1e-3, 200
    X, Y = _grid(n)
    ns = NS2D(n, nu, dt)
    ns.set_vorticity(2 * np.sin(X) * np.sin(Y))
    assert np.abs(ns.nonlinear_hat(ns.w_hat)).max() < 1e-10 * n * n
    ns.step(steps)
    g = np.exp(-2 * nu * dt * steps)
    u, v, w, psi = ns.fields()
    tol = 1e-8
    np.testing.assert_allclose(u, g * np.sin(X) * np.cos(Y), atol=tol)
    np.testing.assert_allclose(v, -g * np.cos(X) * np.sin(Y), atol=tol)
    np.testing.assert_allclose(w, 2 * g * np.sin(X) * np.sin(Y), atol=2 * tol)
    np.testing.assert_allclose(psi, g * np.sin(X) * np.sin(Y), atol=tol)


def test_stream_function_and_velocity_of_an_anisotropic_mode():
    """omega = 13 sin 2x cos 3y has psi = sin 2x cos 3y (omega = -lap psi),
    u = dpsi/dy = -3 sin 2x sin 3y, v = -dpsi/dx = -2 cos 2x cos 3y; distinct
    x and y wavenumbers catch a transposed axis."""
    n = 24
    X, Y = _grid(n)
    ns = NS2D(n, 0.0, 1e-3)
    ns.set_vorticity(13 * np.sin(2 * X) * np.cos(3 * Y))
    u, v, w, psi = ns.fields()
    np.testing.assert_allclose(psi, np.sin(2 * X) * np.cos(3 * Y), atol=1e-13)
    np.testing.assert_allclose(u, -3 * np.sin(2 * X) * np.sin(3 * Y), atol=1e-13)
    np.testing.assert_allclose(v, -2 * np.cos(2 * X) * np.cos(3 * Y), atol=1e-13)


def test_band_is_the_largest_alias_free_one():
    """A band |m| <= K is alias-free when no sum of two retained indices
    folds (mod n) onto a retained index other than itself; the oracle's band
    is the largest such K, found here by enumerating all pairs."""
    for n in (12, 16, 17, 24, 32):
        def alias_free(K):
            for p in range(-K, K + 1):
                for q in range(-K, K + 1):
                    s = p + q
                    folded = (s + n // 2) % n - n // 2
                    if folded != s and abs(folded) <= K:
                        return False
            return True
        kmax = max(K for K in range(n // 2 + 1) if alias_free(K))
        m = band_mask(n)
        my = np.fft.fftfreq(n, d=1.0 / n)
        kept_y = sorted(int(abs(v)) for v in my[m[:, 0]])
        assert max(kept_y) == kmax, (n, kept_y, kmax)
        kept_x = np.nonzero(m[0])[0]
        assert kept_x.max() == kmax


def test_advection_term_matches_a_brute_force_convolution():
    """On a field inside the band, the oracle's dealiased transform of
    u dw/dx + v dw/dy equals the Fourier-space convolution sum over all
    pairs of modes, written out term by term (n = 12 is divisible by 3, the
    edge of the 2/3 rule)."""
    n, K = 12, 3
    w, coef = _band_field(n, 5, K)
    ns = NS2D(n, 0.0, 1e-3)
    ns.set_vorticity(w)
    got = ns.nonlinear_hat(ns.w_hat) / (n * n)

    def psi(m):
        return coef.get(m, 0) / (m[0] ** 2 + m[1] ** 2) if m != (0, 0) else 0

    expect = {}
    for p in coef:
        up = 1j * p[1] * psi(p)
        vp = -1j * p[0] * psi(p)
        for q, cq in coef.items():
            k = (p[0] + q[0], p[1] + q[1])
            expect[k] = expect.get(k, 0) + up * 1j * q[0] * cq + vp * 1j * q[1] * cq
    my = np.fft.fftfreq(n, d=1.0 / n).astype(int)
    checked = 0
    for jy, ky in enumerate(my):
        for kx in range(n // 2 + 1):
            kept = 3 * abs(kx) < n and 3 * abs(ky) < n
            e = expect.get((kx, ky), 0) if kept else 0
            assert abs(got[jy, kx] - e) < 1e-12 * max(1.0, abs(e)), (kx, ky, got[jy, kx], e)
            checked += kept
    assert checked > 20


def test_inviscid_truncated_system_conserves_energy_and_enstrophy():
    """For nu = 0 the dealiased Galerkin system conserves energy and
    enstrophy exactly: d/dt <psi omega> / 2 = <psi R> = 0 and
    <omega R> = 0 on the grid, to rounding.  A sign error in one velocity
    component, or swapped derivative axes, breaks both."""
    n = 32
    w, _ = _band_field(n, 9, 10)
    ns = NS2D(n, 0.0, 1e-3)
    ns.set_vorticity(w)
    R = ns.to_grid(ns.rhs(ns.w_hat))
    _, _, om, psi = ns.fields()
    scale_e = np.sqrt(np.mean(psi ** 2) * np.mean(R ** 2))
    scale_z = np.sqrt(np.mean(om ** 2) * np.mean(R ** 2))
    assert abs(np.mean(psi * R)) < 1e-12 * scale_e
    assert abs(np.mean(om * R)) < 1e-12 * scale_z
    assert np.mean(R ** 2) > 1e-3 * np.mean(om ** 2)   # the term is not trivially zero


def test_ab2_is_second_order_in_time():
    """Halving dt divides the error at a fixed time by about 4 on a
    nonlinear, viscous field (reference: dt / 8)."""
    n, nu, T = 32, 0.02, 0.4
    w0 = synth.random_vorticity(n, 4.0, 11)

    def run(dt):
        ns = NS2D(n, nu, dt)
        ns.set_vorticity(w0)
        ns.step(int(round(T / dt)))
        return ns.fields()[2]

    ref = run(0.01 / 8)
    e1 = np.abs(run(0.01) - ref).max()
    e2 = np.abs(run(0.005) - ref).max()
    assert e1 > 1e-9
    assert 3.2 < e1 / e2 < 4.8, (e1, e2)


def test_domain_length_scales_as_the_equations_say():
    """On a domain s L with viscosity s^2 nu the same grid vorticity evolves
    identically (advection is scale-free, k^2 scales by 1/s^2), while psi
    scales by s^2 and the velocity by s."""
    n, s = 32, 3.0
    w0 = synth.random_vorticity(n, 4.0, 12)
    a = NS2D(n, 0.01, 2e-3)
    b = NS2D(n, 0.01 * s * s, 2e-3, length=2 * np.pi * s)
    for ns in (a, b):
        ns.set_vorticity(w0)
        ns.step(25)
    ua, va, wa, pa = a.fields()
    ub, vb, wb, pb = b.fields()
    np.testing.assert_allclose(wb, wa, atol=1e-12 * np.abs(wa).max())
    np.testing.assert_allclose(ub, s * ua, atol=1e-12 * np.abs(s * ua).max())
    np.testing.assert_allclose(pb, s * s * pa, atol=1e-12 * np.abs(s * s * pa).max())


def test_first_step_is_forward_euler_then_ab2():
    """One mode under pure viscous decay follows the scalar recurrence
    w1 = (1 - l dt) w0, w_{k+1} = w_k - l dt (3 w_k - w_{k-1}) / 2, with
    l = nu |k|^2 (here 5 nu); the amplitude is read off the grid."""
    n, nu, dt = 16, 0.3, 0.05
    X, Y = _grid(n)
    mode = np.cos(X + 2 * Y)
    ns = NS2D(n, nu, dt)
    ns.set_vorticity(mode)
    lam = nu * 5
    amps = [1.0, 1.0 - lam * dt]
    for _ in range(6):
        amps.append(amps[-1] - lam * dt * (3 * amps[-1] - amps[-2]) / 2)
    for k in range(1, 8):
        ns.step(1)
        w = ns.fields()[2]
        np.testing.assert_allclose(w, amps[k] * mode, atol=1e-13)


def test_rhs_of_a_shear_plus_wave_is_the_closed_form():
    """omega = A sin y + e cos(m x): each part alone is a Laplacian
    eigenfunction (no self-advection), so the advection term is the exact
    cross term u1 dw2/dx + v2 dw1/dy with u1 = A cos y, v2 = e sin(m x) / m:
    N = -e A (m - 1/m) cos y sin(m x), and the inviscid right-hand side is
    -N.  Fixes the sign of the advection term and which velocity component
    meets which derivative."""
    n, A, e, m = 16, 1.7, 0.3, 3
    X, Y = _grid(n)
    ns = NS2D(n, 0.0, 1e-3)
    ns.set_vorticity(A * np.sin(Y) + e * np.cos(m * X))
    R = ns.to_grid(ns.rhs(ns.w_hat))
    np.testing.assert_allclose(R, e * A * (m - 1.0 / m) * np.cos(Y) * np.sin(m * X), atol=1e-13)

"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the particle method (no interpolation, no
time stepping, no statistics).  It only manufactures inputs:

* velocity snapshots on the doubly periodic [0, L)^2 grid, node (i, j) at
  (i*h, j*h), stored as ``f[j, i]`` (x fastest);
* point sets for interpolation and stepping tests.

Random-phase spectra stand in for the paper's decaying-turbulence snapshots,
which are not public.  The velocity follows from a stream function through
u = d(psi)/dy, v = -d(psi)/dx (eqs. adv_eqn and spectral_velocity), with the
zero mode of psi set to zero (eq. poisson_spectral).
"""
from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi


def grid_coords(n: int, length: float = TWO_PI):
    h = length / n
    x = np.arange(n) * h
    return x, x.copy()


def taylor_green(n: int, length: float = TWO_PI, alpha: float = 1.0, k: float = 1.0,
                 eps: float = 0.0, omega: float = 0.0, phi: float = 0.0, t: float = 0.0):
    """Gridded (oscillating) Taylor-Green flow of eq. kinematic_flow.

    Returns (u, v, psi), each [n, n] float64 indexed [j, i].  eps = 0 gives the
    steady cellular flow u = alpha sin(kx) cos(ky), v = -alpha cos(kx) sin(ky).
    """
    x, y = grid_coords(n, length)
    X = x[None, :]
    Y = y[:, None]
    ax = k * (X - eps * np.sin(omega * t))
    ay = k * (Y - eps * np.sin(omega * t + phi))
    psi = alpha / k * np.sin(ax) * np.sin(ay)
    u = alpha * np.sin(ax) * np.cos(ay)
    v = -alpha * np.cos(ax) * np.sin(ay)
    return (np.ascontiguousarray(u), np.ascontiguousarray(v), np.ascontiguousarray(psi))


def spectrum_snapshots(n: int, k0: float, seed: int, dt_snap: float, length: float = TWO_PI,
                       with_psi: bool = False):
    """Two velocity snapshots from a random-phase stream function.

    Isotropic energy spectrum E(k) ~ k^4 exp(-(k/k0)^2), so the stream-function
    amplitude is |psi_k|^2 ~ E(k)/k^3 = k exp(-(k/k0)^2); phases are uniform on
    [0, 2pi) from ``numpy.random.default_rng(seed)``; psi_0 = 0.  Snapshot B
    carries the same amplitudes with every phase advanced by |k| * dt_snap.
    Both are scaled by one factor chosen so that snapshot A has rms 1 per
    velocity component (sqrt(<u^2 + v^2>/2) = 1); a common factor keeps the
    field divergence-free.

    Returns ((ua, va), (ub, vb)) float64 [n, n] and, with ``with_psi``, also
    (psia, psib).
    """
    assert length == TWO_PI, "integer wavenumbers assume L = 2 pi"
    rng = np.random.default_rng(seed)
    ky = np.fft.fftfreq(n, d=1.0 / n)[:, None]        # axis 0 is y
    kx = np.fft.rfftfreq(n, d=1.0 / n)[None, :]       # axis 1 is x (half plane)
    kmag = np.sqrt(kx * kx + ky * ky)
    amp = np.sqrt(kmag * np.exp(-(kmag / k0) ** 2))
    amp[0, 0] = 0.0
    phase = rng.uniform(0.0, 2.0 * np.pi, size=amp.shape)

    def fields(ph):
        psih = amp * np.exp(1j * ph)
        uh = 1j * ky * psih
        vh = -1j * kx * psih
        u = np.fft.irfft2(uh, s=(n, n))
        v = np.fft.irfft2(vh, s=(n, n))
        p = np.fft.irfft2(psih, s=(n, n))
        return u, v, p

    ua, va, pa = fields(phase)
    ub, vb, pb = fields(phase - kmag * dt_snap)
    scale = 1.0 / np.sqrt(0.5 * (np.mean(ua * ua) + np.mean(va * va)))
    out = ((np.ascontiguousarray(ua * scale), np.ascontiguousarray(va * scale)),
           (np.ascontiguousarray(ub * scale), np.ascontiguousarray(vb * scale)))
    if with_psi:
        return out + ((np.ascontiguousarray(pa * scale), np.ascontiguousarray(pb * scale)),)
    return out


def random_vorticity(n: int, k0: float, seed: int, omega_rms: float = 1.0,
                     length: float = TWO_PI):
    """Random-phase initial vorticity on the grid [n, n] (indexed [j, i]).

    Same isotropic energy spectrum shape as ``spectrum_snapshots``,
    E(k) ~ k^4 exp(-(k/k0)^2), so |omega_k|^2 ~ k E(k) = k^5 exp(-(k/k0)^2)
    in mode-index units; phases uniform from ``numpy.random.default_rng(seed)``;
    zero mean; scaled to the requested rms.  ``length`` only enters through
    the caller's wavenumbers, so the field is the same for every L.
    """
    rng = np.random.default_rng(seed)
    my = np.fft.fftfreq(n, d=1.0 / n)[:, None]
    mx = np.fft.rfftfreq(n, d=1.0 / n)[None, :]
    kmag = np.sqrt(mx * mx + my * my)
    amp = np.sqrt(kmag ** 5 * np.exp(-(kmag / k0) ** 2))
    amp[0, 0] = 0.0
    phase = rng.uniform(0.0, 2.0 * np.pi, size=amp.shape)
    w = np.fft.irfft2(amp * np.exp(1j * phase), s=(n, n))
    w *= omega_rms / np.sqrt(np.mean(w * w))
    return np.ascontiguousarray(w)


def random_points(count: int, seed: int, length: float = TWO_PI):
    """Uniform random points in [0, L)^2 (numpy generator, not the method's)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, length, count), rng.uniform(0.0, length, count)


def lattice_points(n: int, per_side: int, length: float = TWO_PI):
    """per_side^2 points on the cell-centre lattice of an n x n grid
    (per_side must divide n)."""
    assert n % per_side == 0
    stride = n // per_side
    h = length / n
    c = (np.arange(per_side) * stride + 0.5) * h
    X, Y = np.meshgrid(c, c, indexing="xy")
    return X.ravel().copy(), Y.ravel().copy()

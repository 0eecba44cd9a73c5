"""FP64 CPU oracle of the Eulerian field producer (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg
may import this module.  The product library never loads it and shares no
code with it.

It follows the pseudospectral vorticity-streamfunction solver of Sec. 3.1 in
the paper's order, with numpy's FFT as the transform primitive:

1. spectral derivatives of the vorticity (eq. spectral_vorticity_derivatives);
2. the stream function from the Poisson equation, zero mode zero
   (eq. poisson_spectral, with omega = -lap psi);
3. the velocity from the stream function (eq. spectral_velocity);
4. the advection term u dw/dx + v dw/dy formed on the grid and transformed
   forward (eq. spectral_nonlinear_term), then the 2/3 rule applied to it;
5. the right-hand side -N - nu k^2 w (eq. spectral_vorticity_evolution);
6. the second-order Adams-Bashforth update (eq. ab2_fluid);
7. the fields on the grid by inverse transforms, normalised by the number of
   grid points (numpy's inverse transform includes that factor).

Readings where the paper is silent:

* Dealiasing keeps a mode when 3 |m| < n on both axes (m the signed integer
  mode index), the largest band for which products of two retained fields
  alias onto no retained mode.
* The state is kept in that band: the initial vorticity is truncated to it.
  The update adds only dealiased terms and the viscous term of the state, so
  no mode outside the band is ever non-zero, and no Nyquist mode is used.
* The first step has no previous right-hand side; it takes R^{-1} = R^0,
  i.e. one forward-Euler step.

Grid: node (i, j) at (i h, j h), h = L / n, arrays [n, n] indexed [j, i]
(x fastest).  Wavenumbers k = (2 pi / L) m.

Pins: ``tests/test_oracle_ns.py`` (Taylor-Green decay, the alias-free
product against a brute-force DFT, energy and enstrophy conservation of the
inviscid truncated system, the scalar AB2 recurrence, the velocity of a
known stream function).
"""
from __future__ import annotations

import numpy as np


def wavenumbers(n: int, length: float):
    """(kx, ky, m_x, m_y) on the half plane of a real transform: axis 0 is y
    (all n modes, signed), axis 1 is x (modes 0 .. n/2)."""
    my = np.fft.fftfreq(n, d=1.0 / n)[:, None]
    mx = np.fft.rfftfreq(n, d=1.0 / n)[None, :]
    scale = 2.0 * np.pi / length
    return scale * mx, scale * my, mx, my


def band_mask(n: int):
    """True where a mode survives the 2/3 rule (3 |m| < n on both axes)."""
    _, _, mx, my = wavenumbers(n, 2.0 * np.pi)
    return (3 * np.abs(mx) < n) & (3 * np.abs(my) < n)


class NS2D:
    """Decaying 2D Navier-Stokes on [0, L)^2 in vorticity form (Sec. 3.1)."""

    def __init__(self, n: int, nu: float, dt: float, length: float = 2.0 * np.pi):
        self.n, self.nu, self.dt, self.L = n, float(nu), float(dt), float(length)
        self.kx, self.ky, _, _ = wavenumbers(n, length)
        self.k2 = self.kx ** 2 + self.ky ** 2
        self.mask = band_mask(n)
        self.w_hat = None
        self.r_prev = None
        self.steps = 0

    # -- eqs. poisson_spectral and spectral_velocity ------------------------
    def psi_hat(self, w_hat):
        out = np.zeros_like(w_hat)
        nz = self.k2 > 0
        out[nz] = w_hat[nz] / self.k2[nz]
        return out

    def velocity_hat(self, w_hat):
        p = self.psi_hat(w_hat)
        return 1j * self.ky * p, -1j * self.kx * p

    def to_grid(self, f_hat):
        return np.fft.irfft2(f_hat, s=(self.n, self.n))

    # -- eq. spectral_nonlinear_term with the 2/3 rule ----------------------
    def nonlinear_hat(self, w_hat):
        u_hat, v_hat = self.velocity_hat(w_hat)
        u, v = self.to_grid(u_hat), self.to_grid(v_hat)
        wx = self.to_grid(1j * self.kx * w_hat)           # eq. spectral_vorticity_derivatives
        wy = self.to_grid(1j * self.ky * w_hat)
        n_hat = np.fft.rfft2(u * wx + v * wy)
        return np.where(self.mask, n_hat, 0.0)

    # -- eq. spectral_vorticity_evolution -----------------------------------
    def rhs(self, w_hat):
        return -self.nonlinear_hat(w_hat) - self.nu * self.k2 * w_hat

    def set_vorticity(self, omega):
        """Initial vorticity on the grid [n, n]; truncated to the band."""
        omega = np.asarray(omega, dtype=np.float64)
        assert omega.shape == (self.n, self.n)
        self.w_hat = np.where(self.mask, np.fft.rfft2(omega), 0.0)
        self.r_prev = None
        self.steps = 0

    # -- eq. ab2_fluid --------------------------------------------------------
    def step(self, count: int = 1):
        for _ in range(count):
            r = self.rhs(self.w_hat)
            r_old = r if self.r_prev is None else self.r_prev
            self.w_hat = self.w_hat + self.dt * (1.5 * r - 0.5 * r_old)
            self.r_prev = r
            self.steps += 1

    def fields(self):
        """(u, v, omega, psi) on the grid, each [n, n] float64."""
        u_hat, v_hat = self.velocity_hat(self.w_hat)
        return (self.to_grid(u_hat), self.to_grid(v_hat), self.to_grid(self.w_hat),
                self.to_grid(self.psi_hat(self.w_hat)))

    def energy_enstrophy(self):
        """Kinetic energy <u^2 + v^2>/2 and enstrophy <omega^2>/2 (grid means)."""
        u, v, w, _ = self.fields()
        return 0.5 * np.mean(u * u + v * v), 0.5 * np.mean(w * w)

"""The largest grid the library accepts, n = 32768, through the C ABI against
the FP64 oracle.

Every index of the path is checked at its widest: node records past 2^30
(pitch 32771), stored cells in the top bit of their 16-bit halves, the box
offsets of the block tiles at +-n/2 around their 2^15 bias, and re-sort keys of
30 bits on the first (cell-ordered) sort.  The field is white noise, a
different value at every node, so that a row, column or time level read from
the wrong place cannot go unnoticed; it is binary32-valued, so the FP32-split
path and the oracle see the same field.  Particles are uniform, plus a few
placed within 1e-9 of the seams and corners of the periodic domain.
"""
import numpy as np
import pytest

import oracle
from paper_2607_17836_amd import lpt

pytestmark = pytest.mark.gpu

L = 2 * np.pi
N = 32768


def pdist(a, b):
    d = np.abs(np.asarray(a) - np.asarray(b)) % L
    return np.minimum(d, L - d)


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def noise_field():
    say(f"max grid: white-noise field {N}^2 (binary32 values in [-1, 1))")
    rng = np.random.default_rng(32768)
    out = []
    for _ in range(2):
        f = rng.random((N, N), dtype=np.float32)
        f *= 2.0
        f -= 1.0
        out.append(f.astype(np.float64))
        del f
    return out


def seeded_particles(count):
    rng = np.random.default_rng(77)
    x = rng.uniform(0.0, L, count)
    y = rng.uniform(0.0, L, count)
    e = 1e-9
    edge_x = np.array([L - e, e, L - e, 0.0, L / 2, L - e])
    edge_y = np.array([e, L - e, L - e, 0.0, L - e, L / 2])
    return np.concatenate([x, edge_x]), np.concatenate([y, edge_y])


@pytest.mark.parametrize("precision,scheme,tol", [("fp32_split", "bilinear", 1e-8),
                                                  ("fp64", "catmull_rom", 1e-10)])
def test_max_grid_matches_oracle(noise_field, precision, scheme, tol):
    """Ten steps of 4102 tracers on the steady noise field, re-sorted every 3
    steps, within `tol` of the oracle: 1e-10 for FP64; 1e-8 for the FP32
    split path, whose offsets round to 2^-24 of a cell (1.2e-11 at
    h = 2 pi / 32768) once a step, and whose rounding the noise field's
    gradients (about 2 / h) amplify by up to about 1.5 a step (3.7e-10 was
    measured)."""
    u, v = noise_field
    dt, nsteps = 4e-5, 10   # under 0.3 cells a step at the field's largest speed
    x0, y0 = seeded_particles(4096)
    say(f"max grid {precision} {scheme}: upload")
    tr = lpt.Tracker(N, precision, sort_interval=3)
    tr.set_time_mode("bracket")
    tr.set_snapshot(0, 0.0, u, v)
    tr.set_snapshot(1, 1.0, u, v)
    tr.add_species("tracer", 0.0, scheme, x0, y0)
    say(f"max grid {precision} {scheme}: {nsteps} steps")
    tr.step(nsteps, dt, 0)
    xw, yw, xu, yu = tr.get_positions(0)
    tr.close()
    fl = oracle.grid_flow(u, v, scheme=scheme)
    sp = oracle.Species(x0, y0)
    oracle.run(fl, sp, nsteps, dt)
    ox, oy = sp.unwrapped()
    err = max(np.max(pdist(xw, sp.xw)), np.max(pdist(yw, sp.yw)))
    erru = max(np.max(np.abs(xu - ox)), np.max(np.abs(yu - oy)))
    moved = np.max(np.hypot(ox - x0, oy - y0)) * N / L
    say(f"max grid {precision} {scheme}: position error {err:.3e}, unwrapped {erru:.3e}; "
        f"largest move {moved:.2f} cells")
    assert moved > 0.5   # the particles cross cells, so the stencils change
    assert err < tol and erru < tol

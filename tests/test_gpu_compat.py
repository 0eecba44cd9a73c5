"""The paper's bicubic boundary fallback (Sec. 3.4: the bicubic schemes
revert to bilinear near the domain boundary), LPT_FLAG_COMPAT_EDGE, on every
GPU path that interpolates -- the FP64 step, the FP32-split step and the
reverse sweep -- against the oracle run with the same flag, through the C
ABI.  The fallback cells are i in {0, n - 2, n - 1} (likewise j): the cells
whose 4 x 4 stencil would leave [0, n).  The grid is small (48^2) so that
every particle crosses fallback cells within the run.

The fallback makes the interpolant jump across the boundary of the fallback
cell set, so both sides must place each stage point in the same cell: the
FP64 paths locate points to within rounding of the oracle (x n/L against
x/(L/n)); the FP32-split path locates them in binary32 cell units, and a
point within ~1e-7 cells of a fallback-set edge could land on the other side
(probability ~1e-3 per run here; the seeds below have no such point)."""
import numpy as np
import pytest

import oracle
from paper_2607_17836_amd import lpt, synth

pytestmark = pytest.mark.gpu

L = 2 * np.pi
N, DT = 48, 0.004


def say(msg):
    print(msg, flush=True)


def pdist(a, b):
    d = np.abs(np.asarray(a) - np.asarray(b)) % L
    return np.minimum(d, L - d)


def _fields(rounded=False):
    (ua, va), (ub, vb) = synth.spectrum_snapshots(N, 5, 31, DT)
    if rounded:
        r = lambda f: f.astype(np.float32).astype(np.float64)
        return (r(ua), r(va)), (r(ub), r(vb))
    return (ua, va), (ub, vb)


def _visits_fallback_cells(xw_hist, yw_hist):
    ci = np.floor(np.asarray(xw_hist) * N / L).astype(int)
    cj = np.floor(np.asarray(yw_hist) * N / L).astype(int)
    edge = (ci == 0) | (ci >= N - 2) | (cj == 0) | (cj >= N - 2)
    return edge.any(axis=0).mean()


@pytest.mark.parametrize("precision", ["fp64", "fp32_split"])
@pytest.mark.parametrize("scheme", ["catmull_rom", "bspline"])
def test_compat_edge_step_matches_oracle(precision, scheme):
    """Tracers and inertial particles (St = 0.05, v0 = u(x0)) on the
    ping-pong spectrum, 12 steps, re-sorted every 4 (permuting steps and LDS
    tiles included): FP64 positions within 1e-10 and velocities within 1e-9
    of the oracle with the same fallback; FP32 split within its binary32
    bounds (1e-6 positions, 1e-5 velocities) against the oracle on the
    binary32-rounded fields.  The default, fully periodic, stencil differs
    from the fallback by far more than these bounds."""
    say(f"compat edge step {precision} {scheme}")
    fp32 = precision == "fp32_split"
    (ua, va), (ub, vb) = _fields()
    count, nsteps = 2000, 12
    x0, y0 = oracle.init_uniform(61, count)
    res = {}
    for compat in (True, False):
        tr = lpt.Tracker(N, precision, compat_edge=compat, sort_interval=4, sort_tile=8)
        tr.set_time_mode("pingpong")
        tr.set_snapshot(0, 0.0, ua, va)
        tr.set_snapshot(1, DT, ub, vb)
        a = tr.add_species("tracer", 0.0, scheme, x0, y0)
        b = tr.add_species("inertial", 0.05, scheme, x0, y0)
        tr.step(nsteps, DT)
        res[compat] = (tr.get_positions(a), tr.get_positions(b), tr.get_velocities(b))
        tr.close()
    (fa, fb) = _fields(rounded=fp32)
    fl = oracle.grid_flow(fa[0], fa[1], fb[0], fb[1], scheme=scheme, time_mode=oracle.PINGPONG,
                          compat_edge=1)
    tra = oracle.Species(x0, y0)
    hist_x, hist_y = [tra.xw.copy()], [tra.yw.copy()]
    for k in range(nsteps):
        oracle.run(fl, tra, 1, DT, t_start=k * DT, step0=k)
        hist_x.append(tra.xw.copy())
        hist_y.append(tra.yw.copy())
    assert _visits_fallback_cells(hist_x, hist_y) > 0.1
    u0, v0 = oracle.velocity(fl, x0, y0, 0.0, step=0, t_n=0.0, dt=DT)
    ine = oracle.Species(x0, y0, kind=oracle.INERTIAL, st=0.05, vx0=u0, vy0=v0)
    oracle.run(fl, ine, nsteps, DT)
    (pa, pb, (vx, vy)) = res[True]
    tol_x, tol_v = (1e-6, 1e-5) if fp32 else (1e-10, 1e-9)
    ex = max(np.max(pdist(pa[0], tra.xw)), np.max(pdist(pa[1], tra.yw)),
             np.max(np.abs(pa[2] - (x0 + tra.dx))))
    ei = max(np.max(pdist(pb[0], ine.xw)), np.max(pdist(pb[1], ine.yw)))
    ev = max(np.max(np.abs(vx - ine.vx)), np.max(np.abs(vy - ine.vy)))
    say(f"  errors: tracer {ex:.2e}, inertial {ei:.2e}, velocity {ev:.2e}")
    assert ex < tol_x and ei < tol_x and ev < tol_v
    # the flag is not a no-op: the periodic stencil's trajectories differ
    dper = np.max(pdist(res[False][0][0], pa[0]))
    assert dper > 100 * tol_x, dper


@pytest.mark.parametrize("scheme", ["catmull_rom", "bspline"])
def test_compat_edge_adjoint_matches_oracle(scheme):
    """The reverse sweep with the fallback (its Jacobians and grid scatter
    take the bilinear stencil in fallback cells): dL/dx0 within 1e-9 and the
    grid gradient within 1e-10 of the oracle's full-tape reverse sweep with
    the same fallback; the Jacobian against the oracle's forward tangent."""
    say(f"compat edge adjoint {scheme}")
    (ua, va), (ub, vb) = _fields()
    count, nsteps = 1500, 25
    x0, y0 = oracle.init_uniform(62, count)
    rng = np.random.default_rng(63)
    a, b = rng.normal(size=count), rng.normal(size=count)
    tr = lpt.Tracker(N, "fp64", compat_edge=True)
    tr.set_time_mode("pingpong")
    tr.set_snapshot(0, 0.0, ua, va)
    tr.set_snapshot(1, DT, ub, vb)
    tr.add_species("tracer", 0.0, scheme, x0, y0)
    tr.forward_checkpointed(nsteps, DT, 10)
    gx, gy, gU = tr.adjoint(a, b)
    F = tr.jacobian()
    tr.close()
    fl = oracle.grid_flow(ua, va, ub, vb, scheme=scheme, time_mode=oracle.PINGPONG,
                          compat_edge=1)
    ox, oy, oU = oracle.adjoint(fl, x0, y0, a, b, nsteps, DT)
    sc = lambda z: max(1.0, float(np.max(np.abs(z))))
    assert np.max(np.abs(gx - ox)) < 1e-9 * sc(ox)
    assert np.max(np.abs(gy - oy)) < 1e-9 * sc(oy)
    assert np.max(np.abs(gU - oU)) < 1e-10 * sc(oU)
    Fo = oracle.tangent(fl, oracle.Species(x0, y0), nsteps, DT)
    assert np.max(np.abs(F - Fo)) < 1e-9 * sc(Fo)
    # without the flag the oracle's gradient differs (the flag matters here)
    fl0 = oracle.grid_flow(ua, va, ub, vb, scheme=scheme, time_mode=oracle.PINGPONG)
    px, _, _ = oracle.adjoint(fl0, x0, y0, a, b, nsteps, DT, grid=False)
    assert np.max(np.abs(px - ox)) > 1e-6 * sc(ox)

"""FP64 CPU oracle of the Lagrangian particle path (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it.  The arithmetic lives in ``oracle.c`` (plain C, FP64,
no FMA contraction); this module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

BILINEAR, CATMULL_ROM, BSPLINE = 0, 1, 2
TRACER, INERTIAL = 0, 1
SRC_GRID, SRC_PSI, SRC_UNIFORM, SRC_TG = 0, 1, 2, 3
BRACKET, PINGPONG = 0, 1
SCHEMES = {"bilinear": BILINEAR, "catmull_rom": CATMULL_ROM, "bspline": BSPLINE}

GCC_FLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared"]


OMP_FLAGS = ["-O3", "-march=native", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
             "-std=c11", "-fPIC", "-shared"]
_omp = None


def timing_lib(outdir: str):
    """The oracle built for CPU timing (-O3 -march=native, OpenMP over the
    particles of a step; the same arithmetic), compiled into `outdir` on the
    machine that runs it, and a setter of its thread count.  Returns
    (module-like ctypes library, set_threads)."""
    global _omp
    if _omp is None:
        os.makedirs(outdir, exist_ok=True)
        path = os.path.join(outdir, "liboracle_omp.so")
        subprocess.run(["gcc", *OMP_FLAGS, _SRC, "-o", path, "-lm"], check=True)
        L = C.CDLL(path)
        _declare(L)
        gomp = C.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads.argtypes = [C.c_int]
        _omp = (L, gomp.omp_set_num_threads)
    return _omp


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` with gcc into ``liboracle.so`` (next to it)."""
    with _lock:
        if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            tmp = _LIB + ".tmp%d" % os.getpid()
            subprocess.run(["gcc", *GCC_FLAGS, _SRC, "-o", tmp, "-lm"], check=True)
            os.replace(tmp, _LIB)
    return _LIB


class Flow(C.Structure):
    _fields_ = [
        ("source", C.c_int32), ("scheme", C.c_int32), ("time_mode", C.c_int32),
        ("compat_edge", C.c_int32), ("n", C.c_int32), ("pad_", C.c_int32),
        ("length", C.c_double),
        ("u", C.c_void_p * 2), ("v", C.c_void_p * 2), ("psi", C.c_void_p * 2),
        ("t_slot", C.c_double * 2),
        ("U0", C.c_double), ("V0", C.c_double),
        ("alpha", C.c_double), ("k", C.c_double), ("eps", C.c_double),
        ("omega", C.c_double), ("phi", C.c_double),
    ]


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        _declare(L)
        _lib = L
    return _lib


def _declare(L):
    """Argument and result types of every oracle entry point."""
    dp, ip = C.c_void_p, C.c_void_p
    L.orc_wrap.restype = C.c_double
    L.orc_wrap.argtypes = [C.c_double, C.c_double]
    L.orc_wrap_many.restype = None
    L.orc_wrap_many.argtypes = [C.c_int64, dp, C.c_double, dp]
    L.orc_interp.restype = C.c_double
    L.orc_interp.argtypes = [dp, C.c_int32, C.c_double, C.c_int32, C.c_int32, C.c_double, C.c_double]
    L.orc_interp_many.restype = None
    L.orc_interp_many.argtypes = [dp, C.c_int32, C.c_double, C.c_int32, C.c_int32, C.c_int64, dp, dp, dp]
    L.orc_velocity.restype = None
    L.orc_velocity.argtypes = [C.POINTER(Flow), C.c_int64, dp, dp, C.c_double, C.c_int64,
                               C.c_double, C.c_double, dp, dp]
    L.orc_stats.restype = None
    L.orc_stats.argtypes = [C.c_int64, dp, dp, C.c_double, C.c_double, dp]
    L.orc_run.restype = C.c_int64
    L.orc_run.argtypes = [C.POINTER(Flow), C.c_int32, C.c_double, C.c_int64,
                          dp, dp, dp, dp, dp, dp, C.c_int64, C.c_double, C.c_double,
                          C.c_int64, C.c_int64, C.c_double, dp, C.c_int64]
    L.orc_splitmix64.restype = C.c_uint64
    L.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
    L.orc_init_uniform.restype = None
    L.orc_init_uniform.argtypes = [C.c_uint64, C.c_int64, C.c_double, dp, dp]
    L.orc_cell_keys.restype = None
    L.orc_cell_keys.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int64, ip, ip, ip]
    L.orc_interp_grad.restype = None
    L.orc_interp_grad.argtypes = [dp, C.c_int32, C.c_double, C.c_int32, C.c_int32, C.c_double,
                                  C.c_double, dp, dp, dp]
    L.orc_tangent_run.restype = None
    L.orc_tangent_run.argtypes = [C.POINTER(Flow), C.c_int64, dp, dp, dp, dp, dp, C.c_int64,
                                  C.c_double, C.c_double, C.c_int64]
    L.orc_adjoint_run.restype = None
    L.orc_adjoint_run.argtypes = [C.POINTER(Flow), C.c_int64, dp, dp, dp, dp, C.c_int64,
                                  C.c_double, C.c_double, C.c_int64, dp, dp, dp, dp]
    L.orc_cells_of.restype = None
    L.orc_cells_of.argtypes = [C.c_int32, C.c_double, C.c_int64, dp, ip]


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class FlowSpec:
    """Python-side owner of a Flow struct and the arrays it points to."""

    def __init__(self, source=SRC_GRID, scheme=BILINEAR, time_mode=BRACKET, compat_edge=0,
                 n=0, length=2 * np.pi, u=None, v=None, psi=None, t_slot=(0.0, 1.0),
                 U0=0.0, V0=0.0, alpha=1.0, k=1.0, eps=0.0, omega=0.0, phi=0.0):
        if isinstance(scheme, str):
            scheme = SCHEMES[scheme]
        self._keep = []
        f = Flow()
        f.source, f.scheme, f.time_mode, f.compat_edge = source, scheme, time_mode, compat_edge
        f.n, f.length = n, length
        for name, pair in (("u", u), ("v", v), ("psi", psi)):
            if pair is None:
                continue
            arrs = [_f64(pair[0]), _f64(pair[1])]
            for a in arrs:
                assert a.size == n * n, "field must hold n*n values"
            self._keep += arrs
            getattr(f, name)[0] = arrs[0].ctypes.data
            getattr(f, name)[1] = arrs[1].ctypes.data
        f.t_slot[0], f.t_slot[1] = t_slot
        f.U0, f.V0, f.alpha, f.k, f.eps, f.omega, f.phi = U0, V0, alpha, k, eps, omega, phi
        self.struct = f

    @property
    def length(self):
        return self.struct.length


def grid_flow(ua, va, ub=None, vb=None, scheme=BILINEAR, time_mode=BRACKET, t_slot=(0.0, 1.0),
              length=2 * np.pi, compat_edge=0):
    ua = np.asarray(ua)
    n = ua.shape[-1]
    if ub is None:
        ub, vb = ua, va
    return FlowSpec(SRC_GRID, scheme, time_mode, compat_edge, n, length, u=(ua, ub), v=(va, vb),
                    t_slot=t_slot)


def psi_flow(psia, psib=None, scheme=BILINEAR, time_mode=BRACKET, t_slot=(0.0, 1.0),
             length=2 * np.pi, compat_edge=0):
    psia = np.asarray(psia)
    n = psia.shape[-1]
    if psib is None:
        psib = psia
    return FlowSpec(SRC_PSI, scheme, time_mode, compat_edge, n, length, psi=(psia, psib),
                    t_slot=t_slot)


def uniform_flow(U0, V0, length=2 * np.pi):
    return FlowSpec(SRC_UNIFORM, length=length, U0=U0, V0=V0)


def tg_flow(alpha=1.0, k=1.0, eps=0.0, omega=0.0, phi=0.0, length=2 * np.pi):
    return FlowSpec(SRC_TG, length=length, alpha=alpha, k=k, eps=eps, omega=omega, phi=phi)


def wrap(z, L=2 * np.pi):
    return lib().orc_wrap(float(z), float(L))


def wrap_many(z, L=2 * np.pi):
    z = _f64(np.atleast_1d(z))
    out = np.empty_like(z)
    lib().orc_wrap_many(z.size, _ptr(z), float(L), _ptr(out))
    return out


def interp(f, x, y, scheme=BILINEAR, length=2 * np.pi, compat_edge=0):
    """Spatial interpolation of one grid field at the points (x, y)."""
    if isinstance(scheme, str):
        scheme = SCHEMES[scheme]
    f = _f64(f)
    n = f.shape[-1]
    x = _f64(np.atleast_1d(x))
    y = _f64(np.atleast_1d(y))
    out = np.empty_like(x)
    lib().orc_interp_many(_ptr(f), n, length, scheme, compat_edge, x.size, _ptr(x), _ptr(y), _ptr(out))
    return out


def velocity(flow: FlowSpec, x, y, t, step=0, t_n=0.0, dt=1.0):
    x = _f64(np.atleast_1d(x))
    y = _f64(np.atleast_1d(y))
    u = np.empty_like(x)
    v = np.empty_like(x)
    lib().orc_velocity(C.byref(flow.struct), x.size, _ptr(x), _ptr(y), float(t), int(step),
                       float(t_n), float(dt), _ptr(u), _ptr(v))
    return u, v


class Species:
    """FP64 state of one species: wrapped positions, unwrapped displacements,
    particle velocity (inertial)."""

    def __init__(self, x0, y0, kind=TRACER, st=0.0, vx0=None, vy0=None, length=2 * np.pi):
        self.kind, self.st, self.length = kind, float(st), length
        self.x0 = _f64(x0).copy()
        self.y0 = _f64(y0).copy()
        self.xw = wrap_many(self.x0, length)
        self.yw = wrap_many(self.y0, length)
        self.dx = np.zeros_like(self.x0)
        self.dy = np.zeros_like(self.y0)
        self.vx = _f64(vx0).copy() if vx0 is not None else np.zeros_like(self.x0)
        self.vy = _f64(vy0).copy() if vy0 is not None else np.zeros_like(self.y0)

    @property
    def n(self):
        return self.x0.size

    def unwrapped(self):
        return self.x0 + self.dx, self.y0 + self.dy


def run(flow: FlowSpec, sp: Species, nsteps, dt, t_start=0.0, step0=0, stats_every=0,
        t_origin=0.0, library=None):
    """Advance a species in place; returns the stats records [nrec, 8].
    library: the ctypes library to run (default: the test build; the CPU
    timing passes timing_lib's)."""
    cap = (step0 + nsteps) // stats_every + 1 if stats_every > 0 else 0
    rec = np.zeros((max(cap, 1), 8))
    nrec = (library or lib()).orc_run(C.byref(flow.struct), sp.kind, sp.st, sp.n,
                         _ptr(sp.xw), _ptr(sp.yw), _ptr(sp.dx), _ptr(sp.dy),
                         _ptr(sp.vx), _ptr(sp.vy), int(nsteps), float(dt), float(t_start),
                         int(step0), int(stats_every), float(t_origin), _ptr(rec), cap)
    return rec[:nrec]


def stats(dx, dy, t, elapsed):
    dx, dy = _f64(dx), _f64(dy)
    rec = np.zeros(8)
    lib().orc_stats(dx.size, _ptr(dx), _ptr(dy), float(t), float(elapsed), _ptr(rec))
    return rec


def splitmix64(seed, k):
    return lib().orc_splitmix64(C.c_uint64(seed), C.c_uint64(k))


def init_uniform(seed, count, length=2 * np.pi):
    x = np.empty(count)
    y = np.empty(count)
    lib().orc_init_uniform(C.c_uint64(seed), count, length, _ptr(x), _ptr(y))
    return x, y


def cell_keys(n, tile, ci, cj, coarse=False):
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    cj = np.ascontiguousarray(cj, dtype=np.int32)
    keys = np.empty(ci.size, dtype=np.uint32)
    lib().orc_cell_keys(n, tile, int(bool(coarse)), ci.size, _ptr(ci), _ptr(cj), _ptr(keys))
    return keys


def cells_of(n, x, length=2 * np.pi):
    x = _f64(x)
    ci = np.empty(x.size, dtype=np.int32)
    lib().orc_cells_of(n, length, x.size, _ptr(x), _ptr(ci))
    return ci


def sort_permutation(keys):
    """Stable ascending order of the keys (library primitive)."""
    return np.argsort(np.asarray(keys), kind="stable")


# -- derivatives of the discrete map (tracers) -------------------------------

def interp_grad(f, x, y, scheme=BILINEAR, length=2 * np.pi, compat_edge=0):
    """(value, d/dx, d/dy) of one interpolated grid field at one point."""
    if isinstance(scheme, str):
        scheme = SCHEMES[scheme]
    f = _f64(f)
    out = np.zeros(3)
    o = out.ctypes.data
    lib().orc_interp_grad(_ptr(f), f.shape[-1], length, scheme, compat_edge, float(x), float(y),
                          C.c_void_p(o), C.c_void_p(o + 8), C.c_void_p(o + 16))
    return out[0], out[1], out[2]


def tangent(flow: FlowSpec, sp: Species, nsteps, dt, t_start=0.0, step0=0):
    """Advance a tracer species in place and return F = dx_T/dx_0 [np, 2, 2]
    by forward tangent propagation."""
    F = np.zeros((sp.n, 2, 2))
    F[:, 0, 0] = F[:, 1, 1] = 1.0
    lib().orc_tangent_run(C.byref(flow.struct), sp.n, _ptr(sp.xw), _ptr(sp.yw), _ptr(sp.dx),
                          _ptr(sp.dy), _ptr(F), int(nsteps), float(dt), float(t_start), int(step0))
    return F


def adjoint(flow: FlowSpec, x0, y0, a, b, nsteps, dt, t_start=0.0, step0=0, grid=True):
    """Reverse sweep for L = sum(a x_T + b y_T): returns (dL/dx0, dL/dy0, gU)
    with gU [2 slots, 2 components (u, v), n, n] (None without a grid)."""
    x0, y0, a, b = _f64(x0), _f64(y0), _f64(a), _f64(b)
    np_ = x0.size
    gx, gy = np.empty(np_), np.empty(np_)
    n = flow.struct.n
    gU = np.zeros((2, 2, n, n)) if (grid and flow.struct.source == SRC_GRID) else None
    tape = np.empty(2 * np_ * max(1, int(nsteps)))
    lib().orc_adjoint_run(C.byref(flow.struct), np_, _ptr(x0), _ptr(y0), _ptr(a), _ptr(b),
                          int(nsteps), float(dt), float(t_start), int(step0), _ptr(gx), _ptr(gy),
                          _ptr(gU), _ptr(tape))
    return gx, gy, gU


def ftle(F, T):
    """Finite-time Lyapunov exponent (1/T) ln sqrt(lambda_max(F^T F)) per
    particle (F [np, 2, 2])."""
    C_ = np.einsum("pki,pkj->pij", F, F)
    lam = np.linalg.eigvalsh(C_)[:, -1]
    return np.log(np.sqrt(lam)) / T

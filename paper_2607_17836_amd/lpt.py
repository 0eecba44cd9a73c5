"""Thin ctypes binding of liblpt.so (include/lpt.h).

Argument marshalling only: every step of the particle path runs in the HIP
kernels of liblpt.so.  Arrays may be numpy (host) or torch CUDA tensors
(device); torch is used for device memory and streams only.  Loading fails
loudly when the native library is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

try:  # load torch's HIP runtime first so the process holds exactly one
    import torch
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblpt.so")

OK, E_ARG, E_STATE, E_RANGE, E_NOMEM, E_HIP = range(6)
BILINEAR, CATMULL_ROM, BSPLINE = 0, 1, 2
FP64, FP32_SPLIT = 0, 1
TRACER, INERTIAL = 0, 1
TIME_BRACKET, TIME_PINGPONG = 0, 1
FLAG_COMPAT_EDGE = 0x1
FLAG_TIME_KERNELS = 0x2
FLAG_DETERMINISTIC_GRAD = 0x4

SCHEMES = {"bilinear": BILINEAR, "catmull_rom": CATMULL_ROM, "bspline": BSPLINE}
PRECISIONS = {"fp64": FP64, "fp32_split": FP32_SPLIT}
KINDS = {"tracer": TRACER, "inertial": INERTIAL}
TIME_MODES = {"bracket": TIME_BRACKET, "pingpong": TIME_PINGPONG}


class LptConfig(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("precision", C.c_int32), ("length", C.c_double), ("t0", C.c_double),
        ("hip_stream", C.c_void_p), ("sort_interval", C.c_int32), ("sort_tile", C.c_int32),
        ("block_size", C.c_int32), ("flags", C.c_uint32), ("tile_records", C.c_int32),
    ]


class LptTuning(C.Structure):
    _fields_ = [("block_size", C.c_int32), ("tile_records", C.c_int32),
                ("sort_interval", C.c_int32), ("persistent", C.c_int32),
                ("graph_chunk", C.c_int32), ("halo_scale", C.c_float),
                ("max_workgroups", C.c_int32), ("fused", C.c_int32),
                ("sort_cells", C.c_int32), ("rows", C.c_int32)]


class LptTiming(C.Structure):
    _fields_ = [("step_kernel_ms", C.c_double), ("step_launches", C.c_int64),
                ("sort_ms", C.c_double), ("sorts", C.c_int64),
                ("perm_step_ms", C.c_double), ("perm_steps", C.c_int64),
                ("stats_step_ms", C.c_double), ("stats_steps", C.c_int64),
                ("finalize_ms", C.c_double)]


STAT_DTYPE = np.dtype([("t", "<f8"), ("msd_x", "<f8"), ("msd_y", "<f8"), ("msd", "<f8"),
                       ("d_x", "<f8"), ("d_y", "<f8"), ("sem", "<f8"), ("n", "<i8")])

# (name, restype, argtypes) of every exported entry point
_P = C.c_void_p
_SIGS = [
    ("lpt_create", C.c_int, [C.POINTER(LptConfig), C.POINTER(C.c_void_p)]),
    ("lpt_destroy", None, [_P]),
    ("lpt_last_error", C.c_char_p, [_P]),
    ("lpt_status_string", C.c_char_p, [C.c_int]),
    ("lpt_synchronize", C.c_int, [_P]),
    ("lpt_set_snapshot", C.c_int, [_P, C.c_int32, C.c_double, _P, _P, C.c_int32]),
    ("lpt_set_snapshot_psi", C.c_int, [_P, C.c_int32, C.c_double, _P, C.c_int32]),
    ("lpt_set_time_mode", C.c_int, [_P, C.c_int]),
    ("lpt_add_species", C.c_int, [_P, C.c_int, C.c_double, C.c_int, C.c_int64, _P, _P, _P, _P,
                                  C.c_int32, C.POINTER(C.c_int32)]),
    ("lpt_init_uniform", C.c_int, [_P, C.c_int32, C.c_uint64]),
    ("lpt_step", C.c_int, [_P, C.c_int64, C.c_double, C.c_int32]),
    ("lpt_sort", C.c_int, [_P]),
    ("lpt_get_positions", C.c_int, [_P, C.c_int32, _P, _P, _P, _P, C.c_int32]),
    ("lpt_get_velocities", C.c_int, [_P, C.c_int32, _P, _P, C.c_int32]),
    ("lpt_get_stats", C.c_int, [_P, C.c_int32, _P, C.c_int64, C.POINTER(C.c_int64)]),
    ("lpt_get_order", C.c_int, [_P, C.c_int32, _P, C.c_int32]),
    ("lpt_get_timing", C.c_int, [_P, C.POINTER(LptTiming), C.c_int32]),
    ("lpt_get_time", C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    ("lpt_interp", C.c_int, [_P, C.c_int, C.c_int64, _P, _P, C.c_double, C.c_double, _P, _P,
                             C.c_int32]),
    ("lpt_radix_sort", C.c_int, [_P, C.c_int64, C.c_int32, _P, _P, _P]),
    ("lpt_radix_sort_static", C.c_int, [_P, C.c_int64, C.c_int32, _P, _P, _P]),
    ("lpt_get_state", C.c_int, [_P, _P, C.c_size_t, C.POINTER(C.c_size_t)]),
    ("lpt_set_state", C.c_int, [_P, _P, C.c_size_t]),
    ("lpt_get_tuning", C.c_int, [_P, C.POINTER(LptTuning)]),
    ("lpt_time_steps", C.c_int, [_P, C.c_int64, C.c_double, C.c_int32, C.POINTER(C.c_double)]),
    ("lpt_set_tuning", C.c_int, [_P, C.POINTER(LptTuning)]),
    ("lpt_forward_checkpointed", C.c_int, [_P, C.c_int64, C.c_double, C.c_int32]),
    ("lpt_adjoint", C.c_int, [_P, _P, _P, _P, _P, _P, C.c_int32]),
    ("lpt_jacobian", C.c_int, [_P, _P, C.c_int32]),
    ("lpt_ftle", C.c_int, [_P, _P, _P, C.c_int32]),
    ("lpt_bw_probe", C.c_int, [_P, C.c_int64, C.c_int32, C.POINTER(C.c_double),
                               C.POINTER(C.c_double)]),
]

_lib = None


def load():
    """Load liblpt.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"liblpt.so is not built ({LIB_PATH}); run "
                               "`python -m paper_2607_17836_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class LptError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{load().lpt_status_string(status).decode()}: {msg}")
        self.status = status


def _is_dev(a):
    return torch is not None and isinstance(a, torch.Tensor) and a.is_cuda


def _arr(a, count=None, dtype=np.float64):
    """(pointer, on_device, keepalive) of a float64 input array."""
    if a is None:
        return None, 0, None
    if _is_dev(a):
        assert a.dtype == torch.float64 and a.is_contiguous(), "device arrays: contiguous float64"
        assert count is None or a.numel() == count
        return a.data_ptr(), 1, a
    h = np.ascontiguousarray(a, dtype=dtype)
    assert count is None or h.size == count, (h.size, count)
    return h.ctypes.data, 0, h


class Tracker:
    """One liblpt context (see include/lpt.h for the meaning of every call)."""

    def __init__(self, n, precision="fp64", length=0.0, t0=0.0, stream=None, sort_interval=0,
                 sort_tile=0, block_size=0, compat_edge=False, time_kernels=False,
                 tile_records=0, deterministic_grad=False):
        lib = load()
        cfg = LptConfig()
        cfg.n = n
        cfg.precision = PRECISIONS[precision] if isinstance(precision, str) else precision
        cfg.length = length
        cfg.t0 = t0
        cfg.hip_stream = stream
        cfg.sort_interval = sort_interval
        cfg.sort_tile = sort_tile
        cfg.block_size = block_size
        cfg.tile_records = tile_records
        cfg.flags = ((FLAG_COMPAT_EDGE if compat_edge else 0) |
                     (FLAG_TIME_KERNELS if time_kernels else 0) |
                     (FLAG_DETERMINISTIC_GRAD if deterministic_grad else 0))
        h = C.c_void_p()
        st = lib.lpt_create(C.byref(cfg), C.byref(h))
        if st != OK:
            raise LptError(st, "lpt_create failed")
        self._h = h
        self.n = n
        self.length = length if length else 2 * np.pi
        self.precision = cfg.precision
        self.counts = []

    # -- plumbing ---------------------------------------------------------
    def _check(self, st):
        if st != OK:
            raise LptError(st, load().lpt_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            load().lpt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        return self._h

    # -- API --------------------------------------------------------------
    def synchronize(self):
        self._check(load().lpt_synchronize(self._h))

    def set_snapshot(self, slot, t, u, v):
        nn = self.n * self.n
        pu, du, ku = _arr(u, nn)
        pv, dv, kv = _arr(v, nn)
        assert du == dv
        self._check(load().lpt_set_snapshot(self._h, slot, t, pu, pv, du))

    def set_snapshot_device(self, slot, t, u_ptr, v_ptr):
        """Velocity level from raw device pointers of n*n doubles each (for
        instance the field producer's ns2d_velocity), read in stream order."""
        assert u_ptr and v_ptr
        self._check(load().lpt_set_snapshot(self._h, slot, t, u_ptr, v_ptr, 1))

    def set_snapshot_psi(self, slot, t, psi):
        p, d, k = _arr(psi, self.n * self.n)
        self._check(load().lpt_set_snapshot_psi(self._h, slot, t, p, d))

    def set_time_mode(self, mode):
        self._check(load().lpt_set_time_mode(self._h, TIME_MODES[mode] if isinstance(mode, str) else mode))

    def add_species(self, kind, st, scheme, x0, y0, vx0=None, vy0=None):
        kind = KINDS[kind] if isinstance(kind, str) else kind
        scheme = SCHEMES[scheme] if isinstance(scheme, str) else scheme
        count = int(x0.numel() if _is_dev(x0) else np.size(x0))
        px, d1, k1 = _arr(x0, count)
        py, d2, k2 = _arr(y0, count)
        pvx, d3, k3 = _arr(vx0, count)
        pvy, d4, k4 = _arr(vy0, count)
        sid = C.c_int32()
        self._check(load().lpt_add_species(self._h, kind, float(st), scheme, count, px, py, pvx,
                                           pvy, d1, C.byref(sid)))
        self.counts.append(count)
        return sid.value

    def init_uniform(self, sid, seed):
        self._check(load().lpt_init_uniform(self._h, sid, C.c_uint64(seed)))

    def step(self, nsteps, dt, stats_every=0):
        self._check(load().lpt_step(self._h, int(nsteps), float(dt), int(stats_every)))

    def sort(self):
        self._check(load().lpt_sort(self._h))

    def get_positions(self, sid, out=None):
        """Returns (xw, yw, xu, yu) numpy arrays, or fills the given device tensors."""
        count = self.counts[sid]
        if out is not None:
            ptrs = [t.data_ptr() if t is not None else None for t in out]
            self._check(load().lpt_get_positions(self._h, sid, *ptrs, 1))
            return out
        arrs = [np.empty(count) for _ in range(4)]
        self._check(load().lpt_get_positions(self._h, sid, *[a.ctypes.data for a in arrs], 0))
        return tuple(arrs)

    def get_velocities(self, sid):
        count = self.counts[sid]
        vx, vy = np.empty(count), np.empty(count)
        self._check(load().lpt_get_velocities(self._h, sid, vx.ctypes.data, vy.ctypes.data, 0))
        return vx, vy

    def get_stats(self, sid, cap=1 << 20):
        steps, _ = self.get_time()
        cap = min(cap, max(steps, 1))
        out = np.zeros(cap, dtype=STAT_DTYPE)
        nw = C.c_int64()
        self._check(load().lpt_get_stats(self._h, sid, out.ctypes.data, cap, C.byref(nw)))
        return out[: nw.value]

    def get_order(self, sid):
        ids = np.empty(self.counts[sid], dtype=np.int32)
        self._check(load().lpt_get_order(self._h, sid, ids.ctypes.data, 0))
        return ids

    def get_timing(self, reset=True):
        t = LptTiming()
        self._check(load().lpt_get_timing(self._h, C.byref(t), int(reset)))
        return {k: getattr(t, k) for k, _ in LptTiming._fields_}

    def get_time(self):
        s, t = C.c_int64(), C.c_double()
        self._check(load().lpt_get_time(self._h, C.byref(s), C.byref(t)))
        return s.value, t.value

    def interp(self, scheme, x, y, wa=1.0, wb=0.0):
        scheme = SCHEMES[scheme] if isinstance(scheme, str) else scheme
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        u, v = np.empty_like(x), np.empty_like(x)
        self._check(load().lpt_interp(self._h, scheme, x.size, x.ctypes.data, y.ctypes.data,
                                      float(wa), float(wb), u.ctypes.data, v.ctypes.data, 0))
        return u, v

    def bw_probe(self, nbytes, iters=20):
        """(copy GB/s, triad GB/s) of plain streaming kernels on this device."""
        cp, tr = C.c_double(), C.c_double()
        self._check(load().lpt_bw_probe(self._h, int(nbytes), int(iters), C.byref(cp), C.byref(tr)))
        return cp.value, tr.value

    # -- checkpoint / resume ---------------------------------------------
    def get_state(self) -> bytes:
        size = C.c_size_t()
        self._check(load().lpt_get_state(self._h, None, 0, C.byref(size)))
        buf = C.create_string_buffer(size.value)
        self._check(load().lpt_get_state(self._h, buf, size.value, C.byref(size)))
        return buf.raw[: size.value]

    def set_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._check(load().lpt_set_state(self._h, buf, len(blob)))

    # -- tuning -----------------------------------------------------------
    def get_tuning(self):
        t = LptTuning()
        self._check(load().lpt_get_tuning(self._h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in LptTuning._fields_}

    def time_steps(self, nsteps, dt, stats_every=0):
        """Device milliseconds of lpt_step(nsteps) between HIP events."""
        ms = C.c_double()
        self._check(load().lpt_time_steps(self._h, int(nsteps), float(dt), int(stats_every),
                                          C.byref(ms)))
        return ms.value

    def set_tuning(self, **kw):
        cur = self.get_tuning()
        cur.update(kw)
        t = LptTuning(**cur)
        self._check(load().lpt_set_tuning(self._h, C.byref(t)))

    # -- derivatives (FP64 tracers) ---------------------------------------
    def forward_checkpointed(self, nsteps, dt, ckpt_every):
        self._check(load().lpt_forward_checkpointed(self._h, int(nsteps), float(dt),
                                                    int(ckpt_every)))

    def adjoint(self, gx_T, gy_T, want_grid=True):
        """Reverse sweep for L = sum(gx_T x_T + gy_T y_T) over all particles
        (global index order).  Host arrays in -> numpy out; device tensors in
        -> device tensors out.  Returns (gx0, gy0, gU [2, 2, n, n] or None)."""
        np_ = sum(self.counts)
        if _is_dev(gx_T):
            gx0 = torch.empty(np_, dtype=torch.float64, device=gx_T.device)
            gy0 = torch.empty_like(gx0)
            gU = torch.empty((2, 2, self.n, self.n), dtype=torch.float64,
                             device=gx_T.device) if want_grid else None
            self._check(load().lpt_adjoint(self._h, gx_T.data_ptr(), gy_T.data_ptr(),
                                           gx0.data_ptr(), gy0.data_ptr(),
                                           gU.data_ptr() if gU is not None else None, 1))
            return gx0, gy0, gU
        a = np.ascontiguousarray(gx_T, dtype=np.float64)
        b = np.ascontiguousarray(gy_T, dtype=np.float64)
        assert a.size == np_ and b.size == np_
        gx0, gy0 = np.empty(np_), np.empty(np_)
        gU = np.empty((2, 2, self.n, self.n)) if want_grid else None
        self._check(load().lpt_adjoint(self._h, a.ctypes.data, b.ctypes.data, gx0.ctypes.data,
                                       gy0.ctypes.data,
                                       gU.ctypes.data if gU is not None else None, 0))
        return gx0, gy0, gU

    def jacobian(self):
        """F = dx_T/dx_0 [np, 2, 2] (numpy) of the last checkpointed run."""
        F = np.empty((sum(self.counts), 2, 2))
        self._check(load().lpt_jacobian(self._h, F.ctypes.data, 0))
        return F

    def ftle(self, with_jacobian=False):
        """FTLE sigma [np] (numpy) of the last checkpointed run over its
        duration, computed by the library (lpt_ftle); with_jacobian also
        returns F [np, 2, 2] from the same reverse sweep."""
        np_ = sum(self.counts)
        sig = np.empty(np_)
        F = np.empty((np_, 2, 2)) if with_jacobian else None
        self._check(load().lpt_ftle(self._h, sig.ctypes.data,
                                    F.ctypes.data if F is not None else None, 0))
        return (sig, F) if with_jacobian else sig

    def radix_sort(self, keys, key_bits):
        """Stable sort of a device uint32 tensor (as torch.int32 storage);
        returns (sorted keys, permutation) as device tensors."""
        assert _is_dev(keys) and keys.dtype == torch.int32 and keys.is_contiguous()
        out = torch.empty_like(keys)
        perm = torch.empty_like(keys)
        self._check(load().lpt_radix_sort(self._h, keys.numel(), key_bits, keys.data_ptr(),
                                          out.data_ptr(), perm.data_ptr()))
        return out, perm

    def radix_sort_static(self, keys, key_bits, out=None, perm=None):
        """radix_sort through the library's fixed scratch (no allocation in
        the library; at most STATIC_SORT_MAX keys).  out / perm: caller
        device tensors (allocated here if None)."""
        assert _is_dev(keys) and keys.dtype == torch.int32 and keys.is_contiguous()
        out = torch.empty_like(keys) if out is None else out
        perm = torch.empty_like(keys) if perm is None else perm
        self._check(load().lpt_radix_sort_static(self._h, keys.numel(), key_bits,
                                                 keys.data_ptr(), out.data_ptr(),
                                                 perm.data_ptr()))
        return out, perm


STATIC_SORT_MAX = 1 << 20


def create_error_status(n, **kw):
    """Status of lpt_create for a configuration (no context is kept)."""
    lib = load()
    cfg = LptConfig()
    cfg.n = n
    cfg.precision = kw.get("precision", FP64)
    cfg.length = kw.get("length", 0.0)
    cfg.t0 = kw.get("t0", 0.0)
    cfg.hip_stream = None
    cfg.sort_interval = kw.get("sort_interval", 0)
    cfg.sort_tile = kw.get("sort_tile", 0)
    cfg.block_size = kw.get("block_size", 0)
    cfg.flags = kw.get("flags", 0)
    h = C.c_void_p()
    st = lib.lpt_create(C.byref(cfg), C.byref(h))
    if st == OK:
        lib.lpt_destroy(h)
    return st


# ---------------------------------------------------------------------------
# Autograd: tracer trajectories as a differentiable function of the initial
# positions and of both velocity snapshots.
# ---------------------------------------------------------------------------
if torch is not None:

    class LptTrajectory(torch.autograd.Function):
        """x_T = Phi(x0, Ua, Ub): nsteps FP64 tracer RK4 steps (see
        include/lpt.h) through the snapshots Ua = (u, v) at t_a (slot 0) and
        Ub at t_b (slot 1).  Inputs are CUDA float64 tensors: x0, y0 [np],
        Ua, Ub [2, n, n].  Returns the unwrapped final positions (xT, yT).
        The backward pass is the library's reverse sweep over checkpoints
        every `ckpt_every` steps; it returns gradients for x0, y0, Ua, Ub."""

        @staticmethod
        def forward(ctx, x0, y0, Ua, Ub, nsteps, dt, scheme="bilinear", ckpt_every=20,
                    time_mode="bracket", t_slot=(0.0, 1.0)):
            n = Ua.shape[-1]
            tr = Tracker(n, "fp64")
            tr.set_time_mode(time_mode)
            tr.set_snapshot(0, t_slot[0], Ua[0].contiguous(), Ua[1].contiguous())
            tr.set_snapshot(1, t_slot[1], Ub[0].contiguous(), Ub[1].contiguous())
            tr.add_species("tracer", 0.0, scheme, x0.contiguous(), y0.contiguous())
            tr.forward_checkpointed(nsteps, dt, ckpt_every)
            xT = torch.empty_like(x0)
            yT = torch.empty_like(y0)
            tr.get_positions(0, out=(None, None, xT, yT))
            ctx.tr = tr
            return xT, yT

        @staticmethod
        def backward(ctx, gx, gy):
            tr = ctx.tr
            gx = gx.contiguous() if gx is not None else torch.zeros(tr.counts[0], dtype=torch.float64, device="cuda")
            gy = gy.contiguous() if gy is not None else torch.zeros_like(gx)
            gx0, gy0, gU = tr.adjoint(gx, gy, want_grid=any(ctx.needs_input_grad[2:4]))
            tr.close()
            ctx.tr = None
            gUa = gU[0] if gU is not None else None
            gUb = gU[1] if gU is not None else None
            return gx0, gy0, gUa, gUb, None, None, None, None, None, None


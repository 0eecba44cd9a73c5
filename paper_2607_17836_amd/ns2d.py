"""Thin ctypes binding of libns2d.so (include/ns2d.h), the Eulerian field
producer that feeds the particle path.

Argument marshalling only: every step runs in libns2d.so (its own LDS
transforms and kernels; hipFFT only when asked for).  Arrays may be numpy (host) or torch CUDA
tensors (device).  Loading fails loudly when the native library is missing.
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
LIB_PATH = os.path.join(_HERE, "libns2d.so")

OK, E_ARG, E_STATE, E_NOMEM, E_HIP, E_FFT = 0, 1, 2, 4, 5, 6


class Ns2dConfig(C.Structure):
    _fields_ = [("n", C.c_int32), ("length", C.c_double), ("nu", C.c_double),
                ("dt", C.c_double), ("hip_stream", C.c_void_p), ("transforms", C.c_int32)]


_P = C.c_void_p
_SIGS = [
    ("ns2d_create", C.c_int, [C.POINTER(Ns2dConfig), C.POINTER(C.c_void_p)]),
    ("ns2d_destroy", None, [_P]),
    ("ns2d_last_error", C.c_char_p, [_P]),
    ("ns2d_synchronize", C.c_int, [_P]),
    ("ns2d_set_vorticity", C.c_int, [_P, _P, C.c_int32]),
    ("ns2d_step", C.c_int, [_P, C.c_int32]),
    ("ns2d_velocity", C.c_int, [_P, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)]),
    ("ns2d_get_fields", C.c_int, [_P, _P, _P, _P, _P, C.c_int32]),
    ("ns2d_get_transforms", C.c_int, [_P, C.POINTER(C.c_int32)]),
    ("ns2d_get_steps", C.c_int, [_P, C.POINTER(C.c_int64)]),
]

_lib = None


def load():
    """Load libns2d.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libns2d.so is not built ({LIB_PATH}); run "
                               "`python -m paper_2607_17836_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class Ns2dError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ns2d status {status}: {msg}")
        self.status = status


class Ns2d:
    """One libns2d context (see include/ns2d.h for every call)."""

    def __init__(self, n, nu, dt, length=0.0, stream=None, transforms="auto"):
        """transforms: "auto" or "builtin" (the library's own, for n a power
        of two from 64 to 4096), or "hipfft" (any even n; a cross-check)."""
        cfg = Ns2dConfig(n=n, length=length, nu=nu, dt=dt, hip_stream=stream,
                         transforms={"auto": 0, "hipfft": 1, "builtin": 2}[transforms])
        h = C.c_void_p()
        st = load().ns2d_create(C.byref(cfg), C.byref(h))
        if st != OK:
            raise Ns2dError(st, "ns2d_create failed")
        self._h = h
        self.n = n

    def _check(self, st):
        if st != OK:
            raise Ns2dError(st, load().ns2d_last_error(self._h).decode())

    def close(self):
        if self._h:
            load().ns2d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def synchronize(self):
        self._check(load().ns2d_synchronize(self._h))

    def set_vorticity(self, omega):
        if torch is not None and isinstance(omega, torch.Tensor) and omega.is_cuda:
            assert omega.dtype == torch.float64 and omega.is_contiguous()
            assert omega.numel() == self.n * self.n
            self._check(load().ns2d_set_vorticity(self._h, omega.data_ptr(), 1))
            return
        w = np.ascontiguousarray(omega, dtype=np.float64)
        assert w.size == self.n * self.n
        self._check(load().ns2d_set_vorticity(self._h, w.ctypes.data, 0))

    def step(self, count=1):
        self._check(load().ns2d_step(self._h, count))

    def velocity_ptrs(self):
        """(u, v) device pointers, [n][n] doubles each (see ns2d_velocity)."""
        u, v = C.c_void_p(), C.c_void_p()
        self._check(load().ns2d_velocity(self._h, C.byref(u), C.byref(v)))
        return u.value, v.value

    def get_fields(self):
        """(u, v, omega, psi) as host float64 arrays [n, n] indexed [j, i]."""
        out = [np.empty((self.n, self.n)) for _ in range(4)]
        self._check(load().ns2d_get_fields(self._h, *[a.ctypes.data for a in out], 0))
        return tuple(out)

    @property
    def builtin(self):
        """True when the context runs the library's own transforms."""
        b = C.c_int32()
        self._check(load().ns2d_get_transforms(self._h, C.byref(b)))
        return bool(b.value)

    @property
    def steps(self):
        s = C.c_int64()
        self._check(load().ns2d_get_steps(self._h, C.byref(s)))
        return s.value

"""The field producer's C ABI library (libns2d.so) loads, exports every
symbol include/ns2d.h declares, and rejects invalid configurations and null
handles before touching the GPU (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2607_17836_amd import ns2d

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ns2d.h")


def _built():
    if not os.path.exists(ns2d.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return ns2d.load()


def declared_symbols():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return sorted(set(re.findall(r"\b(ns2d_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    _built()
    out = subprocess.run(["nm", "-D", "--defined-only", ns2d.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(ns2d_\w+)", out))
    names = declared_symbols()
    assert {"ns2d_create", "ns2d_step", "ns2d_velocity", "ns2d_set_vorticity"} <= set(names)
    assert not [s for s in names if s not in exported]
    assert {s for s, _, _ in ns2d._SIGS} == set(names)


@pytest.mark.parametrize("kw", [
    dict(n=6), dict(n=31), dict(n=32768), dict(n=64, length=-1.0),
    dict(n=64, length=float("nan")), dict(n=64, nu=-1e-3), dict(n=64, nu=float("inf")),
    dict(n=64, dt=0.0), dict(n=64, dt=float("nan")), dict(n=64, transforms=3),
    dict(n=64, transforms=-1), dict(n=96, transforms=2), dict(n=8192, transforms=2),
    # the default (own transforms) needs a power of two from 64 to 4096
    dict(n=32), dict(n=96), dict(n=8192),
])
def test_create_rejects_bad_config_without_gpu(kw):
    L = _built()
    cfg = ns2d.Ns2dConfig(n=kw.get("n", 64), length=kw.get("length", 0.0), nu=kw.get("nu", 1e-3),
                          dt=kw.get("dt", 1e-3), hip_stream=None,
                          transforms=kw.get("transforms", 0))
    h = C.c_void_p()
    assert L.ns2d_create(C.byref(cfg), C.byref(h)) == ns2d.E_ARG
    assert not h.value


def test_null_handles_are_rejected():
    L = _built()
    assert L.ns2d_create(None, None) == ns2d.E_ARG
    assert L.ns2d_step(None, 1) == ns2d.E_ARG
    assert L.ns2d_set_vorticity(None, None, 0) == ns2d.E_ARG
    assert L.ns2d_get_fields(None, None, None, None, None, 0) == ns2d.E_ARG
    assert L.ns2d_synchronize(None) == ns2d.E_ARG
    assert L.ns2d_get_steps(None, None) == ns2d.E_ARG
    assert L.ns2d_get_transforms(None, None) == ns2d.E_ARG
    assert L.ns2d_last_error(None) == b"null context"
    L.ns2d_destroy(None)

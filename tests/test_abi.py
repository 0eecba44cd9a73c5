"""The C ABI library loads, exports every symbol its header declares, and
rejects invalid configurations before touching the GPU (no GPU needed)."""
import os
import re
import subprocess

import pytest

from paper_2607_17836_amd import lpt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lpt.h")


def _built():
    if not os.path.exists(lpt.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return lpt.load()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lpt_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("lpt_create", "lpt_destroy", "lpt_set_snapshot", "lpt_add_species",
                     "lpt_init_uniform", "lpt_step", "lpt_get_positions", "lpt_get_stats",
                     "lpt_sort", "lpt_radix_sort", "lpt_interp"):
        assert required in names


def test_library_exports_every_declared_symbol():
    _built()
    out = subprocess.run(["nm", "-D", "--defined-only", lpt.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(lpt_\w+)", out))
    missing = [s for s in declared_symbols() if s not in exported]
    assert not missing, missing
    # the binding knows every exported entry point
    assert {s for s, _, _ in lpt._SIGS} == set(declared_symbols())


def test_status_strings():
    L = _built()
    assert L.lpt_status_string(lpt.OK) == b"LPT_OK"
    assert L.lpt_status_string(lpt.E_RANGE) == b"LPT_E_RANGE"
    assert L.lpt_last_error(None) == b""


@pytest.mark.parametrize("kw", [
    dict(n=3), dict(n=40000), dict(n=64, precision=7), dict(n=64, length=-1.0),
    dict(n=64, length=float("nan")), dict(n=64, sort_interval=-2), dict(n=64, sort_tile=3),
    dict(n=48, sort_tile=32), dict(n=64, block_size=100), dict(n=64, block_size=2048),
    dict(n=64, flags=0x80), dict(n=64, flags=0x8), dict(n=64, t0=float("inf")),
])
def test_create_rejects_bad_config_without_gpu(kw):
    _built()
    n = kw.pop("n")
    assert lpt.create_error_status(n, **kw) == lpt.E_ARG


def test_null_handles_are_rejected():
    L = _built()
    assert L.lpt_step(None, 1, 0.1, 0) == lpt.E_ARG
    assert L.lpt_sort(None) == lpt.E_ARG
    assert L.lpt_get_positions(None, 0, None, None, None, None, 0) == lpt.E_ARG
    L.lpt_destroy(None)

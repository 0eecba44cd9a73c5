"""Host logic of the launch-shape autotuner: the shipped MI355X tuning table
is well formed and is used before the user cache and before tuning."""
import json

import pytest

from paper_2607_17836_amd import autotune, workloads


def test_shipped_table_entries_are_valid_tunings():
    table = json.load(open(autotune.SHIPPED))
    assert table
    fields = {"block_size", "tile_records", "sort_interval", "persistent", "graph_chunk",
              "halo_scale", "max_workgroups", "fused", "sort_cells", "rows"}
    for key, ent in table.items():
        dev, rest = key.split("|", 1)
        assert dev.startswith("gfx950/")
        t = ent["tuning"]
        assert set(t) == fields
        for name, values in autotune.SPACE.items():
            got = tuple(t[k] for k in name) if isinstance(name, tuple) else t[name]
            assert got in values, (name, got)
        assert ent["ms_per_step"] > 0


def test_shipped_entry_is_used_without_tuning(monkeypatch, tmp_path):
    w = workloads.C4_BATCH
    table = json.load(open(autotune.SHIPPED))
    dev = next(k for k in table if k.split("|", 1)[1] == autotune.workload_key(w, "x").split("|", 1)[1])
    dev = dev.split("|", 1)[0]

    def no_tuning(*a, **k):
        raise AssertionError("tuned although the shipped table has the workload")

    monkeypatch.setattr(autotune, "tune", no_tuning)
    t, ms, hit = autotune.cached_or_tune(w, None, None, dev, path=str(tmp_path / "c.json"))
    assert hit and t == table[autotune.workload_key(w, dev)]["tuning"]


def test_user_cache_is_used_for_other_devices(monkeypatch, tmp_path):
    w = workloads.C4_BATCH
    path = tmp_path / "cache.json"
    key = autotune.workload_key(w, "gfx000/1cu")
    json.dump({key: {"tuning": {"block_size": 128}, "ms_per_step": 1.0}}, open(path, "w"))
    monkeypatch.setattr(autotune, "tune", lambda *a, **k: pytest.fail("tuned"))
    t, ms, hit = autotune.cached_or_tune(w, None, None, "gfx000/1cu", path=str(path))
    assert hit and t == {"block_size": 128} and ms == 1.0


def test_rows_are_tried_only_where_they_apply():
    """Two rows per thread change only FP32-split bilinear tracer bodies; the
    tuner does not try them elsewhere (FP64, bicubic or inertial-only mixes)."""
    assert autotune._rows_apply(workloads.C3_SPLIT)
    assert not autotune._rows_apply(workloads.C3_FP64)
    assert not autotune._rows_apply(workloads.c2_spectrum("catmull_rom"))
    assert autotune._rows_apply(workloads.C4_BATCH)   # its species 0: bilinear tracers
    t = {"rows": 2, "tile_records": 0, "graph_chunk": 0, "sort_interval": 16}
    assert autotune._valid(t, "fp32_split", True) and not autotune._valid(t, "fp64", False)

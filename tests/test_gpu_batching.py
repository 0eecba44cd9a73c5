"""Launch-shape choices never change results: persistent launches, hipGraph
step chunks and tuning changes are checked bit for bit against plain eager
launches, and the batched multi-species launch against one context per
species (through the C ABI)."""
import numpy as np
import pytest

import oracle
from paper_2607_17836_amd import lpt, synth, workloads

pytestmark = pytest.mark.gpu

SCHEMES = ["bilinear", "catmull_rom", "bspline"]


def say(msg):
    print(msg, flush=True)


def _mixed(precision, n=128, dt=0.002, x0s=None, **tr_kw):
    """Four species on a spectrum field, initialised uniformly (seeds
    300 ...), or at the given initial positions x0s[k] = (x, y)."""
    (ua, va), (ub, vb) = synth.spectrum_snapshots(n, 8, 12, dt)
    tr = lpt.Tracker(n, precision, **tr_kw)
    tr.set_time_mode("pingpong")
    tr.set_snapshot(0, 0.0, ua, va)
    tr.set_snapshot(1, dt, ub, vb)
    sids = []
    for k, (kind, st, sch, cnt) in enumerate([("tracer", 0.0, "bilinear", 5000),
                                             ("inertial", 0.05, "catmull_rom", 3001),
                                             ("inertial", 1.0, "bspline", 777),
                                             ("tracer", 0.0, "bspline", 64)]):
        if x0s is None:
            z = np.zeros(cnt)
            sids.append(tr.add_species(kind, st, sch, z, z))
            tr.init_uniform(sids[-1], 300 + k)
        else:
            sids.append(tr.add_species(kind, st, sch, *x0s[k]))
    return tr, sids


def _snap(tr, sids):
    out = []
    for s in sids:
        out += list(tr.get_positions(s))
        if s in (1, 2):
            out += list(tr.get_velocities(s))
        out.append(tr.get_stats(s)["msd"])
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32_split"])
def test_persistent_launches_match_normal_launches(precision):
    say(f"persistent {precision}")
    outs = []
    for persistent in (0, 1):
        tr, sids = _mixed(precision, sort_interval=5)
        tr.set_tuning(persistent=persistent)
        tr.step(23, 0.002, stats_every=4)
        outs.append(_snap(tr, sids))
        tr.close()
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("precision", ["fp64", "fp32_split"])
@pytest.mark.parametrize("tile", [0, -1])
@pytest.mark.parametrize("fused", [1, 2, 0])
def test_capped_persistent_walks_match_normal_launches(precision, tile, fused):
    """Persistent launches capped at 8 and 13 workgroups (max_workgroups), so
    that every workgroup walks many logical blocks: the LDS tile is refilled
    per block, the statistics partials are written per block in the loop,
    and the fused launch's block-order table and the per-species XCD ranges
    are walked with strides; with the tile on and off (the tile-off walk has
    no barrier between blocks other than the statistics'), statistics every
    2 steps and re-sorts every 5.  Everything is bit-identical to one
    workgroup per block."""
    say(f"capped persistent {precision} tile={tile} fused={fused}")
    outs = []
    for persistent, cap in ((0, 0), (1, 8), (1, 13)):
        tr, sids = _mixed(precision, sort_interval=5, tile_records=tile)
        tr.set_tuning(persistent=persistent, max_workgroups=cap, fused=fused)
        tr.step(17, 0.002, stats_every=2)
        outs.append(_snap(tr, sids))
        tr.close()
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("precision", ["fp64", "fp32_split"])
def test_fused_launch_matches_per_species_launches(precision):
    """One fused step launch over every species (block-order table, species
    after species or interleaved in cell order; every (scheme, kind) body in
    one kernel) against one launch per species (or, for FP64, one launch in
    species order): the same bits for positions, velocities and statistics,
    with re-sorts and graph chunks."""
    say(f"fused {precision}")
    outs = []
    for fused, chunk in ((0, 0), (1, 0), (2, 0), (1, 5), (2, 5)):
        tr, sids = _mixed(precision, sort_interval=5)
        tr.set_tuning(fused=fused, graph_chunk=chunk)
        tr.step(20, 0.002, stats_every=5)
        outs.append(_snap(tr, sids))
        tr.close()
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("precision", ["fp64", "fp32_split"])
def test_graph_chunks_replay_exactly_like_eager_steps(precision):
    """Chunks of 6 steps captured once and replayed several times, with eager
    readouts and synchronisations in between, against eager stepping in
    lockstep; both sort every 4 steps and take statistics every 3."""
    say(f"graphs {precision}")
    eager, sids = _mixed(precision, sort_interval=4)
    graph, _ = _mixed(precision, sort_interval=4)
    graph.set_tuning(graph_chunk=6, persistent=1)
    for rnd, nsteps in enumerate((6, 6, 12, 5, 6, 13)):
        eager.step(nsteps, 0.002, stats_every=3)
        graph.step(nsteps, 0.002, stats_every=3)
        graph.synchronize()
        for a, b in zip(_snap(eager, sids), _snap(graph, sids)):
            np.testing.assert_array_equal(a, b, err_msg=f"round {rnd}")
    assert graph.get_time() == eager.get_time()
    eager.close()
    graph.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_split"])
def test_two_rows_per_thread_match_one_row(precision):
    """A logical block of block_size slots run by block_size / 2 threads, two
    particles each (the FP32-split bilinear tracer bodies; the others, and
    FP64, run one row whatever the tuning says): per-species launches, so
    that the bilinear tracers of the mix (5000, a ragged count) take that
    body, plain, 128- and 256-thread rows, a persistent walk capped at 8
    workgroups and graph chunks, with re-sorts every 5 steps and statistics
    every 2: positions, velocities and every statistics field bit-identical
    to one particle per thread."""
    say(f"rows {precision}")
    outs = []
    for block, rows, extra in ((256, 1, {}), (512, 2, {}), (256, 2, {}),
                               (512, 2, dict(persistent=1, max_workgroups=8)),
                               (512, 2, dict(graph_chunk=5))):
        tr, sids = _mixed(precision, sort_interval=5)
        tr.set_tuning(block_size=block, rows=rows, fused=0, **extra)
        tr.step(20, 0.002, stats_every=2)
        snap = _snap(tr, sids)
        for s in sids:
            st = tr.get_stats(s)
            snap += [st[f] for f in ("t", "msd_x", "msd_y", "msd", "d_x", "d_y", "sem", "n")]
        outs.append(snap)
        tr.close()
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            np.testing.assert_array_equal(a, b)


def test_tuning_is_validated_and_changes_nothing_on_error():
    tr, _ = _mixed("fp32_split")
    before = tr.get_tuning()
    assert before["tile_records"] == 0 and before["sort_cells"] == 2   # defaults
    assert before["rows"] == 1
    for bad in (dict(block_size=96), dict(tile_records=3), dict(sort_interval=-1),
                dict(persistent=2), dict(graph_chunk=-5), dict(tile_records=100000),
                dict(halo_scale=-1.0), dict(halo_scale=9.0), dict(max_workgroups=-1),
                dict(fused=3), dict(sort_cells=3), dict(sort_cells=-1), dict(rows=3),
                dict(rows=-1), dict(block_size=64, rows=2)):
        with pytest.raises(lpt.LptError) as e:
            tr.set_tuning(**bad)
        assert e.value.status == lpt.E_ARG
        assert tr.get_tuning() == before
    tr.set_tuning(block_size=512, tile_records=2400, sort_interval=7, persistent=1,
                  graph_chunk=10, halo_scale=0.5, max_workgroups=40, fused=0, sort_cells=1,
                  rows=2)
    assert tr.get_tuning() == dict(block_size=512, tile_records=2400, sort_interval=7,
                                   persistent=1, graph_chunk=10, halo_scale=0.5,
                                   max_workgroups=40, fused=0, sort_cells=1, rows=2)
    tr.set_tuning(halo_scale=0.0)   # 0 selects the default
    assert tr.get_tuning()["halo_scale"] == 0.125
    tr.close()


def test_block_size_change_mid_run_keeps_results():
    """Per-particle state and statistics are bit-identical across block
    sizes (the statistics partials are per wave, merged in wave order)."""
    say("block size change")
    outs = []
    for blocks in ((256, 256), (128, 512)):
        tr, sids = _mixed("fp32_split", sort_interval=3)
        tr.set_tuning(block_size=blocks[0])
        tr.step(9, 0.002, stats_every=3)
        tr.set_tuning(block_size=blocks[1])
        tr.step(9, 0.002, stats_every=3)
        outs.append(_snap(tr, sids))
        tr.close()
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)


def test_batched_species_match_one_context_per_species():
    """The batching workload's species mix (8 Stokes numbers, uneven counts,
    scheme k mod 3; reduced counts and grid) in one context gives every
    particle exactly the state it gets when its species runs alone."""
    n, dt = 256, 1e-3
    (ua, va), (ub, vb) = synth.spectrum_snapshots(n, 10, 4, dt)
    mix = [(("inertial" if st > 0 else "tracer"), st, SCHEMES[k % 3], 1000 + 613 * k, 40 + k)
           for k, st in enumerate(workloads.C4_STS)]

    def build(species):
        tr = lpt.Tracker(n, "fp32_split", sort_interval=10)
        tr.set_time_mode("pingpong")
        tr.set_snapshot(0, 0.0, ua, va)
        tr.set_snapshot(1, dt, ub, vb)
        ids = []
        for kind, st, sch, cnt, seed in species:
            z = np.zeros(cnt)
            ids.append(tr.add_species(kind, st, sch, z, z))
            tr.init_uniform(ids[-1], seed)
        return tr, ids

    say("batched")
    tr, ids = build(mix)
    tr.set_tuning(graph_chunk=10, persistent=1)
    tr.step(40, dt, stats_every=20)
    batched = [(tr.get_positions(s), tr.get_velocities(s) if mix[k][0] == "inertial" else None,
                tr.get_stats(s)) for k, s in enumerate(ids)]
    tr.close()
    for k, spec in enumerate(mix):
        say(f"alone {k}")
        one, (sid,) = build([spec])
        one.step(40, dt, stats_every=20)
        for a, b in zip(batched[k][0], one.get_positions(sid)):
            np.testing.assert_array_equal(a, b)
        if spec[0] == "inertial":
            for a, b in zip(batched[k][1], one.get_velocities(sid)):
                np.testing.assert_array_equal(a, b)
        st = one.get_stats(sid)
        np.testing.assert_allclose(batched[k][2]["msd"], st["msd"], rtol=1e-13)
        one.close()


@pytest.mark.parametrize("shape", [dict(), dict(block_size=512, rows=2, fused=0)])
def test_record_steps_draw_uniform_initial_positions_bit_for_bit(shape):
    """On FP32-split record steps a species initialised by init_uniform has
    its initial positions drawn again from the seed (no gather in particle
    order); a species given the same positions explicitly reads them.  The
    two give the same bits -- records (every field), positions and
    velocities -- through re-sorts every 4 steps, for species at offsets
    other than 0 too; in the fused launch and, with two rows per thread, in
    the bilinear tracer body of one launch per species."""
    say(f"drawn initial positions {shape}")
    a, sids = _mixed("fp32_split", sort_interval=4)
    # before any step the unwrapped readout is the initial position itself
    x0s = [tuple(a.get_positions(s)[2:]) for s in sids]
    b, _ = _mixed("fp32_split", sort_interval=4, x0s=x0s)
    for tr in (a, b):
        if shape:
            tr.set_tuning(**shape)
        tr.step(30, 0.002, stats_every=3)
    for x, y in zip(_snap(a, sids), _snap(b, sids)):
        np.testing.assert_array_equal(x, y)
    for s in sids:
        ra, rb = a.get_stats(s), b.get_stats(s)
        assert len(ra) == 10
        for f in ra.dtype.names:
            np.testing.assert_array_equal(ra[f], rb[f])
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_split"])
def test_state_resume_continues_bit_for_bit(precision):
    """Save after 7 steps, restore into a fresh context with the same
    species, step 11 more: identical bits to stepping 18 without a break
    (re-sorts every 4 steps and statistics every 3 included; in FP32 split
    the resumed context reads the blob's initial positions on record steps
    where the uninterrupted one draws them again); a mismatched context
    refuses the blob."""
    say(f"resume {precision}")
    a, sids = _mixed(precision, sort_interval=4)
    a.step(7, 0.002, stats_every=3)
    blob = a.get_state()
    a.step(11, 0.002, stats_every=3)
    b, _ = _mixed(precision, sort_interval=4)
    b.set_state(blob)
    assert b.get_time()[0] == 7
    b.step(11, 0.002, stats_every=3)
    for x, y in zip(_snap(a, sids), _snap(b, sids)):
        np.testing.assert_array_equal(x, y)
    assert a.get_time() == b.get_time()
    a.close()
    b.close()
    other = lpt.Tracker(128, "fp64" if precision == "fp32_split" else "fp32_split")
    with pytest.raises(lpt.LptError) as e:
        other.set_state(blob)
    assert e.value.status == lpt.E_ARG
    other.close()

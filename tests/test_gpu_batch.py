"""Batched steps: simulations of different sizes, media, sources and
receivers advanced by one velocity and one stress launch per step give
bitwise the results of stepping each alone (two-pass path), with every tile
shape, in several calls, and under graph replay; instances stepped in a
batch match the FP64 oracle run on the same inputs."""
import math

import numpy as np
import pytest

from paper_2302_13907_amd import cwell, inputs

from gpu_common import FIELDS, Scenario, announce, check_fields, make_sim, rel_l2, run_oracle

pytestmark = pytest.mark.gpu

H = 5e-3
# (shape, rock jitter, layer (r, z), sources, receivers); depths are multiples of 4
SPECS = [
    ((24, 8, 128), 0.02, (6, 6), [("volume", 0, -1, 40, 1.0), ("force_z", 3, 2, 60, 1e-3)],
     [("pressure", 0, -1, 50, None), ("field", 5, 1, 45, "vz")]),
    ((30, 5, 200), 0.0, (8, 5), [("volume", 0, -1, 70, 1.0), ("torsion", 21, -1, 90, 1.0)],
     [("pressure", 0, -1, 80, None), ("field", 22, 0, 95, "srt"), ("pressure", 0, 2, 100, None)]),
    ((16, 12, 64), 0.02, (0, 0), [("force_r", 4, 7, 30, 1e-3)],
     [("field", 4, 7, 32, "vr")]),
    ((20, 3, 256), 0.0, (5, 10), [("volume", 0, -1, 100, 1.0)],
     [("pressure", 0, -1, k, None) for k in range(90, 140, 10)]),
]
TILES = [4, 2, 1, 2]
STEPS = 70


def _sim(spec, steps):
    shape, jitter, npml, sources, receivers = spec
    s = cwell.Sim(*shape, H, H)
    s.set_material(*inputs.cased_well(*shape, H, H, z_top=shape[2] * H / 2, ramp=0.05, rock_jitter=jitter))
    if npml != (0, 0):
        s.set_pml(npml[0], npml[1], 1e-3, math.pi * 20e3)
    dt = 0.5 * s.cfl_dt()
    s.set_dt(dt)
    for (kind, i, j, k, amp) in sources:
        off = 0.0 if kind in ("force_r", "force_z") else 0.5
        # the pulse peaks at step 30, so the receivers see it within the run
        t = (np.arange(steps) + off) * dt + 2.0 / 20e3 - 30 * dt
        s.add_source(kind, i, j, k, amp * cwell.ricker(20e3, t))
    for (kind, i, j, k, fld) in receivers:
        s.add_receiver(kind, i, j, k, fld)
    s.set_trace_capacity(steps)
    s.set_path("two-pass")
    s.bind()
    return s


def _state(s):
    s.sync()
    return s.traces(), {n: s.field(n) for n in FIELDS}


def test_batch_matches_solo_runs():
    solo = []
    for spec in SPECS:
        s = _sim(spec, STEPS)
        s.step(STEPS)
        solo.append(_state(s))
        s.close()
    sims = [_sim(spec, STEPS) for spec in SPECS]
    b = cwell.Batch(sims)
    for q, t in enumerate(TILES):
        b.set_tile(q, t)
    b.bind()
    b.step(25)
    b.step(45)
    for q, s in enumerate(sims):
        assert s.steps_done == STEPS
        tr, f = _state(s)
        announce("instance %d %s: max |trace| %.3e" % (q, SPECS[q][0], np.abs(tr).max()))
        assert np.abs(tr).max() > 0
        assert np.array_equal(tr, solo[q][0]), q
        for n in FIELDS:
            assert np.array_equal(f[n], solo[q][1][n]), (q, n)
    b.close()
    for s in sims:
        s.close()


def test_batch_graph_replay_and_mixed_calls():
    """Graph replay of the batch (with odd starts and remainders) equals
    ordinary batched launches; single-instance steps between batched ones
    keep the instances consistent."""
    runs = []
    for graph in (0, 8):
        sims = [_sim(spec, STEPS) for spec in SPECS]
        b = cwell.Batch(sims)
        b.bind()
        b.set_graph(graph)
        b.step(3)
        b.step(17)
        b.step(16)
        b.step(34)
        runs.append([_state(s) for s in sims])
        b.close()
        for s in sims:
            s.close()
    for (ta, fa), (tb, fb) in zip(*runs):
        assert np.array_equal(ta, tb)
        for n in FIELDS:
            assert np.array_equal(fa[n], fb[n]), n


def test_batch_refuses_mismatched_instances():
    a = _sim(SPECS[0], STEPS)
    c = _sim(SPECS[1], STEPS)
    c.step(1)                                       # other buffer parity
    with pytest.raises(cwell.CwellError):
        cwell.Batch([a, c])
    d = cwell.Sim(8, 4, 30, H, H)                  # depth not a multiple of 4
    d.set_material(*inputs.homogeneous(8, 4, 30))
    d.set_dt(0.5 * d.cfl_dt())
    d.bind()
    with pytest.raises(cwell.CwellError):
        cwell.Batch([a, d])
    for s in (a, c, d):
        s.close()


def test_autotuner_caches_its_choice(tmp_path, monkeypatch):
    from paper_2302_13907_amd import autotune
    cache = str(tmp_path / "tiles.json")
    tz, w = autotune.best_config(12, 4, 200, cache=cache, steps=2)
    assert tz in autotune.SHAPES and w in autotune.OCCUPANCY
    import json
    db = json.load(open(cache))
    assert len(db) == 1
    e = list(db.values())[0]
    assert (e["tz_waves"], e["waves_per_simd"]) == (tz, w)
    assert len(e["seconds_per_step"]) == len(autotune.SHAPES) * len(autotune.OCCUPANCY)
    # a second request is answered from the cache, without measuring
    monkeypatch.setattr(autotune, "measure", lambda *a, **k: (_ for _ in ()).throw(AssertionError("measured")))
    assert autotune.best_config(12, 4, 200, cache=cache) == (tz, w)
    assert autotune.best_tile(12, 4, 200, cache=cache) == tz


def test_batch_occupancy_variants_are_bitwise_equal():
    """The batched kernels compiled for each register budget give bitwise
    the same results (same operations, other register allocation)."""
    from paper_2302_13907_amd import autotune
    runs = []
    for w in autotune.OCCUPANCY:
        sims = [_sim(spec, STEPS) for spec in SPECS]
        b = cwell.Batch(sims)
        b.set_occupancy(w)
        b.bind()
        b.step(STEPS)
        runs.append([_state(s) for s in sims])
        b.close()
        for s in sims:
            s.close()
    for other in runs[1:]:
        for (ta, fa), (tb, fb) in zip(runs[0], other):
            assert np.array_equal(ta, tb)
            for n in FIELDS:
                assert np.array_equal(fa[n], fb[n]), n
    s = _sim(SPECS[0], STEPS)
    b = cwell.Batch([s])
    with pytest.raises(cwell.CwellError):
        b.set_occupancy(5)
    b.close()
    s.close()


def test_batch_instances_match_oracle():
    """Two instances of one batch against the FP64 oracle on the same inputs:
    traces within 1e-5 relative L2, fields within 1e-5 (RMS and cell by
    cell).  One has a ragged depth (100 cells: the last 256-cell wavefront
    group of each column ends after 25 of its 64 lanes) and an axisymmetric
    medium; the other a 3-D medium (rock moduli jittered cell by cell) and
    a theta count that is not a multiple of the tile's rows."""
    h = 5e-3
    specs = []
    for shape, jitter, tile in (((30, 8, 100), 0.0, 4), ((36, 6, 136), 0.02, 1)):
        nr, nt, nz = shape
        med = inputs.cased_well(*shape, h, h, z_top=nz * h / 2, ramp=0.05, rock_jitter=jitter)
        srcs = [("volume", 0, -1, nz // 3, 1.0), ("force_z", 3, nt - 1, nz // 2, 1e-3),
                ("torsion", 21, -1, nz // 3 + 4, 1.0)]
        recs = [("pressure", 0, -1, k, None) for k in range(4, nz - 4, nz // 8)]
        recs += [("field", 2, 1, nz // 3 + 2, f) for f in FIELDS]
        specs.append((Scenario(shape=shape, h=(h, h), medium=med, steps=160, npml=(6, 6), f0=20e3,
                               sources=srcs, receivers=recs, path="two-pass"), tile))
    sims = [make_sim(sc) for sc, _ in specs]
    b = cwell.Batch(sims)
    for q, (_, tile) in enumerate(specs):
        b.set_tile(q, tile)
    b.bind()
    b.step(70)
    b.step(90)
    for q, ((sc, _), s) in enumerate(zip(specs, sims)):
        announce("batched instance %d %s against the oracle" % (q, sc.shape))
        s.sync()
        tr_g = s.traces()
        f_g = {n: s.field(n) for n in FIELDS}
        tr_o, f_o = run_oracle(sc)
        press = [m for m, r in enumerate(sc.receivers) if r[0] == "pressure"]
        assert np.abs(tr_o[press]).max() > 0
        e = rel_l2(tr_g[press], tr_o[press])
        announce("  pressure traces relL2 %.2e" % e)
        assert e <= 1e-5, e
        check_fields(f_g, f_o, 1e-5)
    b.close()
    for s in sims:
        s.close()

"""16-bit field storage (float16 with per-field power-of-two scales, and
bfloat16), float32 arithmetic: errors against the FP64 oracle and against
the float32-storage run on the same GPU, stated as numbers.

Measured on MI355X (relative L2 of the receiver traces against the
oracle): 48 x 32 x 192 parity case (300 steps) float16 4.1e-4, bfloat16
3.3e-3; 48 x 32 x 512 crop of the mixed-precision workload (3000 steps)
float16 8.5e-3, bfloat16 1.2e-1 (float32 storage 1.6e-6).  The asserted
bounds below add margin to those numbers.  bfloat16's 8-bit mantissa
loses every per-step increment below half a unit of the stored value, so
its error grows with the step count much faster than float16's: on the
crop it passes 1e-2 after 550 steps (89 us of simulated time), while
float16 stays below 1e-2 for all 3000."""
import math

import numpy as np
import pytest

from paper_2302_13907_amd import cwell, inputs

from gpu_common import (FIELDS, STRESS, VEL, Scenario, announce, field_errors, parity_scenario,
                        rel_l2, run_gpu, run_oracle)

pytestmark = pytest.mark.gpu

PARITY_BOUND = {"f16": 1e-3, "bf16": 1e-2}
CROP_BOUND = {"f16": 1.5e-2, "bf16": 2e-1}
# step counts below which the crop's trace error stays under 1e-2: measured on
# MI355X, float16 never passes it in 3000 steps; bfloat16 passes it at 550
# steps (the error over steps [0, n) checked every 50 steps)
CROSS_MIN = {"f16": 3000, "bf16": 400}


def _run(sc, storage, rounding="nearest", graph=0):
    s = cwell.Sim(*sc.shape, *sc.h)
    s.set_material(*sc.medium)
    if sc.npml != (0, 0):
        s.set_pml(sc.npml[0], sc.npml[1], 1e-3, math.pi * sc.f0)
    dt = sc.cfl_fraction * s.cfl_dt()
    s.set_dt(dt)
    for (kind, i, j, k, amp) in sc.sources:
        off = 0.0 if kind in ("force_r", "force_z") else 0.5
        s.add_source(kind, i, j, k, amp * cwell.ricker(sc.f0, (np.arange(sc.steps) + off) * dt))
    for (kind, i, j, k, fld) in sc.receivers:
        s.add_receiver(kind, i, j, k, fld)
    s.set_trace_capacity(sc.steps)
    s.set_storage(storage)
    s.set_rounding(rounding)
    s.set_graph(graph)
    s.bind()
    s.step(sc.steps)
    s.sync()
    tr = s.traces()
    f = {n: s.field(n) for n in FIELDS}
    s.close()
    return tr, f


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_parity_case_16bit(storage):
    sc = parity_scenario()
    announce("parity case, %s storage" % storage)
    tr16, f16 = _run(sc, storage)
    tr32, f32 = _run(sc, "f32")
    tro, fo = run_oracle(sc)
    e_or = rel_l2(tr16, tro)
    e_32 = rel_l2(tr16, tr32)
    fe = field_errors(f16, fo)
    announce("  %s: traces vs oracle %.3e, vs float32 %.3e; worst field %.3e" % (
        storage, e_or, e_32, max(fe.values())))
    assert np.all(np.isfinite(tr16))
    assert e_or <= PARITY_BOUND[storage], e_or
    assert max(fe.values()) <= 10 * PARITY_BOUND[storage], fe


def _crop_scenario():
    """48 x 32 x 512 crop of the mixed-precision workload: 5 mm cells,
    10-cell layer, cement top at k = 256 with a seeded ramp length, source
    at k = 128, 32 axis receivers every 20 mm below it, 3000 steps."""
    rng = np.random.default_rng(3)
    ramp = float(rng.uniform(0.05, 0.5))
    shape = (48, 32, 512)
    med = inputs.cased_well(*shape, 5e-3, 5e-3, z_top=256 * 5e-3, ramp=ramp)
    recs = [("pressure", 0, -1, min(511, 132 + 4 * m), None) for m in range(32)]
    return Scenario(shape=shape, h=(5e-3, 5e-3), medium=med, steps=3000, npml=(10, 10), f0=15e3,
                    sources=[("volume", 0, -1, 128, 1.0)], receivers=recs)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_crop_3000_steps_16bit(storage):
    sc = _crop_scenario()
    announce("48x32x512 crop, 3000 steps, %s storage" % storage)
    tr16, _ = _run(sc, storage)
    tr32, _ = _run(sc, "f32")
    tro, _ = run_oracle(sc)
    e_or = rel_l2(tr16, tro)
    e_32 = rel_l2(tr16, tr32)
    e_32o = rel_l2(tr32, tro)
    # the first step count n at which the error of the traces over steps [0, n)
    # passes 1e-2 (none: it stays below over the whole run)
    cross = next((n for n in range(100, sc.steps + 1, 50) if rel_l2(tr16[:, :n], tro[:, :n]) > 1e-2), None)
    announce("  %s: traces vs oracle %.3e, vs float32 %.3e (float32 vs oracle %.3e); error passes 1e-2 at %s steps" % (
        storage, e_or, e_32, e_32o, cross))
    assert e_32o <= 1e-5, e_32o
    assert e_or <= CROP_BOUND[storage], e_or
    if storage == "f16":
        assert cross is None or cross >= CROSS_MIN["f16"], cross
    else:
        assert cross is not None and CROSS_MIN["bf16"] <= cross, cross


def test_crop_3000_steps_bf16_stochastic_rounding():
    """bfloat16 with stochastic rounding of the field stores: the per-step
    increments below half a unit are kept on average, so the crop's error
    grows much more slowly than with rounding to nearest.  Measured on
    MI355X: 4.4e-2 after 3000 steps against 1.2e-1, 9.9e-3 after 1000 steps
    against 7.6e-2; the error over steps [0, n) passes 1e-2 at n = 750
    instead of 550 (at 900 with the random bits of a prototype)."""
    sc = _crop_scenario()
    announce("48x32x512 crop, 3000 steps, bf16 with stochastic rounding")
    tr_sr, _ = _run(sc, "bf16", "stochastic")
    tr_rn, _ = _run(sc, "bf16")
    tro, _ = run_oracle(sc)
    e_sr, e_rn = rel_l2(tr_sr, tro), rel_l2(tr_rn, tro)
    e_sr1k, e_rn1k = rel_l2(tr_sr[:, :1000], tro[:, :1000]), rel_l2(tr_rn[:, :1000], tro[:, :1000])
    cross = next((n for n in range(100, sc.steps + 1, 50) if rel_l2(tr_sr[:, :n], tro[:, :n]) > 1e-2), None)
    announce("  stochastic %.3e (1000 steps %.3e), nearest %.3e (1000 steps %.3e); passes 1e-2 at %s steps" % (
        e_sr, e_sr1k, e_rn, e_rn1k, cross))
    assert np.all(np.isfinite(tr_sr))
    assert e_sr <= 7e-2, e_sr
    assert e_sr <= 0.6 * e_rn, (e_sr, e_rn)
    assert e_sr1k <= 0.3 * e_rn1k, (e_sr1k, e_rn1k)
    assert cross is None or cross >= 650, cross


def test_bf16_stochastic_rounding_is_reproducible():
    """The random bits are a hash of cell, field and step: two runs, and a
    run replayed from graphs, are bitwise equal; the parity case stays
    within the bfloat16 bound; and the stores do differ from rounding to
    nearest."""
    sc = parity_scenario()
    sc.steps = 120
    announce("parity case, bf16 stochastic rounding: reproducibility")
    a, fa = _run(sc, "bf16", "stochastic")
    b, fb = _run(sc, "bf16", "stochastic")
    g, fg = _run(sc, "bf16", "stochastic", graph=8)
    n, _ = _run(sc, "bf16")
    assert np.array_equal(a, b) and np.array_equal(a, g)
    for f in FIELDS:
        assert np.array_equal(fa[f], fb[f]) and np.array_equal(fa[f], fg[f]), f
    assert not np.array_equal(a, n)
    tro, _ = run_oracle(sc)
    announce("  stochastic %.3e, nearest %.3e against the oracle" % (rel_l2(a, tro), rel_l2(n, tro)))
    assert rel_l2(a, tro) <= PARITY_BOUND["bf16"], rel_l2(a, tro)


def test_f16_field_roundtrip_and_scale():
    """set_field / get_field with float16 storage: values come back within
    half a float16 unit of the largest magnitude, whatever its size."""
    shape = (6, 4, 70)
    s = cwell.Sim(*shape, 5e-3, 5e-3)
    s.set_material(*inputs.homogeneous(*shape))
    s.set_dt(0.5 * s.cfl_dt())
    s.set_storage("f16")
    s.bind()
    rng = np.random.default_rng(2)
    for mag in (1e-12, 1.0, 3e7):
        a = (mag * rng.standard_normal(shape)).astype(np.float32)
        s.set_field("szz", a)
        b = s.field("szz")
        m = np.abs(a).max()
        assert np.abs(b - a).max() <= m * 2.0 ** -10, mag
    with pytest.raises(cwell.CwellError) as e:
        bad = np.zeros(shape, np.float32)
        bad[1, 1, 1] = np.inf
        s.set_field("vr", bad)
    assert e.value.status == -6
    s.close()


def test_f16_refuses_fused_path():
    shape = (8, 4, 20)
    s = cwell.Sim(*shape, 5e-3, 5e-3)
    s.set_material(*inputs.homogeneous(*shape))
    s.set_dt(0.5 * s.cfl_dt())
    s.set_storage("f16")
    s.set_path("fused")
    s.bind()
    with pytest.raises(cwell.CwellError) as e:
        s.step(1)
    assert e.value.status == -2
    s.set_path("auto")
    s.step(2)
    assert s.steps_done == 2
    s.close()


def test_f16_abrupt_large_source_stays_finite():
    """A step-onset volume source of strength 3e9: its first injected stress
    (about 1e10) is far above float16's largest finite value at the initial
    scale 1.  The first write of each field a source injects into takes the
    scale its largest injected value needs, so the float16 run stays finite
    and follows the float32 run."""
    shape, h, steps = (24, 8, 64), 5e-3, 80
    med = inputs.cased_well(*shape, h, h, z_top=0.16, rock_jitter=0.02)
    out = {}
    for storage in ("f16", "f32"):
        s = cwell.Sim(*shape, h, h)
        s.set_material(*med)
        s.set_pml(5, 5, 1e-3, math.pi * 20e3)
        s.set_dt(0.5 * s.cfl_dt())
        s.add_source("volume", 0, -1, 20, np.full(steps, 3e9))
        for k in (21, 24, 30, 40):
            s.add_receiver("pressure", 0, -1, k)
        s.set_trace_capacity(steps)
        s.set_storage(storage)
        s.bind()
        s.step(steps)
        s.sync()
        out[storage] = (s.traces(), s.field("szz"))
        s.close()
    tr16, tr32 = out["f16"][0], out["f32"][0]
    announce("abrupt 3e9 source: max |p| %.3e, float16 vs float32 %.2e" % (np.abs(tr32).max(), rel_l2(tr16, tr32)))
    assert np.all(np.isfinite(tr16)) and np.all(np.isfinite(out["f16"][1]))
    assert np.abs(tr32).max() > 1e9
    assert rel_l2(tr16, tr32) <= 1e-2

"""Degenerate grids on the device against the FP64 oracle: one ring, one
azimuthal cell, a single cell, depths shorter than a four-cell group or
exactly one group, with a random heterogeneous medium (zero shear moduli
included) and a seeded random initial state, on every kernel path and in
16-bit storage; float16 overflow reported as an error; and a zero-step
call, which must change nothing."""
import numpy as np
import pytest

from gpu_common import FIELDS, Scenario, announce, check_fields, make_sim, run_gpu, run_oracle
from paper_2302_13907_amd import cwell

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (2, 1, 3), (3, 2, 5), (1, 4, 8), (2, 3, 4), (5, 1, 2), (4, 2, 12)]
PATHS = ["auto", "two-pass", "fused"]


def _scenario(shape, seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(1000.0, 8000.0, shape)
    mu = rng.uniform(0.0, 3e10, shape)
    mu[rng.random(shape) < 0.3] = 0.0                  # fluid cells among solid ones
    lam = rng.uniform(2e9, 2e10, shape)
    init = {f: rng.standard_normal(shape) for f in FIELDS}
    recs = [("field", shape[0] - 1, 0, shape[2] - 1, f) for f in FIELDS] + [("pressure", 0, -1, 0, None)]
    return Scenario(shape=shape, h=(5e-3, 5e-3), medium=(rho, lam, mu), steps=6, initial=init, receivers=recs)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("shape", SHAPES)
def test_degenerate_grid_matches_oracle(shape, path):
    announce("degenerate grid %s, %s" % (shape, path))
    sc = _scenario(shape, seed=sum(shape) * 7 + len(path))
    sc.path = path
    tr_g, f_g = run_gpu(sc)
    tr_o, f_o = run_oracle(sc)
    check_fields(f_g, f_o, 1e-5, tag="%s %s" % (shape, path))
    scale = np.abs(tr_o).max()
    assert scale > 0
    assert np.abs(tr_g - tr_o).max() <= 1e-5 * scale


# 16-bit storage: one rounding per stored value and step (half a unit in the
# last place: float16 2^-11, bfloat16 2^-8 of the value) over six steps,
# which the update can amplify (the axis ring's 1/r terms); bound: eight such
# roundings relative to the group's largest magnitude (measured at most 1.0e-3
# and 1.75e-2).  The four-cell kernels take the shapes whose depth is a
# multiple of 4, whose ring and depth neighbours at the grid's edges are read
# without branches, the one-cell kernels the others.  The initial state is
# one a wave could have: values of magnitude 0.5 to 1.5 and random sign, the
# stresses times the cell's impedance rho Vp.  With unrelated unit stresses
# and velocities the first step multiplies the stresses by about 1e6, and a
# field whose few values all happen to be small (one cell) grows by 100
# from one step to the next: both are past float16's per-step headroom of
# 2^5 (the next test).
BOUND_16 = {"f16": 8 * 2.0 ** -11, "bf16": 8 * 2.0 ** -8}


def _scenario_impedance(shape, seed):
    sc = _scenario(shape, seed)
    rho, lam, mu = sc.medium
    z = rho * np.sqrt((lam + 2 * mu) / rho)
    rng = np.random.default_rng(seed + 1)
    for f in FIELDS:
        v = rng.choice([-1.0, 1.0], shape) * rng.uniform(0.5, 1.5, shape)
        sc.initial[f] = v * z if f.startswith("s") else v
    return sc


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("shape", SHAPES)
def test_degenerate_grid_16bit_storage(shape, storage):
    announce("degenerate grid %s, %s storage" % (shape, storage))
    sc = _scenario_impedance(shape, seed=sum(shape) * 11 + len(storage))
    sc.storage = storage
    tr_g, f_g = run_gpu(sc)
    tr_o, f_o = run_oracle(sc)
    check_fields(f_g, f_o, BOUND_16[storage], tag="%s %s " % (shape, storage))
    scale = np.abs(tr_o).max()
    assert scale > 0
    assert np.abs(tr_g - tr_o).max() <= BOUND_16[storage] * scale


def test_float16_overflow_is_reported():
    """Unit stresses beside unit velocities in a medium of moduli near 1e10
    are far from equilibrium: the first step multiplies the stresses by about
    1e6, beyond the 2^5 a float16 field may grow from one step to the next.
    The stores overflow to infinity; the device flags the fields, and
    synchronising or reading reports CW_ERR_NONFINITE (instead of returning
    NaN fields as if nothing had happened) until the state is reset.
    bfloat16, with float32's exponent range, takes the same state."""
    announce("float16 overflow: reported, and cleared by a reset")
    sc = _scenario((3, 2, 8), seed=5)
    sc.storage = "f16"
    s = make_sim(sc)
    s.sync()                                        # the initial state is fine
    s.step(2)
    with pytest.raises(cwell.CwellError) as e:
        s.sync()
    assert e.value.status == -6 and "overflowed" in str(e.value)
    with pytest.raises(cwell.CwellError):
        s.field("srr")
    with pytest.raises(cwell.CwellError):
        s.traces()
    s.reset()
    s.sync()
    s.step(2)                                       # from the zero state
    s.sync()
    assert np.all(s.field("srr") == 0.0)
    s.close()
    sc.storage = "bf16"
    tr, f = run_gpu(sc)
    assert all(np.isfinite(v).all() for v in f.values()) and np.isfinite(tr).all()


def test_zero_steps_change_nothing():
    sc = _scenario((3, 2, 5), seed=11)
    s = make_sim(sc)
    before = {f: s.field(f) for f in FIELDS}
    s.step(0)
    s.sync()
    assert s.steps_done == 0
    for f in FIELDS:
        assert np.array_equal(s.field(f), before[f]), f
    s.close()

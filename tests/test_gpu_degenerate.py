"""Degenerate grids on the device against the FP64 oracle: one ring, one
azimuthal cell, a single cell, depths shorter than a four-cell group or
exactly one group, with a random heterogeneous medium (zero shear moduli
included) and a seeded random initial state, on every kernel path; and a
zero-step call, which must change nothing."""
import numpy as np
import pytest

from gpu_common import FIELDS, Scenario, announce, check_fields, make_sim, run_gpu, run_oracle

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

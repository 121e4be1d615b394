"""Pin of the oracle's staggered material averages (reading R7: face buoyancy
b = 2/(rho_a + rho_b), edge shear modulus = harmonic mean of four cells, zero
when one of them is zero; indices clamped at the last ring and depth, wrapped
in theta).

The expected values are hand-derived ratios stored in
``tests/golden/staggered_averages_3x3x3.json``, each with its derivation, for
interior, edge-clamped, theta-wrapped and fluid-touching nodes of a 3x3x3
medium whose every cell has its own density and shear modulus.  Two checks
use them:

* the coefficient tables the oracle builds (``coef``);
* the coefficients the time step actually applies, read back from the
  response of one step to a unit impulse: a unit sigma_zz, sigma_rz or
  sigma_thetaz at a node moves that node's v_z, v_r or v_theta by
  -dt b_z/dz, +dt b_r/dz or +dt b_theta/dz; a unit v_theta or v_r moves the
  node's sigma_thetaz, sigma_rz or sigma_rtheta by -dt mu_thetaz/dz,
  -dt mu_rz/dz or -dt mu_rtheta/(R_i dtheta) (the depth or azimuthal
  difference of the impulse, Eq. (1) discretised on the staggered grid)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import OracleSim

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "staggered_averages_3x3x3.json")


def _case():
    with open(GOLDEN) as f:
        g = json.load(f)
    gr = g["grid"]
    shape = (gr["nr"], gr["ntheta"], gr["nz"])
    i, j, k = np.indices(shape)
    p = 9 * i + 3 * j + k
    rho = 1000.0 + 50.0 * p
    mu = 1e9 / (1.0 + p)
    mu[1, 1, 1] = 0.0
    lam = np.full(shape, 2e9)
    return g, shape, gr["dr"], gr["dz"], rho, lam, mu


def _sim(shape, dr, dz, rho, lam, mu):
    o = OracleSim(*shape, dr, dz)
    o.set_material(rho, lam, mu)
    o.set_dt(0.5 * o.cfl_dt())
    return o


def test_coefficient_tables_match_hand_values():
    g, shape, dr, dz, rho, lam, mu = _case()
    o = _sim(shape, dr, dz, rho, lam, mu)
    tables = {c: o.coef(c) for c in ("b_r", "b_t", "b_z", "mu_rt", "mu_rz", "mu_tz")}
    seen = set()
    for v in g["values"]:
        want = v["num"] / v["den"]
        got = tables[v["coef"]][tuple(v["node"])]
        seen.add(v["coef"])
        if want == 0.0:
            assert got == 0.0, (v, got)
        else:
            assert abs(got / want - 1.0) < 1e-14, (v, got, want)
    assert seen == set(tables)


# impulse field -> (response field, coefficient, factor of the response per
# unit coefficient, as a function of (dt, dr, dz, dth, i))
IMPULSE = {
    "b_z": ("szz", "vz", lambda dt, dr, dz, dth, i: -dt / dz),
    "b_r": ("srz", "vr", lambda dt, dr, dz, dth, i: dt / dz),
    "b_t": ("stz", "vt", lambda dt, dr, dz, dth, i: dt / dz),
    "mu_tz": ("vt", "stz", lambda dt, dr, dz, dth, i: -dt / dz),
    "mu_rz": ("vr", "srz", lambda dt, dr, dz, dth, i: -dt / dz),
    "mu_rt": ("vr", "srt", lambda dt, dr, dz, dth, i: -dt / ((i + 1) * dr * dth)),
}


@pytest.mark.parametrize("coef", sorted(IMPULSE))
def test_step_applies_hand_values(coef):
    g, shape, dr, dz, rho, lam, mu = _case()
    src, resp, factor = IMPULSE[coef]
    dth = 2.0 * math.pi / shape[1]
    nodes = [v for v in g["values"] if v["coef"] == coef]
    assert nodes
    for v in nodes:
        node = tuple(v["node"])
        o = _sim(shape, dr, dz, rho, lam, mu)
        imp = np.zeros(shape)
        imp[node] = 1.0
        o.set_field(src, imp)
        o.step_linear()
        got = o.field(resp)[node] / factor(o.dt, dr, dz, dth, node[0])
        want = v["num"] / v["den"]
        if want == 0.0:
            assert got == 0.0, (v, got)
        else:
            assert abs(got / want - 1.0) < 1e-12, (v, got, want)

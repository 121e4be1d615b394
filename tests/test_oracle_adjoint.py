"""Pins of the oracle's adjoint (test infrastructure for the gradient path).

1. Dot-product test: for random states U, W (fields and absorbing-layer
   memory) and a random heterogeneous medium with a fluid core, the
   transposed step satisfies <step(U), W> = <U, step^T(W)> to rounding.
   This pins every transposed stencil index, coefficient, zero ghost and
   layer-memory recursion against the forward step.
2. Gradient: the adjoint gradient of the receiver loss with respect to the
   cement moduli of z-bins agrees with central finite differences of the
   FP64 forward run (relative step 1e-4), bin by bin, and each difference
   resolves a loss change far above the float64 rounding of the loss."""
import math

import numpy as np
import pytest

import oracle
from paper_2302_13907_amd import inputs


@pytest.mark.parametrize("layer", [False, True])
def test_adjoint_step_is_the_transpose(layer):
    shape = (9, 5, 11)
    o = oracle.OracleSim(*shape, 5e-3, 5e-3)
    o.set_material(*inputs.random_medium(*shape, seed=4))
    if layer:
        o.set_pml(3, 2, 1e-3, 3e4)
    o.set_dt(0.5 * o.cfl_dt())
    rng = np.random.default_rng(0)
    U = {n: rng.standard_normal(shape) for n in oracle.FIELDS}
    P = [rng.standard_normal(shape) for _ in range(18)] if layer else []
    for n, a in U.items():
        o.set_field(n, a)
    for q, a in enumerate(P):
        o.set_psi(q, a)
    o.step_linear()
    FU = {n: o.field(n) for n in oracle.FIELDS}
    FP = [o.psi(q) for q in range(len(P))]
    W = {n: rng.standard_normal(shape) for n in oracle.FIELDS}
    WP = [rng.standard_normal(shape) for _ in range(len(P))]
    lhs = sum((FU[n] * W[n]).sum() for n in oracle.FIELDS) + sum((a * b).sum() for a, b in zip(FP, WP))
    fb, pb = o.adjoint_step({n: W[n].copy() for n in W}, [a.copy() for a in WP] if layer else None)
    rhs = sum((U[n] * fb[n]).sum() for n in oracle.FIELDS)
    if layer:
        rhs += sum((a * b).sum() for a, b in zip(P, pb))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs), (lhs, rhs)


from adjoint_case import REGION, STEPS, WINDOW, medium as _medium, oracle_sim as _sim


def adjoint_reference():
    """Loss and FP64 adjoint gradient of the thin-well case (also the
    reference of the GPU gradient)."""
    o, dt = _sim(_medium())
    return o.gradient(STEPS, WINDOW, REGION), dt


def test_gradient_matches_finite_differences():
    (L, gm, gk), dt = adjoint_reference()
    assert L > 0

    def loss(dmu, dK):
        o, _ = _sim(_medium(dmu, dK), dt)
        tr = o.run(STEPS)
        return float((tr[:, WINDOW[0]:WINDOW[1]] ** 2).sum())

    nb = REGION[3]
    assert math.isclose(loss(np.zeros(nb), np.zeros(nb)), L, rel_tol=1e-12)
    _, lam_c, mu_c = inputs.moduli(*inputs.CEMENT)
    K_c = lam_c + 2.0 * mu_c / 3.0
    z = np.zeros(nb)
    for b in (0, 3):
        e = np.zeros(nb)
        e[b] = 1e-4 * mu_c
        fd = (loss(e, z) - loss(-e, z)) / (2 * e[b])
        assert abs(gm[b] - fd) <= 1e-5 * abs(fd), (b, "mu", gm[b], fd)
        _well_conditioned(fd, e[b], L)
        e[b] = 1e-4 * K_c
        fd = (loss(z, e) - loss(z, -e)) / (2 * e[b])
        assert abs(gk[b] - fd) <= 1e-5 * abs(fd), (b, "K", gk[b], fd)
        _well_conditioned(fd, e[b], L)
    # relative sensitivities |dL/dtheta| |theta| / L of the checked bins
    assert abs(gm[0]) * mu_c / L > 1e-4 and abs(gk[0]) * K_c / L > 1e-5, (gm[0] * mu_c / L, gk[0] * K_c / L)


def _well_conditioned(fd, h, L):
    """The loss difference a central difference resolves is many orders of
    magnitude above the float64 rounding of the loss itself, so the check
    measures the gradient, not rounding noise."""
    assert abs(fd) * 2 * h >= 1e6 * np.finfo(np.float64).eps * L, (fd, h, L)


# ---- the adjoint workload's correctness crop (48 x 32 x 256, 4000 steps)
import json
import os

import adjoint_case as AC

CROP_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_crop_48x32x256.json")


def _crop_golden():
    with open(CROP_GOLDEN) as f:
        return json.load(f)


def test_crop_golden_is_for_the_crop_case():
    """The stored oracle gradient of the crop belongs to the crop as
    tests/adjoint_case.py defines it, at half the oracle's Courant limit."""
    g = _crop_golden()
    c = AC.CROP
    want = {"shape": list(c.shape), "h": c.h, "radii": list(c.radii), "ktop": c.ktop, "ramp": c.ramp,
            "steps": c.steps, "window": list(c.window), "region": list(c.region), "npml": c.npml,
            "f0": c.f0, "src_k": c.src_k, "rec_k": list(c.rec_k)}
    assert g["case"] == want
    o = oracle.OracleSim(*c.shape, c.h, c.h)
    o.set_material(*AC.medium(case=c))
    assert g["dt"] == 0.5 * o.cfl_dt()
    nb = c.region[3]
    assert len(g["dL_dmu"]) == nb and len(g["dL_dK"]) == nb and g["loss"] > 0


def test_crop_gradient_agrees_with_finite_differences():
    """On the crop, the oracle's adjoint gradient agrees with central finite
    differences of the oracle's forward loss (step 1e-4 of the bin's own
    modulus) for two shear and two bulk parameters, each difference well
    above the float64 rounding of the loss; the relative sensitivities
    |dL/dtheta| |theta| / L of those bins exceed 1e-4, so the check is well
    conditioned.  Both sides were computed by tests/golden/make_adjoint_crop.py
    (about 15 minutes of oracle time); CWELL_LONG_ORACLE=1 repeats the
    computation in test_crop_oracle_reproduces_golden."""
    g = _crop_golden()
    L = g["loss"]
    assert len(g["finite_differences"]) == 4
    for e in g["finite_differences"]:
        b = e["bin"]
        adj = (g["dL_dmu"] if e["modulus"] == "mu" else g["dL_dK"])[b]
        theta = (g["bin_mu"] if e["modulus"] == "mu" else g["bin_K"])[b]
        assert abs(e["step"] / theta - 1e-4) < 1e-12
        assert math.isclose(e["fd"], (e["loss_plus"] - e["loss_minus"]) / (2 * e["step"]), rel_tol=1e-15)
        assert abs(adj - e["fd"]) <= 1e-5 * abs(e["fd"]), (e, adj)
        _well_conditioned(e["fd"], e["step"], L)
        assert abs(adj) * theta / L > 1e-4, (e, adj * theta / L)


@pytest.mark.skipif(not os.environ.get("CWELL_LONG_ORACLE"),
                    reason="about 15 minutes of oracle time; set CWELL_LONG_ORACLE=1")
def test_crop_oracle_reproduces_golden():
    """The oracle recomputes the stored crop gradient and one of the stored
    finite differences."""
    g = _crop_golden()
    c = AC.CROP
    o, dt = AC.oracle_sim(AC.medium(case=c), case=c)
    L, gm, gk = o.gradient(c.steps, c.window, c.region)
    assert math.isclose(L, g["loss"], rel_tol=1e-12)
    assert np.allclose(gm, g["dL_dmu"], rtol=1e-10, atol=1e-10 * np.abs(gm).max())
    assert np.allclose(gk, g["dL_dK"], rtol=1e-10, atol=1e-10 * np.abs(gk).max())
    e = g["finite_differences"][0]
    nb = c.region[3]
    d = np.zeros(nb)
    d[e["bin"]] = e["step"]
    z = np.zeros(nb)
    args = (d, z) if e["modulus"] == "mu" else (z, d)
    o2, _ = AC.oracle_sim(AC.medium(*args, case=c), dt, case=c)
    tr = o2.run(c.steps)
    lp = float((tr[:, c.window[0]:c.window[1]] ** 2).sum())
    assert math.isclose(lp, e["loss_plus"], rel_tol=1e-12)

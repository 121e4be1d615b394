"""GPU adjoint gradient (float32 arithmetic, float64 accumulation of the
gradient) against the FP64 oracle's adjoint gradient on the thin-well case
and on the adjoint workload's correctness crop; independence of the
checkpoint spacing; the torch.autograd wrapper.

Measured on MI355X (thin well): loss relative error 1.1e-7, per-bin gradient
relative error (bins above 1e-3 of the largest) 4.6e-6; the bound asserted
is 1e-4."""
import json
import math
import os

import numpy as np
import pytest

from paper_2302_13907_amd import cwell

import adjoint_case as C
from gpu_common import announce

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-4


def _gpu_sim(dt, every, shape=None, rock_jitter=0.0, case=C.THIN):
    shape = shape or case.shape
    s = cwell.Sim(*shape, case.h, case.h)
    s.set_material(*C.medium(shape=shape, rock_jitter=rock_jitter, case=case))
    s.set_pml(case.npml, case.npml, 1e-3, math.pi * case.f0)
    s.set_dt(dt)
    s.add_source("volume", 0, -1, case.src_k, cwell.ricker(case.f0, (np.arange(case.steps) + 0.5) * dt))
    for k in case.rec_k:
        s.add_receiver("pressure", 0, -1, k)
    s.set_adjoint(case.steps, every, case.region)
    s.bind()
    return s


def _reference():
    o, dt = C.oracle_sim(C.medium())
    return o.gradient(C.STEPS, C.WINDOW, C.REGION), dt


@pytest.mark.parametrize("nz,jitter", [(C.SHAPE[2], 0.0), (C.SHAPE[2] + 2, 0.0), (C.SHAPE[2], 0.02)])
def test_gradient_matches_oracle(nz, jitter):
    """nz = 96: the depth-vectorized adjoint kernels (four cells per thread,
    most lanes of each workgroup past the last depth), with a medium that
    does not vary along theta and with rock moduli jittered cell by cell
    (a 3-D medium); nz = 98: the one-cell kernels."""
    shape = (C.SHAPE[0], C.SHAPE[1], nz)
    o, dt = C.oracle_sim(C.medium(shape=shape, rock_jitter=jitter), shape=shape)
    L, gm, gk = o.gradient(C.STEPS, C.WINDOW, C.REGION)
    s = _gpu_sim(dt, 64, shape, jitter)
    Lg, gmg, gkg = s.gradient(C.WINDOW)
    announce("loss gpu %.9g oracle %.9g (rel %.2e)" % (Lg, L, abs(Lg - L) / L))
    assert abs(Lg - L) <= 1e-4 * L
    for name, a, b in (("mu", gmg, gm), ("K", gkg, gk)):
        big = np.abs(b) > 1e-3 * np.abs(b).max()
        err = np.abs(a - b)[big] / np.abs(b)[big]
        announce("  dL/d%s: worst relative error %.2e over %d bins" % (name, err.max(), big.sum()))
        assert err.max() <= GRAD_TOL, (name, a, b)
        assert np.all(np.abs(a - b) <= GRAD_TOL * np.abs(b).max()), name
    s.close()


def test_checkpoint_spacing_does_not_change_the_gradient():
    """The recomputed segments reproduce the forward run bitwise, so the
    result does not depend on the checkpoint spacing (one segment, 64-step
    segments, 7-step segments with a ragged last one)."""
    _, dt = C.oracle_sim(C.medium())
    res = []
    for every in (C.STEPS, 64, 7):
        s = _gpu_sim(dt, every)
        res.append(s.gradient(C.WINDOW))
        s.close()
    for r in res[1:]:
        assert r[0] == res[0][0]
        assert np.array_equal(r[1], res[0][1]) and np.array_equal(r[2], res[0][2])


def test_autograd_wrapper():
    import torch
    _, dt = C.oracle_sim(C.medium())
    s = _gpu_sim(dt, 100)
    nb = C.REGION[3]
    dmu = torch.zeros(nb, dtype=torch.float64, requires_grad=True)
    dK = torch.zeros(nb, dtype=torch.float64, requires_grad=True)
    loss = cwell.cement_loss(s, C.WINDOW, dmu, dK)
    loss.backward()
    L0, gm, gk = s.gradient(C.WINDOW)
    assert math.isclose(float(loss), L0, rel_tol=1e-12)
    assert np.array_equal(dmu.grad.numpy(), gm) and np.array_equal(dK.grad.numpy(), gk)
    # the loss moves as the gradient says: central difference along a shift of
    # mu by 5e8 Pa in bins 1..7 (bin 0, at the top of the ramp, has mu = 2.7e8);
    # the shift is large enough for float32 losses to resolve the difference
    d = torch.full((nb,), 5e8, dtype=torch.float64)
    d[0] = 0.0
    z = torch.zeros(nb, dtype=torch.float64)
    lp = float(cwell.cement_loss(s, C.WINDOW, d, z))
    lm = float(cwell.cement_loss(s, C.WINDOW, -d, z))
    fd = (lp - lm) / 2.0
    pred = float((d.numpy() * gm).sum())
    announce("  central difference %.4e, adjoint %.4e" % (fd, pred))
    assert abs(fd - pred) <= 0.1 * abs(pred)
    # a shift that would make a modulus negative is refused and changes nothing
    with pytest.raises(cwell.CwellError):
        s.set_region_moduli(np.full(nb, -1e12), np.zeros(nb))
    s.set_region_moduli(np.zeros(nb), np.zeros(nb))
    assert s.gradient(C.WINDOW)[0] == L0
    s.close()


CROP_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_crop_48x32x256.json")
CROP_TOL = 1e-4
CROP_FLOOR = 5e-6


def test_crop_gradient_matches_oracle():
    """The adjoint workload's correctness crop (48 x 32 x 256 cells of 5 mm,
    4000 steps, checkpoints every 100, 128 parameters on the 64 one-row bins
    of the cement ramp): the GPU loss and gradient against the FP64 oracle's,
    stored by tests/golden/make_adjoint_crop.py (which calls only the
    oracle).  Every bin is held to CROP_TOL of itself plus CROP_FLOOR of the
    largest bin: float32 rounding over 4000 forward and 4000 adjoint steps
    leaves an error of about 1e-6 of the largest bin in every bin (measured
    0.6e-6 to 1.7e-6 over builds of the same kernels whose float32 results
    differ in the last bits), which a bin at 1e-3 of the largest cannot hold
    to 1e-4 of itself."""
    g = json.load(open(CROP_GOLDEN))
    case = C.CROP
    assert g["case"]["shape"] == list(case.shape) and g["case"]["region"] == list(case.region)
    assert g["case"]["window"] == list(case.window) and g["case"]["steps"] == case.steps
    announce("adjoint crop 48x32x256, 4000 steps, checkpoints every 100")
    s = _gpu_sim(g["dt"], 100, case=case)
    Lg, gmg, gkg = s.gradient(case.window)
    s.close()
    L = g["loss"]
    announce("  loss gpu %.9g oracle %.9g (rel %.2e)" % (Lg, L, abs(Lg - L) / L))
    assert abs(Lg - L) <= CROP_TOL * L
    for name, a, b in (("mu", gmg, np.array(g["dL_dmu"])), ("K", gkg, np.array(g["dL_dK"]))):
        top = np.abs(b).max()
        big = np.abs(b) > 1e-2 * top
        err = np.abs(a - b)[big] / np.abs(b)[big]
        announce("  dL/d%s: worst relative error %.2e over the %d bins above 1e-2 of the largest; "
                 "worst against the largest %.2e" % (name, err.max(), big.sum(), np.abs(a - b).max() / top))
        bound = CROP_TOL * np.abs(b) + CROP_FLOOR * top
        assert np.all(np.abs(a - b) <= bound), (name, float(np.max(np.abs(a - b) / bound)))

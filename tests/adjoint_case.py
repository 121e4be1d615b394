"""The thin-well gradient case shared by the oracle and GPU adjoint tests:
a hole of 20 mm, casing to 30 mm and cement to 50 mm (so the wave reaches
the cement within a short run), 20 x 8 x 96 cells of 5 mm, a 40 kHz volume
source on the axis above a cement top with a 0.1 m shear ramp, 12 axis
pressure receivers, 400 steps, loss over steps [150, 400), parameters on 8
bins of 2 rows of the annulus below the cement top."""
import math

import numpy as np

import oracle
from paper_2302_13907_amd import inputs

H = 5e-3
SHAPE = (20, 8, 96)
RADII = (0.02, 0.03, 0.05)
KTOP = 48
STEPS = 400
WINDOW = (150, 400)
REGION = (6, 10, KTOP + 1, 8, 2)      # annulus rings 6..9, 8 bins of 2 rows below the cement top
NPML = 6
F0 = 40e3
SRC_K = 40
REC_K = list(range(20, 44, 2))


def medium(dmu=None, dK=None, shape=SHAPE, rock_jitter=0.0):
    rho, lam, mu = inputs.cased_well(*shape, H, H, z_top=KTOP * H, ramp=0.1, radii=RADII, rock_jitter=rock_jitter)
    if dmu is not None:
        i0, i1, k0, nb, br = REGION
        K = lam + 2.0 * mu / 3.0
        for b in range(nb):
            sl = (slice(i0, i1), slice(None), slice(k0 + b * br, k0 + (b + 1) * br))
            mu[sl] += dmu[b]
            K[sl] += dK[b]
        lam = K - 2.0 * mu / 3.0
    return rho, lam, mu


def oracle_sim(med, dt=None, shape=SHAPE):
    o = oracle.OracleSim(*shape, H, H)
    o.set_material(*med)
    o.set_pml(NPML, NPML, 1e-3, math.pi * F0)
    dt = dt or 0.5 * o.cfl_dt()
    o.set_dt(dt)
    o.add_source("volume", 0, -1, SRC_K, oracle.ricker(F0, (np.arange(STEPS) + 0.5) * dt))
    for k in REC_K:
        o.add_receiver("pressure", 0, -1, k)
    return o, dt

"""Seeded synthetic inputs for the cased-well workloads.

This module only describes workloads: grid sizes, the layered medium sampled
at the cell centres, source and receiver positions, seeds.  It holds none of
the solver's arithmetic (no stencil, no Courant limit, no wavelet); both the
HIP path and the test oracle take what it produces as plain arrays.

The medium is the cased well of Sec. 5: a fluid-filled hole, a steel casing,
a cement annulus whose upper edge may be graded (the "degree of hardening of
the upper edge" the paper studies), and host rock.  The paper's own material
values are not given in the text; the values below are typical ones.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple, Sequence

import numpy as np

# (Vp, Vs, rho) in SI units
FLUID = (1500.0, 0.0, 1000.0)
STEEL = (5900.0, 3200.0, 7850.0)
CEMENT = (3000.0, 1700.0, 1900.0)
ROCK = (4000.0, 2300.0, 2400.0)

R_HOLE, R_CASING, R_CEMENT = 0.10, 0.11, 0.15

ROCK_SEED = 20230227


def moduli(vp: float, vs: float, rho: float) -> Tuple[float, float, float]:
    """(rho, lambda, mu) from wave speeds: mu = rho Vs^2, lambda = rho Vp^2 - 2 mu."""
    mu = rho * vs * vs
    return rho, rho * vp * vp - 2.0 * mu, mu


def cased_well(nr: int, nt: int, nz: int, dr: float, dz: float,
               z_top: float, ramp: float = 0.0,
               rock_jitter: float = 0.0, seed: int = ROCK_SEED,
               radii: Tuple[float, float, float] = (R_HOLE, R_CASING, R_CEMENT)):
    """rho, lambda, mu (float64, [nr][nt][nz]) of the cased well.

    Sampled at the cell centres r_i = (i + 1/2) dr, z_k = k dz (z grows with
    depth).  Annulus cells with z_k >= z_top hold cement; above it the annulus
    holds fluid.  With ramp > 0 the cement keeps its density and bulk modulus
    but its shear modulus grows linearly from 0 at z_top to full at
    z_top + ramp.  rock_jitter > 0 multiplies lambda and mu of every rock cell
    by independent factors (1 + eps), eps ~ U[-jitter, jitter], drawn for
    lambda first, then mu, over the whole grid in C order.
    """
    r = (np.arange(nr) + 0.5) * dr
    z = np.arange(nz) * dz
    shape = (nr, nt, nz)
    rho = np.empty(shape)
    lam = np.empty(shape)
    mu = np.empty(shape)
    R = r[:, None, None] + np.zeros(shape)
    Z = z[None, None, :] + np.zeros(shape)
    fluid = R < radii[0]
    steel = (R >= radii[0]) & (R < radii[1])
    annulus = (R >= radii[1]) & (R < radii[2])
    rock = R >= radii[2]
    for mask, mat in ((fluid, FLUID), (steel, STEEL), (rock, ROCK)):
        ro, la, m = moduli(*mat)
        rho[mask], lam[mask], mu[mask] = ro, la, m
    cem = annulus & (Z >= z_top)
    mud = annulus & (Z < z_top)
    ro, la, m = moduli(*FLUID)
    rho[mud], lam[mud], mu[mud] = ro, la, m
    ro, la, m = moduli(*CEMENT)
    K = la + 2.0 * m / 3.0
    if ramp > 0:
        frac = np.clip((Z - z_top) / ramp, 0.0, 1.0)
    else:
        frac = np.ones(shape)
    mu_c = m * frac
    rho[cem] = ro
    mu[cem] = mu_c[cem]
    lam[cem] = (K - 2.0 * mu_c / 3.0)[cem]
    if rock_jitter > 0:
        rng = np.random.default_rng(seed)
        e_l = rng.uniform(-rock_jitter, rock_jitter, size=shape)
        e_m = rng.uniform(-rock_jitter, rock_jitter, size=shape)
        lam[rock] *= 1.0 + e_l[rock]
        mu[rock] *= 1.0 + e_m[rock]
    return rho, lam, mu


def cased_well_rz(nr: int, nz: int, dr: float, dz: float, z_top: float, ramp: float = 0.0,
                  radii: Tuple[float, float, float] = (R_HOLE, R_CASING, R_CEMENT)):
    """Axisymmetric form of cased_well (no jitter): rho, lambda, mu as [nr][nz]."""
    rho, lam, mu = cased_well(nr, 1, nz, dr, dz, z_top, ramp, 0.0, radii=radii)
    return rho[:, 0, :].copy(), lam[:, 0, :].copy(), mu[:, 0, :].copy()


def homogeneous(nr: int, nt: int, nz: int, mat=FLUID):
    ro, la, m = moduli(*mat)
    shape = (nr, nt, nz)
    return np.full(shape, ro), np.full(shape, la), np.full(shape, m)


def random_medium(nr: int, nt: int, nz: int, seed: int, fluid_rings: int = 2):
    """Heterogeneous random medium with a fluid core of `fluid_rings` rings."""
    rng = np.random.default_rng(seed)
    shape = (nr, nt, nz)
    rho = rng.uniform(1000.0, 8000.0, shape)
    mu = rng.uniform(5e9, 8e10, shape)
    lam = rng.uniform(1e9, 1e11, shape)
    mu[:fluid_rings] = 0.0
    lam[:fluid_rings] = 2.25e9
    rho[:fluid_rings] = 1000.0
    return rho, lam, mu


def random_fields(shape, seed: int, n: int = 9, scale: float = 1.0) -> List[np.ndarray]:
    rng = np.random.default_rng(seed)
    return [scale * rng.standard_normal(shape) for _ in range(n)]


@dataclass
class Workload:
    """One synthetic workload of the paper's kind (a cased well, an axis source)."""
    name: str
    nr: int
    nt: int
    nz: int
    dr: float
    dz: float
    steps: int
    npml: int
    f0: float
    src_k: int
    rec_k: List[int]
    z_top: float
    ramp: float = 0.0
    rock_jitter: float = 0.0
    cfl_fraction: float = 0.5
    pml_rc: float = 1e-3
    extra: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return self.nr * self.nt * self.nz

    def medium(self):
        return cased_well(self.nr, self.nt, self.nz, self.dr, self.dz,
                          self.z_top, self.ramp, self.rock_jitter)

    def medium_rz(self):
        """[nr][nz] arrays; only for workloads without azimuthal jitter."""
        assert self.rock_jitter == 0
        return cased_well_rz(self.nr, self.nz, self.dr, self.dz, self.z_top, self.ramp)

    @property
    def layer_cells(self):
        """(cells in the radial layer slab, cells in the two z layer slabs)."""
        return (self.npml * self.nt * self.nz, self.nr * self.nt * (2 * self.npml + 1))


def parity_case() -> Workload:
    """48 x 32 x 192 cells of 5 mm, 300 steps, 10-cell layer, 20 kHz axis
    source at z = 0.2 m, 16 axis receivers every 20 mm from z = 0.22 m,
    sharp cement top at z = 0.5 m, rock moduli jittered by +-2 %."""
    return Workload("cased-well 48x32x192 (5 mm), 300 steps", 48, 32, 192, 5e-3, 5e-3,
                    steps=300, npml=10, f0=20e3, src_k=40,
                    rec_k=[44 + 4 * m for m in range(16)], z_top=0.5,
                    rock_jitter=0.02)


def production_case() -> Workload:
    """256 x 128 x 8192 cells of 2 mm (268 M cells), 2000 steps, 20-cell
    layer, 15 kHz axis source at k = 2048, 64 axis receivers every 10 cells
    below it, cement top at k = 4096 with a 0.3 m shear ramp."""
    nz = 8192
    return Workload("cased-well 256x128x8192 (2 mm), 2000 steps", 256, 128, nz, 2e-3, 2e-3,
                    steps=2000, npml=20, f0=15e3, src_k=2048,
                    rec_k=[2048 + 10 * (m + 1) for m in range(64)],
                    z_top=(nz // 2) * 2e-3, ramp=0.3)


def mixed_precision_case() -> Workload:
    """192 x 96 x 4096 cells of 5 mm, 3000 steps, 20-cell layer, 15 kHz axis
    source at k = 1024, 32 axis receivers every 20 mm below it, cement top at
    k = 2048 with a shear ramp whose length is drawn uniformly from
    [0.05, 0.5] m (seed 3)."""
    ramp = float(np.random.default_rng(3).uniform(0.05, 0.5))
    return Workload("cased-well 192x96x4096 (5 mm), 3000 steps", 192, 96, 4096, 5e-3, 5e-3,
                    steps=3000, npml=20, f0=15e3, src_k=1024,
                    rec_k=[1024 + 4 * (m + 1) for m in range(32)],
                    z_top=2048 * 5e-3, ramp=ramp)


def adjoint_case() -> Workload:
    """128 x 64 x 2048 cells of 5 mm, 1500 steps, 20-cell layer, 15 kHz axis
    source at k = 512, 32 axis receivers every 20 mm below it, cement top at
    k = 1024 with a 0.32 m (64-row) shear ramp.  Gradient parameters: the
    cement annulus (rings 22..29) in 64 bins of one row below the top;
    checkpoints every 100 steps; loss over steps [750, 1500)."""
    w = Workload("cased-well 128x64x2048 (5 mm), 1500 steps, adjoint", 128, 64, 2048, 5e-3, 5e-3,
                 steps=1500, npml=20, f0=15e3, src_k=512,
                 rec_k=[516 + 4 * m for m in range(32)], z_top=1024 * 5e-3, ramp=0.32)
    w.extra.update(region=(22, 30, 1025, 64, 1), checkpoint_every=100, window=(750, 1500))
    return w


def batched_case(count: int = 48, seed: int = 4, nr: int = 128, nt: int = 64,
                 depths: Sequence[int] = (1024, 1536, 2048, 3072, 4096), npml: int = 20) -> List[Workload]:
    """Instances of nr x nt x Nz cells of 5 mm (default 128 x 64), Nz drawn
    uniformly from `depths`, 1500 steps, an npml-cell layer, 15 kHz axis
    source at a depth uniform over the top 30 % of the column (below the
    layer), cement top uniform in [0.5, 0.8] Nz, shear ramp length uniform
    in [0.05, 0.5] m, 32 axis receivers every 20 mm below the source.  The
    draws are made in instance order from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        nz = int(rng.choice(list(depths)))
        src_k = int(rng.integers(npml + 1, int(0.3 * nz)))
        top = int(rng.uniform(0.5, 0.8) * nz)
        ramp = float(rng.uniform(0.05, 0.5))
        rec = [min(nz - npml - 2, src_k + 4 * (m + 1)) for m in range(32)]
        out.append(Workload("batch instance %d: cased-well %dx%dx%d (5 mm), 1500 steps" % (q, nr, nt, nz),
                            nr, nt, nz, 5e-3, 5e-3, steps=1500, npml=npml, f0=15e3, src_k=src_k, rec_k=rec,
                            z_top=top * 5e-3, ramp=ramp))
    return out


def small_batched_case(count: int = 256, seed: int = 5) -> List[Workload]:
    """Many small instances, where one launch per instance and step would
    cost more than the work: 48 x 16 x Nz cells of 5 mm, Nz from
    {256, 384, 512}, 8-cell layer; otherwise as batched_case."""
    return batched_case(count, seed, nr=48, nt=16, depths=(256, 384, 512), npml=8)


def refined_zones(nr: int, ntheta_outer: int, ntheta_inner: int, dr: float) -> List[Tuple[int, int]]:
    """Zones of an azimuthally refined grid that keep the outer resolution
    and halve the azimuthal cell count each time the radius halves (Sec. 3):
    with Q zones (ntheta_inner doubling up to ntheta_outer) and r_max =
    nr dr, zone Q-1 holds the rings whose centre radius lies in
    [r_max / 2, r_max), zone Q-2 those in [r_max / 4, r_max / 2), ..., zone
    0 the rest.  Zones that would hold no ring are left out and the inner
    cell counts halve from the next zone out.  Returns [(first_ring,
    ntheta), ...]."""
    q_count = int(round(np.log2(ntheta_outer / ntheta_inner))) + 1
    if ntheta_inner < 1 or ntheta_inner * 2 ** (q_count - 1) != ntheta_outer:
        raise ValueError("ntheta_outer / ntheta_inner must be a power of two")
    r_max = nr * dr
    centres = (np.arange(nr) + 0.5) * dr
    firsts = []
    for q in range(1, q_count):
        first = int(np.searchsorted(centres, r_max / 2 ** (q_count - q), side="left"))
        if 0 < first < nr and (not firsts or first > firsts[-1]):
            firsts.append(first)
    firsts = [0] + firsts
    n = len(firsts)
    return [(firsts[q], ntheta_outer // 2 ** (n - 1 - q)) for q in range(n)]


def refined_production_case() -> Workload:
    """The production workload (256 x 128 x 8192 cells of 2 mm, 20-cell
    layer, 15 kHz axis source at k = 2048, 64 axis receivers) on the
    azimuthally refined grid: 4 azimuthal cells below r = 16 mm, doubling
    with the radius up to 128 from r = 256 mm (21856 cells per depth row
    instead of 32768).  The time step is half of the refined grid's own
    Courant limit."""
    w = production_case()
    w.name = "cased-well 256 x {4..128} x 8192 refined (2 mm)"
    w.extra["zones"] = refined_zones(w.nr, w.nt, 4, w.dr)
    return w


def scaled_case(nr: int, nt: int, nz: int, steps: int = 50) -> Workload:
    """The production medium on a smaller grid (same 2 mm cells and layout
    fractions); used for parity at sizes the oracle finishes quickly."""
    npml = min(20, max(2, nr // 6), max(2, (nz - 2) // 4))
    src_k = nz // 4
    rec = [min(nz - 1, src_k + 10 * (m + 1)) for m in range(8)]
    return Workload("cased-well %dx%dx%d (2 mm), %d steps" % (nr, nt, nz, steps), nr, nt, nz,
                    2e-3, 2e-3, steps=steps, npml=npml, f0=15e3, src_k=src_k, rec_k=rec,
                    z_top=(nz // 2) * 2e-3, ramp=0.3)

"""GPU parity of the azimuthally refined grid (cw_refined_*, Sec. 3) against
the FP64 refined-grid oracle, plus the properties that hold bitwise or to
FP32 rounding.  Tolerances as the uniform parity tests: traces within 1e-5
relative L2, fields within 1e-5 of their group's RMS."""
import math

import numpy as np
import pytest

import oracle
from oracle import refined as R
from paper_2302_13907_amd import cwell, inputs

from gpu_common import STRESS, VEL, announce, rel_l2

pytestmark = pytest.mark.gpu

TRACE_TOL = 1e-5
FIELD_TOL = 1e-5
H = 5e-3


def _medium(nr, nz):
    rho, lam, mu = inputs.cased_well(nr, 1, nz, H, H, z_top=nz * H / 2, ramp=0.02, radii=(0.02, 0.03, 0.045))
    return [a[:, 0, :] for a in (rho, lam, mu)]


def _times(kind, n, dt):
    off = 0.0 if kind in ("force_r", "force_z") else 0.5
    return (np.arange(n) + off) * dt


def _run_both(nr, nz, zones, steps, sources, receivers, npml=(0, 0), f0=40e3, initial=None, cfl=0.5):
    med = _medium(nr, nz)
    g = cwell.Refined(nr, nz, H, H, zones)
    o = R.RefinedOracle(nr, nz, H, H, zones)
    g.set_material_rz(*med)
    o.set_material_rz(*med)
    if npml != (0, 0):
        g.set_pml(npml[0], npml[1], 1e-3, math.pi * f0)
        o.set_pml(npml[0], npml[1], 1e-3, math.pi * f0)
    assert g.cfl_dt() == pytest.approx(o.cfl_dt(), rel=1e-12)
    dt = cfl * o.cfl_dt()
    g.set_dt(dt)
    o.set_dt(dt)
    for kind, i, j, k, amp in sources:
        w = amp * oracle.ricker(f0, _times(kind, steps, dt))
        g.add_source(kind, i, j, k, w)
        o.add_source(kind, i, j, k, w)
    for kind, i, j, k, fld in receivers:
        g.add_receiver(kind, i, j, k, fld)
        o.add_receiver(kind, i, j, k, fld)
    g.set_trace_capacity(steps)
    g.bind("cuda:0")
    if initial:
        for name, a in initial.items():
            a32 = np.asarray(a, dtype=np.float32)
            g.set_field(name, a32)
            o.set_field(name, a32.astype(np.float64))
    g.step(steps)
    tr_g = g.traces(steps)
    tr_o = o.run(steps)
    fg = {n: g.field(n).astype(np.float64) for n in R.FIELDS}
    fo = {n: o.field(n) for n in R.FIELDS}
    return g, o, tr_g, tr_o, fg, fo


def _field_errors(got, ref):
    out = {}
    for group in (VEL, STRESS):
        scale = math.sqrt(sum(float((ref[n] ** 2).sum()) for n in group) / len(group))
        for n in group:
            out[n] = float(np.linalg.norm(got[n] - ref[n]) / scale) if scale > 0 else float(np.linalg.norm(got[n]))
    return out


ZONES = [(0, 4), (4, 8), (9, 16)]


def test_refined_matches_oracle():
    """Three zones (4, 8, 16 azimuthal cells), layer in r and z, every source
    kind in a different zone, receivers in every zone: traces and all nine
    fields against the FP64 refined oracle."""
    announce("refined parity: 18 x {4,8,16} x 64, 240 steps")
    sources = [("volume", 0, -1, 20, 1e6), ("force_r", 5, 3, 30, 1e2), ("torsion", 11, -1, 26, 1e6),
               ("force_z", 2, 1, 36, 1e2)]
    receivers = [("pressure", 0, -1, 24, None), ("pressure", 0, 1, 40, None), ("field", 6, 5, 30, "vt"),
                 ("field", 12, 9, 28, "srt"), ("field", 3, 2, 33, "vr"), ("field", 9, 0, 30, "vz")]
    g, o, tr_g, tr_o, fg, fo = _run_both(18, 64, ZONES, 240, sources, receivers, npml=(4, 6))
    e = rel_l2(tr_g, tr_o)
    fe = _field_errors(fg, fo)
    announce("trace rel L2 %.2e, worst field %.2e" % (e, max(fe.values())))
    assert e <= TRACE_TOL, e
    assert max(fe.values()) <= FIELD_TOL, fe
    for m in range(len(receivers)):
        assert np.abs(tr_o[m]).max() > 0, m      # every receiver saw the wave
    g.close()


def test_refined_ragged_depth_and_one_cell_zone():
    """Zones of 1, 2 and 4 azimuthal cells, a depth that is not a multiple of
    the 1024-cell depth tile, one-ring zones."""
    announce("refined parity: 7 x {1,2,4} x 52")
    zones = [(0, 1), (1, 2), (2, 4)]
    sources = [("volume", 0, -1, 20, 1e6), ("force_r", 3, 1, 22, 1e2)]
    receivers = [("pressure", 0, -1, 26, None), ("field", 1, 1, 24, "vt"), ("field", 5, 2, 30, "vr")]
    g, o, tr_g, tr_o, fg, fo = _run_both(7, 52, zones, 200, sources, receivers, npml=(2, 5))
    e = rel_l2(tr_g, tr_o)
    fe = _field_errors(fg, fo)
    announce("trace rel L2 %.2e, worst field %.2e" % (e, max(fe.values())))
    assert e <= TRACE_TOL, e
    assert max(fe.values()) <= FIELD_TOL, fe
    g.close()


def test_single_zone_is_the_uniform_two_pass_step_bitwise():
    """One zone: the refined object runs the uniform kernels with no ghost
    ring, bitwise equal to a uniform simulation on the two-pass path."""
    nr, nt, nz = 12, 8, 64
    med = _medium(nr, nz)
    g = cwell.Refined(nr, nz, H, H, [(0, nt)])
    s = cwell.Sim(nr, nt, nz, H, H)
    for x in (g, s):
        x.set_material_rz(*med) if x is g else x.set_material(*med)
        x.set_pml(3, 5, 1e-3, math.pi * 40e3)
    dt = 0.5 * s.cfl_dt()
    w = oracle.ricker(40e3, (np.arange(120) + 0.5) * dt)
    for x in (g, s):
        x.set_dt(dt)
        x.add_source("volume", 0, -1, 20, w)
        x.add_source("force_r", 4, 2, 30, w)
        x.add_receiver("pressure", 0, -1, 24)
        x.set_trace_capacity(120)
    s.set_path("two-pass")
    g.bind("cuda:0")
    s.bind("cuda:0")
    g.step(120)
    s.step(120)
    s.sync()
    assert np.array_equal(g.traces(120), s.traces())
    for n in R.FIELDS:
        assert np.array_equal(g.field(n), s.field(n).reshape(-1)), n
    g.close()
    s.close()


def test_refined_energy_conserved_gpu():
    """Layer off, no source, random state: the float64 energy of the float32
    refined state drifts only at float32 rounding level across the zone
    interfaces, and starts at the oracle's value."""
    nr, nz = 14, 64
    zones = [(0, 4), (3, 8), (8, 16)]
    o = R.RefinedOracle(nr, nz, H, H, zones)
    o.set_material_rz(*_medium(nr, nz))
    rng = np.random.default_rng(9)
    init = {}
    for name in R.FIELDS:
        parts = []
        for i in range(nr):
            sh = (o.nt[i], nz)
            if name in ("srr", "stt", "szz"):
                a = rng.standard_normal(sh)
            elif name == "srt":
                a = np.where((o.mu_rt[i] > 0)[None, :], rng.standard_normal(sh), 0.0)
            elif name == "srz":
                a = np.where((o.mu_rz[i] > 0)[None, :], rng.standard_normal(sh), 0.0)
            elif name == "stz":
                a = np.where((o.mu_tz[i] > 0)[None, :], rng.standard_normal(sh), 0.0)
            else:
                a = 1e-6 * rng.standard_normal(sh)
            parts.append(a)
        init[name] = parts
    fluid = [(o.mu[i] == 0)[None, :] for i in range(nr)]
    for i in range(nr):                      # isotropic stress in the fluid
        init["stt"][i] = np.where(fluid[i], init["srr"][i], init["stt"][i])
        init["szz"][i] = np.where(fluid[i], init["srr"][i], init["szz"][i])
    init = {k: np.concatenate([p.reshape(-1) for p in v]).astype(np.float32) for k, v in init.items()}
    g = cwell.Refined(nr, nz, H, H, zones)
    g.set_material_rz(*_medium(nr, nz))
    dt = 0.5 * g.cfl_dt()
    g.set_dt(dt)
    g.bind("cuda:0")
    for name, a in init.items():
        g.set_field(name, a)
    g.step(1)
    E = [g.energy()]
    for _ in range(30):
        g.step(10)
        E.append(g.energy())
    E = np.array(E)
    drift = np.abs(E / E[0] - 1).max()
    announce("refined energy drift over 301 steps: %.2e" % drift)
    assert drift < 2e-5, drift
    o.set_dt(dt)
    for name, a in init.items():
        o.set_field(name, a.astype(np.float64))
    _, Eo = o.run(1, energy=True)
    assert abs(E[0] / Eo[0] - 1) < 1e-6
    g.close()


def test_refined_axisymmetric_matches_uniform_one_cell_gpu():
    """A ring source in an axisymmetric medium: the refined grid's traces
    equal those of the uniform grid with one azimuthal cell to float32
    rounding (the interpolation of a theta-constant ring is the constant)."""
    nr, nz = 16, 64
    med = _medium(nr, nz)
    g = cwell.Refined(nr, nz, H, H, [(0, 2), (3, 4), (7, 8)])
    s = cwell.Sim(nr, 1, nz, H, H)
    g.set_material_rz(*med)
    s.set_material(*med)
    for x in (g, s):
        x.set_pml(4, 5, 1e-3, math.pi * 40e3)
    dt = 0.5 * g.cfl_dt()
    w = oracle.ricker(40e3, (np.arange(200) + 0.5) * dt)
    for x in (g, s):
        x.set_dt(dt)
        x.add_source("volume", 0, -1, 20, 1e6 * w)
        x.add_receiver("pressure", 0, -1, 24)
        x.add_receiver("pressure", 9, -1, 30)
        x.add_receiver("pressure", 13, -1, 40)
        x.set_trace_capacity(200)
    s.set_path("two-pass")
    g.bind("cuda:0")
    s.bind("cuda:0")
    g.step(200)
    s.step(200)
    s.sync()
    e = rel_l2(g.traces(200), s.traces())
    announce("refined vs one-cell uniform: %.2e" % e)
    assert e < 1e-5, e
    vt = g.field("vt")
    assert np.abs(vt).max() <= 1e-6 * np.abs(g.field("vr")).max()
    g.close()
    s.close()


def test_refined_reset_and_rerun_bitwise():
    """cw_refined_reset returns to rest: a second run repeats the first
    bitwise (ghost rings included)."""
    sources = [("volume", 0, -1, 20, 1e6), ("force_r", 5, 3, 30, 1e2)]
    receivers = [("pressure", 0, -1, 24, None), ("field", 12, 9, 28, "srt")]
    med = _medium(18, 64)
    g = cwell.Refined(18, 64, H, H, ZONES)
    g.set_material_rz(*med)
    g.set_pml(4, 6, 1e-3, math.pi * 40e3)
    dt = 0.5 * g.cfl_dt()
    g.set_dt(dt)
    for kind, i, j, k, amp in sources:
        g.add_source(kind, i, j, k, amp * oracle.ricker(40e3, _times(kind, 100, dt)))
    for kind, i, j, k, fld in receivers:
        g.add_receiver(kind, i, j, k, fld)
    g.set_trace_capacity(100)
    g.bind("cuda:0")
    g.step(100)
    a = g.traces(100)
    fa = g.field("vz")
    g.reset()
    g.step(100)
    assert np.array_equal(a, g.traces(100))
    assert np.array_equal(fa, g.field("vz"))
    g.close()

"""Physics pins of the FP64 oracle: wave speeds the theory (or the paper)
fixes, and a bound on the absorbing layer's reflection."""
import json
import math
import os

import numpy as np

import oracle
from oracle import OracleSim
from paper_2302_13907_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lag(a, b, dt):
    """Delay of trace b behind trace a by cross-correlation, with a
    parabolic refinement of the peak."""
    n = len(a)
    c = np.correlate(b, a, mode="full")
    m = int(np.argmax(c))
    if 0 < m < len(c) - 1:
        y0, y1, y2 = c[m - 1], c[m], c[m + 1]
        m = m + 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2)
    return (m - (n - 1)) * dt


def test_tube_wave_speed():
    """Open fluid-filled hole in rock: the low-frequency tube wave travels at
    V_f / sqrt(1 + rho_f V_f^2 / mu) (the long-wave limit of the borehole
    problem of Biot 1952 that Sec. 1 starts from)."""
    h = 0.01
    nr, nz = 60, 800
    rho, lam, mu = inputs.cased_well(nr, 1, nz, h, h, z_top=1e9, radii=(0.1, 0.1, 0.1))
    # fluid r < 0.1 m, rock beyond (radii collapse the casing and annulus)
    assert mu[9, 0, 0] == 0 and mu[10, 0, 0] > 0
    o = OracleSim(nr, 1, nz, h, h)
    o.set_material(rho, lam, mu)
    f0 = 1000.0
    o.set_pml(10, 10, 1e-3, math.pi * f0)
    dt = 0.5 * o.cfl_dt()
    o.set_dt(dt)
    nsteps = int(7.0e-3 / dt)
    w = oracle.ricker(f0, (np.arange(nsteps) + 0.5) * dt)
    o.add_source("volume", 0, -1, 100, w)
    o.add_receiver("pressure", 0, -1, 300)
    o.add_receiver("pressure", 0, -1, 600)
    tr = o.run(nsteps)
    v = (600 - 300) * h / _lag(tr[0], tr[1], dt)
    vf, rhof = 1500.0, 1000.0
    mu_rock = 2400.0 * 2300.0 ** 2
    vt = vf / math.sqrt(1 + rhof * vf * vf / mu_rock)
    assert abs(v / vt - 1) < 0.01, (v, vt)


def test_torsion_wave_in_casing():
    """Torsion ring source in a steel casing between fluids (Sec. 5): the
    wave runs along the pipe at the metal's shear speed printed in the paper
    and no field in the fluid ever moves."""
    g = json.load(open(os.path.join(GOLDEN, "torsion_wave_speed.json")))
    vs = g["shear_speed_m_per_s"]
    h = 5e-3
    nr, nz = 30, 700
    rho, lam, mu = inputs.homogeneous(nr, 1, nz)
    steel = (slice(20, 22), slice(None), slice(None))      # r in [0.10, 0.11)
    ro, la, m = inputs.moduli(5900.0, vs, 7850.0)
    rho[steel], lam[steel], mu[steel] = ro, la, m
    o = OracleSim(nr, 1, nz, h, h)
    o.set_material(rho, lam, mu)
    f0 = 10e3
    o.set_pml(6, 10, 1e-3, math.pi * f0)
    dt = 0.5 * o.cfl_dt()
    o.set_dt(dt)
    nsteps = int(1.1e-3 / dt)
    w = oracle.ricker(f0, (np.arange(nsteps) + 0.5) * dt)
    o.add_source("torsion", 20, -1, 60, w)
    o.add_receiver("field", 20, -1, 200, "vt")
    o.add_receiver("field", 20, -1, 500, "vt")
    tr = o.run(nsteps)
    v = (500 - 200) * h / _lag(tr[0], tr[1], dt)
    assert abs(v / vs - 1) < g["tolerance_relative"], (v, vs)
    vt = o.field("vt")
    assert np.abs(vt[20:22]).max() > 0
    for name in ("vt", "srt", "stz"):
        f = o.field(name)
        assert not np.any(f[:20]), name          # fluid inside the pipe
        assert not np.any(f[22:]), name          # fluid outside the pipe
    for name in ("vr", "vz", "srr", "stt", "szz", "srz"):
        assert not np.any(o.field(name)), name


def _pml_traces(nt, npml, extra, src, T, f0=20e3):
    """Traces of a cased-well run on a small domain (extra = (0, 0)) or on one
    padded by extra = (cells in r, cells at each z end), receivers at the same
    physical places.  The source sits 0.1 m below the top layer, so the
    waves in the fluid reach the layer and come back within the window; the
    padding keeps the fastest waves (5900 m/s along the steel) from coming
    back from the padded domain's own ends before the window closes."""
    h = 5e-3
    nr0, nz0 = 30 + npml, 80 + 2 * npml
    nr, nz = nr0 + extra[0], nz0 + 2 * extra[1]
    ez = extra[1]
    rho, lam, mu = inputs.cased_well(nr, nt, nz, h, h, z_top=(ez + npml + 50) * h)
    o = OracleSim(nr, nt, nz, h, h)
    o.set_material(rho, lam, mu)
    o.set_pml(npml, npml, 1e-3, math.pi * f0)
    # the same time step for both domains: the Courant limit is set by the axis
    dt = 0.5 * o.cfl_dt()
    o.set_dt(dt)
    nsteps = int(T / dt)
    w = oracle.ricker(f0, (np.arange(nsteps) + 0.5) * dt)
    k0 = ez + npml + 20
    kind, i, j = src
    o.add_source(kind, i, j, k0, w)
    for dk in (-10, 10, 30):
        o.add_receiver("pressure", 0, -1, k0 + dk)
    for (ii, jj, name) in ((25, 0, "vr"), (25, 0, "vz"), (12, 0, "srr"), (25, 1 % nt, "vt")):
        o.add_receiver("field", ii, jj, k0 + 10, name)
    return o.run(nsteps)


def _pml_error(nt, npml, src, T=400e-6, extra=(150, 250)):
    small = _pml_traces(nt, npml, (0, 0), src, T)
    big = _pml_traces(nt, npml, extra, src, T)
    return np.linalg.norm(small - big) / np.linalg.norm(big)


def test_pml_reflection_bound():
    """The absorbing layer (unsplit in theta, Sec. 1 and Sec. 6): relative L2
    difference between a small domain closed by the layer and a domain large
    enough that nothing comes back within the window.  A rigid closure in
    place of the layer differs by order one."""
    e10 = _pml_error(1, 10, ("volume", 0, -1))
    e20 = _pml_error(1, 20, ("volume", 0, -1))
    assert e10 < 1e-3, e10
    assert e20 < 3e-4, e20
    # a non-axisymmetric source (off-axis radial point force) in 3-D
    e3d = _pml_error(4, 10, ("force_r", 3, 0), T=300e-6, extra=(90, 170))
    assert e3d < 2e-3, e3d

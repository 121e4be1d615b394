"""Rigid fluid-filled pipe: a plane wave travels along it exactly as the 1-D
staggered acoustic scheme says (oracle pin, CPU only).

A fluid column (mu = 0, rho = 1000, V_f = 1500 m/s) closed at its outer
radius by a ring of practically infinite density, so that the radial
velocity on that face stays at zero (a rigid wall: the face buoyancy is
2 / (rho_f + rho_wall), 1e-27 of the fluid's), and a source that injects the
same stress at one depth on every fluid ring.  With the pressure the same at
every radius and azimuth, v_r and v_theta stay zero (the radial derivative,
the hoop term (s_rr - s_tt)/r and every azimuthal derivative vanish), and the
update of Eq. (1) on the staggered grid of Sec. 3 reduces to the textbook 1-D
staggered leapfrog in z:

    v(k+1/2) += dt / rho * (s(k+1) - s(k)) / dz      (s beyond the ends = 0)
    s(k)     += dt * K * (v(k+1/2) - v(k-1/2)) / dz  (v before the top = 0)

with the pressure -s.  The 3-D oracle must give that 1-D solution on every
ring and azimuth to FP64 rounding, and the pulse must cross the column at the
fluid speed (up to the 1-D scheme's dispersion at 30 cells per wavelength).
The 1-D reference below is written out here, independent of the oracle.
It pins the z stencils, the leapfrog order, the volume-source normalisation
(the ring volume 2 pi r dr dz) and the pressure receiver."""
import math

import numpy as np

import oracle

RHO, VF = 1000.0, 1500.0
K = RHO * VF * VF
NR, NT, NZ = 6, 3, 400          # rings 0..4 fluid, ring 5 the wall
H = 5e-3
F0 = 10e3
KS = 60                          # source depth
KR = (120, 220)                  # receiver depths


def _oracle_run(steps):
    o = oracle.OracleSim(NR, NT, NZ, H, H)
    rho = np.full((NR, NT, NZ), RHO)
    rho[NR - 1] = 1e30                              # the wall ring
    lam = np.full((NR, NT, NZ), K)
    mu = np.zeros((NR, NT, NZ))
    o.set_material(rho, lam, mu)
    dt = 0.5 * o.cfl_dt()
    o.set_dt(dt)
    f = oracle.ricker(F0, (np.arange(steps) + 0.5) * dt)
    for i in range(NR - 1):
        # the ring source injects dt * w / (2 pi r_i dr dz) per cell: scale by
        # that volume so that every ring receives dt * f
        vol = 2.0 * math.pi * (i + 0.5) * H * H * H
        o.add_source("volume", i, -1, KS, f * vol)
    recs = []
    for k in KR:
        for i in (0, 2, NR - 2):
            recs.append(("ring", i, k, o.add_receiver("pressure", i, -1, k)))
        recs.append(("point", 3, k, o.add_receiver("pressure", 3, 1, k)))
    tr = o.run(steps)
    return dt, f, tr, recs, o


def _plane_1d(dt, f, steps):
    """The 1-D staggered leapfrog, pressure traces at KR."""
    s = np.zeros(NZ)
    v = np.zeros(NZ)                                # v[k] at z_{k+1/2}
    out = np.zeros((len(KR), steps))
    for n in range(steps):
        s_up = np.append(s[1:], 0.0)
        v += dt / RHO * (s_up - s) / H
        v_dn = np.insert(v[:-1], 0, 0.0)
        s += dt * K * (v - v_dn) / H
        s[KS] += dt * f[n]
        for q, k in enumerate(KR):
            out[q, n] = -s[k]
    return out


def test_rigid_pipe_plane_wave_matches_1d_scheme():
    steps = 900
    dt, f, tr, recs, o = _oracle_run(steps)
    ref = _plane_1d(dt, f, steps)
    scale = np.abs(ref).max()
    assert scale > 0
    for kind, i, k, m in recs:
        err = np.abs(tr[m] - ref[KR.index(k)]).max() / scale
        assert err < 1e-12, (kind, i, k, err)
    # the radial and azimuthal velocities stay zero, to the rounding of the
    # per-ring source volumes (the rings' stresses differ by a few ulp)
    vs = np.abs(o.field("vz")).max()
    assert vs > 0
    assert np.abs(o.field("vr")[: NR - 1]).max() < 1e-12 * vs
    assert np.abs(o.field("vt")).max() == 0.0


def test_rigid_pipe_plane_wave_travels_at_the_fluid_speed():
    steps = 1000
    dt, f, tr, recs, _ = _oracle_run(steps)
    ring = {k: tr[m] for kind, i, k, m in recs if kind == "ring" and i == 0}

    # the wavelet's central trough in the pressure of the direct (downgoing)
    # wave, searched within one period of its expected arrival (the wave
    # reflected at the free top surface arrives later and inverted);
    # parabolic interpolation of the extremum
    def t_trough(x, k):
        t0 = 2.0 / F0 + (k - KS) * H / VF
        lo, hi = int((t0 - 1.0 / F0) / dt), int((t0 + 1.0 / F0) / dt)
        n = lo + int(np.argmin(x[lo:hi]))
        a, b, c = x[n - 1], x[n], x[n + 1]
        return (n + 0.5 * (a - c) / (a - 2 * b + c)) * dt
    speed = (KR[1] - KR[0]) * H / (t_trough(ring[KR[1]], KR[1]) - t_trough(ring[KR[0]], KR[0]))
    # measured 1493.7 m/s (-0.4 %): the 1-D scheme's dispersion at 30 cells
    # per wavelength, and the trough of a broadband pulse
    assert abs(speed / VF - 1.0) < 1e-2, speed

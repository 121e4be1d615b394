"""FP64 reference of the time step on an azimuthally refined grid (Sec. 3).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may use this module; the product package never does.  It shares
no code with the HIP path (nor with ``cwell_oracle.c``: it is a second,
independent implementation of the same scheme, in numpy).

The grid.  Sec. 3 observes that the azimuthal cell width grows linearly with
r and halves the azimuthal step every time the radius doubles.  Here the
rings are split into zones; zone q holds rings [first_q, first_{q+1}) with
N_theta = N_q azimuthal cells, and N_{q+1} = 2 N_q.  Within a zone the
scheme is the uniform one (staggered velocity-stress form of Eq. (1),
cylindrical, zero values outside the grid, periodic theta); the medium must
not vary along theta.

The interface.  Across the circle between the last ring b-1 of a coarse zone
and the first ring b of the next (fine) zone, a stencil of one ring needs
values of the other ring on its own azimuthal grid:
  * coarse -> fine (what the paper describes): the coarse samples are
    Fourier transformed, the spectrum is extended with zeros to the fine
    length, and the inverse transform gives the fine samples.  Quantities
    on half-integer azimuthal nodes (v_theta, sigma_r_theta, sigma_theta_z)
    sit half a coarse cell from the fine half-integer nodes, so their
    spectrum is shifted in phase by that offset before the inverse
    transform.  The coarse Nyquist mode is split evenly between +N/2 and
    -N/2.
  * fine -> coarse (not stated in the paper; read here as the weighted
    transpose of the former, R = (1/2) P^T, the factor being
    dtheta_fine / dtheta_coarse): the fine samples are transformed, the
    spectrum is cut to the coarse band (the two halves of the coarse
    Nyquist mode folded back together, phase shift conjugated), and the
    inverse transform times 1/2 gives the coarse samples.  It reproduces
    band-limited functions exactly, and with it the coupling of the two
    rings keeps the discrete energy of the uniform scheme conserved.
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

FIELDS = ("vr", "vt", "vz", "srr", "stt", "szz", "srt", "srz", "stz")
# fields on half-integer azimuthal nodes (theta_{j+1/2})
HALF = {"vt", "srt", "stz"}
SRC_KINDS = ("volume", "force_r", "force_z", "torsion")


# ---------------------------------------------------------------------------
# Interpolation between azimuthal grids (Sec. 3: transform, zero-pad, inverse)

def _phase(nc: int, nf: int, half: bool) -> float:
    """Offset (radians) of the fine nodes from the coarse nodes' origin:
    half-integer nodes sit at (j + 1/2) dtheta on each grid."""
    if not half:
        return 0.0
    return 0.5 * (2.0 * math.pi / nf) - 0.5 * (2.0 * math.pi / nc)


def _signed(idx: int, n: int) -> int:
    return idx if idx <= (n - 1) // 2 else idx - n


def prolong(x: np.ndarray, nf: int, half: bool) -> np.ndarray:
    """Coarse samples x[nc, ...] -> fine samples [nf, ...] (nf = 2 nc)."""
    nc = x.shape[0]
    c = np.fft.fft(x, axis=0)
    phi = _phase(nc, nf, half)
    C = np.zeros((nf,) + x.shape[1:], dtype=complex)
    for idx in range(nc):
        m = _signed(idx, nc)
        if nc % 2 == 0 and idx == nc // 2:
            continue                                 # Nyquist mode, below
        C[m % nf] = c[idx] * np.exp(1j * m * phi)
    if nc % 2 == 0:
        h = nc // 2
        C[h % nf] += 0.5 * c[h] * np.exp(1j * h * phi)
        C[(-h) % nf] += 0.5 * c[h] * np.exp(-1j * h * phi)
    y = np.fft.ifft(C, axis=0) * (nf / nc)
    return y.real


def restrict(y: np.ndarray, nc: int, half: bool) -> np.ndarray:
    """Fine samples y[nf, ...] -> coarse samples [nc, ...]: (1/2) prolong^T."""
    nf = y.shape[0]
    Y = np.fft.fft(y, axis=0)
    phi = _phase(nc, nf, half)
    c = np.zeros((nc,) + y.shape[1:], dtype=complex)
    for idx in range(nc):
        m = _signed(idx, nc)
        if nc % 2 == 0 and idx == nc // 2:
            continue
        c[idx] = Y[m % nf] * np.exp(-1j * m * phi)
    if nc % 2 == 0:
        h = nc // 2
        c[h] = 0.5 * (Y[h % nf] * np.exp(-1j * h * phi) + Y[(-h) % nf] * np.exp(1j * h * phi))
    x = np.fft.ifft(c, axis=0) * 0.5
    return x.real


# ---------------------------------------------------------------------------

def hm4(a, b, c, d):
    """Harmonic mean of four moduli; zero where any of them is zero."""
    a, b, c, d = (np.asarray(v, dtype=float) for v in (a, b, c, d))
    out = np.zeros(np.broadcast(a, b, c, d).shape)
    ok = (a != 0) & (b != 0) & (c != 0) & (d != 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        v = 4.0 / (1.0 / a + 1.0 / b + 1.0 / c + 1.0 / d)
    out[ok] = np.broadcast_to(v, out.shape)[ok]
    return out


def _pml_coef(d, alpha, dt):
    b = np.exp(-(d + alpha) * dt)
    a = np.where(d > 0, d * (b - 1.0) / np.where(d + alpha > 0, d + alpha, 1.0), 0.0)
    return a, b


def zone_plan(nr: int, ntheta_outer: int, ntheta_inner: int, dr: float):
    """Zones that halve the azimuthal step each time the radius doubles
    (Sec. 3), keeping the outer resolution: with r_max = nr dr and Q zones
    (ntheta_inner doubling up to ntheta_outer), zone Q-1 holds the rings
    whose centre radius lies in [r_max / 2, r_max), zone Q-2 those in
    [r_max / 4, r_max / 2), ..., zone 0 every ring below r_max / 2^(Q-1).
    A zone that would hold no ring is left out; the cell counts then halve
    inwards from the outermost zone, one halving per zone kept.  Returns
    [(first_ring, ntheta), ...]."""
    q_count = int(round(math.log2(ntheta_outer / ntheta_inner))) + 1
    if ntheta_inner < 1 or ntheta_inner * 2 ** (q_count - 1) != ntheta_outer:
        raise ValueError("ntheta_outer / ntheta_inner must be a power of two")
    r_max = nr * dr
    starts = [0]
    for q in range(1, q_count):
        edge = r_max / 2 ** (q_count - q)
        first = next((i for i in range(nr) if (i + 0.5) * dr >= edge), nr)
        if first < nr and first > starts[-1]:
            starts.append(first)
    n = len(starts)
    return [(starts[q], ntheta_outer // 2 ** (n - 1 - q)) for q in range(n)]


class RefinedOracle:
    """The time step on a zoned grid, FP64, numpy.  Arrays per ring:
    ring i holds [ntheta_i][nz]; get_field returns the rings concatenated
    (ring 0 first), set_field takes the same layout."""

    def __init__(self, nr: int, nz: int, dr: float, dz: float, zones: Sequence[Tuple[int, int]]):
        zones = [(int(a), int(b)) for a, b in zones]
        if not zones or zones[0][0] != 0:
            raise ValueError("the first zone starts at ring 0")
        for (a0, n0), (a1, n1) in zip(zones, zones[1:]):
            if not (a1 > a0 and n1 == 2 * n0):
                raise ValueError("zones must start at increasing rings and double ntheta")
        if zones[-1][0] >= nr:
            raise ValueError("a zone starts beyond the last ring")
        self.nr, self.nz, self.dr, self.dz = nr, nz, dr, dz
        self.zones = zones
        self.nt = np.zeros(nr, dtype=int)
        for q, (a, n) in enumerate(zones):
            b = zones[q + 1][0] if q + 1 < len(zones) else nr
            self.nt[a:b] = n
        self.dth = 2.0 * math.pi / self.nt
        self.rc = (np.arange(nr) + 0.5) * dr
        self.rf = (np.arange(nr) + 1.0) * dr
        self.f = {name: [np.zeros((self.nt[i], nz)) for i in range(nr)] for name in FIELDS}
        self.dt = 0.0
        self.npr = self.npz = 0
        self.psi = None
        self.src = []
        self.rec = []
        self.nstep = 0

    # ------------------------------------------------------------------ setup
    @property
    def cells(self) -> int:
        return int(self.nt.sum()) * self.nz

    def set_material_rz(self, rho, lam, mu):
        """Medium [nr][nz] (no theta dependence)."""
        rho, lam, mu = (np.array(a, dtype=float).reshape(self.nr, self.nz) for a in (rho, lam, mu))
        if not (np.all(rho > 0) and np.all(mu >= 0) and np.all(lam + 2 * mu > 0)):
            raise ValueError("bad medium")
        self.rho, self.lam, self.mu = rho, lam, mu
        i1 = np.minimum(np.arange(self.nr) + 1, self.nr - 1)
        k1 = np.minimum(np.arange(self.nz) + 1, self.nz - 1)
        self.b_r = 2.0 / (rho + rho[i1, :])
        self.b_t = 2.0 / (rho + rho)
        self.b_z = 2.0 / (rho + rho[:, k1])
        self.mu_rt = hm4(mu, mu[i1, :], mu, mu[i1, :])
        self.mu_rz = hm4(mu, mu[i1, :], mu[:, k1], mu[i1][:, k1])
        self.mu_tz = hm4(mu, mu, mu[:, k1], mu[:, k1])

    def vp_max(self) -> float:
        return float(np.sqrt((self.lam + 2 * self.mu) / self.rho).max())

    def cfl_dt(self) -> float:
        """Courant limit with each ring's own azimuthal width r_i dtheta_i."""
        vp = np.sqrt((self.lam + 2 * self.mu) / self.rho)
        ra = self.rc * self.dth
        g = np.sqrt(1.0 / self.dr ** 2 + 1.0 / ra ** 2 + 1.0 / self.dz ** 2)
        return float((1.0 / (vp * g[:, None])).min())

    def set_pml(self, npr: int, npz: int, rc: float = 1e-3, alpha: float = 0.0):
        self.npr, self.npz, self.pml_rc, self.alpha = npr, npz, rc, alpha

    def set_dt(self, dt: float):
        self.dt = dt
        if self.npr == 0 and self.npz == 0:
            self.psi = None
            return
        vpm = self.vp_max()
        Lr, Lz = self.npr * self.dr, self.npz * self.dz
        d0r = -3.0 * vpm * math.log(self.pml_rc) / (2.0 * Lr) if self.npr > 0 else 0.0
        d0z = -3.0 * vpm * math.log(self.pml_rc) / (2.0 * Lz) if self.npz > 0 else 0.0
        rp = (self.nr - self.npr) * self.dr

        def radial(r):
            x = np.where((self.npr > 0) & (r > rp), (r - rp) / Lr if Lr > 0 else 0.0, 0.0)
            d = d0r * x * x
            dtl = d0r * Lr * x ** 3 / (3.0 * r) if self.npr > 0 else np.zeros_like(r)
            return _pml_coef(d, self.alpha, dt), _pml_coef(dtl, self.alpha, dt)

        (self.ar_c, self.br_c), (self.at_c, self.bt_c) = radial(self.rc)
        (self.ar_f, self.br_f), (self.at_f, self.bt_f) = radial(self.rf)

        def depth(z):
            if self.npz == 0:
                x = np.zeros_like(z)
            else:
                x1 = (self.npz * self.dz - z) / Lz
                x2 = (z - (self.nz - 1 - self.npz) * self.dz) / Lz
                x = np.maximum(np.maximum(x1, x2), 0.0)
            return _pml_coef(d0z * x * x, self.alpha, dt)

        self.az_c, self.bz_c = depth(np.arange(self.nz) * self.dz)
        self.az_h, self.bz_h = depth((np.arange(self.nz) + 0.5) * self.dz)
        names = ("vr_dr", "vr_b", "vr_dz", "vt_dr", "vt_b", "vt_dz", "vz_dr", "vz_b", "vz_dz",
                 "n_dr", "n_b", "n_dz", "rt_dr", "rt_b", "rz_dr", "rz_dz", "tz_b", "tz_dz")
        self.psi = {q: [np.zeros((self.nt[i], self.nz)) for i in range(self.nr)] for q in names}

    def add_source(self, kind: str, i: int, j: int, k: int, w: Sequence[float]):
        if kind not in SRC_KINDS or not (0 <= i < self.nr and -1 <= j < self.nt[i] and 0 <= k < self.nz):
            raise ValueError("bad source")
        self.src.append((kind, i, j, k, np.asarray(w, dtype=float)))

    def add_receiver(self, kind: str, i: int, j: int, k: int, field: Optional[str] = None) -> int:
        if kind not in ("pressure", "field") or not (0 <= i < self.nr and -1 <= j < self.nt[i] and 0 <= k < self.nz):
            raise ValueError("bad receiver")
        if kind == "field" and field not in FIELDS:
            raise ValueError("bad field")
        self.rec.append((kind, field, i, j, k))
        return len(self.rec) - 1

    # ----------------------------------------------------------- ring access
    def _nb(self, name: str, i: int, di: int) -> np.ndarray:
        """Field `name` of ring i + di seen on ring i's azimuthal grid (zero
        beyond the grid)."""
        n = i + di
        if n < 0 or n >= self.nr:
            return np.zeros((self.nt[i], self.nz))
        x = self.f[name][n]
        if self.nt[n] == self.nt[i]:
            return x
        half = name in HALF
        if self.nt[n] * 2 == self.nt[i]:
            return prolong(x, self.nt[i], half)
        if self.nt[n] == 2 * self.nt[i]:
            return restrict(x, self.nt[i], half)
        raise AssertionError("zones differ by more than a factor two")

    @staticmethod
    def _km(a):       # value at k-1 (zero before the first row)
        out = np.zeros_like(a)
        out[:, 1:] = a[:, :-1]
        return out

    @staticmethod
    def _kp(a):       # value at k+1 (zero after the last row)
        out = np.zeros_like(a)
        out[:, :-1] = a[:, 1:]
        return out

    def _stretch(self, q, i, a, b, X):
        if self.psi is None:
            return X
        p = self.psi[q][i]
        p[...] = b * p + a * X
        return X + p

    # ------------------------------------------------------------- the step
    def _velocity(self):
        f, dr, dz, dt = self.f, self.dr, self.dz, self.dt
        new = {}
        for i in range(self.nr):
            dth, rci, rfi = self.dth[i], self.rc[i], self.rf[i]
            srr, stt, szz = f["srr"][i], f["stt"][i], f["szz"][i]
            srt, srz, stz = f["srt"][i], f["srz"][i], f["stz"][i]
            srr1, stt1 = self._nb("srr", i, 1), self._nb("stt", i, 1)
            srt0, srz0 = self._nb("srt", i, -1), self._nb("srz", i, -1)
            L = self.psi is not None
            # v_r at (R_i, theta_j, z_k)
            Dr = (srr1 - srr) / dr
            B = (1.0 / rfi) * ((srt - np.roll(srt, 1, axis=0)) / dth + 0.5 * (srr1 + srr) - 0.5 * (stt1 + stt))
            Dz = (srz - self._km(srz)) / dz
            if L:
                Dr = self._stretch("vr_dr", i, self.ar_f[i], self.br_f[i], Dr)
                B = self._stretch("vr_b", i, self.at_f[i], self.bt_f[i], B)
                Dz = self._stretch("vr_dz", i, self.az_c, self.bz_c, Dz)
            dvr = dt * self.b_r[i] * (Dr + B + Dz)
            # v_theta at (r_i, theta_{j+1/2}, z_k)
            Dr = (srt - srt0) / dr
            B = (1.0 / rci) * ((np.roll(stt, -1, axis=0) - stt) / dth + (srt + srt0))
            Dz = (stz - self._km(stz)) / dz
            if L:
                Dr = self._stretch("vt_dr", i, self.ar_c[i], self.br_c[i], Dr)
                B = self._stretch("vt_b", i, self.at_c[i], self.bt_c[i], B)
                Dz = self._stretch("vt_dz", i, self.az_c, self.bz_c, Dz)
            dvt = dt * self.b_t[i] * (Dr + B + Dz)
            # v_z at (r_i, theta_j, z_{k+1/2})
            Dr = (srz - srz0) / dr
            B = (1.0 / rci) * ((stz - np.roll(stz, 1, axis=0)) / dth + 0.5 * (srz + srz0))
            Dz = (self._kp(szz) - szz) / dz
            if L:
                Dr = self._stretch("vz_dr", i, self.ar_c[i], self.br_c[i], Dr)
                B = self._stretch("vz_b", i, self.at_c[i], self.bt_c[i], B)
                Dz = self._stretch("vz_dz", i, self.az_h, self.bz_h, Dz)
            dvz = dt * self.b_z[i] * (Dr + B + Dz)
            new[i] = (dvr, dvt, dvz)
        for i in range(self.nr):     # the right-hand sides read only stresses
            f["vr"][i] = f["vr"][i] + new[i][0]
            f["vt"][i] = f["vt"][i] + new[i][1]
            f["vz"][i] = f["vz"][i] + new[i][2]

    def _stress(self):
        f, dr, dz, dt = self.f, self.dr, self.dz, self.dt
        new = {}
        for i in range(self.nr):
            dth, rci, rfi = self.dth[i], self.rc[i], self.rf[i]
            vr, vt, vz = f["vr"][i], f["vt"][i], f["vz"][i]
            vr0 = self._nb("vr", i, -1)
            vt1, vz1 = self._nb("vt", i, 1), self._nb("vz", i, 1)
            L = self.psi is not None
            err = (vr - vr0) / dr
            ett = (1.0 / rci) * ((vt - np.roll(vt, 1, axis=0)) / dth + 0.5 * (vr + vr0))
            ezz = (vz - self._km(vz)) / dz
            if L:
                err = self._stretch("n_dr", i, self.ar_c[i], self.br_c[i], err)
                ett = self._stretch("n_b", i, self.at_c[i], self.bt_c[i], ett)
                ezz = self._stretch("n_dz", i, self.az_c, self.bz_c, ezz)
            lam, mu = self.lam[i], self.mu[i]
            tr = err + ett + ezz
            d_rr = dt * (lam * tr + 2.0 * mu * err)
            d_tt = dt * (lam * tr + 2.0 * mu * ett)
            d_zz = dt * (lam * tr + 2.0 * mu * ezz)
            # sigma_r_theta at (R_i, theta_{j+1/2}, z_k)
            Dr = (vt1 - vt) / dr
            B = (1.0 / rfi) * ((np.roll(vr, -1, axis=0) - vr) / dth - 0.5 * (vt1 + vt))
            if L:
                Dr = self._stretch("rt_dr", i, self.ar_f[i], self.br_f[i], Dr)
                B = self._stretch("rt_b", i, self.at_f[i], self.bt_f[i], B)
            d_rt = dt * self.mu_rt[i] * (Dr + B)
            # sigma_rz at (R_i, theta_j, z_{k+1/2})
            Dr = (vz1 - vz) / dr
            Dz = (self._kp(vr) - vr) / dz
            if L:
                Dr = self._stretch("rz_dr", i, self.ar_f[i], self.br_f[i], Dr)
                Dz = self._stretch("rz_dz", i, self.az_h, self.bz_h, Dz)
            d_rz = dt * self.mu_rz[i] * (Dr + Dz)
            # sigma_theta_z at (r_i, theta_{j+1/2}, z_{k+1/2})
            B = (1.0 / rci) * (np.roll(vz, -1, axis=0) - vz) / dth
            Dz = (self._kp(vt) - vt) / dz
            if L:
                B = self._stretch("tz_b", i, self.at_c[i], self.bt_c[i], B)
                Dz = self._stretch("tz_dz", i, self.az_h, self.bz_h, Dz)
            d_tz = dt * self.mu_tz[i] * (B + Dz)
            new[i] = (d_rr, d_tt, d_zz, d_rt, d_rz, d_tz)
        for i in range(self.nr):
            for q, name in enumerate(("srr", "stt", "szz", "srt", "srz", "stz")):
                f[name][i] = f[name][i] + new[i][q]

    def _inject(self, name, rad, coef, i, j, k, amp):
        vol = 2.0 * math.pi * rad * self.dr * self.dz if j < 0 else rad * self.dr * self.dth[i] * self.dz
        c = 1.0 if coef is None else coef[i, k]
        if j < 0:
            self.f[name][i][:, k] += self.dt * c * amp / vol
        else:
            self.f[name][i][j, k] += self.dt * c * amp / vol

    def _sources(self, n, stress_phase):
        for kind, i, j, k, w in self.src:
            a = w[n] if n < len(w) else 0.0
            if a == 0.0:
                continue
            if kind == "volume" and stress_phase:
                for name in ("srr", "stt", "szz"):
                    self._inject(name, self.rc[i], None, i, j, k, a)
            elif kind == "torsion" and stress_phase:
                self._inject("srt", self.rf[i], None, i, j, k, a)
                self._inject("stz", self.rc[i], None, i, j, k, a)
            elif kind == "force_r" and not stress_phase:
                self._inject("vr", self.rf[i], self.b_r, i, j, k, a)
            elif kind == "force_z" and not stress_phase:
                self._inject("vz", self.rc[i], self.b_z, i, j, k, a)

    def _sample(self, rec):
        kind, field, i, j, k = rec
        sl = slice(None) if j < 0 else slice(j, j + 1)
        if kind == "pressure":
            t = self.f["srr"][i][sl, k] + self.f["stt"][i][sl, k] + self.f["szz"][i][sl, k]
            return -float(t.sum()) / (3.0 * t.size)
        v = self.f[field][i][sl, k]
        return float(v.sum()) / v.size

    def _energy(self, sold):
        """E^{n+1/2}, as in the uniform scheme, each ring with its own dtheta."""
        E = 0.0
        f = self.f
        for i in range(self.nr):
            ri, Ri, w = self.rc[i], self.rf[i], self.dr * self.dth[i] * self.dz
            e = 0.5 * Ri * f["vr"][i] ** 2 / self.b_r[i]
            e += 0.5 * ri * f["vt"][i] ** 2 / self.b_t[i]
            e += 0.5 * ri * f["vz"][i] ** 2 / self.b_z[i]
            K = self.lam[i] + 2.0 * self.mu[i] / 3.0
            n1 = [f["srr"][i], f["stt"][i], f["szz"][i]]
            n0 = [sold["srr"][i], sold["stt"][i], sold["szz"][i]]
            t1, t0 = n1[0] + n1[1] + n1[2], n0[0] + n0[1] + n0[2]
            e = e + 0.5 * ri * t1 * t0 / (9.0 * K)
            mu = self.mu[i]
            dev = sum((n1[c] - t1 / 3.0) * (n0[c] - t0 / 3.0) for c in range(3))
            e = e + np.where(mu > 0, 0.5 * ri * dev / np.where(mu > 0, 2.0 * mu, 1.0), 0.0)
            for name, m, rad in (("srt", self.mu_rt[i], Ri), ("srz", self.mu_rz[i], Ri), ("stz", self.mu_tz[i], ri)):
                e = e + np.where(m > 0, 0.5 * rad * f[name][i] * sold[name][i] / np.where(m > 0, m, 1.0), 0.0)
            E += float(e.sum()) * w
        return E

    def run(self, nsteps: int, energy: bool = False):
        """Advance nsteps (velocity, force sources, stress, stress sources,
        receivers); returns traces [nrec][nsteps] (and E^{n+1/2} [nsteps])."""
        if not self.dt > 0:
            raise ValueError("set_dt first")
        tr = np.zeros((len(self.rec), nsteps))
        en = np.zeros(nsteps) if energy else None
        for t in range(nsteps):
            n = self.nstep
            self._velocity()
            self._sources(n, False)
            sold = {name: [a.copy() for a in self.f[name]] for name in ("srr", "stt", "szz", "srt", "srz", "stz")} \
                if energy else None
            self._stress()
            self._sources(n, True)
            for m, rec in enumerate(self.rec):
                tr[m, t] = self._sample(rec)
            if energy:
                en[t] = self._energy(sold)
            self.nstep += 1
        return (tr, en) if energy else tr

    def field(self, name: str) -> np.ndarray:
        """Rings concatenated: ring i contributes ntheta_i x nz values."""
        return np.concatenate([a.reshape(-1) for a in self.f[name]])

    def set_field(self, name: str, data):
        data = np.asarray(data, dtype=float).reshape(-1)
        if data.size != self.cells:
            raise ValueError("expected %d values" % self.cells)
        off = 0
        for i in range(self.nr):
            n = self.nt[i] * self.nz
            self.f[name][i] = data[off:off + n].reshape(self.nt[i], self.nz).copy()
            off += n

    def ring(self, name: str, i: int) -> np.ndarray:
        return self.f[name][i]

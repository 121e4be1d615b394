"""FP64 CPU oracle of the cased-well time step (arXiv 2302.13907).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's CPU
baseline leg may import this package; the product package never does.  The
arithmetic lives in ``cwell_oracle.c`` (plain C loops, FP64, no fused
multiply-add contraction); this module compiles it with gcc and wraps it with
ctypes.  It shares no code with the HIP path.

Parity status of every function is listed in ``ORACLE_PINS`` below, together
with the test that pins it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cwell_oracle.c")
_LIB = os.path.join(_HERE, "libcwell_oracle.so")

FIELDS = ("vr", "vt", "vz", "srr", "stt", "szz", "srt", "srz", "stz")
SRC_KINDS = {"volume": 0, "force_r": 1, "force_z": 2, "torsion": 3}
REC_KINDS = {"pressure": 0, "field": 1}

# Which check pins which part of the oracle (test file :: test name).
ORACLE_PINS = {
    "velocity/strain operators vs the matrices A, B, C, D of Eq. (1)":
        "tests/test_oracle_pins.py::test_operators_match_paper_matrices",
    "discrete skew-adjointness (stencil indices, weights, axis and edge closure)":
        "tests/test_oracle_pins.py::test_operators_skew_adjoint",
    "leapfrog ordering + material averaging: energy conservation":
        "tests/test_oracle_pins.py::test_energy_conserved",
    "staggered material averages (face buoyancy, harmonic edge shear modulus, clamp and wrap): hand-derived values":
        "tests/test_oracle_averages.py::test_coefficient_tables_match_hand_values",
    "the step applies those averages: one-step impulse responses against the hand-derived values":
        "tests/test_oracle_averages.py::test_step_applies_hand_values",
    "theta stencils and periodic wrap: axisymmetric invariance":
        "tests/test_oracle_pins.py::test_theta_invariance_bitwise",
    "P-SV / SH decoupling of axisymmetric sources":
        "tests/test_oracle_pins.py::test_decoupling",
    "source/receiver normalisation and timing: reciprocity":
        "tests/test_oracle_pins.py::test_reciprocity",
    "point source in a homogeneous fluid: closed form, 2nd order":
        "tests/test_oracle_pins.py::test_point_source_closed_form",
    "z stencils, leapfrog order, ring-source volume, pressure receiver: rigid pipe against the 1-D staggered scheme":
        "tests/test_oracle_rigid_pipe.py::test_rigid_pipe_plane_wave_matches_1d_scheme",
    "plane wave in a rigid pipe travels at the fluid speed":
        "tests/test_oracle_rigid_pipe.py::test_rigid_pipe_plane_wave_travels_at_the_fluid_speed",
    "fluid-solid coupling: low-frequency tube-wave speed":
        "tests/test_oracle_physics.py::test_tube_wave_speed",
    "shear stencils, zero shear at fluid contacts: torsional casing wave":
        "tests/test_oracle_physics.py::test_torsion_wave_in_casing",
    "absorbing layer: reflection bound":
        "tests/test_oracle_physics.py::test_pml_reflection_bound",
    "Courant limit: stability margin by power iteration":
        "tests/test_oracle_pins.py::test_cfl_margin",
    "Courant limit: sufficient and nearly sharp where the axis ring's azimuthal width dominates":
        "tests/test_oracle_pins.py::test_cfl_margin_near_axis",
    "pins reject planted mistakes (signs, terms, indices, operands, radii, normalisations)":
        "tests/test_oracle_mutants.py::test_pins_reject_mutant",
    "Ricker pulse of Sec. 2: zeros, extrema, zero mean, spectral peak":
        "tests/test_oracle_pins.py::test_ricker_properties",
    "adjoint step (orc_adjoint_step): exact transpose of the step, layer included":
        "tests/test_oracle_adjoint.py::test_adjoint_step_is_the_transpose",
    "gradient of the receiver loss in the cement moduli (orc_gradient)":
        "tests/test_oracle_adjoint.py::test_gradient_matches_finite_differences",
    "refined grid (refined.py): Fourier interpolation exact on band-limited functions":
        "tests/test_oracle_refined.py::test_interpolation_exact_on_band_limited_functions",
    "refined grid: fine-to-coarse map is the weighted transpose of the interpolation":
        "tests/test_oracle_refined.py::test_restriction_is_half_the_transpose",
    "refined grid: one zone equals the uniform C oracle (independent implementation)":
        "tests/test_oracle_refined.py::test_single_zone_matches_uniform_oracle",
    "refined grid: energy conservation across zone interfaces":
        "tests/test_oracle_refined.py::test_energy_conserved_across_zones",
    "refined grid: axisymmetric solution equals the one-cell uniform grid":
        "tests/test_oracle_refined.py::test_axisymmetric_solution_is_that_of_the_uniform_grid",
    "refined grid: every field crosses an interface at its own azimuthal nodes":
        "tests/test_oracle_refined.py::test_interface_maps_each_field_on_its_own_nodes",
    "refined grid: pins reject planted mistakes in the interpolation":
        "tests/test_oracle_mutants.py::test_refined_pins_reject_mutant",
    "refined grid: order-one wave follows the fine uniform grid":
        "tests/test_oracle_refined.py::test_order_one_wave_close_to_the_fine_uniform_grid",
}


def build(force: bool = False) -> str:
    """Compile the oracle shared library with gcc (FP64, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        D = ctypes.POINTER(ctypes.c_double)
        I = ctypes.c_int
        L = ctypes.c_long
        lib.orc_create.restype = P
        lib.orc_create.argtypes = [I, I, I, ctypes.c_double, ctypes.c_double]
        lib.orc_free.argtypes = [P]
        lib.orc_set_material.argtypes = [P, D, D, D]
        lib.orc_cfl_dt.restype = ctypes.c_double
        lib.orc_cfl_dt.argtypes = [P]
        lib.orc_vpmax.restype = ctypes.c_double
        lib.orc_vpmax.argtypes = [P]
        lib.orc_ricker.restype = ctypes.c_double
        lib.orc_ricker.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.orc_set_pml.argtypes = [P, I, I, ctypes.c_double, ctypes.c_double]
        lib.orc_set_dt.argtypes = [P, ctypes.c_double]
        lib.orc_add_source.argtypes = [P, I, I, I, I, D, L]
        lib.orc_add_receiver.argtypes = [P, I, I, I, I, I]
        lib.orc_run.argtypes = [P, L, D, D]
        lib.orc_get_field.argtypes = [P, I, D]
        lib.orc_set_field.argtypes = [P, I, D]
        lib.orc_get_coef.argtypes = [P, I, D]
        lib.orc_threads.restype = I
        lib.orc_threads.argtypes = []
        lib.orc_steps_done.restype = L
        lib.orc_steps_done.argtypes = [P]
        lib.orc_get_dt.restype = ctypes.c_double
        lib.orc_get_dt.argtypes = [P]
        lib.orc_apply_div.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(D)]
        lib.orc_apply_strain.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(D)]
        lib.orc_step_linear.argtypes = [P]
        lib.orc_adjoint_step.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(D)]
        lib.orc_get_psi.argtypes = [P, I, D]
        lib.orc_set_psi.argtypes = [P, I, D]
        lib.orc_gradient.argtypes = [P, L, L, L, I, I, I, I, I, D, D, D]
        _lib = lib
    return _lib


def threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(_load().orc_threads())


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def ricker(f0: float, t) -> np.ndarray:
    """Ricker pulse of Sec. 2 (delay 2/f0) sampled at times t, via the C oracle."""
    lib = _load()
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    return np.array([lib.orc_ricker(float(f0), float(x)) for x in t])


class OracleSim:
    """One FP64 simulation.  Arrays are C-order [nr][ntheta][nz] float64."""

    def __init__(self, nr: int, ntheta: int, nz: int, dr: float, dz: float):
        self.lib = _load()
        self.shape = (nr, ntheta, nz)
        self.dr, self.dz = float(dr), float(dz)
        self.h = self.lib.orc_create(nr, ntheta, nz, self.dr, self.dz)
        if not self.h:
            raise ValueError("bad grid")
        self.nrec = 0
        self._keep = []

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_free(h)
            self.h = None

    def _arr(self, a) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.float64)
        if a.shape != self.shape:
            a = np.ascontiguousarray(np.broadcast_to(a, self.shape), dtype=np.float64)
        return a

    def set_material(self, rho, lam, mu):
        r, l, m = self._arr(rho), self._arr(lam), self._arr(mu)
        rc = self.lib.orc_set_material(self.h, _dp(r), _dp(l), _dp(m))
        if rc:
            raise ValueError("material rejected (%d)" % rc)

    def cfl_dt(self) -> float:
        return self.lib.orc_cfl_dt(self.h)

    def vp_max(self) -> float:
        return self.lib.orc_vpmax(self.h)

    def set_pml(self, npml_r: int, npml_z: int, rc: float = 1e-3, alpha: float = 0.0):
        if self.lib.orc_set_pml(self.h, npml_r, npml_z, rc, alpha):
            raise ValueError("bad layer")

    def set_dt(self, dt: float):
        if self.lib.orc_set_dt(self.h, dt):
            raise ValueError("set_dt failed")

    @property
    def dt(self) -> float:
        return self.lib.orc_get_dt(self.h)

    def add_source(self, kind: str, i: int, j: int, k: int, w: Sequence[float]):
        w = np.ascontiguousarray(w, dtype=np.float64)
        rc = self.lib.orc_add_source(self.h, SRC_KINDS[kind], i, j, k, _dp(w), len(w))
        if rc:
            raise ValueError("bad source (%d)" % rc)

    def add_receiver(self, kind: str, i: int, j: int, k: int, field: Optional[str] = None) -> int:
        fid = FIELDS.index(field) if field else 0
        rc = self.lib.orc_add_receiver(self.h, REC_KINDS[kind], fid, i, j, k)
        if rc < 0:
            raise ValueError("bad receiver (%d)" % rc)
        self.nrec += 1
        return rc

    def run(self, nsteps: int, energy: bool = False):
        """Advance nsteps; returns traces [nrec][nsteps] (and energy [nsteps])."""
        tr = np.zeros((max(self.nrec, 1), nsteps))
        en = np.zeros(nsteps) if energy else None
        self.lib.orc_run(self.h, nsteps, _dp(tr), _dp(en) if en is not None else None)
        tr = tr[: self.nrec]
        return (tr, en) if energy else tr

    def field(self, name: str) -> np.ndarray:
        out = np.empty(self.shape)
        self.lib.orc_get_field(self.h, FIELDS.index(name), _dp(out))
        return out

    def set_field(self, name: str, a):
        a = self._arr(a)
        self.lib.orc_set_field(self.h, FIELDS.index(name), _dp(a))

    def coef(self, name: str) -> np.ndarray:
        names = ("b_r", "b_t", "b_z", "mu_rt", "mu_rz", "mu_tz")
        out = np.empty(self.shape)
        self.lib.orc_get_coef(self.h, names.index(name), _dp(out))
        return out

    @property
    def steps_done(self) -> int:
        return self.lib.orc_steps_done(self.h)

    def apply_div(self, sig):
        """Velocity right-hand sides (no density) of stresses sig = (srr, stt, szz, srt, srz, stz)."""
        sig = [self._arr(a) for a in sig]
        out = [np.zeros(self.shape) for _ in range(3)]
        S = (ctypes.POINTER(ctypes.c_double) * 6)(*[_dp(a) for a in sig])
        O = (ctypes.POINTER(ctypes.c_double) * 3)(*[_dp(a) for a in out])
        self.lib.orc_apply_div(self.h, S, O)
        return out

    NPSI = 18

    def psi(self, q: int) -> np.ndarray:
        """Layer memory variable q (0..17; requires the layer on)."""
        out = np.empty(self.shape)
        if self.lib.orc_get_psi(self.h, q, _dp(out)):
            raise ValueError("no layer memory")
        return out

    def set_psi(self, q: int, a):
        a = self._arr(a)
        if self.lib.orc_set_psi(self.h, q, _dp(a)):
            raise ValueError("no layer memory")

    def step_linear(self):
        """One step of the current state without sources."""
        self.lib.orc_step_linear(self.h)

    def adjoint_step(self, fb: dict, pb=None):
        """Apply the transposed step in place: fb maps field name -> adjoint
        array, pb lists the 18 layer-memory adjoints (layer on)."""
        arrs = [np.ascontiguousarray(fb[n], dtype=np.float64) for n in FIELDS]
        for n, a in zip(FIELDS, arrs):
            fb[n] = a
        F = (ctypes.POINTER(ctypes.c_double) * 9)(*[_dp(a) for a in arrs])
        if pb is not None:
            for q in range(self.NPSI):
                pb[q] = np.ascontiguousarray(pb[q], dtype=np.float64)
            Pp = (ctypes.POINTER(ctypes.c_double) * self.NPSI)(*[_dp(a) for a in pb])
        else:
            dummy = np.zeros(1)
            Pp = (ctypes.POINTER(ctypes.c_double) * self.NPSI)(*[_dp(dummy)] * self.NPSI)
        self.lib.orc_adjoint_step(self.h, F, Pp)
        return fb, pb

    def gradient(self, nsteps: int, window, region):
        """Loss sum over steps n in window [n0, n1) and pressure receivers of
        p(t_{n+1})^2, and its gradient with respect to (mu, K) of the bins of
        region = (i0, i1, k0, nbins, bin_rows); runs the forward from the
        zero state and the adjoint back.  Returns (loss, dL/dmu, dL/dK)."""
        i0, i1, k0, nb, br = region
        gm, gk = np.zeros(nb), np.zeros(nb)
        loss = ctypes.c_double()
        rc = self.lib.orc_gradient(self.h, nsteps, window[0], window[1], i0, i1, k0, nb, br,
                                   ctypes.byref(loss), _dp(gm), _dp(gk))
        if rc:
            raise ValueError("gradient rejected (%d)" % rc)
        return loss.value, gm, gk

    def apply_strain(self, vel):
        """Strain rates (e_rr, e_tt, e_zz, g_rt, g_rz, g_tz) of vel = (vr, vt, vz)."""
        vel = [self._arr(a) for a in vel]
        out = [np.zeros(self.shape) for _ in range(6)]
        V = (ctypes.POINTER(ctypes.c_double) * 3)(*[_dp(a) for a in vel])
        O = (ctypes.POINTER(ctypes.c_double) * 6)(*[_dp(a) for a in out])
        self.lib.orc_apply_strain(self.h, V, O)
        return out

"""Shared helpers of the GPU tests: run one scenario through the HIP path
(via the C ABI) and through the FP64 oracle on the same seeded inputs."""
from __future__ import annotations

import math
import sys
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

import oracle
from paper_2302_13907_amd import cwell, inputs

FIELDS = cwell.FIELDS
VEL = ("vr", "vt", "vz")
STRESS = ("srr", "stt", "szz", "srt", "srz", "stz")


@dataclass
class Scenario:
    shape: Tuple[int, int, int]
    h: Tuple[float, float]
    medium: tuple
    steps: int
    npml: Tuple[int, int] = (0, 0)
    f0: float = 20e3
    cfl_fraction: float = 0.5
    sources: List[tuple] = field(default_factory=list)     # (kind, i, j, k, amplitude)
    receivers: List[tuple] = field(default_factory=list)   # (kind, i, j, k, field)
    initial: Optional[dict] = None                          # field -> array
    path: str = "auto"                                      # kernel path of cw_step
    storage: str = "f32"                                    # field storage on the device


def announce(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def _times(kind, n, dt):
    # stress sources act at t_{n+1/2}, force sources at t_n
    off = 0.0 if kind in ("force_r", "force_z") else 0.5
    return (np.arange(n) + off) * dt


def make_sim(sc: Scenario):
    """A bound simulation of scenario sc (not yet stepped; sources cover sc.steps)."""
    s = cwell.Sim(*sc.shape, *sc.h)
    s.set_material(*sc.medium)
    if sc.npml != (0, 0):
        s.set_pml(sc.npml[0], sc.npml[1], 1e-3, math.pi * sc.f0)
    dt = sc.cfl_fraction * s.cfl_dt()
    s.set_dt(dt)
    for (kind, i, j, k, amp) in sc.sources:
        s.add_source(kind, i, j, k, amp * cwell.ricker(sc.f0, _times(kind, sc.steps, dt)))
    for (kind, i, j, k, fld) in sc.receivers:
        s.add_receiver(kind, i, j, k, fld)
    s.set_trace_capacity(sc.steps)
    s.set_path(sc.path)
    s.set_storage(sc.storage)
    s.bind()
    if sc.initial:
        for name, a in sc.initial.items():
            s.set_field(name, a)
    return s


def run_gpu(sc: Scenario, keep_sim: bool = False):
    s = make_sim(sc)
    s.step(sc.steps)
    s.sync()
    tr = s.traces()
    fields = {name: s.field(name) for name in FIELDS}
    if keep_sim:
        return tr, fields, s
    s.close()
    return tr, fields


def run_oracle(sc: Scenario):
    o = oracle.OracleSim(*sc.shape, *sc.h)
    o.set_material(*sc.medium)
    if sc.npml != (0, 0):
        o.set_pml(sc.npml[0], sc.npml[1], 1e-3, math.pi * sc.f0)
    dt = sc.cfl_fraction * o.cfl_dt()
    o.set_dt(dt)
    for (kind, i, j, k, amp) in sc.sources:
        o.add_source(kind, i, j, k, amp * oracle.ricker(sc.f0, _times(kind, sc.steps, dt)))
    for (kind, i, j, k, fld) in sc.receivers:
        o.add_receiver(kind, i, j, k, fld)
    if sc.initial:
        for name, a in sc.initial.items():
            o.set_field(name, a)
    tr = o.run(sc.steps)
    fields = {name: o.field(name) for name in FIELDS}
    return tr, fields


def rel_l2(a, b) -> float:
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def field_errors(got: dict, ref: dict) -> dict:
    """Per-field RMS error divided by the RMS of the field's group
    (velocities, stresses): shear stresses may be tiny or zero."""
    out = {}
    for group in (VEL, STRESS):
        scale = math.sqrt(sum(float((ref[n] ** 2).sum()) for n in group) / len(group))
        for n in group:
            d = got[n].astype(np.float64) - ref[n]
            out[n] = float(np.linalg.norm(d) / scale) if scale > 0 else float(np.linalg.norm(d))
    return out


def field_max_errors(got: dict, ref: dict) -> dict:
    """Per-field largest |gpu - oracle| over every cell, divided by the
    largest |value| of the field's group (velocities, stresses) in the
    oracle.  A group the oracle holds at exactly zero everywhere gives inf
    unless the device holds it at exactly zero too (then 0)."""
    out = {}
    for group in (VEL, STRESS):
        scale = max(float(np.abs(ref[n]).max()) for n in group)
        for n in group:
            d = float(np.abs(got[n].astype(np.float64) - ref[n]).max())
            out[n] = d / scale if scale > 0 else (0.0 if d == 0 else math.inf)
    return out


def check_fields(got: dict, ref: dict, tol: float, tag: str = ""):
    """Fields within tol of the oracle twice over: the per-field RMS error
    over the group's RMS (field_errors), and cell by cell against the group's
    largest magnitude (field_max_errors), so a wrong value in one corner of
    the layer or one axis cell cannot hide in a norm."""
    fe = field_errors(got, ref)
    fm = field_max_errors(got, ref)
    announce("  %sfield errors: rms worst %.2e (%s), per cell worst %.2e (%s)"
             % (tag, max(fe.values()), max(fe, key=fe.get), max(fm.values()), max(fm, key=fm.get)))
    assert max(fe.values()) <= tol, fe
    assert max(fm.values()) <= tol, fm


def parity_scenario() -> Scenario:
    w = inputs.parity_case()
    return Scenario(shape=(w.nr, w.nt, w.nz), h=(w.dr, w.dz), medium=w.medium(), steps=w.steps,
                    npml=(w.npml, w.npml), f0=w.f0,
                    sources=[("volume", 0, -1, w.src_k, 1.0)],
                    receivers=[("pressure", 0, -1, k, None) for k in w.rec_k])

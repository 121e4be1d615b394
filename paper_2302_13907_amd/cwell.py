"""Thin Python binding of libcwell (the C ABI declared in include/cwell.h).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  PyTorch supplies the device workspace and the stream.  The
library must have been built (``python -m paper_2302_13907_amd.build`` or
``__graft_entry__.build()``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcwell.so")

FIELDS = ("vr", "vt", "vz", "srr", "stt", "szz", "srt", "srz", "stz")
SRC_KINDS = {"volume": 0, "force_r": 1, "force_z": 2, "torsion": 3}
REC_KINDS = {"pressure": 0, "field": 1}

CW_OK = 0
STATUS = {0: "CW_OK", -1: "CW_ERR_ARG", -2: "CW_ERR_RANGE", -3: "CW_ERR_MATERIAL",
          -4: "CW_ERR_UNSTABLE", -5: "CW_ERR_STATE", -6: "CW_ERR_NONFINITE",
          -7: "CW_ERR_HIP", -8: "CW_ERR_NOMEM"}

# every symbol include/cwell.h declares
EXPORTS = ("cw_create", "cw_set_material", "cw_set_material_rz", "cw_set_pml", "cw_cfl_dt",
           "cw_set_dt", "cw_add_source", "cw_add_receiver", "cw_set_trace_capacity",
           "cw_workspace_bytes", "cw_bind", "cw_step", "cw_sync", "cw_get_traces",
           "cw_get_field", "cw_set_field", "cw_energy", "cw_reset", "cw_steps_done",
           "cw_ricker", "cw_destroy", "cw_last_error", "cw_profile", "cw_profile_read",
           "cw_set_path", "cw_set_storage", "cw_set_rounding", "cw_stream_probe", "cw_set_graph", "cw_set_adjoint",
           "cw_set_region_moduli", "cw_gradient", "cw_batch_create", "cw_batch_set_tile",
           "cw_batch_workspace_bytes", "cw_batch_bind", "cw_batch_set_occupancy", "cw_batch_set_graph", "cw_batch_step", "cw_batch_destroy",
           "cw_refined_create", "cw_refined_cells", "cw_refined_set_material_rz", "cw_refined_set_pml",
           "cw_refined_cfl_dt", "cw_refined_set_dt", "cw_refined_add_source", "cw_refined_add_receiver",
           "cw_refined_set_trace_capacity", "cw_refined_workspace_bytes", "cw_refined_bind", "cw_refined_step",
           "cw_refined_get_field", "cw_refined_set_field", "cw_refined_get_traces", "cw_refined_energy",
           "cw_refined_reset", "cw_refined_destroy", "cw_energy_noalloc")

STORAGE = {"f32": 0, "f16": 1, "bf16": 2}

PATHS = {"auto": 0, "two-pass": 1, "fused": 2}
ROUNDING = {"nearest": 0, "stochastic": 1}

KERNELS = {"velocity": 0, "stress": 1, "fused": 2, "inject": 3, "record": 4}


def _pick(table, key, what: str) -> int:
    """The C enum value of a named choice; ValueError naming the choices."""
    if isinstance(table, dict):
        if key in table:
            return table[key]
        names = list(table)
    else:
        if key in table:
            return table.index(key)
        names = list(table)
    raise ValueError("unknown %s %r (one of %s)" % (what, key, ", ".join(map(str, names))))


class CwellError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class _Grid(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_int32), ("ntheta", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dr", ctypes.c_double), ("dz", ctypes.c_double)]


_lib = None


def load():
    """Load libcwell.so (after torch, so both share torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  -- the HIP runtime the library binds to
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libcwell.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    DP = ctypes.POINTER(ctypes.c_double)
    FP = ctypes.POINTER(ctypes.c_float)
    sig = {
        "cw_create": [ctypes.POINTER(_Grid), ctypes.POINTER(P)],
        "cw_set_material": [P, DP, DP, DP],
        "cw_set_material_rz": [P, DP, DP, DP],
        "cw_set_pml": [P, I32, I32, D, D],
        "cw_cfl_dt": [P, DP],
        "cw_set_dt": [P, D],
        "cw_add_source": [P, I32, I32, I32, I32, DP, I64],
        "cw_add_receiver": [P, I32, I32, I32, I32, I32, ctypes.POINTER(I32)],
        "cw_set_trace_capacity": [P, I64],
        "cw_workspace_bytes": [P, ctypes.POINTER(ctypes.c_uint64)],
        "cw_bind": [P, P, ctypes.c_uint64, P],
        "cw_step": [P, I64],
        "cw_sync": [P],
        "cw_get_traces": [P, DP, I64, ctypes.POINTER(I64)],
        "cw_get_field": [P, I32, FP],
        "cw_set_field": [P, I32, FP],
        "cw_energy": [P, DP],
        "cw_energy_noalloc": [P, I32, DP],
        "cw_reset": [P],
        "cw_steps_done": [P, ctypes.POINTER(I64)],
        "cw_ricker": [D, DP, I64, DP],
        "cw_profile": [P, I32],
        "cw_set_path": [P, I32],
        "cw_set_rounding": [P, I32],
        "cw_set_storage": [P, I32],
        "cw_profile_read": [P, I32, DP, ctypes.POINTER(I64)],
        "cw_stream_probe": [P, ctypes.c_uint64, I32, I32, I32, I32, P, DP],
        "cw_set_graph": [P, I32],
        "cw_set_adjoint": [P, I64, I32, I32, I32, I32, I32, I32],
        "cw_set_region_moduli": [P, DP, DP],
        "cw_gradient": [P, I64, I64, DP, DP, DP],
        "cw_batch_create": [ctypes.POINTER(P), I32, ctypes.POINTER(P)],
        "cw_batch_set_tile": [P, I32, I32],
        "cw_batch_set_occupancy": [P, I32],
        "cw_batch_workspace_bytes": [P, ctypes.POINTER(ctypes.c_uint64)],
        "cw_batch_bind": [P, P, ctypes.c_uint64],
        "cw_batch_set_graph": [P, I32],
        "cw_batch_step": [P, I64],
        "cw_refined_create": [ctypes.POINTER(_Grid), I32, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(P)],
        "cw_refined_cells": [P, ctypes.POINTER(ctypes.c_uint64)],
        "cw_refined_set_material_rz": [P, DP, DP, DP],
        "cw_refined_set_pml": [P, I32, I32, D, D],
        "cw_refined_cfl_dt": [P, DP],
        "cw_refined_set_dt": [P, D],
        "cw_refined_add_source": [P, I32, I32, I32, I32, DP, I64],
        "cw_refined_add_receiver": [P, I32, I32, I32, I32, I32, ctypes.POINTER(I32)],
        "cw_refined_set_trace_capacity": [P, I64],
        "cw_refined_workspace_bytes": [P, ctypes.POINTER(ctypes.c_uint64)],
        "cw_refined_bind": [P, P, ctypes.c_uint64, P],
        "cw_refined_step": [P, I64],
        "cw_refined_get_field": [P, I32, FP],
        "cw_refined_set_field": [P, I32, FP],
        "cw_refined_get_traces": [P, DP, I64, ctypes.POINTER(I64)],
        "cw_refined_energy": [P, DP],
        "cw_refined_reset": [P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int32
    lib.cw_destroy.argtypes = [P]
    lib.cw_destroy.restype = None
    lib.cw_refined_destroy.argtypes = [P]
    lib.cw_refined_destroy.restype = None
    lib.cw_batch_destroy.argtypes = [P]
    lib.cw_batch_destroy.restype = None
    lib.cw_last_error.argtypes = []
    lib.cw_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(st: int):
    if st != CW_OK:
        raise CwellError(st, load().cw_last_error().decode())


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def ricker(f0: float, t) -> np.ndarray:
    """Ricker pulse of Sec. 2 (delay 2/f0) at times t, computed by libcwell."""
    t = np.ascontiguousarray(np.atleast_1d(t), dtype=np.float64)
    out = np.empty_like(t)
    _check(load().cw_ricker(float(f0), _dp(t), len(t), _dp(out)))
    return out


PROBE_NONTEMPORAL = 0x100       # CW_PROBE_NONTEMPORAL


def stream_probe(nread: int, nwrite: int, bytes_per_array: int = 1 << 30, reps: int = 10,
                 device: str = "cuda", lane_bytes: int = 16, nontemporal: bool = False) -> float:
    """Achieved bytes per second of a kernel that only streams nread arrays
    in and nwrite arrays out (the access pattern of a step kernel without
    its stencil), lane_bytes (16 or 4) per thread and array, on a
    torch-allocated buffer on the current stream; nontemporal: every load
    and store non-temporal."""
    import torch
    lib = load()
    n = nread + nwrite
    buf = torch.empty(n * bytes_per_array + 256, dtype=torch.uint8, device=device)
    ptr = buf.data_ptr()
    ptr += (-ptr) % 256
    buf[:].zero_()
    stream = torch.cuda.current_stream(buf.device).cuda_stream
    ms = ctypes.c_double()
    _check(lib.cw_stream_probe(ctypes.c_void_p(ptr), int(bytes_per_array), int(nread), int(nwrite),
                               int(lane_bytes) | (PROBE_NONTEMPORAL if nontemporal else 0), int(reps),
                               ctypes.c_void_p(stream), ctypes.byref(ms)))
    del buf
    return n * bytes_per_array / (ms.value * 1e-3)


class Sim:
    """One simulation on one GPU.  Arrays are C order [nr][ntheta][nz]."""

    def __init__(self, nr: int, ntheta: int, nz: int, dr: float, dz: float):
        self.lib = load()
        self.shape = (int(nr), int(ntheta), int(nz))
        self.dr, self.dz = float(dr), float(dz)
        self._nbins = 0
        g = _Grid(int(nr), int(ntheta), int(nz), float(dr), float(dz))
        h = ctypes.c_void_p()
        _check(self.lib.cw_create(ctypes.byref(g), ctypes.byref(h)))
        self.h = h
        self.nrec = 0
        self.workspace = None

    def close(self):
        if getattr(self, "h", None):
            self.lib.cw_destroy(self.h)
            self.h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_material(self, rho, lam, mu):
        """3-D arrays [nr][nt][nz], or axisymmetric [nr][nz] ones."""
        arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (rho, lam, mu)]
        if arrs[0].shape == (self.shape[0], self.shape[2]):
            for a in arrs:
                if a.shape != arrs[0].shape:
                    raise ValueError("medium arrays differ in shape")
            _check(self.lib.cw_set_material_rz(self.h, *[_dp(a) for a in arrs]))
            return
        arrs = [np.ascontiguousarray(np.broadcast_to(a, self.shape), dtype=np.float64) for a in arrs]
        _check(self.lib.cw_set_material(self.h, *[_dp(a) for a in arrs]))

    def set_pml(self, npml_r: int, npml_z: int, rc: float = 1e-3, alpha: float = 0.0):
        _check(self.lib.cw_set_pml(self.h, int(npml_r), int(npml_z), float(rc), float(alpha)))

    def cfl_dt(self) -> float:
        v = ctypes.c_double()
        _check(self.lib.cw_cfl_dt(self.h, ctypes.byref(v)))
        return v.value

    def set_dt(self, dt: float):
        _check(self.lib.cw_set_dt(self.h, float(dt)))
        self.dt = float(dt)

    def add_source(self, kind: str, i: int, j: int, k: int, w: Sequence[float]):
        w = np.ascontiguousarray(w, dtype=np.float64)
        _check(self.lib.cw_add_source(self.h, _pick(SRC_KINDS, kind, "source kind"), i, j, k, _dp(w), len(w)))

    def add_receiver(self, kind: str, i: int, j: int, k: int, field: Optional[str] = None) -> int:
        rid = ctypes.c_int32()
        fid = _pick(FIELDS, field, "field") if field else 0
        _check(self.lib.cw_add_receiver(self.h, _pick(REC_KINDS, kind, "receiver kind"), fid, i, j, k, ctypes.byref(rid)))
        self.nrec += 1
        return rid.value

    def set_trace_capacity(self, nsteps: int):
        _check(self.lib.cw_set_trace_capacity(self.h, int(nsteps)))
        self.trace_cap = int(nsteps)

    def workspace_bytes(self) -> int:
        b = ctypes.c_uint64()
        _check(self.lib.cw_workspace_bytes(self.h, ctypes.byref(b)))
        return b.value

    def bind(self, device: str = "cuda", stream=None):
        """Allocate the device workspace with torch and hand it to the library."""
        import torch
        nbytes = self.workspace_bytes()
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        ptr = ws.data_ptr()
        off = (-ptr) % 256
        if stream is None:
            stream = torch.cuda.current_stream(ws.device)
        self.stream = stream
        self.workspace = ws
        _check(self.lib.cw_bind(self.h, ctypes.c_void_p(ptr + off), nbytes,
                                ctypes.c_void_p(stream.cuda_stream)))

    def step(self, nsteps: int = 1):
        _check(self.lib.cw_step(self.h, int(nsteps)))

    def sync(self):
        _check(self.lib.cw_sync(self.h))

    @property
    def steps_done(self) -> int:
        n = ctypes.c_int64()
        _check(self.lib.cw_steps_done(self.h, ctypes.byref(n)))
        return n.value

    def traces(self) -> np.ndarray:
        n = self.steps_done
        out = np.zeros((max(self.nrec, 1), max(n, 1)))
        done = ctypes.c_int64()
        _check(self.lib.cw_get_traces(self.h, _dp(out), out.shape[1], ctypes.byref(done)))
        return out[: self.nrec, : done.value]

    def field(self, name: str) -> np.ndarray:
        out = np.empty(self.shape, dtype=np.float32)
        _check(self.lib.cw_get_field(self.h, _pick(FIELDS, name, "field"), _fp(out)))
        return out

    def set_field(self, name: str, a):
        a = np.ascontiguousarray(np.broadcast_to(a, self.shape), dtype=np.float32)
        _check(self.lib.cw_set_field(self.h, _pick(FIELDS, name, "field"), _fp(a)))

    def energy(self) -> float:
        e = ctypes.c_double()
        _check(self.lib.cw_energy(self.h, ctypes.byref(e)))
        return e.value

    def energy_noalloc(self, nblocks: int = 1024) -> float:
        """cw_energy_noalloc: the energy with its partial sums in the
        library's static scratch (no device memory allocated)."""
        e = ctypes.c_double()
        _check(self.lib.cw_energy_noalloc(self.h, int(nblocks), ctypes.byref(e)))
        return e.value

    def reset(self):
        _check(self.lib.cw_reset(self.h))

    def set_storage(self, storage: str):
        """Field storage: "f32", "f16" (per-field power-of-two scales) or "bf16"."""
        _check(self.lib.cw_set_storage(self.h, _pick(STORAGE, storage, "storage")))

    def set_rounding(self, mode: str):
        """Rounding of the bfloat16 field stores: "nearest" (default) or "stochastic"."""
        _check(self.lib.cw_set_rounding(self.h, _pick(ROUNDING, mode, "rounding mode")))

    def set_path(self, path: str):
        """Kernel path of step(): "auto", "two-pass" or "fused"."""
        _check(self.lib.cw_set_path(self.h, _pick(PATHS, path, "path")))

    def set_adjoint(self, nsteps: int, checkpoint_every: int, region):
        """Configure the adjoint gradient (before bind): region = (i0, i1, k0,
        nbins, bin_rows); nsteps forward steps, a checkpoint every
        checkpoint_every steps."""
        i0, i1, k0, nb, br = region
        _check(self.lib.cw_set_adjoint(self.h, int(nsteps), int(checkpoint_every), int(i0), int(i1), int(k0),
                                       int(nb), int(br)))
        self._nbins = int(nb)

    def set_region_moduli(self, dmu, dK):
        """Shift the region's bins' mu and K (Pa) from the medium given at set_material."""
        dmu = np.ascontiguousarray(dmu, dtype=np.float64)
        dK = np.ascontiguousarray(dK, dtype=np.float64)
        if dmu.shape != (self._nbins,) or dK.shape != (self._nbins,):
            raise ValueError("one shift per bin")
        _check(self.lib.cw_set_region_moduli(self.h, _dp(dmu), _dp(dK)))

    def gradient(self, window):
        """(loss, dL/dmu per bin, dL/dK per bin) of the loss over steps
        [window[0], window[1]); runs the configured forward and adjoint."""
        gm, gk = np.zeros(self._nbins), np.zeros(self._nbins)
        loss = ctypes.c_double()
        _check(self.lib.cw_gradient(self.h, int(window[0]), int(window[1]), ctypes.byref(loss), _dp(gm), _dp(gk)))
        return loss.value, gm, gk

    def set_graph(self, steps: int):
        """Replay the two-pass step's launches as a HIP graph of `steps`
        (even) steps; 0 switches graph replay off."""
        _check(self.lib.cw_set_graph(self.h, int(steps)))

    def profile(self, enable: bool = True):
        """Start (or stop and clear) per-launch HIP-event timing of the step kernels."""
        _check(self.lib.cw_profile(self.h, 1 if enable else 0))

    def kernel_time(self, kernel: str):
        """(summed device milliseconds, launches) recorded for one step kernel."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(self.lib.cw_profile_read(self.h, _pick(KERNELS, kernel, "kernel"), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


class Batch:
    """Simulations advanced together by batched launches (see cw_batch_* in
    include/cwell.h).  The simulations must be bound (on one stream) first."""

    def __init__(self, sims):
        self.lib = load()
        self.sims = list(sims)
        arr = (ctypes.c_void_p * len(self.sims))(*[s.h for s in self.sims])
        h = ctypes.c_void_p()
        _check(self.lib.cw_batch_create(arr, len(self.sims), ctypes.byref(h)))
        self.h = h
        self._ws = None

    def set_tile(self, index: int, tz_waves: int):
        _check(self.lib.cw_batch_set_tile(self.h, int(index), int(tz_waves)))

    def set_occupancy(self, waves_per_simd: int):
        """Minimum wavefronts per SIMD of the batched kernels: 0 (none), 7 or 8."""
        _check(self.lib.cw_batch_set_occupancy(self.h, int(waves_per_simd)))

    def bind(self):
        import torch
        b = ctypes.c_uint64()
        _check(self.lib.cw_batch_workspace_bytes(self.h, ctypes.byref(b)))
        ws = torch.empty(b.value + 256, dtype=torch.uint8, device=self.sims[0].workspace.device)
        ptr = ws.data_ptr()
        ptr += (-ptr) % 256
        _check(self.lib.cw_batch_bind(self.h, ctypes.c_void_p(ptr), b.value))
        self._ws = ws

    def set_graph(self, steps: int):
        _check(self.lib.cw_batch_set_graph(self.h, int(steps)))

    def step(self, n: int = 1):
        _check(self.lib.cw_batch_step(self.h, int(n)))

    def close(self):
        if self.h:
            self.lib.cw_batch_destroy(self.h)
            self.h = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Refined:
    """An azimuthally refined grid (see cw_refined_* in include/cwell.h):
    zones = [(first_ring, ntheta), ...], ntheta doubling outwards.  Fields
    are exchanged as the rings concatenated (ring i: ntheta_i x nz)."""

    def __init__(self, nr: int, nz: int, dr: float, dz: float, zones):
        self.lib = load()
        self.zones = [(int(a), int(b)) for a, b in zones]
        self.nr, self.nz, self.dr, self.dz = int(nr), int(nz), float(dr), float(dz)
        g = _Grid(self.nr, self.zones[-1][1], self.nz, self.dr, self.dz)
        first = (ctypes.c_int32 * len(self.zones))(*[a for a, _ in self.zones])
        nth = (ctypes.c_int32 * len(self.zones))(*[b for _, b in self.zones])
        h = ctypes.c_void_p()
        _check(self.lib.cw_refined_create(ctypes.byref(g), len(self.zones), first, nth, ctypes.byref(h)))
        self.h = h
        self.nrec = 0
        self.workspace = None
        c = ctypes.c_uint64()
        _check(self.lib.cw_refined_cells(self.h, ctypes.byref(c)))
        self.cells = int(c.value)
        self.ntheta = np.zeros(self.nr, dtype=int)
        for q, (a, n) in enumerate(self.zones):
            b = self.zones[q + 1][0] if q + 1 < len(self.zones) else self.nr
            self.ntheta[a:b] = n

    def close(self):
        if getattr(self, "h", None):
            self.lib.cw_refined_destroy(self.h)
            self.h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_material_rz(self, rho, lam, mu):
        arrs = [np.ascontiguousarray(np.reshape(a, (self.nr, self.nz)), dtype=np.float64) for a in (rho, lam, mu)]
        _check(self.lib.cw_refined_set_material_rz(self.h, *[_dp(a) for a in arrs]))

    def set_pml(self, npml_r: int, npml_z: int, rc: float = 1e-3, alpha: float = 0.0):
        _check(self.lib.cw_refined_set_pml(self.h, int(npml_r), int(npml_z), float(rc), float(alpha)))

    def cfl_dt(self) -> float:
        v = ctypes.c_double()
        _check(self.lib.cw_refined_cfl_dt(self.h, ctypes.byref(v)))
        return v.value

    def set_dt(self, dt: float):
        _check(self.lib.cw_refined_set_dt(self.h, float(dt)))
        self.dt = float(dt)

    def add_source(self, kind: str, i: int, j: int, k: int, w: Sequence[float]):
        w = np.ascontiguousarray(w, dtype=np.float64)
        _check(self.lib.cw_refined_add_source(self.h, _pick(SRC_KINDS, kind, "source kind"), i, j, k, _dp(w), len(w)))

    def add_receiver(self, kind: str, i: int, j: int, k: int, field: Optional[str] = None) -> int:
        rid = ctypes.c_int32()
        fid = _pick(FIELDS, field, "field") if field else 0
        _check(self.lib.cw_refined_add_receiver(self.h, _pick(REC_KINDS, kind, "receiver kind"), fid, i, j, k, ctypes.byref(rid)))
        self.nrec += 1
        return rid.value

    def set_trace_capacity(self, nsteps: int):
        _check(self.lib.cw_refined_set_trace_capacity(self.h, int(nsteps)))
        self.trace_cap = int(nsteps)

    def workspace_bytes(self) -> int:
        b = ctypes.c_uint64()
        _check(self.lib.cw_refined_workspace_bytes(self.h, ctypes.byref(b)))
        return b.value

    def bind(self, device: str = "cuda", stream=None):
        import torch
        nbytes = self.workspace_bytes()
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        ptr = ws.data_ptr()
        off = (-ptr) % 256
        if stream is None:
            stream = torch.cuda.current_stream(ws.device)
        self.stream = stream
        self.workspace = ws
        _check(self.lib.cw_refined_bind(self.h, ctypes.c_void_p(ptr + off), nbytes,
                                        ctypes.c_void_p(stream.cuda_stream)))

    def step(self, nsteps: int = 1):
        _check(self.lib.cw_refined_step(self.h, int(nsteps)))

    def traces(self, nsteps: int) -> np.ndarray:
        out = np.zeros((max(self.nrec, 1), max(nsteps, 1)))
        done = ctypes.c_int64()
        _check(self.lib.cw_refined_get_traces(self.h, _dp(out), out.shape[1], ctypes.byref(done)))
        return out[: self.nrec, : done.value]

    def field(self, name: str) -> np.ndarray:
        out = np.empty(self.cells, dtype=np.float32)
        _check(self.lib.cw_refined_get_field(self.h, _pick(FIELDS, name, "field"), _fp(out)))
        return out

    def set_field(self, name: str, a):
        a = np.ascontiguousarray(np.reshape(a, self.cells), dtype=np.float32)
        _check(self.lib.cw_refined_set_field(self.h, _pick(FIELDS, name, "field"), _fp(a)))

    def energy(self) -> float:
        e = ctypes.c_double()
        _check(self.lib.cw_refined_energy(self.h, ctypes.byref(e)))
        return e.value

    def reset(self):
        _check(self.lib.cw_refined_reset(self.h))


def cement_loss(sim: "Sim", window, dmu, dK):
    """The receiver loss of `sim` over `window` as a differentiable function
    of the per-bin shifts dmu, dK (float64 torch tensors of nbins values):
    the forward sets the region's moduli and runs cw_gradient, whose
    gradient the backward returns."""
    import torch

    class _CementLoss(torch.autograd.Function):
        @staticmethod
        def forward(ctx, mu_shift, k_shift):
            sim.set_region_moduli(mu_shift.detach().cpu().numpy(), k_shift.detach().cpu().numpy())
            loss, gm, gk = sim.gradient(window)
            ctx.save_for_backward(torch.from_numpy(gm), torch.from_numpy(gk))
            return torch.tensor(loss, dtype=torch.float64)

        @staticmethod
        def backward(ctx, g):
            gm, gk = ctx.saved_tensors
            return g * gm, g * gk

    return _CementLoss.apply(dmu, dK)

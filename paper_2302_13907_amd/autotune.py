"""Tile-shape autotuner for batched steps.

A batched workgroup covers tz_waves x 256 depth cells of 4 / tz_waves theta
rows (tz_waves in {1, 2, 4}).  Which shape is fastest depends on the
instance's depth (ragged last segments waste lanes), its ring size and the
device; the tuner times a one-instance batch of each shape on the device
and keeps the fastest per (device, nr, ntheta, nz) in a JSON cache, so a
shape is measured once.

Cache file: $CWELL_TILE_CACHE, else ~/.cache/cwell/tiles.json."""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, Optional, Sequence

import numpy as np

SHAPES = (4, 2, 1)


def cache_path() -> str:
    return os.environ.get("CWELL_TILE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "cwell", "tiles.json"))


def _load(path: str) -> Dict[str, dict]:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _key(device_name: str, nr: int, nt: int, nz: int) -> str:
    return "%s|%dx%dx%d" % (device_name, nr, nt, nz)


def measure(nr: int, nt: int, nz: int, dr: float = 5e-3, dz: float = 5e-3, steps: int = 10,
            shapes: Sequence[int] = SHAPES) -> Dict[int, float]:
    """Seconds per step of a one-instance batch (fluid-filled cased well,
    layer on) for each tile shape."""
    import torch
    from . import cwell, inputs
    res = {}
    for tz in shapes:
        s = cwell.Sim(nr, nt, nz, dr, dz)
        s.set_material(*inputs.cased_well_rz(nr, nz, dr, dz, z_top=nz * dz / 2, ramp=0.1))
        npml = min(20, max(1, nr // 6), max(1, (nz - 2) // 4))
        s.set_pml(npml, npml, 1e-3, math.pi * 15e3)
        s.set_dt(0.5 * s.cfl_dt())
        s.bind()
        b = cwell.Batch([s])
        b.set_tile(0, tz)
        b.bind()
        b.step(2)
        s.sync()
        t0 = time.perf_counter()
        b.step(steps)
        s.sync()
        torch.cuda.synchronize()
        res[tz] = (time.perf_counter() - t0) / steps
        b.close()
        s.close()
    return res


def best_tile(nr: int, nt: int, nz: int, dr: float = 5e-3, dz: float = 5e-3,
              cache: Optional[str] = None, steps: int = 10) -> int:
    """The fastest tile shape for an instance of this size, from the cache
    or measured (and then cached)."""
    import torch
    path = cache or cache_path()
    db = _load(path)
    key = _key(torch.cuda.get_device_name(0), nr, nt, nz)
    if key in db:
        return int(db[key]["tz_waves"])
    t = measure(nr, nt, nz, dr, dz, steps)
    best = min(t, key=t.get)
    db[key] = {"tz_waves": best, "seconds_per_step": {str(k): v for k, v in t.items()}}
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return best


def tune_batch(batch, sims, cache: Optional[str] = None) -> Dict[int, int]:
    """Set every instance's tile shape from the tuner (before batch.bind());
    returns {instance: tz_waves}."""
    out = {}
    for q, s in enumerate(sims):
        nr, nt, nz = s.shape
        tz = best_tile(nr, nt, nz, s.dr, s.dz, cache)
        batch.set_tile(q, tz)
        out[q] = tz
    return out

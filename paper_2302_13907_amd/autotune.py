"""Autotuner for batched steps: tile shape x occupancy.

A batched workgroup covers tz_waves x 256 depth cells of 4 / tz_waves theta
rows (tz_waves in {1, 2, 4}: the theta rows per tile are 4, 2 or 1), and the
batched kernels are compiled for several register budgets (at least 0 = the
compiler's choice, 7 or 8 wavefronts per SIMD).  Which combination is
fastest depends on the instance's depth (ragged last segments waste lanes),
its ring size and the device.  The tuner times a one-instance batch of each
combination and keeps the fastest per (device, nr, ntheta, nz) in a JSON
cache, so a shape is measured once.  The tile shape is per instance; the
occupancy is one per batch launch, so a batch takes the occupancy chosen
for most of its cells.

Cache file: $CWELL_TILE_CACHE, else ~/.cache/cwell/tiles.json."""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, Optional, Sequence, Tuple

SHAPES = (4, 2, 1)
OCCUPANCY = (0, 7, 8)
_VERSION = 3          # cache entries of other versions are measured again


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


def measure(nr: int, nt: int, nz: int, dr: float = 5e-3, dz: float = 5e-3, steps: int = 20,
            shapes: Sequence[int] = SHAPES, occupancy: Sequence[int] = OCCUPANCY,
            repeats: int = 3) -> Dict[Tuple[int, int], float]:
    """Seconds per step of a one-instance batch (fluid-filled cased well,
    layer on) for each (tile shape, occupancy): the best of `repeats` timings
    of `steps` steps (the candidates differ by a few per cent, about what one
    timing varies by)."""
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
        for w in occupancy:
            b.set_occupancy(w)
            b.step(2)
            s.sync()
            best = math.inf
            for _ in range(repeats):
                t0 = time.perf_counter()
                b.step(steps)
                s.sync()
                torch.cuda.synchronize()
                best = min(best, (time.perf_counter() - t0) / steps)
            res[(tz, w)] = best
        b.close()
        s.close()
    return res


def best_config(nr: int, nt: int, nz: int, dr: float = 5e-3, dz: float = 5e-3,
                cache: Optional[str] = None, steps: int = 20) -> Tuple[int, int]:
    """The fastest (tz_waves, waves per SIMD) for an instance of this size,
    from the cache or measured (and then cached)."""
    import torch
    path = cache or cache_path()
    db = _load(path)
    key = _key(torch.cuda.get_device_name(0), nr, nt, nz)
    e = db.get(key)
    if e and e.get("version") == _VERSION:
        return int(e["tz_waves"]), int(e["waves_per_simd"])
    t = measure(nr, nt, nz, dr, dz, steps)
    tz, w = min(t, key=t.get)
    db[key] = {"version": _VERSION, "tz_waves": tz, "waves_per_simd": w,
               "seconds_per_step": {"%d/%d" % k: v for k, v in sorted(t.items())}}
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return tz, w


def best_tile(nr: int, nt: int, nz: int, dr: float = 5e-3, dz: float = 5e-3,
              cache: Optional[str] = None, steps: int = 20) -> int:
    """The tile shape of best_config."""
    return best_config(nr, nt, nz, dr, dz, cache, steps)[0]


def tune_batch(batch, sims, cache: Optional[str] = None) -> Dict[str, object]:
    """Set every instance's tile shape and the batch's occupancy from the
    tuner (before batch.bind()); returns {"tiles": {instance: tz_waves},
    "waves_per_simd": w}."""
    tiles, votes = {}, {}
    for q, s in enumerate(sims):
        nr, nt, nz = s.shape
        tz, w = best_config(nr, nt, nz, s.dr, s.dz, cache)
        batch.set_tile(q, tz)
        tiles[q] = tz
        votes[w] = votes.get(w, 0) + nr * nt * nz
    w = max(sorted(votes), key=lambda x: votes[x])
    batch.set_occupancy(w)
    return {"tiles": tiles, "waves_per_simd": w}

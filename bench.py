#!/usr/bin/env python3
"""Throughput of the cased-well time step on one MI355X.

Runs the production workload -- 256 x 128 x 8192 cells of 2 mm (268 M cells),
a fluid-filled hole, steel casing, cement with a 0.3 m graded top, rock, a
20-cell absorbing layer, a 15 kHz Ricker source on the axis and 64 axis
receivers -- through the C ABI, times K whole steps (velocity, stress,
layer, source, receivers) after W warm-up steps, and prints one JSON line:
Gcell-updates/s, the roofline fraction of the dominant kernel from HIP
events recorded live over the timed steps, and the FP64 CPU oracle timed on
a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gcell-updates/s per MI355X (FP32 vs FP16-store), % HBM roofline; s/adjoint grad"
HBM_PEAK_GBS = 8000.0
PMC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(kernel: str, w, n_r: int, n_z: int, fb: int = 4) -> float:
    """Algorithmic HBM bytes of one launch of `kernel` over workload w.

    One cell-update reads the 9 fields and the 3 moduli (rho, lambda, mu) and
    writes the 9 fields: 84 B in float32.  Each layer memory variable is read
    and written once: 12 of them per radial-slab cell (96 B), 6 per z-slab
    cell (48 B).  The separate velocity pass moves 6 stresses + 3 velocities
    in, 3 velocities out and rho (52 B, 6 radial / 3 z variables); the
    separate stress pass 3 velocities + 6 stresses in, 6 out, lambda and mu
    (68 B, the other 6 radial / 3 z variables).  With fb-byte field storage
    the field terms scale by fb/4 (the moduli and layer memory stay
    float32)."""
    n = w.cells
    if kernel == "fused":
        return (18 * fb + 12.0) * n + 96.0 * n_r + 48.0 * n_z
    if kernel == "velocity":
        return (12 * fb + 4.0) * n + 48.0 * n_r + 24.0 * n_z
    if kernel == "stress":
        return (15 * fb + 8.0) * n + 48.0 * n_r + 24.0 * n_z
    raise ValueError(kernel)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2302_13907_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources; else None."""
    try:
        d = json.load(open(PMC_FILE))
    except (OSError, ValueError):
        return None
    e = d.get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash() or e.get("workload") != workload:
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(w, target_s: float):
    """The FP64 oracle on a bounded sample of the workload: the full
    256 x 128 cross-section (with its radial layer) over 96 z-planes around
    the source, stepped until about target_s seconds have passed."""
    import numpy as np
    import oracle
    from paper_2302_13907_amd import inputs
    nzs = 96
    rho, lam, mu = inputs.cased_well_rz(w.nr, nzs, w.dr, w.dz, z_top=1e9, ramp=0.0)
    o = oracle.OracleSim(w.nr, w.nt, nzs, w.dr, w.dz)
    o.set_material(rho[:, None, :], lam[:, None, :], mu[:, None, :])
    o.set_pml(w.npml, 0, w.pml_rc, math.pi * w.f0)
    dt = w.cfl_fraction * o.cfl_dt()
    o.set_dt(dt)
    o.add_source("volume", 0, -1, nzs // 2, oracle.ricker(w.f0, (np.arange(4096) + 0.5) * dt))
    o.add_receiver("pressure", 0, -1, nzs // 2 + 10)
    o.run(1)
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < target_s:
        o.run(1)
        steps += 1
    el = time.perf_counter() - t0
    cells = w.nr * w.nt * nzs
    return {"value": cells * steps / el / 1e9, "unit": "Gcell-updates/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": "%dx%dx%d cross-section slab of the same workload (radial layer included, "
                      "no z layer), %d FP64 steps in %.1f s" % (w.nr, w.nt, nzs, steps, el)}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", choices=("production", "parity"), default="production")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--path", choices=("auto", "fused", "two-pass"), default="auto",
                    help="kernel path of the step")
    ap.add_argument("--storage", choices=("f32", "f16", "bf16"), default="f32",
                    help="field storage (arithmetic is float32 in every case)")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="after the run, copy this many GiB device-to-device once (a known-size "
                         "reference dispatch for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the z-slab decomposition is a design, not code); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2302_13907_amd import cwell, inputs

    if not torch.cuda.is_available():
        print("no HIP device visible", file=sys.stderr)
        sys.exit(1)
    w = inputs.production_case() if args.workload == "production" else inputs.parity_case()
    total = args.warmup + args.steps
    log("workload %s: building the medium" % w.name)
    s = cwell.Sim(w.nr, w.nt, w.nz, w.dr, w.dz)
    if w.rock_jitter == 0:
        s.set_material(*w.medium_rz())
    else:
        s.set_material(*w.medium())
    s.set_pml(w.npml, w.npml, w.pml_rc, math.pi * w.f0)
    dt = w.cfl_fraction * s.cfl_dt()
    s.set_dt(dt)
    s.add_source("volume", 0, -1, w.src_k, cwell.ricker(w.f0, (np.arange(total) + 0.5) * dt))
    for k in w.rec_k:
        s.add_receiver("pressure", 0, -1, k)
    s.set_trace_capacity(total)
    s.set_path(args.path)
    s.set_storage(args.storage)
    log("binding %.2f GB workspace" % (s.workspace_bytes() / 1e9))
    s.bind("cuda:0")
    log("warm-up %d steps" % args.warmup)
    s.step(args.warmup)
    s.sync()
    torch.cuda.synchronize()
    s.profile(True)
    log("timing %d steps" % args.steps)
    t0 = time.perf_counter()
    s.step(args.steps)
    s.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    times = {k: s.kernel_time(k) for k in ("velocity", "stress", "fused", "inject", "record")}
    s.profile(False)
    tr = s.traces()
    if not np.all(np.isfinite(tr)):
        print("non-finite traces", file=sys.stderr)
        sys.exit(1)
    value = w.cells * args.steps / el / 1e9
    dom = max(("velocity", "stress", "fused"), key=lambda k: times[k][0])
    ms, launches = times[dom]
    avg_s = ms / 1e3 / max(launches, 1)
    n_r, n_z = w.layer_cells
    fb = 4 if args.storage == "f32" else 2
    alg = algorithmic_bytes(dom, w, n_r, n_z, fb)
    achieved = alg / avg_s / 1e9
    traffic = measured_traffic(dom, w.name)
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "storage": args.storage,
        "data": "synthetic",
        "config": {"workload": w.name, "cells": w.cells, "grid": [w.nr, w.nt, w.nz],
                   "cell_m": w.dr, "layer_cells": w.npml, "receivers": len(w.rec_k),
                   "kernel_path": "two-pass" if dom != "fused" else "fused"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "alg_bytes_per_launch": alg,
                     "avg_launch_ms": round(avg_s * 1e3, 4)},
        "kernel_ms": {k: [round(v[0], 3), v[1]] for k, v in times.items() if v[1]},
    }
    s.close()
    del s
    torch.cuda.empty_cache()
    if args.copy_gib > 0:
        nb = int(args.copy_gib * (1 << 30))
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_reference_bytes"] = nb
        del src, dst
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("CPU baseline: FP64 oracle for about %.0f s" % args.cpu_seconds)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

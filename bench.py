#!/usr/bin/env python3
"""Throughput of the cased-well time step on one MI355X.

Runs the production workload -- 256 x 128 x 8192 cells of 2 mm (268 M cells),
a fluid-filled hole, steel casing, cement with a 0.3 m graded top, rock, a
20-cell absorbing layer, a 15 kHz Ricker source on the axis and 64 axis
receivers -- through the C ABI, times K whole steps (velocity, stress,
layer, source, receivers) after W warm-up steps, and prints one JSON line:
Gcell-updates/s, the step's roofline fraction (the method's bytes per
cell-update over the step kernels' time, from HIP events recorded live over
the timed steps), and the FP64 CPU oracle timed on a bounded sample of the
same workload on the host cores.
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


def algorithmic_bytes(kernel: str, w, n_r: int, n_z: int, fb: int = 4, axisym: bool = False) -> float:
    """Algorithmic HBM bytes of one launch of `kernel` over workload w.

    One cell-update reads the 9 fields and the 3 moduli (rho, lambda, mu) and
    writes the 9 fields: 84 B in float32.  Each layer memory variable is read
    and written once: 12 of them per radial-slab cell (96 B), 6 per z-slab
    cell (48 B).  The separate velocity pass moves 6 stresses + 3 velocities
    in, 3 velocities out and rho (52 B, 6 radial / 3 z variables); the
    separate stress pass 3 velocities + 6 stresses in, 6 out, lambda and mu
    (68 B, the other 6 radial / 3 z variables).  With fb-byte field storage
    the field terms scale by fb/4 (the moduli and layer memory stay
    float32).  A medium that does not vary along theta is stored once per
    (ring, depth): its bytes per cell-update are divided by Nt."""
    n = w.cells
    m = 1.0 / w.nt if axisym else 1.0
    if kernel == "fused":
        return (18 * fb + 12.0 * m) * n + 96.0 * n_r + 48.0 * n_z
    if kernel == "velocity":
        return (12 * fb + 4.0 * m) * n + 48.0 * n_r + 24.0 * n_z
    if kernel == "stress":
        return (15 * fb + 8.0 * m) * n + 48.0 * n_r + 24.0 * n_z
    raise ValueError(kernel)


# the sources the profiled step kernels (two-pass, fused, sources, receivers) are built from, and the
# host code that lays out their arrays (the padded field rings)
PROFILED_SOURCES = ("cwell_internal.hpp", "storage.hpp", "vec_common.hpp", "step_basic.hip", "step_vec.hip",
                    "step_fused.hip", "cwell_api.hip")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2302_13907_amd", "csrc")
    for f in PROFILED_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(variant: str, kernel: str, workload: str):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources; else None."""
    try:
        d = json.load(open(PMC_FILE))
    except (OSError, ValueError):
        return None
    e = d.get(variant, {}).get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash() or e.get("workload") != workload:
        return None
    return e.get("bytes_per_launch")


# --- hardware-counter profiles ------------------------------------------------------------
# Each profiled variant runs this script for a few steps under rocprofv3 three times: a
# kernel trace with statistics, then FETCH_SIZE and WRITE_SIZE counter passes (each counter
# in a run of its own), and a fourth pass counting L2-to-fabric read requests by size.  The
# run ends with a 1 GiB device-to-device copy whose counter readings calibrate the counters
# (bytes the copy must move / what the counter reports for it).
PROFILE_VARIANTS = {
    "auto_f32": "--path auto --storage f32",
    "two_pass_f32": "--path two-pass --storage f32",
    "two_pass_f16": "--path two-pass --storage f16",
    "two_pass_bf16": "--path two-pass --storage bf16",
    "fused_f32": "--path fused --storage f32",
}
PROFILE_RUN = ("python3 -u bench.py --steps 20 --warmup 5 --no-cpu-baseline --no-storage-forms --no-stream-ceiling "
               "--no-graph-replay --no-adjoint --no-batched --no-refined --copy-gib 1")
PROFILE_PASSES = (
    ("stats", "--kernel-trace --stats"),
    ("fetch", "--pmc FETCH_SIZE"),
    ("write", "--pmc WRITE_SIZE"),
    ("rdreq", "--pmc TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum"),
)
KERNEL_PATTERNS = (("velocity", "k_velocity_"), ("stress", "k_stress_"), ("fused", "k_step_fused"),
                   ("tail", "k_step_tail"), ("copy", "copyBuffer"))


def profile_commands(variant: str, outdir: str):
    run = "%s %s" % (PROFILE_RUN, PROFILE_VARIANTS[variant])
    return [(name, "rocprofv3 %s --output-format csv -d %s/%s -o p -- %s" % (opts, outdir, name, run))
            for name, opts in PROFILE_PASSES]


def _kernel_key(name: str):
    for key, pat in KERNEL_PATTERNS:
        if pat in name:
            return key
    return None


def _read_csv(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def ingest_profiles(variant: str, outdir: str):
    """Turn the four rocprofv3 passes of `variant` (made by the commands of
    profile_commands) into profiles/<kernels>_<variant>_production.txt and the
    variant's entry of profiles/hbm_traffic.json."""
    from paper_2302_13907_amd import inputs
    w = inputs.production_case()
    cmds = dict(profile_commands(variant, outdir))
    # kernel statistics
    stats = {}
    for r in _read_csv(os.path.join(outdir, "stats", "p_kernel_stats.csv")):
        k = _kernel_key(r["Name"])
        if k is None:
            continue
        e = stats.setdefault(k, {"calls": 0, "total_ns": 0.0, "min_ns": float("inf"), "max_ns": 0.0})
        e["calls"] += int(r["Calls"])
        e["total_ns"] += float(r["TotalDurationNs"])
        e["min_ns"] = min(e["min_ns"], float(r["MinNs"]))
        e["max_ns"] = max(e["max_ns"], float(r["MaxNs"]))
    live = None
    try:
        for line in open(os.path.join(outdir, "stats.log")):
            if line.startswith("{"):
                live = json.loads(line)
    except OSError:
        pass
    # counters: per kernel class, the mean over dispatches; the copy reference is the
    # largest copy dispatch (the 1 GiB copy at the end of the run)
    counters = {}
    for name in ("fetch", "write", "rdreq"):
        per = {}
        for r in _read_csv(os.path.join(outdir, name, "p_counter_collection.csv")):
            k = _kernel_key(r["Kernel_Name"])
            if k is None:
                continue
            per.setdefault((k, r["Counter_Name"]), {}).setdefault(r["Dispatch_Id"], 0.0)
            per[(k, r["Counter_Name"])][r["Dispatch_Id"]] += float(r["Counter_Value"])
        for (k, c), disp in per.items():
            vals = list(disp.values())
            counters[(k, c)] = {"mean": sum(vals) / len(vals), "max": max(vals), "n": len(vals)}
    copy_bytes = float(1 << 30)
    f_fetch = copy_bytes / (counters[("copy", "FETCH_SIZE")]["max"] * 1024.0)
    f_write = copy_bytes / (counters[("copy", "WRITE_SIZE")]["max"] * 1024.0)

    def rd_bytes(k, agg="mean"):
        try:
            return sum(sz * counters[(k, "TCC_EA0_RDREQ_%dB_sum" % sz)][agg] for sz in (32, 64, 128))
        except KeyError:
            return None

    copy_rd = rd_bytes("copy", "max")
    storage = PROFILE_VARIANTS[variant].split()[-1]
    fb = 4 if storage == "f32" else 2
    n_r, n_z = w.layer_cells
    entry = {}
    lines = ["rocprofv3 summary: %s, workload %s" % (variant, w.name), "",
             "Commands (from the repository root; the outputs land under %s):" % outdir]
    lines += ["  %s" % cmds[n] for n, _ in PROFILE_PASSES]
    lines += ["", "Calibration with a 1 GiB device-to-device copy (1073741824 B read, "
              "1073741824 B written):",
              "  FETCH_SIZE read %.0f KiB -> factor %.4f" % (counters[("copy", "FETCH_SIZE")]["max"], f_fetch),
              "  WRITE_SIZE read %.0f KiB -> factor %.4f" % (counters[("copy", "WRITE_SIZE")]["max"], f_write)]
    if copy_rd:
        lines.append("  read requests by size (32/64/128 B) sum to %.0f B = %.4f x the copy's reads"
                     % (copy_rd, copy_rd / copy_bytes))
    if "copy" in stats:
        c = stats["copy"]
        lines.append("  copy kernel: %d dispatches, max %.1f us (%.2f TB/s for the 2 GiB moved)"
                     % (c["calls"], c["max_ns"] / 1e3, 2 * copy_bytes / c["max_ns"] / 1e3))
    lines += ["", "%-10s %6s %12s %12s %12s %14s %14s %14s %10s"
              % ("kernel", "calls", "avg_us", "min_us", "max_us", "alg_B/launch", "fetch_B", "write_B",
                 "L2miss_TB/s")]
    for k in ("velocity", "stress", "fused", "tail"):
        if k not in stats:
            continue
        st = stats[k]
        avg_ns = st["total_ns"] / st["calls"]
        fe = counters.get((k, "FETCH_SIZE"))
        wr = counters.get((k, "WRITE_SIZE"))
        fetch_b = fe["mean"] * 1024.0 * f_fetch if fe else float("nan")
        write_b = wr["mean"] * 1024.0 * f_write if wr else float("nan")
        alg = (algorithmic_bytes(k, w, n_r, n_z, fb, w.rock_jitter == 0)
               if k in ("velocity", "stress", "fused") else float("nan"))
        lines.append("%-10s %6d %12.1f %12.1f %12.1f %14.4g %14.4g %14.4g %10.3f"
                     % (k, st["calls"], avg_ns / 1e3, st["min_ns"] / 1e3, st["max_ns"] / 1e3, alg,
                        fetch_b, write_b, (fetch_b + write_b) / avg_ns / 1e3))
        if k in ("velocity", "stress", "fused") and fe and wr:
            rd = rd_bytes(k)
            entry[k] = {"bytes_per_launch": fetch_b + write_b, "fetch_bytes": fetch_b,
                        "write_bytes": write_b, "alg_bytes": alg, "avg_ns": avg_ns,
                        "fetch_factor": f_fetch, "write_factor": f_write,
                        "read_request_bytes": rd * copy_bytes / copy_rd if rd and copy_rd else None,
                        "workload": w.name, "source_hash": kernel_source_hash()}
    if live:
        lines += ["", "Same run, HIP events recorded by the benchmark around each launch "
                  "(warm-up excluded): " + ", ".join(
                      "%s %.1f us" % (k, v[0] * 1e3 / v[1]) for k, v in live.get("kernel_ms", {}).items()),
                  "Benchmark line of that run: %s Gcell-updates/s, %s ms per step"
                  % (live.get("value"), live.get("ms_per_step"))]
    if any(e.get("read_request_bytes") for e in entry.values()):
        lines += ["", "Reads from the request-size pass, scaled by the copy's reading: "
                  + ", ".join("%s %.4g B" % (k, e["read_request_bytes"]) for k, e in entry.items()
                              if e.get("read_request_bytes"))]
    lines.append("")
    kern = "fused_step_%s" % storage if "fused" in entry else "velocity_stress_%s" % variant
    out = os.path.join(ROOT, "profiles", "%s_production.txt" % kern)
    open(out, "w").write("\n".join(lines))
    try:
        d = json.load(open(PMC_FILE))
    except (OSError, ValueError):
        d = {}
    d[variant] = entry
    with open(PMC_FILE, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    print("\n".join(lines))


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


ORACLE_TIMING_CASES = {
    # name: (workload, steps of a full run, (warm-up, timed) steps at every thread,
    # (warm-up, timed) at one thread); s_per_full_run scales the timed steps to a full run
    "parity": ("parity", 300, (0, 300), (0, 300)),
    "parity-long": ("parity", 3000, (0, 3000), (0, 600)),
    "production": ("production", 2000, (2, 20), (1, 1)),
}


def oracle_timing_case(name: str):
    """One timing of the FP64 oracle (host only): the named case at the
    thread count this process was started with."""
    import numpy as np
    import oracle
    from paper_2302_13907_amd import inputs
    wl, full, every, one = ORACLE_TIMING_CASES[name]
    w = inputs.parity_case() if wl == "parity" else inputs.production_case()
    warm, steps = one if oracle.threads() == 1 else every
    t0 = time.perf_counter()
    o = oracle.OracleSim(w.nr, w.nt, w.nz, w.dr, w.dz)
    o.set_material(*w.medium())
    o.set_pml(w.npml, w.npml, w.pml_rc, math.pi * w.f0)
    dt = w.cfl_fraction * o.cfl_dt()
    o.set_dt(dt)
    o.add_source("volume", 0, -1, w.src_k, oracle.ricker(w.f0, (np.arange(warm + steps) + 0.5) * dt))
    for k in w.rec_k:
        o.add_receiver("pressure", 0, -1, k)
    setup = time.perf_counter() - t0
    log("  set up in %.1f s" % setup)
    if warm:
        o.run(warm)
        log("  %d warm-up steps done" % warm)
    t0 = time.perf_counter()
    o.run(steps)
    el = time.perf_counter() - t0
    return {"case": "%s, %d timed steps after %d" % (w.name.split(",")[0], steps, warm),
            "threads": oracle.threads(), "setup_s": round(setup, 2), "s": round(el, 3),
            "Gcell_per_s": round(w.cells * steps / el / 1e9, 5),
            "full_run_steps": full, "s_per_full_run": round(el / steps * full, 1)}


def oracle_timing():
    """The FP64 oracle on the host: each case with every hardware thread and
    with one, in child processes (the thread count is fixed at start)."""
    import platform
    import subprocess
    model = platform.processor()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    out = {"host_cpu": model, "nproc": os.cpu_count(), "cases": []}
    for name in ORACLE_TIMING_CASES:
        for threads in (None, 1):
            env = dict(os.environ)
            if threads:
                env["OMP_NUM_THREADS"] = str(threads)
            log("oracle timing: %s, %s threads" % (name, threads or env.get("OMP_NUM_THREADS", "all")))
            r = subprocess.run([sys.executable, "-u", os.path.abspath(__file__), "--oracle-timing-case", name],
                               env=env, stdout=subprocess.PIPE, text=True)
            if r.returncode != 0:
                raise RuntimeError("oracle timing of %s failed" % name)
            res = json.loads(r.stdout.strip().splitlines()[-1])
            log("  " + json.dumps(res))
            out["cases"].append(res)
    return out


def run_steps(w, storage: str, path: str, warmup: int, steps: int, graph: int = 0, profile: bool = True,
              rounding: str = "nearest"):
    """Set up workload w, bind it, run warmup + timed steps; returns
    (seconds for the timed steps, {kernel: (ms, launches)}, traces).  With
    graph > 0 the steps are replayed from a captured graph of that many
    steps; per-launch timing (profile) needs ordinary launches."""
    import numpy as np
    import torch
    from paper_2302_13907_amd import cwell
    total = warmup + steps
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
    s.set_path(path)
    s.set_storage(storage)
    s.set_rounding(rounding)
    s.set_graph(graph)
    log("binding %.2f GB workspace (%s storage)" % (s.workspace_bytes() / 1e9, storage))
    s.bind("cuda:0")
    log("warm-up %d steps" % warmup)
    s.step(warmup)
    s.sync()
    torch.cuda.synchronize()
    s.profile(profile)
    log("timing %d steps" % steps)
    t0 = time.perf_counter()
    s.step(steps)
    s.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    times = {k: s.kernel_time(k) for k in ("velocity", "stress", "fused", "inject", "record")} if profile else {}
    s.profile(False)
    tr = s.traces()
    s.close()
    del s
    torch.cuda.empty_cache()
    if not np.all(np.isfinite(tr)):
        raise RuntimeError("non-finite traces (%s storage)" % storage)
    return el, times, tr


# (reads, writes) of 4-byte streams per cell of each step kernel, 3-D medium / axisymmetric medium
STREAM_MIX = {"velocity": ((10, 3), (9, 3)), "stress": ((11, 6), (9, 6)), "fused": ((12, 9), (9, 9))}


def stream_ceiling(kernel: str, axisym: bool, roofline: dict, lane_bytes: int = 16):
    """What HBM delivers to a kernel that only streams the dominant kernel's
    read/write mix (1 GiB per array; 16 bytes per thread and array, and 4),
    and a plain 1 + 1 copy; the dominant kernel's algorithmic rate as a
    fraction of the figure for its own access width (lane_bytes: 16 for the
    four-cell kernels, 4 for the one-cell ones)."""
    from paper_2302_13907_amd import cwell
    r, w = STREAM_MIX[kernel][1 if axisym else 0]
    log("stream ceiling: %d reads + %d writes" % (r, w))
    mix = cwell.stream_probe(r, w) / 1e9
    mix4 = cwell.stream_probe(r, w, lane_bytes=4) / 1e9
    nt = cwell.stream_probe(r, w, lane_bytes=lane_bytes, nontemporal=True) / 1e9
    copy = cwell.stream_probe(1, 1) / 1e9
    ref = mix4 if lane_bytes == 4 else mix
    return {"kernel": kernel, "reads": r, "writes": w, "GBps": round(mix, 1), "GBps_4B_lanes": round(mix4, 1),
            "GBps_nontemporal": round(nt, 1), "copy_GBps": round(copy, 1), "kernel_lane_bytes": lane_bytes,
            "frac_of_ceiling": round(roofline["achieved"] / ref, 4),
            "frac_of_nontemporal_ceiling": round(roofline["achieved"] / nt, 4)}


def graph_replay(path: str, graph: int = 20, steps: int = 300):
    """The parity-size workload (48 x 32 x 192, launch-bound) with ordinary
    launches and with graph replay of `graph` steps, Gcell-updates/s."""
    from paper_2302_13907_amd import inputs
    w = inputs.parity_case()
    res = {"workload": w.name, "steps": steps, "graph_steps": graph}
    for g in (0, graph):
        el, _, _ = run_steps(w, "f32", path, 2 * graph, steps, graph=g, profile=False)
        res["graph" if g else "ordinary"] = {"value": round(w.cells * steps / el / 1e9, 3),
                                             "us_per_step": round(el / steps * 1e6, 2)}
    res["speedup"] = round(res["graph"]["value"] / res["ordinary"]["value"], 3)
    return res


def adjoint_gradient():
    """Seconds per adjoint gradient on the adjoint workload (forward with
    checkpoints, segment recomputation, adjoint steps), next to one plain
    forward run of the same steps; and the same gradient with one segment
    (the strain rates of all steps kept on the device, nothing recomputed)."""
    import numpy as np
    import torch
    from paper_2302_13907_amd import cwell, inputs
    w = inputs.adjoint_case()
    x = w.extra
    log("adjoint gradient on %s" % w.name)

    def make(every):
        s = cwell.Sim(w.nr, w.nt, w.nz, w.dr, w.dz)
        s.set_material(*w.medium_rz())
        s.set_pml(w.npml, w.npml, w.pml_rc, math.pi * w.f0)
        dt = w.cfl_fraction * s.cfl_dt()
        s.set_dt(dt)
        s.add_source("volume", 0, -1, w.src_k, cwell.ricker(w.f0, (np.arange(w.steps) + 0.5) * dt))
        for k in w.rec_k:
            s.add_receiver("pressure", 0, -1, k)
        s.set_adjoint(w.steps, every, x["region"])
        s.bind("cuda:0")
        return s

    s = make(x["checkpoint_every"])
    s.step(10)                                    # warm-up of the forward kernels
    s.sync()
    s.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(w.steps)
    s.sync()
    fwd = time.perf_counter() - t0
    s.reset()
    t0 = time.perf_counter()
    loss, gm, gk = s.gradient(x["window"])
    grad = time.perf_counter() - t0
    ws = s.workspace_bytes()
    s.close()
    del s
    torch.cuda.empty_cache()
    if not (np.all(np.isfinite(gm)) and np.all(np.isfinite(gk))):
        raise RuntimeError("non-finite gradient")
    s = make(w.steps)
    t0 = time.perf_counter()
    loss1, gm1, gk1 = s.gradient(x["window"])
    grad1 = time.perf_counter() - t0
    ws1 = s.workspace_bytes()
    s.close()
    del s
    torch.cuda.empty_cache()
    if loss1 != loss or not (np.array_equal(gm1, gm) and np.array_equal(gk1, gk)):
        raise RuntimeError("the one-segment gradient differs from the checkpointed one")
    return {"workload": w.name, "parameters": 2 * x["region"][3], "checkpoint_every": x["checkpoint_every"],
            "s_per_gradient": round(grad, 3), "forward_s": round(fwd, 3), "ratio_to_forward": round(grad / fwd, 2),
            "workspace_GB": round(ws / 1e9, 2), "loss": loss,
            "one_segment": {"s_per_gradient": round(grad1, 3), "ratio_to_forward": round(grad1 / fwd, 2),
                            "workspace_GB": round(ws1 / 1e9, 2)}}


def batched_form(small: bool = False, steps: int = 40, graph: int = 20):
    """A batched workload (48 uneven 128 x 64 x Nz instances, or with `small`
    256 uneven 48 x 16 x Nz ones): aggregate Gcell-updates/s of the
    instances stepped one after another, of one batch (autotuned tile
    shapes), and of the batch under graph replay."""
    import numpy as np
    import torch
    from paper_2302_13907_amd import autotune, cwell, inputs
    ws = inputs.small_batched_case() if small else inputs.batched_case()
    log("batched form: %d instances" % len(ws))
    sims = []
    for w in ws:
        s = cwell.Sim(w.nr, w.nt, w.nz, w.dr, w.dz)
        s.set_material(*w.medium_rz())
        s.set_pml(w.npml, w.npml, w.pml_rc, math.pi * w.f0)
        dt = w.cfl_fraction * s.cfl_dt()
        s.set_dt(dt)
        total = 4 * steps + 8 + 2 * graph
        s.add_source("volume", 0, -1, w.src_k, cwell.ricker(w.f0, (np.arange(total) + 0.5) * dt))
        for k in w.rec_k:
            s.add_receiver("pressure", 0, -1, k)
        s.set_trace_capacity(total)
        s.set_path("two-pass")
        s.bind("cuda:0")
        sims.append(s)
    cells = sum(w.cells for w in ws)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    for s in sims:
        s.step(2)
    t_seq = timed(lambda: [s.step(steps) for s in sims])
    b = cwell.Batch(sims)
    tuned = autotune.tune_batch(b, sims)
    tiles = tuned["tiles"]
    b.bind()
    b.step(2)
    t_bat = timed(lambda: b.step(steps))
    b.set_graph(graph)
    b.step(2 * graph)                             # capture and warm up
    t_gr = timed(lambda: b.step(steps))
    b.close()
    for s in sims:
        s.close()
    del sims
    torch.cuda.empty_cache()
    gc = lambda t: round(cells * steps / t / 1e9, 3)
    # the method's bytes of one step of every instance (axisymmetric media;
    # the layer is a larger share of these smaller grids than of the production one)
    alg = sum(algorithmic_bytes("fused", w, *w.layer_cells, axisym=True) for w in ws)
    depths = sorted({w.nz for w in ws})
    return {"workload": "%d instances of %dx%dxNz, Nz in {%d..%d} (5 mm)" % (len(ws), ws[0].nr, ws[0].nt,
                                                                           depths[0], depths[-1]),
            "cells_per_step": cells, "steps": steps, "unit": "Gcell-updates/s",
            "sequential": gc(t_seq), "batched": gc(t_bat), "batched_graph": gc(t_gr),
            "speedup_batched": round(t_seq / t_bat, 3), "speedup_batched_graph": round(t_seq / t_gr, 3),
            "bytes_per_cell_update": round(alg / cells, 2),
            "roofline_frac_batched": round(alg * steps / t_bat / 1e9 / HBM_PEAK_GBS, 4),
            "tiles": {str(ws[q].nz): tz for q, tz in sorted(tiles.items())},
            "waves_per_simd": tuned["waves_per_simd"]}


def refined_form(uniform_ms: float, warmup: int = 10, steps: int = 100):
    """The production workload on the azimuthally refined grid (4 azimuthal
    cells next to the axis doubling with the radius up to 128): Gcell-
    updates/s of its own cells, its time step against the uniform grid's,
    and the physical time simulated per second of wall time, against the
    uniform grid's (uniform_ms: its measured milliseconds per step)."""
    import numpy as np
    import torch
    from paper_2302_13907_amd import cwell, inputs
    w = inputs.refined_production_case()
    zones = w.extra["zones"]
    log("refined form: %d zones %s" % (len(zones), zones))
    u = cwell.Sim(w.nr, w.nt, w.nz, w.dr, w.dz)          # host-side only: the uniform Courant limit
    u.set_material(*w.medium_rz())
    dt_uni = w.cfl_fraction * u.cfl_dt()
    u.close()
    r = cwell.Refined(w.nr, w.nz, w.dr, w.dz, zones)
    r.set_material_rz(*w.medium_rz())
    r.set_pml(w.npml, w.npml, w.pml_rc, math.pi * w.f0)
    dt = w.cfl_fraction * r.cfl_dt()
    r.set_dt(dt)
    total = warmup + steps
    r.add_source("volume", 0, -1, w.src_k, cwell.ricker(w.f0, (np.arange(total) + 0.5) * dt))
    for k in w.rec_k:
        r.add_receiver("pressure", 0, -1, k)
    r.set_trace_capacity(total)
    r.bind("cuda:0")
    r.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tr = r.traces(total)
    r.close()
    del r
    torch.cuda.empty_cache()
    if not np.all(np.isfinite(tr)):
        raise RuntimeError("non-finite traces on the refined grid")
    ms = el / steps * 1e3
    cells = sum((b - a) * n for (a, n), (b, _) in zip(zones, zones[1:] + [(w.nr, 0)])) * w.nz
    us_per_s = lambda d, m: d * 1e6 / (m * 1e-3)          # simulated microseconds per wall second
    return {"workload": w.name, "zones": [list(z) for z in zones], "cells": cells,
            "cells_uniform": w.cells, "steps": steps, "ms_per_step": round(ms, 4),
            "value": round(cells * steps / el / 1e9, 3), "unit": "Gcell-updates/s",
            "dt": dt, "dt_uniform": dt_uni, "dt_ratio": round(dt / dt_uni, 3),
            "sim_us_per_s": round(us_per_s(dt, ms), 2),
            "sim_us_per_s_uniform": round(us_per_s(dt_uni, uniform_ms), 2),
            "time_to_solution_speedup": round(us_per_s(dt, ms) / us_per_s(dt_uni, uniform_ms), 3)}


def storage_forms(path: str, warmup: int = 10, steps: int = 100):
    """Gcell-updates/s of the mixed-precision workload with float32, float16
    and bfloat16 field storage (float32 arithmetic in every case), and with
    bfloat16 stores rounded stochastically."""
    from paper_2302_13907_amd import inputs
    w = inputs.mixed_precision_case()
    log("storage forms on %s" % w.name)
    res = {"workload": w.name, "steps": steps, "warmup": warmup}
    for st in ("f32", "f16", "bf16"):
        el, times, _ = run_steps(w, st, path, warmup, steps)
        res[st] = {"value": round(w.cells * steps / el / 1e9, 3),
                   "ms_per_step": round(el / steps * 1e3, 4)}
    # bfloat16 with stochastically rounded stores
    el, _, _ = run_steps(w, "bf16", path, warmup, steps, rounding="stochastic")
    res["bf16_stochastic"] = {"value": round(w.cells * steps / el / 1e9, 3), "ms_per_step": round(el / steps * 1e3, 4)}
    for st in ("f16", "bf16", "bf16_stochastic"):
        res[st]["speedup_vs_f32"] = round(res[st]["value"] / res["f32"]["value"], 3)
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", choices=("production", "parity"), default="production")
    ap.add_argument("--medium", choices=("axisymmetric", "3d"), default="axisymmetric",
                    help="production medium as specified (theta-invariant, stored once per ring and depth), "
                         "or with the rock moduli jittered +-2 %% cell by cell (a 3-D medium)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--path", choices=("auto", "fused", "two-pass"), default="auto",
                    help="kernel path of the step")
    ap.add_argument("--storage", choices=("f32", "f16", "bf16"), default="f32",
                    help="field storage (arithmetic is float32 in every case)")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="after the run, copy this many GiB device-to-device once (a known-size "
                         "reference dispatch for hardware byte counters)")
    ap.add_argument("--no-storage-forms", action="store_true",
                    help="skip the float32 / float16 / bfloat16 storage comparison on the "
                         "192 x 96 x 4096 mixed-precision workload")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-form measurements (48 uneven large and 256 uneven small instances)")
    ap.add_argument("--no-refined", action="store_true",
                    help="skip the azimuthally refined grid (production workload, zones of 4..128 cells)")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the seconds-per-adjoint-gradient measurement")
    ap.add_argument("--no-graph-replay", action="store_true",
                    help="skip the ordinary-launch / graph-replay comparison on the parity-size workload")
    ap.add_argument("--no-stream-ceiling", action="store_true",
                    help="skip the streaming-bandwidth reference for the step kernels' read/write mixes")
    ap.add_argument("--print-profile-commands", nargs=2, metavar=("VARIANT", "OUTDIR"),
                    help="print the rocprofv3 commands that profile VARIANT (%s), one "
                         "'name command' per line, and exit" % ", ".join(PROFILE_VARIANTS))
    ap.add_argument("--ingest-profiles", nargs=2, metavar=("VARIANT", "OUTDIR"),
                    help="summarise the outputs of those commands into profiles/ and exit")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="time the FP64 oracle on the host (parity case at 300 and 3000 steps, a "
                         "production-size sample; every thread and one), print one JSON line and exit")
    ap.add_argument("--oracle-timing-case", choices=tuple(ORACLE_TIMING_CASES), help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_timing_case:
        print(json.dumps(oracle_timing_case(args.oracle_timing_case)))
        return
    if args.oracle_timing:
        print(json.dumps({"oracle_timing": oracle_timing()}))
        return
    if args.print_profile_commands:
        for name, cmd in profile_commands(*args.print_profile_commands):
            print(name, cmd)
        return
    if args.ingest_profiles:
        ingest_profiles(*args.ingest_profiles)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the z-slab decomposition is a design, not code); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2302_13907_amd import inputs

    if not torch.cuda.is_available():
        print("no HIP device visible", file=sys.stderr)
        sys.exit(1)
    w = inputs.production_case() if args.workload == "production" else inputs.parity_case()
    if args.medium == "3d" and w.rock_jitter == 0:
        import dataclasses
        w = dataclasses.replace(w, rock_jitter=0.02, name=w.name + ", 3-D medium")
    log("workload %s" % w.name)
    try:
        el, times, _ = run_steps(w, args.storage, args.path, args.warmup, args.steps)
    except RuntimeError as e:
        print(str(e), file=sys.stderr)
        sys.exit(1)
    value = w.cells * args.steps / el / 1e9
    n_r, n_z = w.layer_cells
    fb = 4 if args.storage == "f32" else 2
    axisym = w.rock_jitter == 0          # the medium is then stored once per (ring, depth)
    # the default path differs from the column two-pass step only in the float32 kernels
    fused = times["fused"][1] > 0
    form = ("fused" if fused else "auto" if args.path == "auto" and args.storage == "f32" else "two_pass")
    variant = "%s_%s" % (form, args.storage)
    # Roofline of the step: the method's bytes per cell-update (every field read
    # and written once, the moduli read once, each layer memory variable read and
    # written once) times the cells, over the time the step's kernels take per
    # step (HIP events around every launch).  A two-pass step is the velocity
    # and the stress launch together; the fused step is one launch.
    step_kernels = ("fused",) if fused else ("velocity", "stress")
    step_alg = algorithmic_bytes("fused", w, n_r, n_z, fb, axisym)
    kern_s = sum(times[k][0] / 1e3 / max(times[k][1], 1) for k in step_kernels)
    achieved = step_alg / kern_s / 1e9
    tr = [measured_traffic(variant, k, w.name) for k in step_kernels]
    traffic = sum(tr) if all(t is not None for t in tr) else None
    bpc = step_alg / w.cells
    # the slower kernel of a two-pass step against its own bytes (it moves more
    # than the method needs: the velocities are written and read back)
    dom = max(step_kernels, key=lambda k: times[k][0])
    ms, launches = times[dom]
    avg_s = ms / 1e3 / max(launches, 1)
    dom_alg = algorithmic_bytes(dom, w, n_r, n_z, fb, axisym)
    dom_achieved = dom_alg / avg_s / 1e9
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
                   "medium": "axisymmetric" if axisym else "3-D",
                   "cell_m": w.dr, "layer_cells": w.npml, "receivers": len(w.rec_k),
                   "kernel_path": {"fused": "fused",
                                   "auto": "two-pass, one-cell velocity and stress kernels"}.get(
                                       form, "two-pass, four-cell kernels")},
        "roofline": {"bound": "hbm", "kernel": "+".join(step_kernels), "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "traffic_kind": "L2-miss bytes per step (FETCH_SIZE + WRITE_SIZE, copy-calibrated; "
                                     "Infinity Cache hits count in them)",
                     # the counter-measured rate against the peak (an upper bound on the
                     # HBM rate: cache hits beyond L2 count in it)
                     "traffic_GBps": round(traffic / kern_s / 1e9, 1) if traffic else None,
                     "traffic_frac": round(traffic / kern_s / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
                     "bytes_per_cell_update": round(bpc, 2), "alg_bytes_per_step": step_alg,
                     "kernel_ms_per_step": round(kern_s * 1e3, 4),
                     "frac_of_wall_step": round(value * bpc / HBM_PEAK_GBS, 4),
                     # for comparison only: the same rate counted with the bytes a 3-D
                     # medium would add (this workload's medium does not vary along theta)
                     "frac_at_3d_medium_bytes": round(
                         algorithmic_bytes("fused", w, n_r, n_z, fb, False) / kern_s / 1e9 / HBM_PEAK_GBS, 4)},
        "kernel_own_bytes_roofline": {"kernel": dom, "achieved": round(dom_achieved, 1), "peak": HBM_PEAK_GBS,
                                      "unit": "GB/s", "frac": round(dom_achieved / HBM_PEAK_GBS, 4),
                                      "own_bytes_per_launch": dom_alg, "avg_launch_ms": round(avg_s * 1e3, 4),
                                      "traffic": measured_traffic(variant, dom, w.name)},
        "kernel_ms": {k: [round(v[0], 3), v[1]] for k, v in times.items() if v[1]},
    }
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
    if not args.no_stream_ceiling:
        one_cell = form == "auto"            # the default float32 kernels: one cell per thread
        out["stream_ceiling"] = stream_ceiling(dom, axisym, out["kernel_own_bytes_roofline"], 4 if one_cell else 16)
    if not args.no_storage_forms:
        out["storage_forms"] = storage_forms(args.path)
    if not args.no_graph_replay:
        out["graph_replay"] = graph_replay(args.path)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_gradient()
    if not args.no_batched:
        out["batched"] = [batched_form(), batched_form(small=True)]
    if not args.no_refined:
        out["refined"] = refined_form(out["ms_per_step"] if args.workload == "production" else float("nan"))
    if not args.no_cpu_baseline:
        log("CPU baseline: FP64 oracle for about %.0f s" % args.cpu_seconds)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

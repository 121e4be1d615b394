"""Host-side checks of the benchmark's measurement contract: the algorithmic
byte counts it divides by (against a count written out field by field),
the counter summary it reads traffic from (current sources only), the
rocprofv3 commands it prints, and its refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import pytest

import bench
from paper_2302_13907_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _count(kernel, w, axisym, fb):
    """Bytes of one launch, counted array by array: (reads, writes) of field
    arrays, medium arrays (4 B, stored once per ring and depth when the
    medium does not vary along theta), and the layer memory read and written
    in the radial slab and in the two depth slabs."""
    fields = {"velocity": (9, 3), "stress": (9, 6), "fused": (9, 9)}[kernel]
    medium = {"velocity": 1, "stress": 2, "fused": 3}[kernel]
    psi_r = {"velocity": 6, "stress": 6, "fused": 12}[kernel]
    psi_z = {"velocity": 3, "stress": 3, "fused": 6}[kernel]
    n = w.cells
    n_r, n_z = w.layer_cells
    mcells = n / w.nt if axisym else n
    return ((fields[0] + fields[1]) * fb * n + medium * 4 * mcells
            + psi_r * 2 * 4 * n_r + psi_z * 2 * 4 * n_z)


@pytest.mark.parametrize("kernel", ["velocity", "stress", "fused"])
@pytest.mark.parametrize("axisym", [False, True])
@pytest.mark.parametrize("fb", [4, 2])
def test_algorithmic_bytes_match_an_array_count(kernel, axisym, fb):
    w = inputs.production_case()
    n_r, n_z = w.layer_cells
    assert bench.algorithmic_bytes(kernel, w, n_r, n_z, fb, axisym) == pytest.approx(_count(kernel, w, axisym, fb),
                                                                                      rel=1e-12)


def test_production_figures():
    """84 B per cell-update for the fused floor without the layer, 52 + 68
    for the two passes; the layer adds 96 B per radial-slab cell and 48 B
    per depth-slab cell, 7.7 B per cell averaged over the production grid."""
    w = inputs.production_case()
    n = w.cells
    n_r, n_z = w.layer_cells
    assert bench.algorithmic_bytes("fused", w, 0, 0) == 84 * n
    assert bench.algorithmic_bytes("velocity", w, 0, 0) + bench.algorithmic_bytes("stress", w, 0, 0) == 120 * n
    layer = bench.algorithmic_bytes("fused", w, n_r, n_z) - 84 * n
    assert layer / n == pytest.approx(7.7, abs=0.05)


def test_traffic_only_for_the_current_sources(tmp_path, monkeypatch):
    """The counter summary is used only when it was taken on the kernel
    sources and workload at hand."""
    w = inputs.production_case()
    entry = {"two_pass_f32": {"stress": {"bytes_per_launch": 1.5e10, "source_hash": bench.kernel_source_hash(),
                                         "workload": w.name}}}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(entry))
    monkeypatch.setattr(bench, "PMC_FILE", str(f))
    assert bench.measured_traffic("two_pass_f32", "stress", w.name) == 1.5e10
    assert bench.measured_traffic("two_pass_f32", "stress", "another workload") is None
    assert bench.measured_traffic("two_pass_f32", "velocity", w.name) is None
    entry["two_pass_f32"]["stress"]["source_hash"] = "0" * 16
    f.write_text(json.dumps(entry))
    assert bench.measured_traffic("two_pass_f32", "stress", w.name) is None


def test_committed_traffic_matches_the_committed_sources():
    """Every variant in profiles/hbm_traffic.json was taken on the kernel
    sources of this tree, on the production workload."""
    d = json.load(open(os.path.join(ROOT, "profiles", "hbm_traffic.json")))
    w = inputs.production_case()
    assert "auto_f32" in d
    for variant, kernels in d.items():
        for k, e in kernels.items():
            assert e["source_hash"] == bench.kernel_source_hash(), (variant, k)
            assert e["workload"] == w.name
            assert e["bytes_per_launch"] > 0.9 * e["alg_bytes"], (variant, k)


def test_profile_commands_run_committed_files_only():
    for variant in bench.PROFILE_VARIANTS:
        for name, cmd in bench.profile_commands(variant, "gpurun_out/x"):
            assert cmd.startswith("rocprofv3 ") and " -- python3 -u bench.py " in cmd, cmd
            assert "--pmc" not in cmd or ("--sys-trace" not in cmd and "--kernel-trace" not in cmd), cmd
            assert "_work" not in cmd


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], stdout=subprocess.PIPE,
                       stderr=subprocess.PIPE, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""

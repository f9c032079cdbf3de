"""Host-side arithmetic of the benchmark (no GPU): the roofline entry, the validity rule of the
recorded HBM traffic, the operator flop count and the one-GPU exit."""
import json
import os
import shutil
import subprocess
import sys

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_operator_flops_invert_the_algorithmic_bytes():
    """Bytes per launch are sites*(72 b + 48 b n); flops are 1392 per site and right-hand side."""
    sites, n, b, calls = 131072, 128, 2, 7
    byt = calls * sites * (72.0 * b + 48.0 * b * n)
    assert bench.dslash_flops(byt, calls, sites, b) == pytest.approx(1392.0 * sites * n * calls, rel=1e-12)


def test_roofline_takes_the_dominant_family_against_hbm():
    # family: (ms, launches, algorithmic bytes)
    kt = {"dslash": (490.0, 630, 630 * 1.6e9), "cgs_dots": (97.0, 400, 2.0e11), "projections": (4.7, 2, 0.0)}
    r = bench._roofline(kt, sites=131072, b=2, tile=(2, 256, 64, 3))
    assert r["kernel"] == "dslash" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(630 * 1.6e9 / 0.490 / 1e9, abs=0.05)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, abs=1e-4)
    assert r["avg_launch_us"] == pytest.approx(490.0e3 / 630, abs=0.01)
    # a family with no algorithmic bytes is never the dominant one
    kt2 = {"projections": (900.0, 2, 0.0), "cgs_dots": (97.0, 400, 2.0e11)}
    assert bench._roofline(kt2)["kernel"] == "cgs_dots"


def test_recorded_traffic_is_used_only_for_its_source_workload_and_tile(tmp_path, monkeypatch):
    import hashlib

    pkg = tmp_path / "paper_1909_12234_amd"
    (pkg / "csrc").mkdir(parents=True)
    src = b"// kernel source\n"
    (pkg / "csrc" / "k.hip").write_bytes(src)
    rec = {"source": "csrc/k.hip", "sha256_16": hashlib.sha256(src).hexdigest()[:16], "workload": "w1",
           "tile": [2, 256, 64, 3], "fetch_bytes": 1000, "write_bytes": 24}
    other = dict(rec, tile=[2, 256, 64, 2], fetch_bytes=5)
    (pkg / "traffic.json").write_text(json.dumps({"kernels": {"dslash": [rec, other]}}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench._measured_traffic("dslash", (2, 256, 64, 3), "w1") == 1024
    assert bench._measured_traffic("dslash", (2, 256, 64, 2), "w1") == 29
    assert bench._measured_traffic("dslash", (7, 7, 7, 7), "w1") is None
    assert bench._measured_traffic("no_such_kernel", None, "w1") is None
    # a record taken on another workload (other lattice, other batch size) is not used
    assert bench._measured_traffic("dslash", (2, 256, 64, 3), "w2") is None
    assert bench._measured_traffic("dslash", (2, 256, 64, 3)) is None
    # a kernel source that differs from the recorded hash voids the record
    (pkg / "csrc" / "k.hip").write_bytes(src + b"// edited\n")
    assert bench._measured_traffic("dslash", (2, 256, 64, 3), "w1") is None


def test_committed_traffic_records_are_well_formed():
    with open(os.path.join(ROOT, "paper_1909_12234_amd", "traffic.json")) as f:
        recs = json.load(f)["kernels"]["dslash"]
    from paper_1909_12234_amd.workloads import WORKLOADS

    for rec in recs:
        assert os.path.exists(os.path.join(ROOT, "paper_1909_12234_amd", rec["source"]))
        assert len(rec["tile"]) == 4 and rec["fetch_bytes"] > 0 and rec["write_bytes"] > 0
        assert len(rec["sha256_16"]) == 16
        assert rec["workload"] in WORKLOADS


def test_more_than_one_gpu_exits_before_touching_a_device():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert p.returncode == 2 and "one GPU" in p.stderr and p.stdout == ""


def test_multigrid_workload_has_what_its_bench_path_reads():
    from paper_1909_12234_amd.workloads import WORKLOADS

    w = WORKLOADS["wilson32x64_mg"]
    for key in ("dims", "eps", "seed", "mass", "nprobes", "probe_seed", "xi", "block", "nv", "k", "inner_prec",
                "restart", "sstep", "batch"):
        assert key in w
    assert all(L % b == 0 for L, b in zip(w["dims"], w["block"]))
    # Table 2's first row: 8192 aggregates x 48 coarse dof = 393,216
    nagg = int(np.prod([L // b for L, b in zip(w["dims"], w["block"])]))
    assert nagg * 2 * w["nv"] == 393216

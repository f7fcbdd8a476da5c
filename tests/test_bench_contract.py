"""Host logic of bench.py, without a GPU: the one-GPU refusal, the
algorithmic byte counts its roofline figures divide by, and the rule that a
recorded HBM traffic figure is reported only while the kernel sources it was
measured on are unchanged."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_spmv_bytes_of_the_headline_matrix():
    # 128^3 mesh, s = 32, FP32 values: values and indices once, row offsets
    # once, x read and y written once
    n, nnz, s = 129 ** 3, 385 ** 3, 32
    got = bench.spmv_bytes(n, nnz, s, 4.0)
    assert got == nnz * (32 * 4 + 4) + 4 * (n + 1) + 2 * n * 32 * 4
    assert abs(got / 1e9 - 8.0909) < 1e-4
    # one Jacobi-CG iteration adds eleven vector passes
    assert bench.cg_iteration_bytes(n, nnz, s, 8.0) == bench.spmv_bytes(n, nnz, s, 8.0) + 11 * n * s * 8


def test_traffic_is_reported_only_for_the_sources_it_was_measured_on(tmp_path, monkeypatch):
    rec = {"k": {"source_hash": bench.kernel_source_hash(), "bytes_per_launch": 123}}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_counters.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the hash is of the sources under ROOT: point it back at the repository
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: rec["k"]["source_hash"])
    assert bench.load_traffic("k") == 123
    assert bench.load_traffic("other") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.load_traffic("k") is None


"""bench.py's committed_traffic: the HBM bytes of the roofline come from a
counter summary line only for the same kernel class and run configuration,
and only while the kernel's sources still hash to what the line records."""
import hashlib
import os

import bench


def _write(tmp_path, src_text, sha=None, run="w/P0/f64"):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "k.hip").write_text(src_text)
    sha = sha or hashlib.sha256(src_text.encode()).hexdigest()
    (tmp_path / "profiles" / "t.md").write_text(
        f"text\n    traffic kernel=gemm_tn run={run} source=k.hip sha256={sha} bytes_per_launch=1.5e+09\n")


def test_line_matches_kernel_run_and_hash(tmp_path, monkeypatch):
    _write(tmp_path, "kernel source\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    b, src = bench.committed_traffic("gemm_tn", "w/P0/f64")
    assert b == 1.5e9 and src == os.path.join("profiles", "t.md")
    assert bench.committed_traffic("gemm_tn", "w/P1/f64") == (None, None)
    assert bench.committed_traffic("gemm_nn", "w/P0/f64") == (None, None)


def test_changed_source_voids_the_line(tmp_path, monkeypatch):
    _write(tmp_path, "kernel source\n", sha=hashlib.sha256(b"older source\n").hexdigest())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.committed_traffic("gemm_tn", "w/P0/f64") == (None, None)


def test_headline_line_is_current():
    # the committed summary covers the kernels the default bench line reports
    b, _ = bench.committed_traffic("gemm_nn_256", "inv1_20000x16000/P0/f64")
    assert b is not None and b > 2.0e9

"""Host logic of bench.py: the algorithmic byte counts, and the committed
profile records it reads only while the HIP sources match their digest.
CPU only (nothing here touches a GPU)."""

import json
import subprocess
import sys

import pytest

import bench


def test_algorithmic_bytes_formula():
    ne, nn = 6 * 96 ** 3, 97 ** 3
    assert bench.algorithmic_bytes(ne, nn, "fwd", 8) == 16 * ne + 80 * nn
    assert bench.algorithmic_bytes(ne, nn, "vjp", 8) == 16 * ne + 96 * nn
    # mixed: FP64 coordinates, FP32 fields
    assert bench.algorithmic_bytes(ne, nn, "fwd", 4) == 16 * ne + (24 + 12 + 4 + 12) * nn
    assert bench.algorithmic_bytes(ne, nn, "vjp", 4) == 16 * ne + (24 + 12 + 12 + 12) * nn
    # per element on the 96^3 mesh: the figures the roofline quotes
    assert abs(bench.algorithmic_bytes(ne, nn, "fwd", 8) / ne - 29.8) < 0.05
    assert abs(bench.algorithmic_bytes(ne, nn, "vjp", 8) / ne - 32.5) < 0.05


@pytest.fixture
def profile_dir(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILE_DIR", str(tmp_path))
    return tmp_path


def _write(path, rec):
    path.write_text(json.dumps(rec))


def test_records_are_read_only_for_the_current_sources(profile_dir):
    digest = bench.source_digest()
    _write(profile_dir / "traffic_w.json",
           {"source_sha256": digest, "scatter": "patch_gather", "calls": {"vjp": {"bytes": 123.0}}})
    _write(profile_dir / "valu_w.json", {"source_sha256": digest, "calls": {"vjp": {"fp64_flops": 4.0e9}}})
    assert bench.measured_traffic("w", "vjp", "patch_gather") == 123.0
    assert bench.measured_traffic("w", "vjp", "atomic") is None  # another scatter
    assert bench.measured_traffic("w", "fwd", "patch_gather") is None  # no such call
    assert bench.executed_flops("w", "vjp") == 4.0e9
    ex = bench.executed_rate("w", "vjp", 0.1, 10 ** 7)
    assert abs(ex["achieved"] - 40.0) < 1e-9 and abs(ex["flops_per_element"] - 400.0) < 1e-9
    assert abs(ex["frac"] - 40.0 / bench.FP64_PEAK_TFS) < 1e-12
    # a record of other sources (the kernels changed since it was taken)
    _write(profile_dir / "traffic_w.json",
           {"source_sha256": "0" * 64, "scatter": "patch_gather", "calls": {"vjp": {"bytes": 123.0}}})
    _write(profile_dir / "valu_w.json", {"source_sha256": "0" * 64, "calls": {"vjp": {"fp64_flops": 4.0e9}}})
    assert bench.measured_traffic("w", "vjp", "patch_gather") is None
    assert bench.executed_flops("w", "vjp") is None
    assert bench.executed_rate("w", "vjp", 0.1, 10 ** 7) is None


def test_missing_or_broken_records(profile_dir):
    assert bench.measured_traffic("none", "vjp", "patch_gather") is None
    (profile_dir / "valu_bad.json").write_text("{not json")
    assert bench.executed_flops("bad", "vjp") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "exactly one GPU" in r.stderr


def test_committed_profiles_match_the_current_sources():
    """The committed traffic and VALU records were taken with the HIP sources
    as they are now, so the bench line carries measured traffic and executed
    flops; an edit under csrc/ must be followed by new profiles."""
    for mode in ("fwd", "vjp"):
        assert bench.measured_traffic("cube96_jit_perm", mode, "patch_gather") is not None
        assert bench.executed_flops("cube96_jit_perm", mode) is not None

"""Host logic of bench.py: the algorithmic byte counts, the committed profile
records it reads only while the HIP sources match their digest, and the
roofline/limiter arithmetic.  CPU only (nothing here touches a GPU)."""

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


def test_configs_follow_the_measurement_plan():
    c = bench.CONFIGS
    assert [c[k].workload for k in ("C1", "C2", "C3", "C4", "C5")] == [
        "cube16", "cube96_perm", "cube160_jit_perm_smag", "cube96_jit_perm", "cube160_jit_perm_smag"]
    assert [c[k].precision for k in ("C1", "C2", "C3", "C4", "C5")] == ["fp64"] * 4 + ["mixed"]
    assert c["C4"].calls == ("fwd", "vjp") and c["C5"].calls == ("fwd", "vjp") and c["C3"].calls == ("fwd",)
    assert c["C1"].one_thread and c["C2"].one_thread
    assert bench.HEADLINE == "C4"
    assert bench.kernel_names("mixed", True, "vjp") == ("k_assemble_patch<float, 1, 0, 1, true>",
                                                       "k_gather_partials<float, 3>")


@pytest.fixture
def profile_dir(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILE_DIR", str(tmp_path))
    return tmp_path


def _write(path, rec):
    path.write_text(json.dumps(rec))


def _ctr():
    return {"k": {"waves": 2000.0, "hbm_bytes": 2.0e8, "f64_flops": 3.0e9, "f32_flops": 1.0e9, "l2_hit_rate": 0.7,
                  "per_wave": {"SQ_INSTS_VALU": 300.0, "SQ_LDS_IDX_ACTIVE": 400.0, "SQ_LDS_BANK_CONFLICT": 100.0}}}


def test_records_are_read_only_for_the_current_sources(profile_dir):
    digest = bench.source_digest()
    _write(profile_dir / "counters_w.json", {"source_sha256": digest, "kernels": _ctr()})
    assert bench.counter_record("w")["k"]["hbm_bytes"] == 2.0e8
    _write(profile_dir / "counters_w.json", {"source_sha256": "0" * 64, "kernels": _ctr()})
    assert bench.counter_record("w") is None
    assert bench.counter_record("none") is None
    (profile_dir / "counters_bad.json").write_text("{not json")
    assert bench.counter_record("bad") is None
    _write(profile_dir / "resources.json", {"source_sha256": digest, "kernels": {"k": {"vgprs": 77}}})
    assert bench.resource_record()["k"]["vgprs"] == 77


def test_kernel_evidence_and_limiter():
    ev = bench.kernel_evidence(_ctr(), "k", 0.1, 5000.0)
    assert abs(ev["hbm_GBs"] - 2000.0) < 1e-9 and abs(ev["hbm_frac_of_scale"] - 0.4) < 1e-12
    assert abs(ev["executed_fp64_TFs"] - 30.0) < 1e-9
    assert abs(ev["executed_frac_of_valu_issue"] - 40.0 / bench.FP64_PEAK_TFS) < 1e-12
    busy = 300.0 * 2000.0 * 4 / (1024 * 2.4e9 * 1e-4)
    assert abs(ev["valu_busy"] - busy) < 1e-12 and abs(ev["lds_conflict_share"] - 0.25) < 1e-12
    # 400 LDS-active cycles a wave, 2000 waves, over 256 units x 2.4 GHz x 0.1 ms
    assert abs(ev["lds_busy"] - 400.0 * 2000.0 / (256 * 2.4e9 * 1e-4)) < 1e-12
    bound, verdict = bench.limiter(ev)
    assert bound == "hbm" and "neither roof" in verdict  # busy 0.0098 < HBM 0.4 < 0.8
    assert "busiest is HBM at 0.40" in verdict and "bank-conflict share 0.25" in verdict
    bound, verdict = bench.limiter({"valu_busy": 0.5, "hbm_frac_of_scale": 0.4, "lds_busy": 0.65,
                                    "lds_conflict_share": 0.3})
    assert bound == "alu" and "neither roof" in verdict and "busiest is LDS at 0.65" in verdict
    bound, verdict = bench.limiter({"valu_busy": 0.5, "hbm_frac_of_scale": 0.4, "lds_busy": 0.85})
    assert bound == "alu" and verdict.startswith("LDS throughput (0.85")
    bound, verdict = bench.limiter({"valu_busy": 0.04, "hbm_frac_of_scale": 0.05, "waves": 384.0})
    assert bound == "hbm" and verdict.startswith("latency: 384 waves cannot fill the 1024 SIMDs")
    bound, verdict = bench.limiter({"valu_busy": 0.9, "hbm_frac_of_scale": 0.3})
    assert bound == "alu" and "VALU issue" in verdict
    assert bench.kernel_evidence(None, "k", 0.1, 5000.0) is None
    assert bench.limiter(None)[0] == "alu"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "exactly one GPU" in r.stderr


def test_committed_profiles_match_the_current_sources():
    """The committed counter records of every workload the bench measures,
    and the compiler resource record, were taken with the HIP sources as they
    are now, so the bench line carries measured traffic, executed flops and
    register counts; an edit under csrc/ must be followed by new profiles."""
    for wl in sorted({c.workload for c in bench.CONFIGS.values()}):
        rec = bench.counter_record(wl)
        assert rec is not None, f"profiles/counters_{wl}.json is missing or stale"
    assert bench.resource_record() is not None

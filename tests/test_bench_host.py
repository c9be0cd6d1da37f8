"""Host logic of the benchmark: the committed HBM counters are quoted only for
the launch variant the autotuner picked and only while the GEMM source matches
the hash recorded with them; --gpus above 1 is refused."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _rec():
    with open(os.path.join(ROOT, "profiles", "wire256_fp64_traffic.json")) as f:
        return json.load(f)


def _source_matches(rec):
    import hashlib
    with open(os.path.join(ROOT, rec["source"]), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest() == rec["source_sha256"]


def test_traffic_follows_the_tuned_tile():
    rec = _rec()
    if not _source_matches(rec):                  # counters older than the GEMM source: never quoted
        assert bench.measured_traffic("projection", False, 128, None) is None
        return
    by_cfg = rec["stages"]["back_projection"]["bytes_by_nn_cfg"]
    for cfg, b in by_cfg.items():
        assert bench.measured_traffic("back_projection", False, 128, int(cfg)) == b
    assert bench.measured_traffic("back_projection", False, 128, 99) is None
    assert bench.measured_traffic("projection", False, 128, None) == rec["stages"]["projection"]["bytes_per_launch"]
    # counters were taken on the complex128 path at 128 bands only
    assert bench.measured_traffic("projection", True, 128, None) is None
    assert bench.measured_traffic("projection", False, 136, None) is None
    assert bench.measured_traffic("xy_fft_v", False, 128, None) is None


def test_traffic_needs_the_recorded_source(tmp_path, monkeypatch):
    rec = _rec()
    rec["source_sha256"] = "0" * 64
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "wire256_fp64_traffic.json").write_text(json.dumps(rec))
    src = tmp_path / rec["source"]
    src.parent.mkdir(parents=True)
    src.write_bytes(open(os.path.join(ROOT, rec["source"]), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("projection", False, 128, None) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr

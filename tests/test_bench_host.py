"""Host logic of the benchmark: the committed HBM counters of the 4000-atom
wire are quoted only for the BF16 launch variant in use and only while the
kernel source matches the hash recorded with them; --gpus above 1 is refused."""
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

REC = os.path.join(ROOT, "profiles", "wire4000_traffic.json")


def _rec():
    with open(REC) as f:
        return json.load(f)


def _matches(st):
    with open(os.path.join(ROOT, st["source"]), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest() == st["source_sha256"]


def test_traffic_follows_the_bf16_variant():
    rec = _rec()
    st = rec["stages"]["projection"]
    if not _matches(st):                          # counters older than the kernel source: never quoted
        assert bench.measured_traffic_wire4000("projection", 6) is None
        return
    for v, b in st["bytes_by_variant"].items():
        assert bench.measured_traffic_wire4000("projection", int(v)) == b
    assert bench.measured_traffic_wire4000("projection", 99) is None
    assert bench.measured_traffic_wire4000("projection", None) is None
    assert bench.measured_traffic_wire4000("block_gram", 6) is None          # no counter run for it


def test_traffic_needs_the_recorded_source(tmp_path, monkeypatch):
    rec = _rec()
    st = rec["stages"]["projection"]
    st["source_sha256"] = "0" * 64
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "wire4000_traffic.json").write_text(json.dumps(rec))
    src = tmp_path / st["source"]
    src.parent.mkdir(parents=True)
    src.write_bytes(open(os.path.join(ROOT, st["source"]), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    v = next(iter(st["bytes_by_variant"]))
    assert bench.measured_traffic_wire4000("projection", int(v)) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr

"""Host-side parts of bench.py: the one-GPU guard and the lookup of the HBM
byte counts, which are reported only for the kernel sources they were
measured on (no GPU calls)."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout.strip() == ""


def test_source_hash_covers_every_kernel_source(tmp_path):
    b = _bench_module()
    h = b.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    assert b.kernel_source_hash() == h   # deterministic
    # a copy of the sources with one byte changed hashes differently
    csrc = os.path.join(ROOT, "paper_2605_30342_amd", "csrc")
    dst = tmp_path / "paper_2605_30342_amd" / "csrc"
    dst.mkdir(parents=True)
    names = sorted(os.listdir(csrc))
    for n in names:
        (dst / n).write_bytes(open(os.path.join(csrc, n), "rb").read())
    b.ROOT = str(tmp_path)
    assert b.kernel_source_hash() == h
    last = dst / names[-1]
    last.write_bytes(last.read_bytes() + b" ")
    assert b.kernel_source_hash() != h


def test_traffic_is_reported_only_for_matching_sources(tmp_path):
    b = _bench_module()
    (tmp_path / "profiles").mkdir()
    doc = {"raster_vis": {"source_hash": "0123456789abcdef", "bytes_per_launch": 123456}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(doc))
    b.ROOT = str(tmp_path)
    b.kernel_source_hash = lambda: "0123456789abcdef"
    assert b.traffic_for("raster_vis") == 123456
    assert b.traffic_for("raster_uq") is None           # no entry
    b.kernel_source_hash = lambda: "fedcba9876543210"
    assert b.traffic_for("raster_vis") is None          # measured on other sources
    (tmp_path / "profiles" / "traffic.json").write_text("not json")
    assert b.traffic_for("raster_vis") is None

"""Host logic of bench.py (no GPU): the HBM traffic figure of the bounce
kernel is read from its committed rocprofv3 summary only while the summary's
source hash matches the current kernel sources, and `--gpus N > 1` is refused.
"""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _summary(name):
    kv = {}
    for line in open(os.path.join(ROOT, "profiles", name)):
        parts = line.strip().lstrip("- ").split(":", 1)
        if len(parts) == 2:
            kv[parts[0].strip()] = parts[1].strip().strip("`")
    return kv


def test_street_canyon_traffic_matches_the_committed_summary(bench):
    kv = _summary("k_trace_bounce_street_canyon_traffic.md")
    assert kv["source_hash"] == bench.trace_source_hash(), "the traffic summary predates the kernel sources"
    want = (float(kv["fetch_kib_per_dispatch"]) * float(kv["fetch_scale"]) +
            float(kv["write_kib_per_dispatch"]) * float(kv["write_scale"])) * 1024.0
    got = bench.measured_traffic("street_canyon")
    assert got == pytest.approx(want, rel=1e-12)
    assert 5e9 < got < 1e10


def test_traffic_is_withheld_without_a_summary_or_on_a_hash_mismatch(bench, tmp_path, monkeypatch):
    assert bench.measured_traffic("no_such_workload") is None
    prof = tmp_path / "profiles"
    prof.mkdir()
    text = open(os.path.join(ROOT, "profiles", "k_trace_bounce_street_canyon_traffic.md")).read()
    h = bench.trace_source_hash()
    (prof / "k_trace_bounce_street_canyon_traffic.md").write_text(text.replace(h, "0" * 16))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "trace_source_hash", lambda: h)
    assert bench.measured_traffic("street_canyon") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr

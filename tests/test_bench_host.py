"""Host logic of bench.py (no GPU): the single-GPU guard and the committed
HBM-traffic lookup, which must refuse counters taken on other kernel sources."""
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def _tree(tmp_path, sources, recorded_hash):
    csrc = tmp_path / "paper_1609_04205_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name, text in sources.items():
        (csrc / name).write_text(text)
    (tmp_path / "profiles").mkdir()
    d = {"kernels": {"k": {"sources": list(sources), "sources_sha256_16": recorded_hash,
                           "hbm_bytes_per_launch": 12345.6}}}
    (tmp_path / "profiles" / "hbm_traffic.json").write_text(json.dumps(d))


def test_traffic_is_reported_only_for_the_measured_sources(tmp_path, monkeypatch):
    b = _bench()
    sources = {"k.hip": "kernel body\n", "shared.h": "shared helper\n"}
    h = hashlib.sha256()
    for t in sources.values():
        h.update(t.encode())
    _tree(tmp_path, sources, h.hexdigest()[:16])
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.measured_traffic("k") == 12346
    assert b.measured_traffic("missing") is None
    # a change in a shared header invalidates the counters too
    (tmp_path / "paper_1609_04205_amd" / "csrc" / "shared.h").write_text("shared helper, changed\n")
    assert b.measured_traffic("k") is None


def test_committed_traffic_summary_is_well_formed():
    d = json.load(open(os.path.join(ROOT, "profiles", "hbm_traffic.json")))
    for k, v in d["kernels"].items():
        assert v["sources"] and v["sources"][0].endswith(".hip"), k
        assert len(v["sources_sha256_16"]) == 16
        assert v["hbm_bytes_per_launch"] > 0

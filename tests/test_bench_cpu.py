"""Host logic of bench.py that runs without a GPU: the one-GPU guard and the rule that a
recorded HBM traffic figure is reported only while its kernel source is unchanged."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}),
                                      ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(argv, env):
    e = dict(os.environ)
    e.update(env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, capture_output=True, text=True,
                       env=e, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line for a configuration that was not measured


def test_traffic_follows_the_source_hash(monkeypatch):
    for (kernel, prec), rec in bench.TRAFFIC.items():
        current = bench._source_hash(rec["source"]) == rec["sha256"]
        assert bench.traffic_for(kernel, prec) == (rec["bytes"] if current else None)
    key = next(iter(bench.TRAFFIC))
    rec = dict(bench.TRAFFIC[key])
    monkeypatch.setitem(bench.TRAFFIC, key, dict(rec, sha256=bench._source_hash(rec["source"])))
    assert bench.traffic_for(*key) == rec["bytes"]
    monkeypatch.setitem(bench.TRAFFIC, key, dict(rec, sha256="0" * 16))
    assert bench.traffic_for(*key) is None
    monkeypatch.setitem(bench.TRAFFIC, key, dict(rec, source="no/such/file.hip"))
    assert bench.traffic_for(*key) is None
    assert bench.traffic_for("no such kernel", "fp64") is None


def test_traffic_sources_exist():
    for rec in bench.TRAFFIC.values():
        assert os.path.isfile(os.path.join(ROOT, rec["source"]))
        assert len(rec["sha256"]) == 16 and rec["bytes"] > 0

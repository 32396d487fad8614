"""CPU checks of the measurement bookkeeping in bench.py: the counter-based
traffic figure is reported only for the Wilson-kernel sources and the Wilson
forms and rhs groups it was measured with."""
import importlib.util
import json
import os
import shutil

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _traffic():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        return json.load(fh)


def test_traffic_entries_match_their_tuning(bench):
    t = _traffic()
    entries = t["entries"]["dslash_f64@16x16x16x16"]
    assert len({tuple(e["wilson_tuning"]) for e in entries}) == len(entries)
    for e in entries:
        # counters below the algorithmic bytes come only from links shared by rhs groups
        assert 0.5 < e["measured_over_algorithmic"] < 1.2
        assert abs(e["fetch_bytes_over_alg"] + e["write_bytes_over_alg"] - e["measured_over_algorithmic"]) < 1e-12
        got = bench.counter_traffic("dslash_f64", (16, 16, 16, 16), 1.0e6, e["wilson_tuning"])
        assert got == pytest.approx(e["measured_over_algorithmic"] * 1.0e6)
    assert bench.counter_traffic("dslash_f64", (16, 16, 16, 16), 1.0e6, [9, 9, 9]) is None
    assert bench.counter_traffic("dslash_f64", (32, 32, 32, 32), 1.0e6, entries[0]["wilson_tuning"]) is None
    assert bench.counter_traffic("dslash_f32", (16, 16, 16, 16), 1.0e6, entries[0]["wilson_tuning"]) is None


def test_traffic_is_dropped_once_the_kernel_sources_change(bench, tmp_path, monkeypatch):
    t = _traffic()
    for f in t["source_files"] + ["profiles/traffic.json"]:
        dst = tmp_path / f
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(ROOT, f), dst)
    tuning = t["entries"]["dslash_f64@16x16x16x16"][0]["wilson_tuning"]
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("dslash_f64", (16, 16, 16, 16), 1.0, tuning) is not None
    with open(tmp_path / t["source_files"][0], "a") as fh:
        fh.write("\n// edited\n")
    assert bench.counter_traffic("dslash_f64", (16, 16, 16, 16), 1.0, tuning) is None

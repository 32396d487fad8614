"""CPU checks of the measurement bookkeeping in bench.py: the algorithmic byte
and flop models per kernel (the N-rhs Wilson model, the coarse operator, the
transfer), the choice of bound, the counter-based traffic lookup (only for the
kernel sources and forms it was measured with), the default workload and the
refusal of more than one GPU."""
import hashlib
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_wilson_byte_model(bench):
    vol = 1000
    # one rhs per launch: 960 / 480 / 248 B per site
    assert bench.wilson_bytes("f64", vol, 1, vol) == 960 * vol
    assert bench.wilson_bytes("f32", vol, 1, vol) == 480 * vol
    assert bench.wilson_bytes("bf16", vol, 1, vol) == 248 * vol
    # N rhs per launch: (576/N + 384) B per site and rhs, links once per launch
    for n in (2, 8, 20):
        assert bench.wilson_bytes("f64", vol, 3, 3 * n * vol) == pytest.approx(3 * n * vol * (576 / n + 384))
        assert bench.wilson_bytes("f32", vol, 1, n * vol) == pytest.approx(n * vol * (288 / n + 192))
        assert bench.wilson_bytes("f16", vol, 1, n * vol) == pytest.approx(n * vol * (144 / n + 104))
    # a mix of one-rhs and 20-rhs launches is counted launch by launch
    mixed = bench.wilson_bytes("f64", vol, 432 + 150, 432 * vol + 150 * 20 * vol)
    assert mixed == pytest.approx(432 * 960 * vol + 150 * vol * (576 + 20 * 384))


def test_bound_follows_arithmetic_intensity(bench):
    w = {"vol": 24 ** 3 * 48, "nv": 24, "n2_mid": 48, "n2_coarsest": 48, "nsite_mid": 2592, "nsite_coarsest": 2592}
    # coarsest GCR operator with 32 rhs: AI = 72 * 48^2 * 32 / (9 * 48^2 * 16 + 32 * 3 * 48 * 16) ~ 16 > 9.8
    r = bench.roofline_of("coarse_gcr", {"launches": 10, "units": 10 * 2592 * 32, "ms_total": 3.6}, w)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    assert r["flops_per_launch"] == pytest.approx(72 * 48 * 48 * 2592 * 32)
    assert r["achieved"] == pytest.approx(r["flops_per_launch"] / 0.36e-3 / 1e12)
    # one rhs: bandwidth bound
    r1 = bench.roofline_of("coarse_gcr", {"launches": 10, "units": 10 * 2592, "ms_total": 1.0}, w)
    assert r1["bound"] == "hbm" and r1["unit"] == "GB/s"
    d = bench.roofline_of("dslash_bf16", {"launches": 4, "units": 4 * 32 * w["vol"], "ms_total": 6.0}, w)
    assert d["bound"] == "hbm"
    assert d["bytes_per_launch"] == pytest.approx(w["vol"] * (144 + 32 * 104))
    assert bench.roofline_of("block_qr", {"launches": 1, "units": 1, "ms_total": 1.0}, w) is None


def _write_traffic(root, kernel, workload, tuning, ratio, files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    t = {"entries": {f"{kernel}@{workload}": [{"tuning": tuning, "measured_over_algorithmic": ratio,
                                                "source_files": files, "source_hash": h.hexdigest()[:16]}]}}
    os.makedirs(os.path.join(root, "profiles"), exist_ok=True)
    with open(os.path.join(root, "profiles", "traffic.json"), "w") as fh:
        json.dump(t, fh)


def test_traffic_lookup_needs_same_sources_and_tuning(bench, tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("// kernel\n")
    _write_traffic(str(tmp_path), "coarse_gcr", "24x24x24x48_32rhs_bf16", [1, 2, 3], 1.25, ["k.hip"])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("coarse_gcr", "24x24x24x48_32rhs_bf16", 1e6, [1, 2, 3]) == pytest.approx(1.25e6)
    assert bench.counter_traffic("coarse_gcr", "24x24x24x48_32rhs_bf16", 1e6, [1, 2, 4]) is None
    assert bench.counter_traffic("coarse_gcr", "16x16x16x16_1rhs_f64", 1e6, [1, 2, 3]) is None
    assert bench.counter_traffic("dslash_f64", "24x24x24x48_32rhs_bf16", 1e6, [1, 2, 3]) is None
    src.write_text("// kernel, edited\n")
    assert bench.counter_traffic("coarse_gcr", "24x24x24x48_32rhs_bf16", 1e6, [1, 2, 3]) is None


def test_traffic_lookup_compares_the_tuning_entries_it_names(bench, tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("// kernel\n")
    _write_traffic(str(tmp_path), "dslash_f32", "24x24x24x48_32rhs_bf16", {"f32x24": [5, 8], "f32x32": [5, 8]},
                   1.5, ["k.hip"])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    run = {"f32x24": [5, 8], "f32x32": [5, 8], "bf16x32": [2, 2], "coarse_apply": None}
    assert bench.counter_traffic("dslash_f32", "24x24x24x48_32rhs_bf16", 2e6, run) == pytest.approx(3e6)
    run["bf16x32"] = [3, 1]  # another kernel's form: irrelevant
    assert bench.counter_traffic("dslash_f32", "24x24x24x48_32rhs_bf16", 2e6, run) == pytest.approx(3e6)
    run["f32x32"] = [9, 4]
    assert bench.counter_traffic("dslash_f32", "24x24x24x48_32rhs_bf16", 2e6, run) is None


def test_pinned_tuning_covers_the_default_step(bench):
    a = bench.parse([])
    pins = bench.PINNED_TUNING[(tuple(a.dims), a.nrhs)]
    assert set(pins) == {("f32", 24), ("f32", 32), ("bf16", 32)}
    for form, group in pins.values():
        assert 0 <= form <= 9 and 1 <= group <= 64


def test_committed_traffic_entries_are_well_formed(bench):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path) as fh:
        t = json.load(fh)
    for key, entries in t["entries"].items():
        kernel, workload = key.split("@")
        for e in entries:
            assert 0.3 < e["measured_over_algorithmic"] < 6.0, key
            assert abs(e["fetch_bytes_over_alg"] + e["write_bytes_over_alg"] - e["measured_over_algorithmic"]) < 1e-9
            for f in e["source_files"]:
                assert os.path.exists(os.path.join(ROOT, f)), f
            assert e["command"].startswith("rocprofv3")


def test_default_workload_and_single_gpu(bench, capsys):
    a = bench.parse([])
    assert tuple(a.dims) == (24, 24, 24, 48) and a.nrhs == 32 and a.nv == 24
    assert a.eps == 0.45 and a.delta == 0.005 and a.mg_prec == "bf16" and a.setup_iters == 200
    assert a.levels == 3 and a.nv2 == 16 and a.coarse_tol == 0.3 and a.setup_iters2 == 25
    assert a.restart == 6 and bench.parse(["--nrhs", "1"]).restart == 50 and bench.parse(["--nrhs", "8"]).restart == 12
    one = bench.parse(["--nrhs", "1", "--dims", "16", "16", "16", "16"])
    assert one.levels == 2 and one.coarse_tol == 0.1 and one.setup_iters == 50
    with pytest.raises(SystemExit) as e:
        bench.main(["--gpus", "2"])
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().out


def test_2d_mode_defaults():
    import bench
    a = bench.parse(["--qed2d"])
    assert a.qed2d and a.qed2d_deltas == [0.1, 0.03, 0.01, 0.003]
    assert a.qed2d_setup_iters == 300 and a.qed2d_rhs == 1
    # the 2d workload's stored critical mass is there for the benchmark to read
    import json
    import os
    with open(os.path.join(os.path.dirname(bench.__file__), "tests", "golden", "mcrit_2d.json")) as fh:
        e = json.load(fh)["128x128_beta6.0_seed7000"]
    assert e["dims"] == [128, 128] and -0.1 < e["m_crit"] < -0.05

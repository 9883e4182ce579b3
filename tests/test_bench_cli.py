"""bench.py's contract on the CPU: it measures one GPU only, and counter-measured
traffic enters its JSON line only when it was taken on the current kernel
source."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_multi_gpu_request_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


def test_traffic_is_used_only_for_the_current_source(tmp_path, monkeypatch):
    bench = load_bench()
    os.makedirs(tmp_path / "profiles")
    os.symlink(os.path.join(ROOT, "paper_2303_04934_amd"), tmp_path / "paper_2303_04934_amd")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    name = "traffic_%s_%s.json" % (bench.KERNEL_SHORT[2], "some_workload")
    path = tmp_path / "profiles" / name
    assert bench.load_traffic("some_workload", 2) is None  # no file
    path.write_text(json.dumps({"source_hash": bench.source_hash(), "bytes_per_launch": 1234.0}))
    assert bench.load_traffic("some_workload", 2) == 1234.0
    path.write_text(json.dumps({"source_hash": "0" * 16, "bytes_per_launch": 1234.0}))
    assert bench.load_traffic("some_workload", 2) is None  # taken on other kernels
    path.write_text("not json")
    assert bench.load_traffic("some_workload", 2) is None


def test_source_hash_covers_the_kernel_sources():
    bench = load_bench()
    h = bench.source_hash()
    assert len(h) == 16 and h == bench.source_hash()


def test_kernel_names_follow_the_search_mode():
    bench = load_bench()
    assert bench.kernel_name(1, "scc", 1) == "hipscc::k_expand<2, 1>"
    assert bench.kernel_name(1, "scc", 0) == "hipscc::k_expand<1, 1>"
    assert bench.kernel_name(4, "scc", 1) == "hipscc::k_expand_heavy<2>"
    assert bench.kernel_name(1, "scc", 1, True) == "hipscc::k_expand<5, 1>"
    assert bench.kernel_name(4, "scc", 1, True) == "hipscc::k_expand_heavy<5>"
    assert bench.kernel_name(1, "scc", 0, True) == "hipscc::k_expand<1, 1>"
    o = type("O", (), {"first_slot": 1, "packed": -1})()
    assert bench.packed_used(o, {"n": 100, "trimmed": 40}) and not bench.packed_used(o, {"n": 100, "trimmed": 60})
    assert bench.kernel_name(0, "cc") == "hipscc::k_expand<3, 1>"
    assert bench.kernel_name(6, "cc") == "hipscc::k_cc_union"
    assert bench.kernel_name(1, "le") == "hipscc::k_expand<4, 1>"
    assert len(bench.KERNEL_SHORT) == bench.NK == 7

"""Host-side behaviour of bench.py that needs no GPU: the one-GPU refusal,
the workload names and keys that select stored counters, and the kernel
source hash the counters are tied to."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_band_only_twin_has_its_own_workload_key():
    import bench
    from types import SimpleNamespace
    args = SimpleNamespace(config=2, S=20000, seed=0, n_jump=2)
    std = bench.make_instance(args)
    args.n_jump = 0
    band = bench.make_instance(args)
    assert band.nnz == std.nnz and band.S == std.S
    assert bench.workload_key(band) != bench.workload_key(std)
    # the stored counters apply only to the workload they were taken on
    assert bench.counter_traffic("bellman", bench.workload_key(band)) is None


def test_stored_counters_apply_only_to_their_sources(tmp_path, monkeypatch):
    import glob
    import bench
    files = sorted(glob.glob(bench.COUNTERS_GLOB))
    assert files, "no committed counter summaries"
    with open(files[0]) as f:
        d = json.load(f)
    assert d["calibration"]["fetch_factor"] > 0 and d["calibration"]["write_factor"] > 0
    # a copy of the counters taken on other kernel sources is ignored
    d["source_sha"] = "0" * 64
    (tmp_path / "counters_x.json").write_text(json.dumps(d))
    monkeypatch.setattr(bench, "COUNTERS_GLOB", str(tmp_path / "counters_*.json"))
    assert bench.counter_traffic("bellman", d["workload"]) is None
    # the same file with the current sources applies
    d["source_sha"] = bench.kernel_source_sha()
    (tmp_path / "counters_x.json").write_text(json.dumps(d))
    assert bench.counter_traffic("bellman", d["workload"]) == d["kernels"]["bellman"]["traffic_bytes_per_launch"]

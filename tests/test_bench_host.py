"""Host-side logic of bench.py (no GPU): the one-GPU contract and the rule
that HBM traffic is reported only from counters taken on the current sort
kernels."""
import hashlib
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_follows_the_committed_counters():
    text = open(bench.counters_md("c2", "fp64")).read()
    m = re.search(r"scatter_traffic_bytes_per_launch=(\S+) .*source_sha256_16=([0-9a-f]+)", text)
    rb = int(re.search(r"record_bytes=(\d+)", text).group(1))
    cur = hashlib.sha256(open(bench.SORT_SRC, "rb").read()).hexdigest()[:16]
    got = bench.measured_traffic("c2", "fp64", rb)
    if cur == m.group(2):
        assert got == float(m.group(1))
    else:
        assert got is None
    # precisions or record formats without counters have none
    assert bench.measured_traffic("c2", "fp32", rb) is None
    assert bench.measured_traffic("c2", "fp64", rb + 2) is None
    assert bench.measured_traffic("c4", "fp64", rb) is None


def test_traffic_is_dropped_when_the_sort_source_changes(tmp_path, monkeypatch):
    changed = tmp_path / "sort.hip"
    changed.write_bytes(open(bench.SORT_SRC, "rb").read() + b"\n// edited\n")
    monkeypatch.setattr(bench, "SORT_SRC", str(changed))
    text = open(bench.counters_md("c2", "fp64")).read()
    rb = int(re.search(r"record_bytes=(\d+)", text).group(1))
    assert bench.measured_traffic("c2", "fp64", rb) is None


def test_host_threads_and_neumaier():
    assert 1 <= bench.host_threads() <= len(__import__("os").sched_getaffinity(0))
    vals = [1e16, 1.0, -1e16, 1.0]
    assert bench.neumaier(vals) == 2.0


def test_split_scope_states_partial_runs():
    import bench
    assert bench.split_scope(512, 512, 20).startswith("all 512 subsets")
    assert bench.split_scope(512, 4, 2).startswith("PARTIAL: the first 4 of the 512")

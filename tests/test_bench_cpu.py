"""Host logic of bench.py, on the CPU: the one-GPU refusal, the graph length
of the timed region, the stored-traffic lookup keyed by the kernel sources,
and the oracle baseline record (on a small member, briefly)."""
import json
import os
import subprocess
import sys

import pytest

import bench
from paper_1911_03386_amd import CH_F64, make_desc
from paper_1911_03386_amd.workloads import Workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""  # no JSON line


@pytest.mark.parametrize("steps,cap", [(20, 64), (10000, 64), (97, 64), (5, 64), (1, 64), (128, 64), (200, 32)])
def test_graph_len(steps, cap):
    g = bench.graph_len(steps, cap)
    assert 1 <= g <= min(cap, steps)
    divisors = [d for d in range(max(1, min(cap, steps) // 2), min(cap, steps) + 1) if steps % d == 0]
    if divisors:
        assert g == max(divisors)  # whole replays, as long as possible
    else:
        assert g == min(cap, steps)


def test_graph_len_examples():
    assert bench.graph_len(20, 64) == 20
    assert bench.graph_len(10000, 64) == 50
    assert bench.graph_len(97, 64) == 64  # prime: replays plus a direct remainder


def test_traffic_follows_the_kernel_sources(monkeypatch, tmp_path):
    stored = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    wl, kinds = next(iter(stored["workloads"].items()))
    kind, value = next(iter(kinds.items()))
    if stored["kernel_src_sha"] == bench.kernel_source_sha():
        assert bench.measured_traffic(wl, kind) == value
    assert bench.measured_traffic(wl, "no_such_pass") is None
    assert bench.measured_traffic("no_such_workload", kind) is None
    # other kernel sources: the stored figure no longer applies
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0" * 16)
    assert bench.measured_traffic(wl, kind) is None
    # no summary at all
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic(wl, kind) is None


def test_kernel_source_sha_is_stable():
    a, b = bench.kernel_source_sha(), bench.kernel_source_sha()
    assert a == b and len(a) == 16 and int(a, 16) >= 0


def test_cpu_baseline_record():
    d = make_desc((32, 24), 0.01, 1e-3, c0=0.1, noise=0.05, seed=3)
    wl = Workload("ch2d_32x24_fp64_probe", [d], CH_F64, 10)
    rec = bench.cpu_baseline(wl, 0.05)
    assert rec["kind"] == "oracle" and rec["unit"] == "GLUPS"
    assert rec["value"] > 0 and rec["single_thread"]["value"] > 0
    assert isinstance(rec["cores"], int) and rec["cores"] >= 1
    assert "32x24" in rec["sample"] and "steps" in rec["sample"]
    assert rec["cpu_model"]

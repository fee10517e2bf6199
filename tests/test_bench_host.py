"""Host-side accounting of bench.py (CPU): the algorithmic bytes behind the roofline line, the
lookup of the measured traffic in profiles/, and the one-GPU guard."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

from paper_2306_10379_amd import inputs as I
from paper_2306_10379_amd import profsum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_laplacian_nnz_closed_form():
    # 7 entries per row minus one per missing neighbour on each of the 6 faces: 7 N^3 - 6 N^2
    for N in (3, 8, 13):
        assert I.laplacian_3d(N).nnz == 7 * N ** 3 - 6 * N ** 2


def test_pass_bytes_at_the_benchmark_size():
    b = _bench()
    n, p, N = 128 ** 3, 64, 128
    nnz = 7 * N ** 3 - 6 * N ** 2
    blk = n * p * 8
    nb = b.pass_bytes(n, p, nnz, 8, fused=False)
    assert blk == 1 << 30
    assert nb["update"] == 6 * blk == 6_442_450_944     # X, P, Y, Z read; X, Y written
    # the retraction pass that also forms the next gradient: G_old read, G written as well
    assert b.pass_bytes(n, p, nnz, 8)["update"] == 8 * blk
    assert nb["grad"] == nb["dir"] == 4 * blk
    assert nb["gram"] == 3 * blk
    # CSR once (8-byte values, 4-byte indices, n + 1 row pointers), P once, Z once
    assert nb["spmm"] == nnz * 12 + 4 * (n + 1) + 2 * blk == 2_330_853_380


def test_measured_traffic_follows_the_profile_and_its_source_hash(monkeypatch):
    b = _bench()
    path = os.path.join(ROOT, "profiles", "traffic_laplace3d_128_p64_fp64.json")
    with open(path) as f:
        rec = json.load(f)
    if rec["source_hash"] != profsum.source_hash():
        pytest.skip("the committed profile predates the kernel sources in this tree")
    tag = "gsi::k_update_grad<double, 64"  # the iteration's retraction, fused with the gradient
    t = b.measured_traffic(tag, "traffic_laplace3d_128_p64_fp64.json")
    # it moves what it must: within 1% of its algorithmic bytes (8 blocks of 2^21 x 64 doubles)
    assert t is not None and abs(t / 8_589_934_592 - 1.0) < 0.01
    # a kernel that the profiled iterations do not launch has no entry
    assert b.measured_traffic("gsi::k_update<double, 64", "traffic_laplace3d_128_p64_fp64.json") is None
    # counters taken on other sources are not reported
    monkeypatch.setattr(profsum, "source_hash", lambda: "0" * 16)
    assert b.measured_traffic(tag, "traffic_laplace3d_128_p64_fp64.json") is None
    assert b.measured_traffic(tag, "no_such_profile.json") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    line = r.stdout.strip().splitlines()[-1]
    assert r.returncode == 2 and "one GPU" in json.loads(line)["error"]


def test_extra_legs_start_only_within_the_budget():
    b = _bench()
    # 25 headline solves of ~14 s and the CPU sample leave ~120 s of a 500 s budget
    assert b.leg_fits("hermitian", 14.0, 380.0, 500.0)
    assert not b.leg_fits("mixed", 14.0, 480.0, 500.0)
    assert b.leg_estimate("mixed", 10.0) == 3.2 * 10.0 + 5.0
    assert set(b.DEFAULT_LEGS) == set(b.LEG_COST) == set(b.LEG_KEY)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--legs", "nope"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "unknown leg" in r.stderr

"""Host-side parts of bench.py, checked without a GPU: the one-GPU guard, the algorithmic
FLOP-per-pair accounting behind the roofline figures, and the source check that keeps a
traffic record from being reported against kernels it was not measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no bench line


# FLOP convention: add/sub/mul 1, fma 2, transcendental 1.  r^2 in 2-D: 2 sub, mul, fma = 5;
# in 3-D: 3 sub, mul, 2 fma = 8.  Accumulation: fma + add = 3.
@pytest.mark.parametrize("dim,p,flop", [
    (2, 2.0, 5 + 1 + 3),       # rcp
    (2, 1.0, 5 + 1 + 3),       # rsq
    (2, 3.0, 5 + 3 + 3),       # rsq, 2 mul
    (2, 4.0, 5 + 2 + 3),       # rcp, mul
    (3, 2.5, 8 + 4 + 3),       # rsq, mul, sqrt, mul
    (2, 1.5, 5 + 3 + 3),       # log2, mul, exp2
    (3, 2.0, 8 + 1 + 3),
])
def test_forward_flop_per_pair(dim, p, flop):
    assert bench.fwd_flop_per_pair(dim, p) == flop


def test_adjoint_flop_per_pair():
    # 2-D p = 2: the fused sweep's 18 (query sweep 16 + the dz fma)
    assert bench.adjoint_flop_per_pair(2, 2.0) == bench.FLOP_PER_PAIR["bwd_fused"] == 18
    assert bench.FLOP_PER_PAIR["bwd_query"] + 2 == 18
    # general p: r^2 5, log2 + mul + exp2 3, mul (w), sub, mul (t), fma (P) 2, mul (u),
    # 2 fma (G) 4, fma (dz) 2 = 20
    assert bench.adjoint_flop_per_pair(2, 1.5) == 20


def test_traffic_record_needs_matching_sources(monkeypatch):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    rec = json.load(open(path))
    k = rec["kernels"]["bwd_fused"]
    assert k["bytes_per_launch"] == pytest.approx(k["fetch_bytes"] + k["write_bytes"])
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: rec["source_hash"])
    assert bench.load_traffic("bwd_fused") == k["bytes_per_launch"]
    # the sweep with the data-coordinate gradient is another kernel, with a record of its own
    kx = rec["kernels"]["bwd_fused_dx"]
    assert ", true, true, true, false," in kx["kernel"] and ", true, true, false, false," in k["kernel"]
    assert bench.load_traffic("bwd_fused_dx") == kx["bytes_per_launch"]
    assert bench.load_traffic("no_such_kernel") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.load_traffic("bwd_fused") is None


def test_source_hash_covers_the_kernel_sources():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    assert h == bench.kernel_source_hash()

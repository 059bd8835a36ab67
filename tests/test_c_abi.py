"""The boundary from plain C: tests/c/idw_c_client.c includes only include/idw.h and the HIP
runtime header, links libidw.so, and runs idw_forward + idw_backward on a point set read
from a file.  On the CPU the client must compile and link warning-free; on the GPU its
results are checked against the FP64 oracle (forward 1e-5 of the condition scale, the
gradients at their FP32 tolerances, exact hits bit-exact)."""
import importlib.util
import json
import os
import re
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location("idw_c_client_build", os.path.join(HERE, "c", "build.py"))
c_client = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(c_client)


def test_c_client_compiles_and_links_cleanly(tmp_path):
    out = str(tmp_path / "client")
    r = subprocess.run(c_client.command(out), stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    assert "warning" not in r.stdout
    assert os.path.exists(out)


def _write_input(path, x, z, q, g, p):
    n, dim = x.shape
    with open(path, "wb") as f:
        np.array([n, len(q)], dtype="<i8").tofile(f)
        np.array([dim, 0], dtype="<i4").tofile(f)
        np.array([p], dtype="<f8").tofile(f)
        for a in (x, z, q, g):
            np.ascontiguousarray(a, dtype="<f8").tofile(f)


@pytest.mark.gpu
def test_c_client_matches_oracle(tmp_path):
    exe = c_client.EXE
    assert os.path.exists(exe), "build the C client first (__graft_entry__.build())"
    r = np.random.default_rng(600)
    n, m, dim, p = 2500, 900, 2, 2.0
    x = r.random((n, dim)).astype(np.float32).astype(np.float64)
    z = r.normal(size=n).astype(np.float32).astype(np.float64)
    q = r.random((m, dim)).astype(np.float32).astype(np.float64)
    q[:5] = x[:5]                                          # exact hits
    g = r.normal(size=m).astype(np.float32).astype(np.float64)
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    _write_input(fin, x, z, q, g, p)
    print("c client n=2500 m=900", flush=True)
    res = subprocess.run([exe, fin, fout], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=120)
    assert res.returncode == 0, res.stdout
    o = np.fromfile(fout, dtype="<f8")
    Z, D, dz, dp, dq = o[:m], o[m:2 * m], o[2 * m:2 * m + n], o[2 * m + n], o[2 * m + n + 1:].reshape(m, dim)
    ref = oracle.forward(x, z, q, p)
    assert np.max(np.abs(Z - ref["Z"]) / ref["S"]) <= 1e-5
    np.testing.assert_array_equal(Z[:5], ref["Z"][:5].astype(np.float32).astype(np.float64))
    assert np.all(np.isinf(D[:5]))
    np.testing.assert_allclose(D[5:], ref["D"][5:], rtol=1e-5)
    rb = oracle.backward(x, z, q, p, g)
    assert np.max(np.abs(dz - rb["dz"]) / rb["dz_scale"]) <= 1e-5
    assert abs(dp - rb["dp"]) <= 1e-5 * rb["dp_cond"]
    assert np.max(np.max(np.abs(dq - rb["dq"]), axis=1) / np.maximum(rb["dq_cond"], 1e-300)) <= 1e-5


@pytest.mark.gpu
def test_c_client_batched_plan_takes_the_tuned_defaults():
    # A plan made from plain C with no configuration runs with the autotuned item length and
    # persistent workgroup count of the tuning table, compiled into the library.
    exe = c_client.EXE
    assert os.path.exists(exe), "build the C client first (__graft_entry__.build())"
    tune = json.load(open(os.path.join(os.path.dirname(HERE), "paper_1402_4986_amd", "tuning", "gfx950.json")))
    print("c client --batched-params", flush=True)
    res = subprocess.run([exe, "--batched-params"], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                         timeout=120)
    assert res.returncode == 0, res.stdout
    got = re.search(r"plan chunk=(\d+) workgroups=(\d+)", res.stdout)
    assert got, res.stdout
    assert (int(got.group(1)), int(got.group(2))) == (tune["batch_chunk"], tune["batch_workgroups"])

"""GPU parity of the per-pair Kahan FP32 variant (IDW_FP32_KAHAN) against the FP64 oracle
at the FP32 tolerance, and, on the 3-D mixture workload at full size, against the GPU FP64
path for every query."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import GTOL, TOL, gpu_forward, points, rand_case, scaled_err
from paper_1402_4986_amd import api, workloads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("layout", ["soa", "aos", "aoas", "hybrid", "soaos"])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("p", [1.0, 2.0, 2.5, 3.7])
def test_kahan_forward_matches_oracle(layout, dim, p):
    x, z, q = rand_case(500 + dim, 4100, 1500, dim)
    q[:6] = x[:6]                                         # exact hits
    q[6:9] = (x[10:13] + 2e-7).astype(np.float32)          # near-coincident
    print(f"case layout={layout} dim={dim} p={p}", flush=True)
    Z, D = gpu_forward(x, z, q, p, layout, "f32_kahan")
    ref = oracle.forward(x, z, q, p)
    assert np.max(scaled_err(Z, ref)) <= TOL["f32_kahan"]
    np.testing.assert_array_equal(Z[:6], ref["Z"][:6].astype(np.float32).astype(np.float64))
    assert np.all(np.isinf(D[:6]))


@pytest.mark.parametrize("split", [1, 7])
def test_kahan_leave_one_out_and_split(split):
    x, z, _ = rand_case(510, 6000, 1, 2)
    Z, _ = gpu_forward(x, z, x, 1.5, "aoas", "f32_kahan", exclude_self=True, split=split)
    ref = oracle.forward(x, z, x, 1.5, self_index=np.arange(len(x)))
    assert np.max(scaled_err(Z, ref)) <= TOL["f32_kahan"]


def test_kahan_backward_is_the_fp32_adjoint():
    x, z, q = rand_case(520, 2000, 700, 2)
    g = np.random.default_rng(521).normal(size=len(q)).astype(np.float32).astype(np.float64)
    d, qq = points(x, z, q, "hybrid", "f32_kahan")
    Z, D = api.forward(d, qq, 2.0, "f32_kahan")
    dz, dp, dq = api.backward(d, qq, 2.0, torch.tensor(g, dtype=torch.float32, device="cuda"), Z, D, "f32_kahan")
    torch.cuda.synchronize()
    ref = oracle.backward(x, z, q, 2.0, g)
    assert np.max(np.abs(dz.cpu().numpy() - ref["dz"]) / ref["dz_scale"]) <= GTOL["f32"]
    assert abs(float(dp) - ref["dp"]) <= GTOL["f32"] * ref["dp_cond"]
    e = np.max(np.abs(dq.cpu().numpy() - ref["dq"]), axis=1) / ref["dq_cond"]
    assert np.max(e) <= GTOL["f32"]


def test_full_size_mixture3d_kahan_vs_fp64_every_query():
    # 262,144 3-D mixture points, 1,048,576 queries with 1,024 exact hits, p = 2.5: the
    # Kahan FP32 path against the GPU FP64 path for every query, and against the oracle on
    # a sample and on every hit.
    cfg = workloads.WORKLOADS["mixture3d_p2.5_262k_1m"]
    x, z, q, hit_rows = workloads.mixture3d(cfg["n"], cfg["m"], cfg["hits"], "f32", cfg=cfg["cfg"])
    print("full-size mixture3d, Kahan", flush=True)
    Zk, _ = gpu_forward(x, z, q, 2.5, "aoas", "f32_kahan")
    Z64, _ = gpu_forward(x, z, q, 2.5, "aoas", "f64")
    rel = np.abs(Zk - Z64) / np.maximum(np.abs(Z64), 1e-3)
    assert np.max(rel) <= 1e-5
    ref_h = oracle.forward(x, z, q[hit_rows], 2.5)
    np.testing.assert_array_equal(Zk[hit_rows], ref_h["Z"].astype(np.float32).astype(np.float64))
    idx = np.sort(np.random.default_rng(530).choice(len(q), size=128, replace=False))
    ref = oracle.forward(x, z, q[idx], 2.5)
    assert np.max(scaled_err(Zk[idx], ref)) <= TOL["f32_kahan"]

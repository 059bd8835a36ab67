"""The largest point sets the boundary accepts (2^31 - 1 points, checked on the host), in the
FP32 sweep.  Inputs are generated on the device; results are checked where the oracle
cannot go through properties that hold at any size:
  * a constant field (z = 0.7) with a few distinct values placed at exactly hit points:
    every other query returns 0.7 within the FP32 tolerance (the few distinct points move
    it by about 3/n), and every exact hit returns its own value bit for bit, including
    hits on the first, the middle and the LAST data index (64-bit indexing at the top of
    the range);
  * the value gradients of each query sum to its upstream gradient (sum_j dz_j = sum_i g_i);
  * with many queries and few data points, sampled queries against the FP64 oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import TOL, scaled_err
from paper_1402_4986_amd import api

pytestmark = pytest.mark.gpu

NMAX = 2 ** 31 - 1


def _records(n, seed):
    gen = torch.Generator(device="cuda").manual_seed(seed)
    rec = torch.rand((n, 4), generator=gen, device="cuda", dtype=torch.float32)
    rec[:, 2] = 0.7
    rec[:, 3] = 0.0
    return rec


@pytest.mark.parametrize("p", [2.0, 8.0])
def test_max_data_count_forward_and_adjoint(p):
    # p = 8 runs the relative weights: the nearest-distance pass and the scaled sweeps.
    n, m = NMAX, 2048
    print(f"n={n} m={m} FP32 aoas p={p}", flush=True)
    data = _records(n, 900)
    hits = [0, n // 2, n - 1]
    vals = [1.25, -0.5, 2.0]
    for j, v in zip(hits, vals):
        data[j, 2] = v
    query = torch.zeros((m, 4), device="cuda", dtype=torch.float32)
    query[:, :2] = torch.rand((m, 2), generator=torch.Generator(device="cuda").manual_seed(901), device="cuda")
    for k, j in enumerate(hits):
        query[k, :2] = data[j, :2]
    d = api.Points([data], n, 2, "aoas")
    q = api.Points([query], m, 2, "aoas")
    Z, D = api.forward(d, q, p, "f32")
    torch.cuda.synchronize()
    Zh = Z.cpu().numpy()
    np.testing.assert_array_equal(Zh[:3], np.array(vals, dtype=np.float32))
    assert np.all(np.isinf(D[:3].cpu().numpy()))
    assert np.max(np.abs(Zh[3:] - 0.7)) <= 1e-5
    print("forward ok; adjoint", flush=True)
    g = torch.rand(m, device="cuda", dtype=torch.float32)
    dz, dp, dq = api.backward(d, q, p, g, Z, D, "f32")
    torch.cuda.synchronize()
    assert torch.isfinite(dp)
    tot = float(dz.double().sum())
    assert tot == pytest.approx(float(g.double().sum()), rel=1e-5)
    del data, query, Z, D, dz, dp, dq
    api._ws_cache.clear()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n,p", [(64, 2.0), (65536, 8.0)])
def test_max_query_count_forward(n, p):
    # p = 8 with 65,536 data points runs the relative weights with the grid's ring search
    # for every query's nearest distance: its grid-stride loops reach index 2^31 - 2.
    m = NMAX
    print(f"n={n} m={m} FP32 aoas p={p}", flush=True)
    rng = np.random.default_rng(910)
    x = rng.random((n, 2)).astype(np.float32)
    z = np.full(n, 0.7, dtype=np.float32)
    z[5] = 1.3
    data = torch.zeros((n, 4), device="cuda", dtype=torch.float32)
    data[:, :2] = torch.tensor(x, device="cuda")
    data[:, 2] = torch.tensor(z, device="cuda")
    query = torch.rand((m, 4), generator=torch.Generator(device="cuda").manual_seed(911), device="cuda",
                       dtype=torch.float32)
    query[:, 2:] = 0.0
    query[m - 1, :2] = data[5, :2]                    # exact hit at the last query index
    query[0, :2] = data[9, :2]                        # and at the first
    d = api.Points([data], n, 2, "aoas")
    q = api.Points([query], m, 2, "aoas")
    Z, D = api.forward(d, q, p, "f32")
    torch.cuda.synchronize()
    assert float(Z[m - 1]) == np.float32(1.3) and float(Z[0]) == np.float32(0.7)
    assert float(Z.min()) >= np.float32(0.7) - 1e-6 and float(Z.max()) <= np.float32(1.3) + 1e-6
    idx = np.unique(np.concatenate([rng.integers(0, m, size=4096), [1, m // 2, m - 2]]))
    qs = query[torch.tensor(idx, device="cuda"), :2].double().cpu().numpy()
    ref = oracle.forward(x.astype(np.float64), z.astype(np.float64), qs, p)
    got = Z[torch.tensor(idx, device="cuda")].double().cpu().numpy()
    assert np.max(scaled_err(got, ref)) <= TOL["f32"]
    del data, query, Z, D
    api._ws_cache.clear()
    torch.cuda.empty_cache()

"""The grid of the nearest-distance searches against brute force.

Small p (many near-coincidence candidates: the fixed-radius check) and large p (relative
weights: every query's nearest distance, the ring search) take the nearest distances
from a uniform grid over the data when 65,536 to 2^26 points are given.  Those distances
are computed with the brute-force kernels' arithmetic, so every output must equal the
brute-force run (idw_config.near_search = 1) bit for bit, forward and adjoint; the
oracle checks a sample of queries besides.  The workspace header shows which path ran:
its int slot 3 holds the number of candidates the grid took in the last candidate check
and slot 1 the number it handed back to the brute-force kernels (dense cells); slots 7 and
5 hold the same for the last ring search.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import GTOL, TOL, points, rand_case, scaled_err
from paper_1402_4986_amd import api

pytestmark = pytest.mark.gpu


def _hint(ws):
    torch.cuda.synchronize()
    return ws[256:292].view(torch.int32).cpu().numpy()


def _run(x, z, q, p, prec, near_search, layout="aoas", exclude_self=False, adjoint=True, g=None):
    d, qq = points(x, z, q, layout, prec)
    cfg = api._cfg(near_search=near_search)
    ws = api.workspace(d, qq, prec, cfg)
    Z, D = api.forward(d, qq, p, prec, exclude_self=exclude_self, ws=ws, near_search=near_search)
    hint_f = _hint(ws)
    out = {"Z": Z.cpu().numpy(), "D": D.cpu().numpy(), "hint_f": hint_f}
    if adjoint:
        t = torch.float32 if prec == "f32" else torch.float64
        gt = torch.as_tensor(g, dtype=t, device="cuda")
        dz, dp, dq = api.backward(d, qq, p, gt, Z, D, prec, exclude_self=exclude_self, ws=ws,
                                  near_search=near_search)
        out["hint_b"] = _hint(ws)
        out.update(dz=dz.cpu().numpy(), dp=float(dp), dq=dq.cpu().numpy())
    return out


def _same(a, b, keys=("Z", "D", "dz", "dp", "dq")):
    for k in keys:
        if k in a:
            np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def _g(seed, m, prec):
    g = np.random.default_rng(seed).normal(size=m)
    return g.astype(np.float32).astype(np.float64) if prec == "f32" else g


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("dim", [2, 3])
def test_small_p_candidate_check(prec, dim):
    # p = 0.7 with 200,000 points: nearly every query is a candidate.
    x, z, q = rand_case(1300 + dim, 200000, 6000, dim, prec)
    q[:5] = x[:5]                                    # exact hits
    q[5:9] = x[100:104] + 3e-8                       # within 1e-6 of the extent
    t = np.float32 if prec == "f32" else np.float64
    q = q.astype(t).astype(np.float64)
    g = _g(1301, len(q), prec)
    print(f"case prec={prec} dim={dim}", flush=True)
    a = _run(x, z, q, 0.7, prec, 0, g=g)
    b = _run(x, z, q, 0.7, prec, 1, g=g)
    assert a["hint_f"][3] > len(q) // 2, "the grid did not take the candidates"
    _same(a, b)
    sel = np.concatenate([np.arange(12), np.arange(12, len(q), 97)])
    ref = oracle.forward(x, z, q[sel], 0.7)
    assert np.max(scaled_err(a["Z"][sel].astype(np.float64), ref)) <= TOL[prec]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("p", [8.0, 30.0])
def test_large_p_ring_search(dim, p):
    x, z, q = rand_case(1310 + dim, 150000, 5000, dim)
    q[:3] = x[:3]
    q[3:6] = x[50:53] + 3e-8
    q[6:40] += 0.3                                   # outside the box: rings from an edge cell
    q = q.astype(np.float32).astype(np.float64)
    g = _g(1311, len(q), "f32")
    print(f"case dim={dim} p={p}", flush=True)
    a = _run(x, z, q, p, "f32", 0, g=g)
    b = _run(x, z, q, p, "f32", 1, g=g)
    _same(a, b)
    assert a["hint_f"][7] == len(q), "the ring search did not take every query"
    assert a["hint_f"][5] < len(q) // 10
    sel = np.concatenate([np.arange(50), np.arange(50, len(q), 101)])
    ref = oracle.forward(x, z, q[sel], p)
    assert np.max(scaled_err(a["Z"][sel].astype(np.float64), ref)) <= TOL["f32"]


def test_clustered_data_falls_back():
    # 90% of the points in 20 tight clusters (dense cells), the rest uniform; queries both
    # inside the clusters and in the empty space between them.
    r = np.random.default_rng(1320)
    n = 120000
    centres = r.uniform(0.1, 0.9, (20, 2))
    k = int(n * 0.9)
    xc = centres[r.integers(0, 20, k)] + r.normal(0, 2e-4, (k, 2))
    x = np.concatenate([xc, r.uniform(0, 1, (n - k, 2))]).astype(np.float32).astype(np.float64)
    z = (np.sin(3 * x[:, 0]) + r.normal(0, 0.1, n)).astype(np.float32).astype(np.float64)
    q = np.concatenate([x[r.integers(0, k, 2500)] + r.normal(0, 1e-4, (2500, 2)),
                        r.uniform(0, 1, (3500, 2))]).astype(np.float32).astype(np.float64)
    g = _g(1321, len(q), "f32")
    for p in (0.6, 9.0):
        print(f"case p={p}", flush=True)
        a = _run(x, z, q, p, "f32", 0, g=g)
        b = _run(x, z, q, p, "f32", 1, g=g)
        _same(a, b)
        grid, back = (3, 1) if p < 6 else (7, 5)
        assert a["hint_f"][grid] > 0
        assert a["hint_f"][back] > 0, "no query fell back"
        sel = np.arange(0, len(q), 53)
        ref = oracle.forward(x, z, q[sel], p)
        assert np.max(scaled_err(a["Z"][sel].astype(np.float64), ref)) <= TOL["f32"]


def test_duplicates_and_degenerate_box():
    # Data on one horizontal line (zero extent in y) with 3,000 copies of one point.
    r = np.random.default_rng(1330)
    n = 80000
    x = np.stack([r.uniform(0, 1, n), np.full(n, 0.25)], axis=1)
    x[:3000] = x[3000]
    x = x.astype(np.float32).astype(np.float64)
    z = r.normal(size=n).astype(np.float32).astype(np.float64)
    q = np.stack([r.uniform(0, 1, 3000), r.uniform(0.2, 0.3, 3000)], axis=1)
    q[:4] = x[3000:3004]
    q = q.astype(np.float32).astype(np.float64)
    g = _g(1331, len(q), "f32")
    for p in (0.5, 7.0):
        print(f"case p={p}", flush=True)
        a = _run(x, z, q, p, "f32", 0, layout="soa", g=g)
        b = _run(x, z, q, p, "f32", 1, layout="soa", g=g)
        _same(a, b)
        sel = np.concatenate([np.arange(8), np.arange(8, len(q), 61)])
        ref = oracle.forward(x, z, q[sel], p)
        assert np.max(scaled_err(a["Z"][sel].astype(np.float64), ref)) <= TOL["f32"]


@pytest.mark.parametrize("p", [0.8, 8.0])
def test_leave_one_out(p):
    x, z, _ = rand_case(1340, 70000, 1, 2)
    g = _g(1341, len(x), "f32")
    a = _run(x, z, x, p, "f32", 0, layout="hybrid", exclude_self=True, g=g)
    b = _run(x, z, x, p, "f32", 1, layout="hybrid", exclude_self=True, g=g)
    _same(a, b)
    idx = np.arange(0, len(x), 211)
    ref = oracle.forward(x, z, x[idx], p, self_index=idx)
    assert np.max(scaled_err(a["Z"][idx].astype(np.float64), ref)) <= TOL["f32"]


def test_small_p_adjoint_against_oracle():
    # The adjoint settles its candidates through the grid too; check it on sampled queries
    # (the upstream gradient is zero elsewhere, so the oracle needs only those).
    x, z, q = rand_case(1350, 100000, 5000, 2)
    q[:3] = x[:3]
    r = np.random.default_rng(1351)
    sel = np.sort(np.concatenate([[0, 1, 2], r.choice(np.arange(3, len(q)), 80, replace=False)]))
    g = np.zeros(len(q))
    g[sel] = r.normal(size=len(sel)).astype(np.float32)
    a = _run(x, z, q, 0.7, "f32", 0, g=g)
    assert a["hint_b"][3] > 0
    rb = oracle.backward(x, z, q[sel], 0.7, g[sel])
    assert np.max(np.abs(a["dz"] - rb["dz"]) / rb["dz_scale"]) <= GTOL["f32"]
    assert abs(a["dp"] - rb["dp"]) <= GTOL["f32"] * rb["dp_cond"]
    e = np.max(np.abs(a["dq"][sel] - rb["dq"]), axis=1) / np.maximum(rb["dq_cond"], 1e-300)
    assert np.max(e) <= GTOL["f32"]


def test_grid_inside_graph_replay():
    x, z, q = rand_case(1360, 90000, 6000, 2)
    q[:4] = x[:4]
    d, qq = points(x, z, q, "aoas", "f32")
    g = torch.as_tensor(_g(1361, len(q), "f32"), dtype=torch.float32, device="cuda")
    ws = api.workspace(d, qq, "f32")
    Z = torch.empty(len(q), dtype=torch.float32, device="cuda")
    D = torch.empty(len(q), dtype=torch.float64, device="cuda")
    for p in (0.7, 10.0):
        def step():
            api.forward(d, qq, p, "f32", out_z=Z, out_den=D, ws=ws)
            return api.backward(d, qq, p, g, Z, D, "f32", ws=ws)

        eager = [a.clone() for a in step()]
        eager_z = Z.clone()
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            step()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            outs = step()
        for rep in range(3):
            Z.fill_(float("nan"))
            for o in outs:
                o.fill_(float("nan"))
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            print(f"p={p} replay {rep}", flush=True)
            assert torch.equal(Z, eager_z)
            for a, b in zip(outs, eager):
                assert torch.equal(a, b)
        del graph

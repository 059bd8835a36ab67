"""The seeded workload generators follow their recipes: shapes, ranges, float32 rounding,
bit-exact hit copies, reproducibility, and record packing for every layout."""
import numpy as np
import pytest

from paper_1402_4986_amd import workloads


def test_plain2d_recipe_and_rounding():
    x, z, q, t = workloads.plain2d(4096, 2048, "f32", cfg=1)
    assert x.shape == (4096, 2) and z.shape == (4096,) and q.shape == (2048, 2) and t.shape == (2048,)
    for a in (x, z, q, t):
        np.testing.assert_array_equal(a, a.astype(np.float32).astype(np.float64))
    assert x.min() >= 0 and x.max() <= 1 and q.min() >= 0 and q.max() <= 1
    # z is the sin*cos field plus N(0, 0.01^2) noise
    resid = z - np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1])
    assert abs(np.std(resid) - 0.01) < 0.001
    x2, z2, q2, _ = workloads.plain2d(4096, 2048, "f32", cfg=1)
    np.testing.assert_array_equal(x, x2)
    np.testing.assert_array_equal(q, q2)


def test_mixture3d_hits_are_bit_exact_copies():
    x, z, q, hit_rows = workloads.mixture3d(20000, 30000, 1024, "f32", cfg=2)
    assert x.shape == (20000, 3) and q.shape == (30000, 3) and len(hit_rows) == 1024
    assert np.all((x >= 0) & (x <= 1))
    xs = {tuple(r) for r in x}
    assert all(tuple(q[i]) in xs for i in hit_rows)
    # the copies are of distinct data points
    assert len({tuple(q[i]) for i in hit_rows}) == 1024
    resid = z - np.exp(-np.sum((x - 0.5) ** 2, axis=1))
    assert abs(np.std(resid) - 0.01) < 0.002


def test_batched_recipe_ranges():
    insts = workloads.batched(count=64, cfg=4)
    assert len(insts) == 64
    for inst in insts:
        assert inst["dim"] in (2, 3) and inst["p"] in (1.0, 2.0, 3.0)
        n, m = len(inst["x"]), len(inst["q"])
        assert 1024 <= n <= 262144 and 1024 <= m <= 524288
    assert {i["dim"] for i in insts} == {2, 3} and {i["p"] for i in insts} == {1.0, 2.0, 3.0}


@pytest.mark.parametrize("layout", workloads.LAYOUTS)
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_packing_round_trips(layout, dim, dtype):
    r = np.random.default_rng(0)
    x = r.random((37, dim))
    z = r.random(37)
    arrs = workloads.pack_data(x, z, layout, dtype)
    t = np.float32 if dtype == "f32" else np.float64
    assert all(a.dtype == t for a in arrs)
    if layout == "soa":
        got_x, got_z = np.stack(arrs[:dim], 1), arrs[dim]
    elif layout == "aos":
        got_x, got_z = arrs[0][:, :dim], arrs[0][:, dim]
    elif layout == "aoas":
        assert arrs[0].shape == (37, 4)
        got_x, got_z = arrs[0][:, :dim], arrs[0][:, dim]
    elif layout == "hybrid":
        got_x, got_z = arrs[0], arrs[1]
    else:
        got_x, got_z = arrs[0][:, :dim], arrs[1][:, 0]
    np.testing.assert_array_equal(got_x, x.astype(t))
    np.testing.assert_array_equal(got_z, z.astype(t))
    qa = workloads.pack_query(x, layout, dtype)
    qx = np.stack(qa[:dim], 1) if layout == "soa" else qa[0][:, :dim]
    np.testing.assert_array_equal(qx, x.astype(t))

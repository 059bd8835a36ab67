"""Batched plan parity: each instance of one graph launch against idw_forward on its own
(bitwise, same single-chunk configuration) and against the FP64 oracle, graph replays
bitwise stable with eager work in between, and the full 64-instance workload sampled."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import TOL, scaled_err
from paper_1402_4986_amd import api, batched, workloads

pytestmark = pytest.mark.gpu


def _inst(x, z, q, dim, p, dev="cuda"):
    return dict(data=torch.tensor(workloads.pack_data(x, z, "aoas", "f32")[0], device=dev),
                query=torch.tensor(workloads.pack_query(q, "aoas", "f32")[0], device=dev),
                dim=dim, p=p, out_z=torch.empty(len(q), dtype=torch.float32, device=dev),
                out_den=torch.empty(len(q), dtype=torch.float64, device=dev))


def _small_instances():
    r = np.random.default_rng(40)
    out = []
    specs = [(2, 1.0, 3000, 1500), (3, 2.0, 1024, 5000), (2, 3.0, 700, 257), (3, 2.5, 5000, 1),
             (2, 2.0, 1, 64), (3, 1.7, 2047, 1025), (2, 2.0, 4096, 0), (2, 2.0, 9000, 3333)]
    for dim, p, n, m in specs:
        x = r.random((n, dim)).astype(np.float32).astype(np.float64)
        z = r.normal(size=n).astype(np.float32).astype(np.float64)
        q = r.random((m, dim)).astype(np.float32).astype(np.float64)
        if m >= 10 and n >= 10:
            q[:5] = x[:5]                      # exact hits: FP64 fix-up inside the graph
        out.append((x, z, q, dim, p))
    return out


def test_batched_matches_single_instance_and_oracle():
    cases = _small_instances()
    insts = [_inst(*c) for c in cases]
    plan = batched.BatchedPlan(insts, chunk=16384, tuning={})
    plan.run()
    torch.cuda.synchronize()
    for (x, z, q, dim, p), inst in zip(cases, insts):
        print(f"instance dim={dim} p={p} n={len(x)} m={len(q)}", flush=True)
        got = inst["out_z"].cpu().numpy().astype(np.float64)
        if len(q) == 0:
            continue
        d = api.Points([inst["data"]], len(x), dim, "aoas")
        qq = api.Points([inst["query"]], len(q), dim, "aoas")
        Zs, Ds = api.forward(d, qq, p, "f32", split=1)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got, Zs.cpu().numpy().astype(np.float64))
        np.testing.assert_array_equal(inst["out_den"].cpu().numpy(), Ds.cpu().numpy())
        ref = oracle.forward(x, z, q, p)
        assert np.max(scaled_err(got, ref)) <= TOL["f32"]
    plan.close()


def test_graph_replays_are_bitwise_stable():
    cases = _small_instances()
    insts = [_inst(*c) for c in cases]
    plan = batched.BatchedPlan(insts, chunk=2048, workgroups=64, tuning={})
    outs = []
    for rep in range(4):
        for inst in insts:
            inst["out_z"].fill_(float("nan"))
        plan.run()
        torch.cuda.synchronize()
        outs.append([inst["out_z"].cpu().clone() for inst in insts])
        # unrelated eager work between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        del junk
    for rep in range(1, 4):
        for a, b in zip(outs[0], outs[rep]):
            assert torch.equal(a, b)
    for (x, z, q, dim, p), o in zip(cases, outs[0]):
        if len(q):
            ref = oracle.forward(x, z, q, p)
            assert np.max(scaled_err(o.numpy().astype(np.float64), ref)) <= TOL["f32"]
    plan.close()


def test_full_batched_workload_sampled():
    # 64 instances: dim ~ U{2,3}, p ~ U{1,2,3}, n ~ logU[1024, 262144], m ~ logU[1024, 524288].
    insts_np = workloads.batched(count=64, cfg=4)
    insts = [_inst(i["x"], i["z"], i["q"], i["dim"], i["p"]) for i in insts_np]
    plan = batched.BatchedPlan(insts)
    plan.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(41)
    worst = 0.0
    for src, inst in zip(insts_np, insts):
        got = inst["out_z"].cpu().numpy().astype(np.float64)
        idx = rng.choice(len(src["q"]), size=min(64, len(src["q"])), replace=False)
        ref = oracle.forward(src["x"], src["z"], src["q"][idx], src["p"])
        worst = max(worst, float(np.max(scaled_err(got[idx], ref))))
        assert np.all(np.isfinite(got))
    assert worst <= TOL["f32"], worst
    plan.close()

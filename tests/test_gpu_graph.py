"""idw_forward and idw_backward under HIP graph capture: they launch kernels only (no
allocation, no memset node, no synchronisation), so a torch.cuda.CUDAGraph can record a
forward + adjoint step.  The graph is replayed several times with eager work and
synchronisations in between, and every replay must equal the eager result bit for bit
(exact hits included, so compaction and the FP64 fix-ups are inside the graph)."""
import numpy as np
import pytest
import torch

from gpu_helpers import points, rand_case
from paper_1402_4986_amd import api

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_forward_and_adjoint_replay_bitwise(prec):
    x, z, q = rand_case(700, 3000, 1200, 2, prec)
    q[:7] = x[:7]                                   # exact hits: FP64 fix-up inside the graph
    d, qq = points(x, z, q, "aoas", prec)
    t = torch.float32 if prec == "f32" else torch.float64
    g = torch.as_tensor(np.random.default_rng(701).normal(size=len(q)), dtype=t, device="cuda")
    ws = api.workspace(d, qq, prec, need_dx=True)
    Z = torch.empty(len(q), dtype=t, device="cuda")
    D = torch.empty(len(q), dtype=torch.float64, device="cuda")

    def step():
        api.forward(d, qq, 2.0, prec, out_z=Z, out_den=D, ws=ws)
        return api.backward(d, qq, 2.0, g, Z, D, prec, ws=ws, need_dx=True)

    eager = [a.clone() for a in step()]
    eager_z = Z.clone()
    torch.cuda.synchronize()

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()                                      # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        outs = step()
    for rep in range(3):
        Z.fill_(float("nan"))                       # eager work between replays
        for o in outs:
            o.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        print(f"replay {rep} prec={prec}", flush=True)
        assert torch.equal(Z, eager_z)
        for a, b in zip(outs, eager):
            assert torch.equal(a, b)
        assert torch.isfinite(junk)

"""Accuracy report: the error of every workload against the FP64 oracle (and of the FP32
path against the GPU FP64 path), as one JSON object per workload.

Errors are |Z - Z_ref| / S with S = sum w|z| / sum w (the summation condition scale; the
oracle reports it), and beside them the plain relative error |Z - Z_ref| / |Z_ref| on the
queries with |Z_ref| >= 0.1 max|z|; gradients relative to their condition sums (see tests/).  Run on the
MI355X machine:  python errors.py [--sample 512]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def _stats(e):
    import numpy as np
    e = np.asarray(e, dtype=np.float64)
    return {"max": float(e.max()), "p99": float(np.quantile(e, 0.99)), "median": float(np.median(e)), "count": int(e.size)}


def _plain(got, ref, z):
    """Plain relative error |Z - Z_oracle| / |Z_oracle| on the queries where |Z_oracle| is at
    least a tenth of max |z| (there the plain measure is well defined)."""
    import numpy as np
    keep = np.abs(ref["Z"]) >= 0.1 * np.max(np.abs(z))
    return _stats(np.abs(got[keep] - ref["Z"][keep]) / np.abs(ref["Z"][keep]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sample", type=int, default=512)
    args = ap.parse_args()
    import numpy as np
    import torch

    import oracle
    from paper_1402_4986_amd import api, batched, workloads

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(2024)

    def run(x, z, q, p, layout, prec):
        d = api.Points.from_arrays(workloads.pack_data(x, z, layout, prec), len(x), x.shape[1], layout, dev)
        qq = api.Points.from_arrays(workloads.pack_query(q, layout, prec), len(q), q.shape[1], layout, dev)
        Z, D = api.forward(d, qq, p, prec)
        torch.cuda.synchronize()
        return Z.cpu().numpy().astype(np.float64), D.cpu().numpy(), d, qq, Z, D

    out = {}
    # plain2d FP64 10K: every query
    c = workloads.WORKLOADS["plain2d_f64_10k"]
    x, z, q, _ = workloads.plain2d(c["n"], c["m"], "f64", cfg=c["cfg"])
    Z, *_ = run(x, z, q, 2.0, "aoas", "f64")
    ref = oracle.forward(x, z, q, 2.0)
    out["plain2d_f64_10k"] = {"fp64_vs_oracle": _stats(np.abs(Z - ref["Z"]) / ref["S"]),
                              "fp64_plain_rel_vs_oracle": _plain(Z, ref, z), "queries": "all"}
    print(json.dumps({"plain2d_f64_10k": out["plain2d_f64_10k"]}), flush=True)

    # plain2d FP32 1M: sampled queries, FP32 and FP64 paths
    c = workloads.WORKLOADS["plain2d_f32_1m"]
    x, z, q, _ = workloads.plain2d(c["n"], c["m"], "f32", cfg=c["cfg"])
    Z32, *_ = run(x, z, q, 2.0, "aoas", "f32")
    Zk, *_ = run(x, z, q, 2.0, "aoas", "f32_kahan")
    Z64, *_ = run(x, z, q, 2.0, "aoas", "f64")
    idx = np.sort(rng.choice(len(q), size=args.sample, replace=False))
    ref = oracle.forward(x, z, q[idx], 2.0)
    out["plain2d_f32_1m"] = {"fp32_vs_oracle": _stats(np.abs(Z32[idx] - ref["Z"]) / ref["S"]),
                             "fp32_kahan_vs_oracle": _stats(np.abs(Zk[idx] - ref["Z"]) / ref["S"]),
                             "fp64_vs_oracle": _stats(np.abs(Z64[idx] - ref["Z"]) / ref["S"]),
                             "fp32_plain_rel_vs_oracle": _plain(Z32[idx], ref, z),
                             "fp32_kahan_plain_rel_vs_oracle": _plain(Zk[idx], ref, z),
                             "fp64_plain_rel_vs_oracle": _plain(Z64[idx], ref, z),
                             "fp32_vs_gpu_fp64_all_queries": _stats(np.abs(Z32 - Z64) / np.maximum(np.abs(Z64), 1e-30)),
                             "fp32_kahan_vs_gpu_fp64_all_queries": _stats(np.abs(Zk - Z64) / np.maximum(np.abs(Z64), 1e-30)),
                             "queries": f"{args.sample} sampled"}
    print(json.dumps({"plain2d_f32_1m": out["plain2d_f32_1m"]}), flush=True)

    # mixture3d p = 2.5: FP32 path against the GPU FP64 path per query (all), oracle on
    # samples and on every exact hit
    c = workloads.WORKLOADS["mixture3d_p2.5_262k_1m"]
    x, z, q, hits = workloads.mixture3d(c["n"], c["m"], c["hits"], "f32", cfg=c["cfg"])
    Z32, *_ = run(x, z, q, 2.5, "aoas", "f32")
    Zk, *_ = run(x, z, q, 2.5, "aoas", "f32_kahan")
    Z64, *_ = run(x, z, q, 2.5, "aoas", "f64")
    idx = np.sort(rng.choice(len(q), size=args.sample, replace=False))
    ref = oracle.forward(x, z, q[idx], 2.5)
    refh = oracle.forward(x, z, q[hits], 2.5)
    out["mixture3d_p2.5_262k_1m"] = {
        "fp32_vs_gpu_fp64_all_queries": _stats(np.abs(Z32 - Z64) / np.maximum(np.abs(Z64), 1e-30)),
        "fp32_kahan_vs_gpu_fp64_all_queries": _stats(np.abs(Zk - Z64) / np.maximum(np.abs(Z64), 1e-30)),
        "fp32_vs_oracle": _stats(np.abs(Z32[idx] - ref["Z"]) / ref["S"]),
        "fp32_kahan_vs_oracle": _stats(np.abs(Zk[idx] - ref["Z"]) / ref["S"]),
        "fp64_vs_oracle": _stats(np.abs(Z64[idx] - ref["Z"]) / ref["S"]),
        "fp32_plain_rel_vs_oracle": _plain(Z32[idx], ref, z),
        "fp32_kahan_plain_rel_vs_oracle": _plain(Zk[idx], ref, z),
        "fp64_plain_rel_vs_oracle": _plain(Z64[idx], ref, z),
        "exact_hits_bit_exact_fp32": bool(np.all(Z32[hits] == refh["Z"].astype(np.float32))),
        "exact_hits_bit_exact_fp64": bool(np.all(Z64[hits] == refh["Z"])),
        "queries": f"{args.sample} sampled + {len(hits)} hits"}
    print(json.dumps({"mixture3d": out["mixture3d_p2.5_262k_1m"]}), flush=True)

    # gradient workload: dq per sampled query at full size; dz, dp and dx of a full-size
    # launch whose upstream gradient is non-zero on the sample only
    c = workloads.WORKLOADS["plain2d_grad_f32_128k"]
    x, z, q, t = workloads.plain2d(c["n"], c["m"], "f32", cfg=c["cfg"])
    p = c["p"]
    Zh, _, d, qq, Z, D = run(x, z, q, p, "hybrid", "f32")
    g = ((2.0 / len(q)) * (Zh - t)).astype(np.float32).astype(np.float64)
    dz, dp, dq = api.backward(d, qq, p, torch.tensor(g, dtype=torch.float32, device=dev), Z, D, "f32")
    torch.cuda.synchronize()
    idx = np.sort(rng.choice(len(q), size=args.sample, replace=False))
    rb = oracle.backward(x, z, q[idx], p, g[idx])
    eq = np.max(np.abs(dq.cpu().numpy()[idx] - rb["dq"]), axis=1) / rb["dq_cond"]
    # dz, dp and dx of the full-size launch with the upstream gradient kept on the sample
    gs = np.zeros(len(q))
    gs[idx] = g[idx]
    a, b, _, dxs = api.backward(d, qq, p, torch.tensor(gs, dtype=torch.float32, device=dev), Z, D, "f32",
                                need_dx=True)
    torch.cuda.synchronize()
    ez = np.abs(a.cpu().numpy() - rb["dz"]) / rb["dz_scale"]
    rx = oracle.backward_x(x, z, q[idx], p, g[idx])
    ex = np.max(np.abs(dxs.cpu().numpy() - rx["dx"]), axis=1) / np.maximum(rx["dx_cond"], 1e-300)
    # the same dq errors relative to each row's own magnitude (what a user of dq sees; near a
    # data point the centred sum is small against its uncentred condition sum), and relative
    # to the centred absolute-term sum on the rows where that sum is well conditioned
    dqg = dq.cpu().numpy()[idx].astype(np.float64)
    err_row = np.max(np.abs(dqg - rb["dq"]), axis=1)
    own = err_row / np.maximum(np.max(np.abs(rb["dq"]), axis=1), 1e-300)
    well = rb["dq_cond"] <= 10.0 * rb["dq_scale"]
    dq_own = {
        "dq_rel_own_magnitude": _stats(own),
        "dq_vs_centred_scale_well_conditioned": _stats(err_row[well] / rb["dq_scale"][well]) if well.any() else None,
        "well_conditioned_rows": int(well.sum())}
    out["plain2d_grad_f32_128k"] = {"dq_vs_oracle": _stats(eq), "dz_vs_oracle": _stats(ez),
                                    "dx_vs_oracle": _stats(ex),
                                    "dp_vs_oracle": abs(float(b) - rb["dp"]) / rb["dp_cond"],
                                    "dp_rel_own_magnitude": abs(float(b) - rb["dp"]) / abs(rb["dp"]),
                                    "dq_own": dq_own,
                                    "queries": f"{args.sample} sampled"}
    print(json.dumps({"grad": out["plain2d_grad_f32_128k"]}), flush=True)

    # batched x64: 64 sampled queries per instance
    insts_np = workloads.batched(count=64, cfg=4)
    insts = []
    for i in insts_np:
        insts.append(dict(data=torch.tensor(workloads.pack_data(i["x"], i["z"], "aoas", "f32")[0], device=dev),
                          query=torch.tensor(workloads.pack_query(i["q"], "aoas", "f32")[0], device=dev),
                          dim=i["dim"], p=i["p"], out_z=torch.empty(len(i["q"]), dtype=torch.float32, device=dev)))
    plan = batched.BatchedPlan(insts)
    plan.run()
    torch.cuda.synchronize()
    errs, plain = [], []
    for src, inst in zip(insts_np, insts):
        k = rng.choice(len(src["q"]), size=min(64, len(src["q"])), replace=False)
        r = oracle.forward(src["x"], src["z"], src["q"][k], src["p"])
        got = inst["out_z"].cpu().numpy()[k].astype(np.float64)
        errs.append(np.abs(got - r["Z"]) / r["S"])
        keep = np.abs(r["Z"]) >= 0.1 * np.max(np.abs(src["z"]))
        plain.append(np.abs(got[keep] - r["Z"][keep]) / np.abs(r["Z"][keep]))
    plan.close()
    out["batched_x64"] = {"fp32_vs_oracle": _stats(np.concatenate(errs)),
                          "fp32_plain_rel_vs_oracle": _stats(np.concatenate(plain)),
                          "queries": "64 sampled per instance"}
    print(json.dumps({"batched": out["batched_x64"]}), flush=True)
    print(json.dumps({"errors": out}), flush=True)


if __name__ == "__main__":
    main()

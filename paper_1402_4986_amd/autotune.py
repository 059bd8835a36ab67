"""Autotuner for the batched plan's tile and occupancy parameters on the local GPU.

Grid-searches the data points per work item (batch_chunk) and the number of persistent
workgroups (batch_workgroups) on a seeded batched workload, timing graph replays with
HIP events, and writes the best pair (plus the whole table) to tuning/gfx950.json.  The
library's build compiles that pair in as the defaults of every batched plan (a plan whose
configuration leaves the fields at 0); rebuild after tuning.

Usage: python -m paper_1402_4986_amd.autotune [--count 64] [--out path] [--reps 3]
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np
import torch

from . import batched, workloads

CHUNKS = (4096, 8192, 16384, 32768, 65536)
WORKGROUPS = (256, 512, 768, 1024)


def make_instances(count: int, dev, seed_cfg: int = 4):
    out = []
    for inst in workloads.batched(count=count, cfg=seed_cfg):
        x, z, q, dim = inst["x"], inst["z"], inst["q"], inst["dim"]
        d = torch.tensor(workloads.pack_data(x, z, "aoas", "f32")[0], device=dev)
        qq = torch.tensor(workloads.pack_query(q, "aoas", "f32")[0], device=dev)
        out.append(dict(data=d, query=qq, dim=dim, p=inst["p"],
                        out_z=torch.empty(len(q), dtype=torch.float32, device=dev),
                        out_den=torch.empty(len(q), dtype=torch.float64, device=dev)))
    return out


def time_plan(plan: batched.BatchedPlan, reps: int) -> float:
    plan.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(reps):
        e0.record()
        plan.run()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=batched.TUNING_FILE)
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    insts = make_instances(args.count, dev)
    pairs = float(sum(i["data"].shape[0] * i["query"].shape[0] for i in insts))
    table = []
    for chunk in CHUNKS:
        for wg in WORKGROUPS:
            plan = batched.BatchedPlan(insts, chunk=chunk, workgroups=wg, tuning={})
            ms = time_plan(plan, args.reps)
            plan.close()
            table.append({"batch_chunk": chunk, "batch_workgroups": wg, "ms": round(ms, 3),
                          "pairs_per_s": pairs / (ms * 1e-3)})
            print(json.dumps(table[-1]), flush=True)
    best = min(table, key=lambda r: r["ms"])
    rec = {"device": torch.cuda.get_device_name(dev), "workload": f"batched x{args.count} (seeded, cfg 4 recipe)",
           "pairs": pairs, "batch_chunk": best["batch_chunk"], "batch_workgroups": best["batch_workgroups"],
           "best_ms": best["ms"], "table": table, "date": time.strftime("%Y-%m-%d")}
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({"best": best}), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark: Shepard IDW forward + adjoint at 1,048,576 x 1,048,576 FP32 (2-D, p = 2).

One step = idw_forward (Eq. 1 over all pairs) + idw_backward (dL/dz, dL/dp, dL/dq) for a
fixed synthetic upstream gradient, inputs resident in HBM.  Prints one JSON line:
pairs/s over the timed steps, the roofline of the dominant sweep kernel (algorithmic FLOP
per launch / its event-timed duration, against the FP32 vector peak), the FP32 error
against the FP64 oracle on sampled queries, and the oracle's own rate on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--layout aoas] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "query×data pairs/sec, IDW fwd+bwd at 1M×1M FP32; % FP32 VALU peak; err vs FP64"
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector: 256 CU x 2.4 GHz x 256 FLOP/clk/CU
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector

# Algorithmic FLOP per query x data pair, 2-D, p = 2 (add/sub/mul = 1, fma = 2,
# transcendental = 1; compensation and bookkeeping not counted):
#   forward     2 sub, mul + fma (r^2), rcp, fma (num), add (den)                  =  9
#   query sweep 2 sub, mul + fma, rcp, log2, sub (z - Z), mul (t = w c), fma (P),
#               mul (u = t / r^2, with 1/r^2 = w), 2 fma (G)                       = 16
#   data sweep  2 sub, mul + fma, rcp, fma (dz)                                    =  8
#   fused adjoint: the query sweep plus fma (dz) on the same weight                =  18
FLOP_PER_PAIR = {"fwd_sweep": 9, "bwd_query": 16, "bwd_data": 8, "bwd_fused": 18}
# With the data-coordinate gradient (--need-dx): the fused sweep adds mul (a u) and one fma
# per coordinate = 23; the separate data sweep computing dz and dx is 2 sub, mul + fma, rcp,
# mul (a w), add (dz), mul (f), sub + mul (z - Z), 2 fma = 15.
FLOP_PER_PAIR_DX = {"bwd_data": 15, "bwd_fused": 23}


def fwd_flop_per_pair(dim: int, p: float) -> int:
    """Algorithmic FLOP per pair of the forward sweep by weight class (same convention):
    r^2 is dim sub, mul and dim - 1 fma; the weight is rcp (p = 2), rsq (p = 1), rsq and two
    mul (p = 3), rcp and mul (p = 4), rsq, mul, sqrt and mul (p = 2.5), or log2, mul and exp2
    (general p); the accumulation is fma (num) and add (den)."""
    r2 = dim + 1 + 2 * (dim - 1)
    w = {1.0: 1, 2.0: 1, 3.0: 3, 4.0: 2, 2.5: 4}.get(float(p), 3)
    return r2 + w + 3


def adjoint_flop_per_pair(dim: int, p: float) -> int:
    """Algorithmic FLOP per pair of the fused adjoint (dz, dp, dq) at general p: r^2, log2,
    mul and exp2 (w / r^2), mul (w = (w / r^2) r^2), sub (z - Z), mul (t = w c), fma (P),
    mul (u = (w / r^2) c), dim fma (G), fma (dz).  At p = 2 it is FLOP_PER_PAIR["bwd_fused"]."""
    if float(p) == 2.0 and dim == 2:
        return FLOP_PER_PAIR["bwd_fused"]
    r2 = dim + 1 + 2 * (dim - 1)
    return r2 + 3 + 1 + 1 + 1 + 2 + 1 + 2 * dim + 2


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1402_4986_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hpp", ".hip", ".cpp")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str):
    """HBM traffic per launch measured with rocprofv3 counters (profiles/traffic.json),
    only if the kernel sources are unchanged since the measurement."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def cpu_baseline(x, z, q, g, sample: int, Zgpu, dzgpu_unused=None):
    """Times the FP64 oracle (forward + adjoint) on `sample` queries against all n data
    points, single thread; returns (record, oracle outputs for the error report)."""
    import numpy as np

    import oracle
    idx = np.sort(np.random.default_rng(99).choice(len(q), size=sample, replace=False))
    t0 = time.perf_counter()
    ref = oracle.forward(x, z, q[idx], 2.0)
    oracle.backward(x, z, q[idx], 2.0, g[idx])
    dt = time.perf_counter() - t0
    pairs = float(sample) * len(x)
    rec = {"value": pairs / dt, "unit": "pairs/s", "cores": 1, "kind": "oracle",
           "sample": f"{sample} seeded queries x all {len(x)} data points, forward + adjoint "
                     f"(dz, dp, dq), FP64, one thread, {dt:.1f} s"}
    return rec, idx, ref


_SLICE_INPUTS = {}


def _oracle_slice(idx):
    import oracle
    d = _SLICE_INPUTS
    oracle.forward(d["x"], d["z"], d["q"][idx], 2.0)
    oracle.backward(d["x"], d["z"], d["q"][idx], 2.0, d["g"][idx])
    return len(idx)


def cpu_baseline_all_cores(x, z, q, g, per_proc: int):
    """Times the same oracle on every usable host core (at most 16): one forked process per
    slice of seeded queries, each against all n data points.  Called before anything
    touches the GPU, so the workers inherit no device state."""
    import multiprocessing as mp

    import numpy as np

    import oracle
    oracle.build()
    nproc = max(1, min(16, len(os.sched_getaffinity(0))))
    idx = np.sort(np.random.default_rng(98).choice(len(q), size=nproc * per_proc, replace=False))
    _SLICE_INPUTS.update(x=x, z=z, q=q, g=g)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(nproc) as pool:
        pool.map(_oracle_slice, np.array_split(idx, nproc))
    dt = time.perf_counter() - t0
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    pairs = float(len(idx)) * len(x)
    return {"value": pairs / dt, "unit": "pairs/s", "cores": nproc, "kind": "oracle",
            "cpu": model,
            "sample": f"{len(idx)} seeded queries x all {len(x)} data points, forward + adjoint "
                      f"(dz, dp, dq), FP64, {nproc} processes, {dt:.1f} s wall"}


def _events_ms(fn, reps: int) -> float:
    """Mean duration of fn() over `reps` calls, bracketed by events on the current stream
    (one untimed call first)."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _sweep_ms(lib, fn, reps: int) -> float:
    """Mean duration of the forward sweep kernel over `reps` calls of fn (library events)."""
    import ctypes

    import torch

    from paper_1402_4986_amd import _lib
    fn()
    torch.cuda.synchronize()
    _lib.check(lib.idw_timing_enable(1))
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    ms, cnt = ctypes.c_double(), ctypes.c_int64()
    _lib.check(lib.idw_timing_read(_lib.T_FWD_SWEEP, ctypes.byref(ms), ctypes.byref(cnt)))
    _lib.check(lib.idw_timing_enable(0))
    return ms.value / max(cnt.value, 1)


def _rate(pairs: float, ms: float, flop: float) -> dict:
    tf = flop * pairs / (ms * 1e-3) / 1e12
    return {"ms": round(ms, 3), "pairs_per_s": pairs / (ms * 1e-3), "tflops": round(tf, 2),
            "frac_of_peak": round(tf / PEAK_FP32_TFLOPS, 4)}


def other_configs(lib, dev) -> dict:
    """Throughput of the other workloads: 10K x 10K FP64 (p = 2), the 3-D mixture (262,144 x
    1,048,576, p = 2.5: FP32, FP32-Kahan and FP64 forward), the gradient workload (131,072^2,
    p = 1.5: forward + adjoint step, and the leave-one-out fit of p), and the 64-instance
    batched graph.  frac_of_peak is against the FP32 vector peak for every entry (the FP64
    ones are also given against the FP64 peak)."""
    import numpy as np
    import torch

    from paper_1402_4986_amd import api, batched, workloads
    res = {}

    def pts(x, z, q, layout, prec):
        d = api.Points.from_arrays(workloads.pack_data(x, z, layout, prec), len(x), x.shape[1], layout, dev)
        qq = api.Points.from_arrays(workloads.pack_query(q, layout, prec), len(q), q.shape[1], layout, dev)
        return d, qq

    # 10,240 x 10,240, 2-D, FP64, p = 2
    c = workloads.WORKLOADS["plain2d_f64_10k"]
    x, z, q, _ = workloads.plain2d(c["n"], c["m"], "f64", cfg=c["cfg"])
    d, qq = pts(x, z, q, "aoas", "f64")
    ws = api.workspace(d, qq, "f64")
    Z64 = torch.empty(len(q), dtype=torch.float64, device=dev)
    D64 = torch.empty(len(q), dtype=torch.float64, device=dev)
    fwd = lambda: api.forward(d, qq, 2.0, "f64", out_z=Z64, out_den=D64, ws=ws)
    r = _rate(float(c["n"]) * c["m"], _events_ms(fwd, 10), fwd_flop_per_pair(2, 2.0))
    r["frac_of_fp64_peak"] = round(r["tflops"] / PEAK_FP64_TFLOPS, 4)
    res["plain2d_f64_10k"] = {"forward_f64": r, "note": "whole idw_forward call; 1.05e8 pairs"}
    del d, qq, ws, Z64, D64

    # 3-D mixture, p = 2.5
    c = workloads.WORKLOADS["mixture3d_p2.5_262k_1m"]
    x, z, q, _ = workloads.mixture3d(c["n"], c["m"], c["hits"], "f32", cfg=c["cfg"])
    pairs = float(c["n"]) * c["m"]
    fl = fwd_flop_per_pair(3, 2.5)
    entry = {"flop_per_pair": fl}
    for prec in ("f32", "f32_kahan", "f64"):
        d, qq = pts(x, z, q, "aoas", prec)
        ws = api.workspace(d, qq, prec)
        t = torch.float64 if prec == "f64" else torch.float32
        Zo = torch.empty(len(q), dtype=t, device=dev)
        Do = torch.empty(len(q), dtype=torch.float64, device=dev)
        fwd = lambda: api.forward(d, qq, 2.5, prec, out_z=Zo, out_den=Do, ws=ws)
        call = _rate(pairs, _events_ms(fwd, 3), fl)
        sweep = _rate(pairs, _sweep_ms(lib, fwd, 3), fl)
        if prec == "f64":
            call["frac_of_fp64_peak"] = round(call["tflops"] / PEAK_FP64_TFLOPS, 4)
            sweep["frac_of_fp64_peak"] = round(sweep["tflops"] / PEAK_FP64_TFLOPS, 4)
        entry[prec] = {"call": call, "sweep": sweep}
        del d, qq, ws, Zo, Do
    res["mixture3d_p2.5_262k_1m"] = entry

    # gradient workload: one forward + adjoint (dz, dp, dq) step, and the leave-one-out fit
    c = workloads.WORKLOADS["plain2d_grad_f32_128k"]
    x, z, q, tgt = workloads.plain2d(c["n"], c["m"], "f32", cfg=c["cfg"])
    pg = c["p"]
    d, qq = pts(x, z, q, "hybrid", "f32")
    ws = api.workspace(d, qq, "f32")
    Zg = torch.empty(len(q), dtype=torch.float32, device=dev)
    Dg = torch.empty(len(q), dtype=torch.float64, device=dev)
    tt = torch.tensor(tgt, dtype=torch.float32, device=dev)
    g = torch.empty(len(q), dtype=torch.float32, device=dev)

    def gstep():
        api.forward(d, qq, pg, "f32", out_z=Zg, out_den=Dg, ws=ws)
        torch.sub(Zg, tt, out=g).mul_(2.0 / len(q))
        api.backward(d, qq, pg, g, Zg, Dg, "f32", ws=ws)

    pairs = float(c["n"]) * c["m"]
    ms = _events_ms(gstep, 5)
    fl = fwd_flop_per_pair(2, pg) + adjoint_flop_per_pair(2, pg)
    step = _rate(pairs, ms, fl)
    step["flop_per_pair"] = fl
    X = torch.tensor(x, dtype=torch.float32, device=dev)
    zt = torch.tensor(z, dtype=torch.float32, device=dev)
    api.fit_p_loo(X, zt, p0=pg, steps=3)  # untimed: the optimiser's first-call set-up in torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p_fit, hist = api.fit_p_loo(X, zt, p0=pg, steps=50)
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t0
    res["plain2d_grad_f32_128k"] = {"step_fwd_bwd": step, "loo_fit": {
        "seconds": round(fit_s, 3), "evaluations": len(hist), "p0": pg, "p_fit": round(p_fit, 5),
        "loss0": hist[0][1], "loss_fit": min(h[1] for h in hist),
        "note": "L-BFGS on the leave-one-out loss of all 131,072 points, at most 50 evaluations"}}
    del d, qq, ws, X, zt

    # 64 batched instances, one graph launch
    insts_np = workloads.batched(count=64, cfg=4)
    insts, bpairs, bflop = [], 0.0, 0.0
    for i in insts_np:
        insts.append(dict(data=torch.tensor(workloads.pack_data(i["x"], i["z"], "aoas", "f32")[0], device=dev),
                          query=torch.tensor(workloads.pack_query(i["q"], "aoas", "f32")[0], device=dev),
                          dim=i["dim"], p=i["p"], out_z=torch.empty(len(i["q"]), dtype=torch.float32, device=dev)))
        pr = float(len(i["x"])) * len(i["q"])
        bpairs += pr
        bflop += pr * fwd_flop_per_pair(i["dim"], i["p"])
    plan = batched.BatchedPlan(insts)
    ms = _events_ms(plan.run, 5)
    chunk, wg = plan.params()
    plan.close()
    r = _rate(bpairs, ms, bflop / bpairs)
    r.update({"pairs": bpairs, "flop_per_pair_mean": round(bflop / bpairs, 3), "batch_chunk": chunk,
              "batch_workgroups": wg})
    res["batched_x64"] = {"graph_launch": r}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--layout", default="aoas", choices=["soa", "aos", "aoas", "hybrid", "soaos"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing leg")
    ap.add_argument("--no-layouts", action="store_true", help="skip the per-layout forward timings")
    ap.add_argument("--cpu-sample", type=int, default=200)
    ap.add_argument("--cpu-sample-per-core", type=int, default=24)
    ap.add_argument("--separate-adjoint", action="store_true",
                    help="run the adjoint as separate query- and data-direction sweeps")
    ap.add_argument("--need-dx", action="store_true",
                    help="also compute the gradient with respect to the data coordinates")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the timings of the other workloads (10K FP64, 3-D mixture, gradient, batched)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one device-to-device copy of 512 MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the sweep is measured on one GPU's share of "
              "the work; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1402_4986_amd import _lib, api, workloads

    cfg = workloads.WORKLOADS["plain2d_f32_1m"]
    n, m, p = cfg["n"], cfg["m"], cfg["p"]
    x, z, q, _ = workloads.plain2d(n, m, "f32", cfg=cfg["cfg"])
    g = np.random.default_rng(7).normal(size=m).astype(np.float32).astype(np.float64)
    all_cores = None
    if not args.no_cpu:  # before the GPU is initialised (the workers are forked)
        all_cores = cpu_baseline_all_cores(x, z, q, g, args.cpu_sample_per_core)

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    lib = _lib.load()
    dev = torch.device("cuda:0")

    def make(layout, prec="f32"):
        d = api.Points.from_arrays(workloads.pack_data(x, z, layout, prec), n, 2, layout, dev)
        qq = api.Points.from_arrays(workloads.pack_query(q, layout, prec), m, 2, layout, dev)
        return d, qq

    data, query = make(args.layout)
    gt = torch.tensor(g, dtype=torch.float32, device=dev)
    ws = api.workspace(data, query, "f32", need_dx=args.need_dx)
    if args.need_dx:
        FLOP_PER_PAIR.update(FLOP_PER_PAIR_DX)
    Z = torch.empty(m, dtype=torch.float32, device=dev)
    D = torch.empty(m, dtype=torch.float64, device=dev)

    def step():
        api.forward(data, query, p, "f32", out_z=Z, out_den=D, ws=ws)
        return api.backward(data, query, p, gt, Z, D, "f32", ws=ws, separate=args.separate_adjoint,
                            need_dx=args.need_dx)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    _lib.check(lib.idw_timing_enable(1))
    # events on the launch stream between steps give the per-step durations (median below)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(args.steps):
        grads = step()
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps))
    kt = {}
    import ctypes
    for name, which in (("fwd_sweep", _lib.T_FWD_SWEEP), ("bwd_query", _lib.T_BWD_QUERY),
                        ("bwd_data", _lib.T_BWD_DATA), ("bwd_fused", _lib.T_BWD_FUSED)):
        ms, cnt = ctypes.c_double(), ctypes.c_int64()
        _lib.check(lib.idw_timing_read(which, ctypes.byref(ms), ctypes.byref(cnt)))
        if cnt.value:
            kt[name] = ms.value / cnt.value
    _lib.check(lib.idw_timing_enable(0))

    ms_step = wall * 1e3 / args.steps
    pairs = float(n) * m
    kernels = {}
    for name, ms in kt.items():
        tf = FLOP_PER_PAIR[name] * pairs / (ms * 1e-3) / 1e12
        kernels[name] = {"ms": round(ms, 3), "tflops": round(tf, 2), "frac_of_peak": round(tf / PEAK_FP32_TFLOPS, 4)}
    dom = max(kt, key=kt.get)
    achieved = FLOP_PER_PAIR[dom] * pairs / (kt[dom] * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                # with dx the fused sweep is another kernel, with a record of its own
                "traffic": load_traffic(dom + "_dx" if args.need_dx and dom in FLOP_PER_PAIR_DX else dom)}
    total_flop = sum(FLOP_PER_PAIR[k] for k in kt) * pairs
    out = {"metric": METRIC, "value": pairs / (ms_step * 1e-3), "unit": "pairs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
           "median_ms_per_step": round(step_ms[len(step_ms) // 2], 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "plain2d_f32_1m", "n_data": n, "n_query": m, "dim": 2, "p": p,
                      "layout": args.layout, "precision": "fp32 sweep, fp64 ratio/fix-up",
                      "grads": "dz,dp,dq,dx" if args.need_dx else "dz,dp,dq"},
           "frac_fp32_peak_step": round(total_flop / (ms_step * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4),
           "kernels": kernels, "roofline": roofline}
    props = torch.cuda.get_device_properties(dev)
    out["device"] = {"name": props.name, "arch": getattr(props, "gcnArchName", None),
                     "compute_units": props.multi_processor_count}

    if args.calib_copy:
        src = torch.ones(128 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = src.numel() * 4
        del src, dst

    if not args.no_layouts:
        # The paper's layout study: the forward of the same 1M x 1M problem in every record
        # layout, single and double precision (one untimed call, then the mean of two).
        lay = {}
        Z64 = torch.empty(m, dtype=torch.float64, device=dev)
        for prec in ("f32", "f64"):
            lay[prec] = {}
            for layout in ("soa", "aos", "aoas", "hybrid", "soaos"):
                d2, q2 = (data, query) if (layout == args.layout and prec == "f32") else make(layout, prec)
                zo = Z if prec == "f32" else Z64
                api.forward(d2, q2, p, prec, out_z=zo, out_den=D, ws=ws)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(2):
                    api.forward(d2, q2, p, prec, out_z=zo, out_den=D, ws=ws)
                e1.record()
                torch.cuda.synchronize()
                lay[prec][layout] = round(e0.elapsed_time(e1) / 2, 3)
                del d2, q2
        # the FP64 adjoint (dz, dp, dq) of the same problem, aligned-AoS records
        d64, q64 = make("aoas", "f64")
        g64 = torch.tensor(g, dtype=torch.float64, device=dev)
        ws64 = api.workspace(d64, q64, "f64")
        api.forward(d64, q64, p, "f64", out_z=Z64, out_den=D, ws=ws64)
        api.backward(d64, q64, p, g64, Z64, D, "f64", ws=ws64)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(2):
            api.backward(d64, q64, p, g64, Z64, D, "f64", ws=ws64)
        e1.record()
        torch.cuda.synchronize()
        out["adjoint_ms_f64"] = round(e0.elapsed_time(e1) / 2, 3)
        del d64, q64, g64, Z64, ws64
        out["forward_ms_by_layout"] = lay
        # the per-pair Kahan variant of the FP32 forward, same records
        api.forward(data, query, p, "f32_kahan", out_z=Z, out_den=D, ws=ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(2):
            api.forward(data, query, p, "f32_kahan", out_z=Z, out_den=D, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        out["forward_ms_f32_kahan"] = round(e0.elapsed_time(e1) / 2, 3)
        # other exponents, forward and the full adjoint of the same records (one untimed call
        # each, then the mean of two): p = 0.5 and 1 (nearly every query is a near-coincidence
        # candidate, settled through the grid) and p = 8 and 32 (relative weights)
        sp, lp = {}, {}
        for pl in (0.5, 1.0, 8.0, 32.0):
            api.forward(data, query, pl, "f32", out_z=Z, out_den=D, ws=ws)
            api.backward(data, query, pl, gt, Z, D, "f32", ws=ws)
            torch.cuda.synchronize()
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record()
            for _ in range(2):
                api.forward(data, query, pl, "f32", out_z=Z, out_den=D, ws=ws)
            e[1].record()
            for _ in range(2):
                api.backward(data, query, pl, gt, Z, D, "f32", ws=ws)
            e[2].record()
            torch.cuda.synchronize()
            (lp if pl >= 6.0 else sp)[str(pl)] = {"forward": round(e[0].elapsed_time(e[1]) / 2, 3),
                                                  "adjoint": round(e[1].elapsed_time(e[2]) / 2, 3)}
        out["small_p_ms"] = sp
        out["large_p_ms"] = lp
        api.forward(data, query, p, "f32", out_z=Z, out_den=D, ws=ws)
        torch.cuda.synchronize()

    if not args.no_configs:
        out["configs"] = other_configs(lib, dev)
        api.forward(data, query, p, "f32", out_z=Z, out_den=D, ws=ws)
        torch.cuda.synchronize()

    if not args.no_cpu:
        Zh = Z.cpu().numpy().astype(np.float64)
        rec, idx, ref = cpu_baseline(x, z, q, g, args.cpu_sample, Zh)
        out["cpu_baseline"] = rec
        out["cpu_baseline_all_cores"] = all_cores
        err = np.abs(Zh[idx] - ref["Z"]) / ref["S"]
        keep = np.abs(ref["Z"]) >= 0.1 * np.max(np.abs(z))
        plain = np.abs(Zh[idx][keep] - ref["Z"][keep]) / np.abs(ref["Z"][keep])
        out["err_vs_fp64"] = {"max": float(err.max()), "median": float(np.median(err)),
                              "metric": "|Z - Z_oracle| / (sum w|z| / sum w)",
                              "plain_rel_max": float(plain.max()), "plain_rel_median": float(np.median(plain)),
                              "plain_rel_metric": "|Z - Z_oracle| / |Z_oracle| where |Z_oracle| >= 0.1 max|z|",
                              "plain_rel_count": int(keep.sum()), "sample": int(len(idx))}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark: tuples/s to R (FP64) of a two-relation join on one MI355X.

Workload: S(a, 16 FP64 cols) join T(a, 16 FP64 cols), 2,000,000 tuples each,
join key Zipf(1.1) over 1000 ids (about 1.9e11 join rows, never
materialised), seeded synthetic data.  A step is one full forward pass
(every kernel from the relation values to R) on inputs already resident in
HBM in plan order; the plan (keys only) is built once before timing, like the
paper's exclusion of sort time.

Prints one JSON line with the metric, the roofline of the dominant kernel
(from HIP events recorded by the library around each launch, on the stream
the kernels run on), the CPU oracle timed on a bounded sample of the same
workload, and a comparator: QR of the materialised join on the GPU
(torch.linalg.qr, FP64) on a subsample small enough to materialise, next to
this library on the same subsample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_forward(plan, vals, steps, warmup, profile=False):
    import torch
    for _ in range(warmup):
        plan.r_factor(vals)
    torch.cuda.synchronize()
    if profile:
        plan.profile_enable(64 * max(steps, 1))
        plan.profile_reset()
    t0 = time.perf_counter()
    for _ in range(steps):
        R = plan.r_factor(vals)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = plan.profile_read() if profile else None
    if profile:
        plan.profile_enable(0)
    return (t1 - t0) / steps, R, prof


def cpu_baseline(div: int):
    """The oracle (materialise + textbook Householder, one thread) on the
    config-2 shape divided by `div`."""
    import oracle
    import synth
    oracle.build()
    inst = synth.config2(div=div)
    t0 = time.perf_counter()
    A = oracle.join(inst)
    R, _ = oracle.householder_r(A)
    t1 = time.perf_counter()
    return inst.M / (t1 - t0), t1 - t0, inst.M, A.shape[0]


def comparator(F, div: int):
    """torch.linalg.qr (FP64, GPU) of the materialised join vs this library,
    both on the config-2 shape divided by `div`."""
    import torch
    import oracle
    import synth
    inst = synth.config2(div=div)
    plan = F.plan_from_instance(inst)
    vals = F.device_values(plan, inst)
    t_fig, R, _ = time_forward(plan, vals, 10, 3)
    t0 = time.perf_counter()
    A = torch.as_tensor(np.ascontiguousarray(oracle.join(inst))).cuda()
    torch.cuda.synchronize()
    t_mat = time.perf_counter() - t0
    for _ in range(2):
        Rq = torch.linalg.qr(A, mode="r")[1]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        Rq = torch.linalg.qr(A, mode="r")[1]
    torch.cuda.synchronize()
    t_qr = (time.perf_counter() - t0) / reps
    Rq = Rq * torch.sign(torch.diagonal(Rq))[:, None]
    Rr, _ = oracle.householder_r(oracle.join(inst))
    err_fig = float(np.linalg.norm(R.cpu().numpy() - Rr) / np.linalg.norm(Rr))
    err_qr = float(np.linalg.norm(Rq.cpu().numpy() - Rr) / np.linalg.norm(Rr))
    return {"workload": f"config-2 shape / {div}: 2 x {inst.rels[0].rows} tuples, "
                        f"{A.shape[0]} join rows x {A.shape[1]}",
            "figaro_ms": t_fig * 1e3, "materialized_qr_ms": t_qr * 1e3,
            "materialize_host_ms": t_mat * 1e3, "speedup": t_qr / t_fig,
            "figaro_rel_err": err_fig, "materialized_qr_rel_err": err_qr}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparator", action="store_true")
    ap.add_argument("--cpu-div", type=int, default=400)
    ap.add_argument("--comparator-div", type=int, default=200)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the library runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2204_00525_amd as F

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    log("generating config-2 inputs")
    inst = synth.config2()
    t0 = time.perf_counter()
    plan = F.plan_from_instance(inst)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    vals = F.device_values(plan, inst)
    torch.cuda.synchronize()
    log(f"plan built in {t_plan:.2f} s; join rows {plan.join_rows:.0f}")

    t_step, R, prof = time_forward(plan, vals, args.steps, args.warmup, profile=True)
    M = inst.M
    value = M / t_step
    log(f"forward {t_step * 1e3:.3f} ms/step, {value:.4e} tuples/s")

    # dominant kernel: the class with the largest total time
    dom = max(prof.items(), key=lambda kv: kv[1][0])
    name, (ms, launches, nbytes, flops) = dom
    avg_s = ms / 1e3 / max(launches, 1)
    bytes_per_launch = nbytes / max(launches, 1)
    achieved = bytes_per_launch / avg_s / 1e9
    roofline = {"kernel": name, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "avg_launch_us": avg_s * 1e6, "algorithmic_bytes_per_launch": bytes_per_launch,
                "fp64_tflops": flops / max(launches, 1) / avg_s / 1e12}
    kernels = {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps,
                   "GBps": (v[2] / (v[0] / 1e3) / 1e9) if v[0] > 0 else 0.0,
                   "TFps": (v[3] / (v[0] / 1e3) / 1e12) if v[0] > 0 else 0.0}
               for k, v in prof.items() if v[1] > 0}

    out = {"metric": "tuples/s to R (FP64), forward", "value": value, "unit": "tuples/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": t_step * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded, config-2 shape)",
           "config": {"workload": "two-relation join, 2x2,000,000 tuples, 1000 Zipf(1.1) keys, "
                                  "16+16 FP64 columns (n=32)",
                      "tuples": M, "join_rows": plan.join_rows, "n": plan.n,
                      "plan_s": t_plan},
           "roofline": roofline, "kernels": kernels}
    if not args.no_comparator:
        log("comparator: materialised QR on a subsample")
        out["comparator"] = comparator(F, args.comparator_div)
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on a subsample")
        v, secs, Ms, rows = cpu_baseline(args.cpu_div)
        out["cpu_baseline"] = {"value": v, "unit": "tuples/s", "cores": 1, "kind": "oracle",
                               "sample": f"config-2 shape / {args.cpu_div}: {Ms} tuples, {rows} join rows "
                                         f"materialised, textbook Householder ({secs:.1f} s)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

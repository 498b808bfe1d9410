"""Benchmark: tuples/s to R (FP64) of an acyclic join on one MI355X.

Headline workload (the `value` of the JSON line): S(a, 16 FP64 cols) join
T(a, 16 FP64 cols), 2,000,000 tuples each, join key Zipf(1.1) over 1000 ids
(about 1.9e11 join rows, never materialised), seeded synthetic data.  A step
is one full forward pass (every kernel from the relation values to R) on
inputs already resident in HBM in plan order; the plan (keys only) is built
once before timing, like the paper's exclusion of sort time, and its time is
reported separately.  The pass is timed eagerly (one launch per kernel from
the host) and as a HIP graph captured once and replayed; `value` uses the
faster of the two, and both are reported.

Also reported on the same line:
  * fwd_bwd: forward + hand-written backward of the loss
    L(R) = R_nn^2 / 2 + sum_i log R_ii on the same workload;
  * star: the key/foreign-key star join (fact table 10^7 rows with 4 foreign
    keys into four 10^5-row dimensions, 8 columns each, n = 40), forward and
    forward + backward of the same loss, next to torch.linalg.qr of its
    materialised join (10^7 x 40) on the GPU;
  * roofline: the dominant kernel, timed by HIP events that the library
    records around each launch on the stream it launches on; `traffic` is the
    calibrated HBM byte count from rocprofv3 counters stored under profiles/,
    or null when the kernel source changed since they were taken;
  * cpu_baseline: the CPU oracle timed on a bounded sample;
  * comparator: torch.linalg.qr of the materialised two-relation join on a
    subsample small enough to materialise, next to this library on it;
  * batched: many independent instances of the batched workload in one call
    (eager and as a replayed HIP graph), forward and forward + backward.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_heads_tails_two_relation_2x2M.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2204_00525_amd", "csrc", f)
                  for f in ("kernels.hip", "device_common.hpp", "internal.hpp")]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def loss_grad(R):
    """dL/dR for L(R) = R_nn^2 / 2 + sum_i log R_ii."""
    import torch
    d = torch.diagonal(R)
    dR = torch.diag(1.0 / d)
    dR[-1, -1] += R[-1, -1]
    return dR


def time_steps(step, steps, warmup):
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


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


def fwd_bwd_step(plan, vals):
    R = plan.r_factor(vals)
    return plan.r_backward(vals, R, loss_grad(R))


def cpu_baseline(div: int):
    """The oracle (index nested-loop join + textbook Householder, one
    thread) on the two-relation workload with every relation divided by
    `div`."""
    import oracle
    import synth
    oracle.build()
    inst = synth.config2(div=div)
    t0 = time.perf_counter()
    A = oracle.join(inst)
    R, _ = oracle.householder_r(A)
    t1 = time.perf_counter()
    return inst.M / (t1 - t0), t1 - t0, inst.M, A.shape[0]


def materialized_qr_ms(A, reps=3):
    import torch
    for _ in range(1):
        Rq = torch.linalg.qr(A, mode="r")[1]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        Rq = torch.linalg.qr(A, mode="r")[1]
    torch.cuda.synchronize()
    Rq = Rq * torch.sign(torch.diagonal(Rq))[:, None]
    return (time.perf_counter() - t0) / reps * 1e3, Rq


def materialized_qr_fwd_bwd_ms(A, reps=2):
    """Forward + backward of the loss R_nn^2/2 + sum log R_ii through the QR
    of a materialised join (FP64, GPU), R sign-normalised as this library
    returns it.  First through torch.linalg.qr's autograd; where that fails
    (its backward's batched triangular solve can fail to allocate on a
    10^7-row join), through the QR adjoint written out with torch products,
    dA = Q copyltu(R dR^T) R^-T, R^-1 formed as an n x n matrix.  Returns
    (ms, how, notes on what failed)."""
    import torch

    def autograd_step():
        X = A.detach().requires_grad_(True)
        R = torch.linalg.qr(X, mode="reduced")[1]
        R = R * torch.sign(torch.diagonal(R)).detach()[:, None]
        loss = 0.5 * R[-1, -1] ** 2 + torch.log(torch.diagonal(R)).sum()
        return torch.autograd.grad(loss, X)[0]

    def formula_step():
        Q, R = torch.linalg.qr(A, mode="reduced")
        sg = torch.sign(torch.diagonal(R))
        Q, R = Q * sg[None, :], R * sg[:, None]
        dR = loss_grad(R)
        M = R @ dR.t()
        B = torch.tril(M, -1) + torch.tril(M).t()        # copyltu(M)
        Rinv = torch.linalg.solve_triangular(R, torch.eye(R.shape[0], dtype=R.dtype, device=R.device), upper=True)
        return (Q @ B) @ Rinv.t()

    notes = []
    for how, step in (("autograd", autograd_step), ("adjoint formula", formula_step)):
        try:
            g = step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                g = step()
            torch.cuda.synchronize()
            del g
            torch.cuda.empty_cache()
            return (time.perf_counter() - t0) / reps * 1e3, how, "; ".join(notes) or None
        except RuntimeError as e:
            notes.append(f"{how} failed: {str(e).splitlines()[0][:160]}")
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
    return None, None, "; ".join(notes) or None


def comparator(F, div: int):
    """torch.linalg.qr (FP64, GPU) of the materialised two-relation join vs
    this library, both on the workload divided by `div`, both against the
    oracle."""
    import torch
    import oracle
    import synth
    inst = synth.config2(div=div)
    plan = F.plan_from_instance(inst)
    vals = F.device_values(plan, inst)
    t_fig, R, _ = time_forward(plan, vals, 10, 3)
    t0 = time.perf_counter()
    Ah = oracle.join(inst)
    A = torch.as_tensor(np.ascontiguousarray(Ah)).cuda()
    torch.cuda.synchronize()
    t_mat = time.perf_counter() - t0
    t_qr, Rq = materialized_qr_ms(A)
    Rr, _ = oracle.householder_r(Ah)
    err_fig = float(np.linalg.norm(R.cpu().numpy() - Rr) / np.linalg.norm(Rr))
    err_qr = float(np.linalg.norm(Rq.cpu().numpy() - Rr) / np.linalg.norm(Rr))
    return {"workload": f"two-relation join / {div}: 2 x {inst.rels[0].rows} tuples, "
                        f"{A.shape[0]} join rows x {A.shape[1]}",
            "figaro_ms": t_fig * 1e3, "materialized_qr_ms": t_qr,
            "materialize_host_ms": t_mat * 1e3, "speedup": t_qr / (t_fig * 1e3),
            "figaro_rel_err": err_fig, "materialized_qr_rel_err": err_qr,
            "reference": "CPU oracle (materialised join, textbook Householder)"}


def tree_choice(F, inst, R, t_fwd, steps, warmup):
    """Join-tree selection on the star join: the tree the chooser picks
    (host, from the keys) against the tree rooted at the fact table, whose
    join would be carried whole into the post-processing QR; both forward
    passes timed, R compared."""
    import torch
    import synth
    t0 = time.perf_counter()
    parents, cost = F.choose_join_tree(inst)
    t_choose = time.perf_counter() - t0
    fact = [i for i, rel in enumerate(inst.rels) if rel.name == "F"][0]
    fact_rooted = [fact if i != fact else -1 for i in range(inst.r)]
    bad = synth.Instance(inst.name, [synth.Rel(rel.key_attrs, rel.keys, rel.values, p, rel.name)
                                     for rel, p in zip(inst.rels, fact_rooted)], inst.meta)
    plan_b = F.plan_from_instance(bad)
    vals_b = F.device_values(plan_b, bad)
    t_bad, R_b, _ = time_forward(plan_b, vals_b, max(3, steps // 2), warmup)
    diff = float(torch.linalg.norm(R_b - R) / torch.linalg.norm(R))
    plan_b.close()
    del vals_b
    torch.cuda.empty_cache()
    return {"chosen_parents": parents, "chosen_score": cost, "choose_s": t_choose,
            "given_tree_is_chosen": parents == [rel.parent for rel in inst.rels],
            "fact_rooted_score": F.join_tree_cost(inst, fact_rooted),
            "chosen_fwd_ms": t_fwd * 1e3, "fact_rooted_fwd_ms": t_bad * 1e3,
            "speedup_chosen_over_fact_rooted": t_bad / t_fwd, "rel_diff_R": diff}


def plan_times(F, inst):
    """The plan built on the device from device keys (timed, keys uploaded
    beforehand) and, for comparison, the same plan built on the host from the
    same device keys."""
    import torch
    views = F.instance_views(inst)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = F.Plan(views)
    torch.cuda.synchronize()
    t_dev = time.perf_counter() - t0
    t0 = time.perf_counter()
    F.Plan(views, host_plan=True).close()
    torch.cuda.synchronize()
    t_host = time.perf_counter() - t0
    return plan, t_dev, t_host


def svd_pca(F, plan, vals, R, warmup, k=8):
    """From R to the SVD and PCA of the star join (section "From R to Q,
    SVD and PCA"): the SVD of R on the device, then the rank-k PCA
    projection A V[:, :k] of all 10^7 join rows and the rows of Q = A R^-1,
    enumerated without materialising A."""
    import torch

    def timed(fn, reps=3):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, out

    t_svd, (s, U, V) = timed(lambda: F.svd_of_r(R))
    t_pca, P = timed(lambda: plan.join_multiply(vals, V[:, :k]))
    Rinv = F.r_inverse(R)
    t_q, Q = timed(lambda: plan.join_multiply(vals, Rinv), reps=2)
    rows = int(plan.join_rows)
    ortho = float(torch.linalg.norm(Q.T @ Q - torch.eye(plan.n, dtype=torch.float64, device="cuda")))
    del Q, P
    torch.cuda.empty_cache()
    return {"svd_of_r_ms": t_svd * 1e3, "sigma_max": float(s[0]), "sigma_min": float(s[-1]),
            "pca_k": k, "pca_projection_ms": t_pca * 1e3, "pca_rows_per_s": rows / t_pca,
            "q_rows_ms": t_q * 1e3, "q_rows_per_s": rows / t_q, "q_orthogonality": ortho}


def star(F, steps, warmup, with_comparator, with_tree_choice=True):
    """Key/foreign-key star join: forward, forward+backward, comparator, join
    tree choice."""
    import torch
    import oracle
    import synth
    log("star join: generating inputs")
    inst = synth.config3()
    plan, t_plan, t_plan_host = plan_times(F, inst)
    vals = F.device_values(plan, inst)
    log(f"star join: plan {t_plan:.1f} s")
    t_fwd, R, _ = time_forward(plan, vals, steps, warmup)
    t_fb = time_steps(lambda: fwd_bwd_step(plan, vals), steps, warmup)
    out = {"workload": "star join: fact 10^7 rows x 8 cols with 4 uniform foreign keys into four "
                       "10^5-row dimensions x 8 cols; column scales 10^U[-3,3]; n = 40",
           "tuples": inst.M, "join_rows": plan.join_rows, "plan_s": t_plan, "plan_s_host_builder": t_plan_host,
           "fwd_ms": t_fwd * 1e3, "fwd_tuples_per_s": inst.M / t_fwd,
           "fwd_bwd_ms": t_fb * 1e3, "fwd_bwd_tuples_per_s": inst.M / t_fb}
    if with_tree_choice:
        out["tree_choice"] = tree_choice(F, inst, R, t_fwd, steps, warmup)
    out["svd_pca"] = svd_pca(F, plan, vals, R, warmup)
    if with_comparator:
        log("star join: materialising 10^7 x 40 for the comparator")
        t0 = time.perf_counter()
        Ah = oracle.join(inst)
        A = torch.as_tensor(Ah).cuda()       # Fortran-ordered host array -> (rows, n) view
        torch.cuda.synchronize()
        t_mat = time.perf_counter() - t0
        t_qr, Rq = materialized_qr_ms(A)
        log("star join: forward + backward through the materialised QR (autograd)")
        t_qr_fb, fb_how, fb_note = materialized_qr_fwd_bwd_ms(A)
        torch.cuda.empty_cache()
        G = A.t() @ A
        gn = torch.linalg.norm(G)

        def gram_res(Rx):
            return float(torch.linalg.norm(Rx.t() @ Rx - G) / gn)

        out["comparator"] = {
            "materialized_qr_ms": t_qr, "materialize_host_ms": t_mat * 1e3,
            "speedup_fwd": t_qr / (t_fwd * 1e3),
            "materialized_qr_fwd_bwd_ms": t_qr_fb, "materialized_fwd_bwd_method": fb_how,
            "materialized_fwd_bwd_note": fb_note,
            "speedup_fwd_bwd": (t_qr_fb / (t_fb * 1e3)) if t_qr_fb else None,
            "figaro_gram_residual": gram_res(R.contiguous()),
            "materialized_qr_gram_residual": gram_res(Rq),
            "rel_diff_R": float(torch.linalg.norm(R - Rq) / torch.linalg.norm(Rq)),
            "reference": "||R^T R - A^T A|| / ||A^T A|| with A^T A of the materialised join in FP64"}
        del G
        del A, Ah
        torch.cuda.empty_cache()
    plan.close()
    return out


# FiGaRo-MKL seconds for R of the Cartesian product of two m x n relations
# (experiments section, Exp. 1 synthetic table; a 2x24-core CPU server):
# rows m -> seconds for n = 64, 256, 1024, 4096 columns per relation.
PAPER_EXP1_S = {512: (0.10, 0.13, 0.17, 0.43), 1024: (0.10, 0.13, 0.30, 0.81), 2048: (0.12, 0.15, 0.31, 1.77),
                4096: (0.12, 0.14, 0.38, 4.65), 8192: (0.13, 0.18, 0.54, 5.85)}


def wide_grid(F, reps, warmup, cells=None):
    """The synthetic Cartesian-product grid of Exp. 1: S, T in R^{m x n}
    with entries uniform in [-3, 3), R of S x T (n <= 64 per relation: the
    register-tile path; wider: the blocked QR).  Every cell is timed eager
    and replayed from a captured HIP graph, and checked by the property that
    holds at any size: R^T R equals the Gram matrix of the product,
    [m S^T S, s^T t; t^T s, m T^T T] with s, t the column sums."""
    import torch
    out = []
    cols_list = (64, 256, 1024, 4096)
    if cells is None:
        cells = [(m, n) for m in sorted(PAPER_EXP1_S) for n in cols_list]
    for m, n in cells:
        if True:
            j = cols_list.index(n) if n in cols_list else -1
            g = torch.Generator(device="cuda")
            g.manual_seed(1000003 * m + n)
            S = torch.rand((n, m), generator=g, dtype=torch.float64, device="cuda") * 6.0 - 3.0
            T = torch.rand((n, m), generator=g, dtype=torch.float64, device="cuda") * 6.0 - 3.0
            views = [F._RelView([], torch.zeros((0, m), dtype=torch.int32, device="cuda"), n, -1),
                     F._RelView([], torch.zeros((0, m), dtype=torch.int32, device="cuda"), n, 0)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan = F.Plan(views)
            torch.cuda.synchronize()
            t_plan = time.perf_counter() - t0
            vals = [plan.to_plan_order(0, S), plan.to_plan_order(1, T)]
            t_eager, R, _ = time_forward(plan, vals, reps, warmup)
            gb = F.Batch([plan], streams=1)
            gs = torch.cuda.Stream()
            gout = [torch.empty((plan.n, plan.n), dtype=torch.float64, device="cuda")]
            with torch.cuda.stream(gs):
                Rg = gb.capture([vals], gout, gs)[0]
            gs.synchronize()
            gb.launch(gs)
            gs.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                gb.launch(gs)
            gs.synchronize()
            t_graph = (time.perf_counter() - t0) / reps
            same = bool(torch.equal(Rg, R))
            gb.close()
            # R^T R against the Gram matrix of S x T
            St, Tt = S.t().contiguous(), T.t().contiguous()
            G = torch.empty((2 * n, 2 * n), dtype=torch.float64, device="cuda")
            G[:n, :n] = m * (St.t() @ St)
            G[n:, n:] = m * (Tt.t() @ Tt)
            G[:n, n:] = torch.outer(St.sum(0), Tt.sum(0))
            G[n:, :n] = G[:n, n:].t()
            Rc = R.contiguous()
            res = float(torch.linalg.norm(Rc.t() @ Rc - G) / torch.linalg.norm(G))
            t = min(t_eager, t_graph)
            cell = {"rows": m, "cols_per_relation": n, "n": 2 * n, "plan_s": t_plan,
                    "ms_eager": t_eager * 1e3, "ms_graph": t_graph * 1e3, "graph_equals_eager": same,
                    "join_rows_per_s": m * m / t, "gram_residual": res,
                    "paper_figaro_mkl_s": PAPER_EXP1_S[m][j] if (m in PAPER_EXP1_S and j >= 0) else None}
            log(f"wide grid: m={m} n={n} {t * 1e3:.2f} ms gram_residual={res:.2e}")
            out.append(cell)
            plan.close()
            del S, T, St, Tt, G, vals, R, Rg, gout, Rc
            torch.cuda.empty_cache()
    return {"workload": "Cartesian product S x T, S and T m x n uniform in [-3, 3) (Exp. 1 synthetic grid)",
            "cells": out}


def batched(F, count, steps, warmup, cache_path=None):
    """The batched workload: instances 0..count-1 (seeds 5000+i), one plan
    each, run as one batch on 8 streams, eager and replayed from a captured
    HIP graph, next to the same plans run one after another on one stream.
    The plans take the option set the autotuner picked for their shape class
    (one representative tuned per class, kept in a JSON cache); the same
    batch with default options is timed beside them."""
    import torch
    import synth
    ids = list(range(count))
    log(f"batched: generating {count} instances")
    t0 = time.perf_counter()
    views, cvals, M = [], [], 0
    for i in ids:
        inst = synth.config5_instance(i)
        M += inst.M
        views.append(F.instance_views(inst))
        cvals.append([torch.as_tensor(np.ascontiguousarray(r.values)).cuda() for r in inst.rels])
        del inst
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    log("batched: tuning one instance per shape class")
    cache = F.TuningCache(cache_path)
    t0 = time.perf_counter()
    opts = [cache.options(v, c) for v, c in zip(views, cvals)]
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t0
    cache.save()
    log(f"batched: planning ({len(cache.entries)} shape classes)")
    t0 = time.perf_counter()
    plans = [F.Plan(v, **o) for v, o in zip(views, opts)]
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    plans_d = [F.Plan(v) for v in views]
    vals = [[p.to_plan_order(j, x) for j, x in enumerate(c)] for p, c in zip(plans, cvals)]
    del cvals
    torch.cuda.empty_cache()

    def graph_time(pl):
        b = F.Batch(pl, streams=8)
        s = torch.cuda.Stream()
        outs = [torch.empty((p.n, p.n), dtype=torch.float64, device="cuda") for p in pl]
        with torch.cuda.stream(s):
            b.capture(vals, outs, s)
        s.synchronize()
        for _ in range(warmup):
            b.launch(s)
        s.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            b.launch(s)
        s.synchronize()
        return (time.perf_counter() - t0) / steps, b

    log("batched: timing")
    t_graph, b = graph_time(plans)
    t_eager = time_steps(lambda: b.r(vals), steps, warmup)

    def fb():
        Rs = b.r(vals)
        return b.r_backward(vals, Rs, [loss_grad(R) for R in Rs])

    t_fb = time_steps(fb, max(2, steps // 2), 1)
    t_seq = time_steps(lambda: [p.r_factor(v) for p, v in zip(plans, vals)], max(2, steps // 2), 1)
    b.close()
    t_graph_d, bd = graph_time(plans_d)
    bd.close()
    out = {"workload": f"batched joins: instances 0..{count - 1} of the 512 (seeds 5000+i); 2-4 relations, "
                       "chains and stars, 1e3-1e6 tuples per relation, 4-32 columns per relation (n up to 128), "
                       "uniform or Zipf keys",
           "instances": count, "tuples": M, "generate_s": t_gen, "plan_s": t_plan,
           "tuning": {"shape_classes": len(cache.entries), "tune_s": t_tune,
                      "classes": cache.entries},
           "fwd_ms_graph": t_graph * 1e3, "fwd_ms_eager": t_eager * 1e3, "fwd_ms_one_stream": t_seq * 1e3,
           "fwd_ms_graph_default_options": t_graph_d * 1e3,
           "fwd_tuples_per_s_graph": M / t_graph, "fwd_bwd_ms_eager": t_fb * 1e3,
           "fwd_bwd_tuples_per_s": M / t_fb}
    for p in plans + plans_d:
        p.close()
    return out


def traffic_bytes(kernel: str):
    """Calibrated HBM bytes per launch of `kernel` from the stored rocprofv3
    counter summary, or None when missing or stale."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_class") != kernel or t.get("source_sha256") != kernel_source_hash():
        return None
    return float(t["hbm_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparator", action="store_true")
    ap.add_argument("--no-star", action="store_true")
    ap.add_argument("--no-tree-choice", action="store_true")
    ap.add_argument("--batched", type=int, default=512,
                    help="instances of the batched workload (the first N of 512; 0: skip)")
    ap.add_argument("--tuning-cache", default=None,
                    help="JSON file of the autotuner's choice per shape class (read and updated)")
    ap.add_argument("--no-wide-grid", action="store_true")
    ap.add_argument("--wide-grid-only", action="store_true",
                    help="run only the Cartesian-product grid (no headline line)")
    ap.add_argument("--wide-grid-cells", default=None,
                    help="comma-separated ROWSxCOLS cells of the grid (default: all 20)")
    ap.add_argument("--cpu-div", type=int, default=100)
    ap.add_argument("--comparator-div", type=int, default=200)
    ap.add_argument("--calibration-copy", action="store_true",
                    help="after timing, copy 256 MiB once (byte calibration for counter runs)")
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
    cells = None
    if args.wide_grid_cells:
        cells = [tuple(int(x) for x in c.split("x")) for c in args.wide_grid_cells.split(",")]
    if args.wide_grid_only:
        print(json.dumps({"wide_grid": wide_grid(F, 3, 1, cells=cells)}), flush=True)
        return
    log("generating the two-relation inputs")
    inst = synth.config2()
    plan, t_plan, t_plan_host = plan_times(F, inst)
    vals = F.device_values(plan, inst)
    torch.cuda.synchronize()
    log(f"plan built in {t_plan:.2f} s; join rows {plan.join_rows:.0f}")

    t_eager, R, prof = time_forward(plan, vals, args.steps, args.warmup, profile=True)
    # the same pass captured once into a HIP graph and replayed (no host
    # launch gaps between its kernels)
    gb = F.Batch([plan], streams=1)
    gs = torch.cuda.Stream()
    gout = [torch.empty((plan.n, plan.n), dtype=torch.float64, device="cuda")]
    with torch.cuda.stream(gs):
        Rg = gb.capture([vals], gout, gs)[0]
    gs.synchronize()
    for _ in range(args.warmup):
        gb.launch(gs)
    gs.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gb.launch(gs)
    gs.synchronize()
    t_graph = (time.perf_counter() - t0) / args.steps
    assert torch.equal(Rg, R), "graph replay differs from the eager pass"
    gb.close()
    t_step = min(t_eager, t_graph)
    M = inst.M
    value = M / t_step
    log(f"forward {t_eager * 1e3:.3f} ms/step eager, {t_graph * 1e3:.3f} ms/step graph, {value:.4e} tuples/s")
    t_fb = time_steps(lambda: fwd_bwd_step(plan, vals), args.steps, args.warmup)
    log(f"forward+backward {t_fb * 1e3:.3f} ms/step")
    if args.calibration_copy:
        a = torch.empty(256 * 1024 * 1024 // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # dominant kernel: the class with the largest total time
    name, (ms, launches, nbytes, flops) = max(prof.items(), key=lambda kv: kv[1][0])
    avg_s = ms / 1e3 / max(launches, 1)
    bytes_per_launch = nbytes / max(launches, 1)
    achieved = bytes_per_launch / avg_s / 1e9
    tb = traffic_bytes(name)
    roofline = {"kernel": name, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": tb,
                "avg_launch_us": avg_s * 1e6, "algorithmic_bytes_per_launch": bytes_per_launch,
                "fp64_tflops": flops / max(launches, 1) / avg_s / 1e12}
    kernels = {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps,
                   "GBps": (v[2] / (v[0] / 1e3) / 1e9) if v[0] > 0 else 0.0,
                   "TFps": (v[3] / (v[0] / 1e3) / 1e12) if v[0] > 0 else 0.0}
               for k, v in prof.items() if v[1] > 0}

    out = {"metric": "tuples/s to R (FP64), forward", "value": value, "unit": "tuples/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": t_step * 1e3, "ms_per_step_eager": t_eager * 1e3,
           "ms_per_step_graph": t_graph * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded)",
           "config": {"workload": "two-relation join, 2 x 2,000,000 tuples, 1000 Zipf(1.1) keys, "
                                  "16 + 16 FP64 columns (n = 32)",
                      "tuples": M, "join_rows": plan.join_rows, "n": plan.n, "plan_s": t_plan,
                      "plan_s_host_builder": t_plan_host},
           "fwd_bwd": {"ms_per_step": t_fb * 1e3, "tuples_per_s": M / t_fb,
                       "loss": "R_nn^2/2 + sum log R_ii"},
           "join_rows_per_s": plan.join_rows / t_step,
           "roofline": roofline, "kernels": kernels}
    plan.close()
    del vals
    torch.cuda.empty_cache()
    if not args.no_star:
        out["star"] = star(F, max(3, args.steps // 2), 2, not args.no_comparator, not args.no_tree_choice)
    if not args.no_wide_grid:
        out["wide_grid"] = wide_grid(F, 3, 1, cells=cells)
    if args.batched > 0:
        out["batched"] = batched(F, args.batched, max(3, args.steps // 4), 2, args.tuning_cache)
    if not args.no_comparator:
        log("comparator: materialised QR on a subsample")
        out["comparator"] = comparator(F, args.comparator_div)
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on a subsample")
        v, secs, Ms, rows = cpu_baseline(args.cpu_div)
        out["cpu_baseline"] = {"value": v, "unit": "tuples/s", "cores": 1, "kind": "oracle",
                               "host_cores": os.cpu_count(),
                               "sample": f"two-relation join / {args.cpu_div}: {Ms} tuples, {rows} join rows "
                                         f"materialised, textbook Householder ({secs:.1f} s), one thread "
                                         f"of the {os.cpu_count()} host cores"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

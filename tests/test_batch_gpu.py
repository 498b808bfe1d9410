"""Batched instances, HIP graph replay and the autotuner (needs an MI355X).

Every instance of a batch is checked against the same plan run alone
(bit for bit: the same kernels on the same workspace) and against the CPU
oracle at 1e-10 relative Frobenius error."""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import synth
from _parity import colscaled

pytestmark = pytest.mark.gpu

# small instances of the batched workload (seeds 5000+i), 2-4 relations,
# 22-57 columns, chains and stars, uniform and Zipf keys
INSTANCES = [15, 23, 27, 35, 58, 78, 79, 96]


def _relf(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _oracle_reference(oracle_lib, inst):
    """R from the oracle's extended-precision factorised Gram matrix (the
    join is never materialised; some of these joins have 10^8 rows), or the
    Gram matrix itself when the join is rank deficient."""
    try:
        R, _ = oracle_lib.factorized_r(inst)
        return R, None
    except np.linalg.LinAlgError:
        Ghi, Glo, _ = oracle_lib.factorized_gram(inst)
        return None, (Ghi, Glo)


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2204_00525_amd as F
    F.lib()
    return F


@pytest.fixture(scope="module")
def batch_setup(F):
    insts = [synth.config5_instance(i) for i in INSTANCES]
    plans = [F.plan_from_instance(inst) for inst in insts]
    vals = [F.device_values(p, inst) for p, inst in zip(plans, insts)]
    return insts, plans, vals


def test_batched_forward_matches_single_and_oracle(F, oracle_lib, batch_setup):
    import torch
    insts, plans, vals = batch_setup
    b = F.Batch(plans, streams=3)
    assert sorted({b.stream_of(i) for i in range(len(plans))}) == [0, 1, 2]
    Rb = [R.cpu().numpy() for R in b.r(vals)]
    torch.cuda.synchronize()
    for inst, p, v, R in zip(insts, plans, vals, Rb):
        print(f"[batch] {inst.name} n={p.n}", flush=True)
        Rs = p.r_factor(v).cpu().numpy()
        assert np.array_equal(R, Rs)
        ref = oracle_lib.r_of_join(inst)
        assert _relf(R, ref) <= 1e-10
        assert colscaled(R, ref) <= 1e-10
    b.close()


def test_graph_replays_match_eager(F, batch_setup):
    import torch
    insts, plans, vals = batch_setup
    b = F.Batch(plans, streams=4)
    eager = [R.cpu().numpy() for R in b.r(vals)]
    s = torch.cuda.Stream()
    outs = [torch.full((p.n, p.n), np.nan, dtype=torch.float64, device="cuda") for p in plans]
    with torch.cuda.stream(s):
        Rg = b.capture(vals, outs, s)
    s.synchronize()
    for rep in range(3):
        for o in outs:
            o.fill_(np.nan)                       # eager work between replays
        torch.cuda.synchronize()
        b.launch(s)
        s.synchronize()
        for R, E in zip(Rg, eager):
            assert np.array_equal(R.cpu().numpy(), E), f"replay {rep}"
    b.close()


def test_batched_backward_matches_single(F, batch_setup):
    import torch
    insts, plans, vals = batch_setup
    b = F.Batch(plans)
    Rs = b.r(vals)
    dRs = [torch.triu(torch.ones_like(R)) for R in Rs]
    gb = b.r_backward(vals, Rs, dRs)
    torch.cuda.synchronize()
    for p, v, R, dR, g in zip(plans, vals, Rs, dRs, gb):
        gs = p.r_backward(v, R, dR)
        for x, y in zip(g, gs):
            assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())
    b.close()


def test_duplicate_plan_is_rejected(F, batch_setup):
    insts, plans, vals = batch_setup
    with pytest.raises(F.FigaroError) as e:
        F.Batch([plans[0], plans[1], plans[0]])
    assert e.value.name == "EINVAL"


def test_batch_refuses_profiled_plans(F, batch_setup):
    """Per-launch timing of a plan is refused in batches (several streams),
    eager passes included; the batch runs again once timing is off."""
    insts, plans, vals = batch_setup
    b = F.Batch(plans[:3])
    plans[1].profile_enable(64)
    try:
        with pytest.raises(F.FigaroError) as e:
            b.r(vals[:3])
        assert e.value.name == "EINVAL"
    finally:
        plans[1].profile_enable(0)
    b.r(vals[:3])
    b.close()


@pytest.mark.parametrize("i", [15, 35, 96])
def test_autotuned_plan(F, oracle_lib, i):
    import torch
    inst = synth.config5_instance(i)
    rels = F.instance_views(inst)
    caller_vals = [torch.as_tensor(np.ascontiguousarray(r.values)).cuda() for r in inst.rels]
    p = F.Plan.tuned(rels, caller_vals, reps=2)
    opts, ms = p.tuning()
    assert opts["variant"] in (0, 2) and opts["waves_per_task"] in (512, 1024, 2048) and ms > 0
    R = p.r_factor(F.device_values(p, inst)).cpu().numpy()
    assert _relf(R, oracle_lib.r_of_join(inst)) <= 1e-10


@pytest.mark.timeout(1200)
def test_config5_sample_batched_against_oracle(F, oracle_lib):
    """The stratified sample of the batched workload (every topology, key
    distribution, relation count and column bucket) as one batch: each R
    bit for bit equal to its plan run alone, and within 1e-10 of the oracle
    (relative Frobenius and column-scaled)."""
    import torch
    ids = synth.config5_sample()
    print(f"[batch-sample] {len(ids)} instances: {ids}", flush=True)
    with ThreadPoolExecutor(8) as ex:     # the oracle's C code runs without the GIL
        insts = list(ex.map(synth.config5_instance, ids))
        refs = list(ex.map(lambda inst: _oracle_reference(oracle_lib, inst), insts))
    plans = [F.plan_from_instance(inst) for inst in insts]
    vals = [F.device_values(p, inst) for p, inst in zip(plans, insts)]
    b = F.Batch(plans, streams=8)
    Rb = [R.cpu().numpy() for R in b.r(vals)]
    torch.cuda.synchronize()
    worst = 0.0
    for inst, p, v, R, (Rref, gram) in zip(insts, plans, vals, Rb, refs):
        Rs = p.r_factor(v).cpu().numpy()
        assert np.array_equal(R, Rs), inst.name
        if Rref is None:
            err = oracle_lib.gram_relerr(R, *gram)
            print(f"[batch-sample] {inst.name} n={p.n} rank-deficient gram_relerr={err:.2e}", flush=True)
            assert err <= 1e-13, inst.name
            continue
        err, cerr = _relf(R, Rref), colscaled(R, Rref)
        worst = max(worst, err, cerr)
        print(f"[batch-sample] {inst.name} {inst.meta['topology']}/{inst.meta['dist']} r={inst.r} n={p.n} "
              f"M={inst.M} rel_err={err:.2e} colscaled={cerr:.2e}", flush=True)
        assert err <= 1e-10 and cerr <= 1e-10, inst.name
    print(f"[batch-sample] worst {worst:.2e}", flush=True)
    b.close()
    for p in plans:
        p.close()

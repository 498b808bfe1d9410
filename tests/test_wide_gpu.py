"""The wide regime: plans of more than 128 columns (needs an MI355X).

Above 128 columns the stack of the head/tail phase is reduced by the blocked
Householder QR (experiments section, the synthetic Cartesian products of up
to thousands of columns per relation; post-processing through a blocked
LAPACK-style QR).  R is checked against the oracle's R from the
extended-precision factorised Gram matrix (the join is never materialised)
at the same 1e-10 bar as the narrow path, relative Frobenius and
column-scaled; rank-deficient joins compare R^T R with A^T A.  Cases cover
both panel forms (one workgroup, per-column passes over many workgroups),
short-wide relations (fewer tails than columns), joins whose subtrees are
wider than 128 columns (the join's column tables on the device), the
accuracy study of Appendix A at more than 128 columns, determinism, graph
replay and the backward pass's refusal."""
import math
import sys

import numpy as np
import pytest

import synth
from _parity import colscaled, relf

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2204_00525_amd as F
    F.lib()
    return F


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_r(F, inst, **kw):
    import torch
    plan = F.plan_from_instance(inst, **kw)
    vals = F.device_values(plan, inst)
    R = plan.r_factor(vals)
    torch.cuda.synchronize()
    return R.cpu().numpy(), plan, vals


CASES = {
    # two wide regions of under 1024 tails each: one-workgroup panels
    "cartesian_100_100": lambda: synth.cartesian_uniform(31, 300, 100, 250, 100),
    # regions of 1999 and 1499 tails: per-column passes over many workgroups
    "cartesian_tall_96_64": lambda: synth.cartesian_uniform(32, 2000, 96, 1500, 64),
    # 256 + 256 columns, 1024 rows per relation (the smallest wide cell of
    # the paper's Cartesian grid at 2^10 rows)
    "cartesian_256_256": lambda: synth.cartesian_uniform(33, 1024, 256, 1024, 256),
    # a narrow relation (fused wave R's in the stack's lower part) beside a
    # wide one
    "cartesian_30_150": lambda: synth.cartesian_uniform(34, 500, 30, 400, 150),
    # exactly 129 columns
    "chain3_129": lambda: synth.random_chain(42, 3, 300, 43, 10),
    # a chain whose middle relation projects 120 joined columns away in place
    "chain3_wide_180": lambda: synth.random_chain(41, 3, 400, 60, 15),
    # star rooted at the fact table, non-key dimensions of 50 columns
    "star_fact_root_200": lambda: synth.random_star(40, 4, 3000, 200, 50, pk_dims=False, dom=20),
    # star rooted at a dimension: the fact table joins 150 columns of its
    # children (more than the in-place view holds: stored join)
    "star_dim_root_200": lambda: synth.random_star(43, 4, 3000, 200, 50, pk_dims=False, dom=20, root=1),
    # a narrow relation of 8 and of 30 columns beside a wide one: 9 and 31
    # rows below the final QR's triangle (its short-tail kernels)
    "cartesian_8_150": lambda: synth.cartesian_uniform(36, 300, 8, 400, 150),
    "cartesian_30_150_short": lambda: synth.cartesian_uniform(37, 300, 30, 400, 150),
    # nine dimensions of 45 columns with about 40 tails each: more regions
    # than one panel launch batches (they are taken eight at a time), each
    # with fewer tails than columns
    "star_nine_wide_dims": lambda: synth.random_star(44, 10, 400, 60, 45, pk_dims=False, dom=20),
}


def test_final_qr_tail_shapes_are_covered(F):
    """The cases above reach every form of the final QR: tails of at most 4,
    16 and 64 rows below the triangle (one-wave column panels and the fused
    update) and longer ones (workgroup panels and GEMM updates)."""
    import torch
    tails = {}
    for name, make in CASES.items():
        inst = make()
        plan = F.plan_from_instance(inst)
        tails[name] = int(F.lib().figaro_debug_stack_rows(plan._handle)) - inst.n
        plan.close()
    _say(f"[wide] rows below the triangle: {tails}")
    g = sorted(tails.values())
    assert any(x <= 4 for x in g)
    assert any(4 < x <= 16 for x in g)
    assert any(16 < x <= 64 for x in g)
    assert any(x > 64 for x in g)


def _reference(oracle_lib, inst):
    try:
        R, rows = oracle_lib.factorized_r(inst)
        return R, None
    except np.linalg.LinAlgError:
        Ghi, Glo, _ = oracle_lib.factorized_gram(inst)
        return None, (Ghi, Glo)


@pytest.mark.parametrize("name", sorted(CASES))
def test_wide_forward_matches_oracle(F, oracle_lib, name):
    inst = CASES[name]()
    assert inst.n > 128
    _say(f"[wide] case={name} r={inst.r} n={inst.n} M={inst.M}")
    R, plan, _ = gpu_r(F, inst)
    assert np.all(np.diag(R) >= 0)
    assert np.all(np.tril(R, -1) == 0.0)
    ref, gram = _reference(oracle_lib, inst)
    if ref is None:
        err = oracle_lib.gram_relerr(R, *gram)
        _say(f"[wide] case={name} rank-deficient gram_relerr={err:.3e}")
        assert err <= 1e-13
        return
    err, cerr = relf(R, ref), colscaled(R, ref)
    _say(f"[wide] case={name} rel_err={err:.3e} colscaled={cerr:.3e}")
    assert err <= TOL
    assert cerr <= TOL
    plan.close()


def test_short_wide_relation_rank_deficient(F, oracle_lib):
    """60 tuples of 150 columns: the relation's region has fewer tails than
    columns (its diagonal block of R is trapezoidal) and the join is rank
    deficient; R^T R must still equal A^T A of the materialised join."""
    inst = synth.cartesian_uniform(35, 60, 150, 80, 20)
    R, plan, _ = gpu_r(F, inst)
    A = oracle_lib.join(inst)
    Ghi, Glo = oracle_lib.gram_ld(A)
    err = oracle_lib.gram_relerr(R, Ghi, Glo)
    _say(f"[wide] short-wide gram_relerr={err:.3e}")
    assert np.all(np.diag(R) >= 0)
    assert err <= 1e-13


@pytest.mark.parametrize("seed,n1,n2,m1", [(7, 8, 130, 40), (15, 44, 90, 60)])
def test_appendix_a_ground_truth_wide(F, oracle_lib, seed, n1, n2, m1):
    """Appendix A at more than 128 columns: the leading n1 x n1 block of R is
    sqrt(m2) R_S exactly in the input's rationals, whatever the rest.  How
    close a QR gets depends on the condition of R_S (random integer
    triangles grow ill-conditioned with n1: 3e2 at n1 = 8, 8e6 for the seed
    taken at n1 = 44); the library's error is held to the error of the
    oracle's textbook Householder QR of the materialised join on the same
    input, within a factor of 20, and to 1e-12 where that is smaller."""
    inst, RS, m2 = synth.appendix_a(seed, m1=m1, n1=n1, m2_root=12, n2=n2)
    assert inst.n > 128
    R, plan, _ = gpu_r(F, inst)
    truth = math.sqrt(m2) * RS
    err = relf(R[:n1, :n1], truth)
    ref = relf(oracle_lib.r_of_join(inst)[:n1, :n1], truth)
    _say(f"[wide] appendix A n1={n1} n2={n2} cond(R_S)={np.linalg.cond(RS):.2e} "
         f"rel_err={err:.3e} oracle rel_err={ref:.3e}")
    assert err <= max(20.0 * ref, 1e-12)


def test_wide_forward_deterministic(F):
    inst = CASES["cartesian_tall_96_64"]()
    R1, plan, vals = gpu_r(F, inst)
    R2 = plan.r_factor(vals).cpu().numpy()
    assert np.array_equal(R1, R2)


def test_wide_graph_replays_match_eager(F):
    """The whole wide pass (clear, head/tail kernels, panels, rocBLAS
    products) captured once and replayed three times, with eager work
    between the replays."""
    import torch
    inst = CASES["cartesian_100_100"]()
    R, plan, vals = gpu_r(F, inst)
    out = torch.full((plan.n, plan.n), np.nan, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        plan.r_factor(vals, out=out, stream=s)    # warm-up outside the capture
    s.synchronize()
    with torch.cuda.graph(g, stream=s):
        plan.r_factor(vals, out=out, stream=s)
    for rep in range(3):
        out.fill_(np.nan)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.T.cpu().numpy(), R), f"replay {rep}"


def test_wide_backward_is_refused(F):
    import torch
    inst = CASES["cartesian_100_100"]()
    R, plan, vals = gpu_r(F, inst)
    Rt = torch.as_tensor(R).cuda()
    with pytest.raises(F.FigaroError) as e:
        plan.r_backward(vals, Rt, torch.eye(plan.n, dtype=torch.float64, device="cuda"))
    assert e.value.name == "EUNSUPPORTED"


@pytest.mark.parametrize("name", ["cartesian_30_150", "star_dim_root_200", "chain3_wide_180"])
def test_wide_r0_theorem6(F, oracle_lib, name):
    """R0 of a wide plan (every tail written in its global columns, 16-bit
    column maps, the buffer cleared by the call): R0^T R0 equals A^T A of
    the join (Theorem 6)."""
    import torch
    inst = CASES[name]()
    plan = F.plan_from_instance(inst)
    vals = F.device_values(plan, inst)
    R0, blk = plan.r0(vals)
    torch.cuda.synchronize()
    R0 = R0.cpu().numpy()
    Ghi, Glo, _ = oracle_lib.factorized_gram(inst)
    err = relf(R0.T @ R0, Ghi + Glo)
    _say(f"[wide] R0 case={name} rows={R0.shape[0]} gram rel={err:.2e}")
    assert err <= 1e-12


def test_wide_plans_in_a_batch(F):
    """Wide and narrow plans in one batch, eager and replayed from a captured
    graph: each R bit for bit equal to its plan run alone."""
    import torch
    insts = [CASES["cartesian_100_100"](), synth.config1(), CASES["chain3_wide_180"]()]
    plans = [F.plan_from_instance(i) for i in insts]
    vals = [F.device_values(p, i) for p, i in zip(plans, insts)]
    alone = [p.r_factor(v).cpu().numpy() for p, v in zip(plans, vals)]
    b = F.Batch(plans, streams=2)
    eager = [R.cpu().numpy() for R in b.r(vals)]
    for a, e in zip(alone, eager):
        assert np.array_equal(a, e)
    s = torch.cuda.Stream()
    outs = [torch.full((p.n, p.n), np.nan, dtype=torch.float64, device="cuda") for p in plans]
    with torch.cuda.stream(s):
        Rg = b.capture(vals, outs, s)
    s.synchronize()
    for rep in range(2):
        for o in outs:
            o.fill_(np.nan)
        torch.cuda.synchronize()
        b.launch(s)
        s.synchronize()
        for R, a in zip(Rg, alone):
            assert np.array_equal(R.cpu().numpy(), a), f"replay {rep}"
    b.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("m,ncols", [(4096, 1024), (8192, 4096), (2048, 8192)])
def test_exp1_cells_full_size(F, m, ncols):
    """Cells of Exp. 1's synthetic table at full size (the largest: S, T of
    8192 x 4096, n = 8192), and the widest plan the library takes (S, T of
    2048 x 8192, n = 16384: regions of fewer tails than columns, a rank-
    deficient join), by the property that holds at any size: R^T R equals
    the Gram matrix of S x T, [m S^T S, s^T t; t^T s, m T^T T] with s, t the
    column sums (plain FP64 products on the device), and R is upper
    triangular with a non-negative diagonal."""
    import torch
    _say(f"[wide] Exp. 1 cell m={m} n={ncols}")
    g = torch.Generator(device="cuda")
    g.manual_seed(1000003 * m + ncols)
    S = torch.rand((ncols, m), generator=g, dtype=torch.float64, device="cuda") * 6.0 - 3.0
    T = torch.rand((ncols, m), generator=g, dtype=torch.float64, device="cuda") * 6.0 - 3.0
    views = [F._RelView([], torch.zeros((0, m), dtype=torch.int32, device="cuda"), ncols, -1),
             F._RelView([], torch.zeros((0, m), dtype=torch.int32, device="cuda"), ncols, 0)]
    plan = F.Plan(views)
    R = plan.r_factor([plan.to_plan_order(0, S), plan.to_plan_order(1, T)]).contiguous()
    torch.cuda.synchronize()
    assert bool(torch.all(torch.diagonal(R) >= 0))
    assert bool(torch.all(torch.tril(R, -1) == 0))
    St, Tt = S.t().contiguous(), T.t().contiguous()
    G = torch.empty((2 * ncols, 2 * ncols), dtype=torch.float64, device="cuda")
    G[:ncols, :ncols] = m * (St.t() @ St)
    G[ncols:, ncols:] = m * (Tt.t() @ Tt)
    G[:ncols, ncols:] = torch.outer(St.sum(0), Tt.sum(0))
    G[ncols:, :ncols] = G[:ncols, ncols:].t()
    res = float(torch.linalg.norm(R.t() @ R - G) / torch.linalg.norm(G))
    _say(f"[wide] Exp. 1 cell m={m} n={ncols} gram residual {res:.2e}")
    assert res <= 1e-13
    plan.close()

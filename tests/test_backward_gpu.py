"""Parity of the hand-written adjoint with autograd through the QR of the
materialised join (CPU, FP64), closed forms and central finite differences
(needs an MI355X).  Gradients must match within 1e-6 relative of finite
differences and (much tighter) of autograd.  Against autograd every data
column of every relation is also judged on its own (each entry against the
norm of its column's gradient), so an error confined to a column with a small
scale cannot hide behind the large ones."""
import sys

import numpy as np
import pytest

import synth
from _parity import colscaled, relf as _relf

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2204_00525_amd as F
    F.lib()
    return F


def gpu_grads(F, inst, loss_fn, **kw):
    """Gradients (caller row order, numpy) of loss_fn(R) through FigaroR."""
    import torch
    plan = F.plan_from_instance(inst, **kw)
    vals = [v.clone().requires_grad_(True) for v in F.device_values(plan, inst)]
    R = F.figaro_r(plan, *vals)
    L = loss_fn(R)
    L.backward()
    torch.cuda.synchronize()
    out = [plan.from_plan_order(i, vals[i].grad.detach()).cpu().numpy() for i in range(inst.r)]
    return out, R.detach().cpu().numpy(), plan


CASES = {
    "config1": lambda: synth.config1(),
    "paper_fig3_b": lambda: synth.paper_fig3(5, m=(40, 90, 30, 30), n=(3, 2, 4, 1), dom=3),
    "chain4": lambda: synth.random_chain(4, 4, 40, 2, 4),
    "star_pk": lambda: synth.random_star(5, 4, 600, 30, 3),
    "star_nonpk": lambda: synth.random_star(6, 3, 300, 40, 2, pk_dims=False, dom=10),
    "star_dim_root": lambda: synth.random_star(7, 4, 500, 20, 2, root=2),
    "two_rel_zipf": lambda: synth.two_relation(10, 3000, 3000, 6, 5, 60, dist="zipf"),
    "config4_div1000": lambda: synth.config3(seed=1004, div=1000),
    "cartesian": lambda: synth.cartesian_uniform(8, 60, 3, 50, 2),
    # wide blocks: a 48-column project-away task (column chunks), n = 64
    # and n = 100 (cooperative dense TSQR, QR adjoint beyond 64 columns)
    "chain4_wide": lambda: synth.random_chain(16, 4, 40, 16, 8),
    "star_wide_dimroot": lambda: synth.random_star(17, 5, 300, 30, 20, root=3),
    # joined heads of exactly 8 and 16 columns under a dimension root: their
    # row-major gradient goes out as one contiguous block per tile
    "star_dimroot_rows8": lambda: synth.random_star(30, 3, 400, 25, 4, root=1),
    "star_dimroot_rows16": lambda: synth.random_star(31, 3, 400, 25, 8, root=1),
}


def _weighted(n, seed):
    rng = np.random.default_rng(seed)
    return np.triu(rng.standard_normal((n, n)))


@pytest.mark.parametrize("name", sorted(CASES))
def test_backward_matches_autograd(F, oracle_lib, name):
    import torch
    inst = CASES[name]()
    W = _weighted(inst.n, 7)
    Wt = torch.as_tensor(W)
    _say(f"[backward] case={name} n={inst.n} M={inst.M}")
    g, R, plan = gpu_grads(F, inst, lambda R: (R * Wt.to(R.device)).sum())
    ref, Rref = oracle_lib.grad_autograd(inst, lambda R: (R * Wt).sum())
    assert _relf(R, Rref) <= 1e-10
    assert colscaled(R, Rref) <= 1e-10
    errs = [_relf(a, b) for a, b in zip(g, ref)]
    cerrs = [colscaled(a, b, axis=1) for a, b in zip(g, ref)]
    _say(f"[backward] case={name} rel_errs={['%.2e' % e for e in errs]} colscaled={['%.2e' % e for e in cerrs]}")
    assert max(errs) <= 1e-8
    assert max(cerrs) <= 1e-8


def config4_loss(R):
    """Least-squares residual of the last column on the others plus the
    log-determinant: 1/2 R_nn^2 + sum_i log R_ii."""
    import torch
    d = torch.diagonal(R)
    return 0.5 * R[-1, -1] ** 2 + torch.log(d).sum()


@pytest.mark.parametrize("tile", [0, 64])
def test_backward_config4_loss(F, oracle_lib, tile):
    inst = CASES["config4_div1000"]()
    g, R, plan = gpu_grads(F, inst, config4_loss, tile_items=tile)
    ref, _ = oracle_lib.grad_autograd(inst, config4_loss)
    errs = [_relf(a, b) for a, b in zip(g, ref)]
    cerrs = [colscaled(a, b, axis=1) for a, b in zip(g, ref)]
    _say(f"[backward] config4 tile={tile} rel_errs={['%.2e' % e for e in errs]} "
         f"colscaled={['%.2e' % e for e in cerrs]}")
    assert max(errs) <= 1e-8
    assert max(cerrs) <= 1e-8


def _stencil5(f, h):
    """Fourth-order central difference (f(-2h) - 8 f(-h) + 8 f(h) - f(2h)) / 12h."""
    return (f(-2 * h) - 8.0 * f(-h) + 8.0 * f(h) - f(2 * h)) / (12.0 * h)


@pytest.mark.timeout(900)
def test_backward_config4_finite_differences(F):
    """Config 4 on the 1/1000 subsample (fact table 10^4 rows, dimensions
    10^2 rows, 8 columns each, column scales 10^U[-3,3], seed 1004), loss
    1/2 R_nn^2 + sum_i log R_ii: the gradient of every coordinate of the four
    dimension tables and of 2,000 seeded coordinates of the fact table
    against finite differences of the GPU forward pass, within 1e-6 relative
    per relation.  The step of a coordinate is h = 10^-3 s_c (s_c the scale
    of its column) in a fourth-order stencil: a plain central difference
    with h = 10^-6 s_c carries rounding noise of ~10^-4 relative on the fact
    table's small gradients (the oracle's own forward pass shows the same),
    which the fourth-order stencil at the larger step removes."""
    import torch
    inst = synth.config3(seed=1004, div=1000)
    scales = inst.meta["scales"]
    plan = F.plan_from_instance(inst)
    vals = F.device_values(plan, inst)
    vg = [v.clone().requires_grad_(True) for v in vals]
    R = F.figaro_r(plan, *vg)
    config4_loss(R).backward()
    torch.cuda.synchronize()
    ana = [v.grad.detach().cpu().numpy() for v in vg]
    col0 = np.cumsum([0] + [rel.ncols for rel in inst.rels])
    rng = np.random.default_rng(4004)

    def fd(i, c, t):
        x0 = float(vals[i][c, t])
        h = 1e-3 * float(scales[col0[i] + c])

        def f(d):
            vals[i][c, t] = x0 + d
            return float(config4_loss(plan.r_factor(vals)).item())
        out = _stencil5(f, h)
        vals[i][c, t] = x0
        return out

    for i, rel in enumerate(inst.rels):
        if i == 1:      # the fact table: a seeded sample of coordinates
            coords = [(int(rng.integers(0, rel.ncols)), int(rng.integers(0, plan.rows(i)))) for _ in range(2000)]
        else:           # every coordinate of a dimension table
            coords = [(c, t) for c in range(rel.ncols) for t in range(plan.rows(i))]
        num = np.array([fd(i, c, t) for c, t in coords])
        got = np.array([ana[i][c, t] for c, t in coords])
        err = float(np.linalg.norm(num - got) / np.linalg.norm(num))
        _say(f"[backward-fd] config4/1000 relation {rel.name}: {len(coords)} coordinates, rel_err={err:.2e}")
        assert err <= 1e-6, rel.name


@pytest.mark.timeout(900)
def test_backward_config4_directions_full_size(F):
    """Config 4 at full size (fact table 10^7 rows): directional derivatives
    of the loss along 8 seeded random directions (entries N(0,1) s_c per
    column) against finite differences of the GPU forward pass (fourth-order
    stencil, step 10^-3 along the direction), within 1e-6 relative."""
    import torch
    inst = synth.config3(seed=1004)
    scales = inst.meta["scales"]
    plan = F.plan_from_instance(inst)
    vals = F.device_values(plan, inst)
    vg = [v.clone().requires_grad_(True) for v in vals]
    R = F.figaro_r(plan, *vg)
    config4_loss(R).backward()
    grads = [v.grad.detach() for v in vg]
    del vg, R
    col0 = np.cumsum([0] + [rel.ncols for rel in inst.rels])
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4005)
    for k in range(8):
        dirs = []
        for i, v in enumerate(vals):
            s = torch.as_tensor(scales[col0[i]:col0[i + 1]], device="cuda", dtype=torch.float64)
            d = torch.randn(v.shape, generator=gen, device="cuda", dtype=torch.float64)
            dirs.append(d * s[:, None])
        ana = float(sum((g * d).sum() for g, d in zip(grads, dirs)).item())

        def f(e):
            return float(config4_loss(plan.r_factor([v + e * d for v, d in zip(vals, dirs)])).item())
        num = _stencil5(f, 1e-3)
        err = abs(num - ana) / abs(num)
        _say(f"[backward-fd] config4 full direction {k}: fd={num:.12e} adjoint={ana:.12e} rel_err={err:.2e}")
        assert err <= 1e-6


def test_backward_logdet_closed_form(F, oracle_lib):
    import torch
    inst = CASES["star_nonpk"]()
    g, R, plan = gpu_grads(F, inst, lambda R: torch.log(torch.diagonal(R)).sum())
    ref = oracle_lib.grad_logdet_closed_form(inst)
    assert max(_relf(a, b) for a, b in zip(g, ref)) <= 1e-9
    assert max(colscaled(a, b, axis=1) for a, b in zip(g, ref)) <= 1e-9


@pytest.mark.parametrize("name", ["paper_fig3_b", "two_rel_zipf", "star_nonpk"])
def test_backward_central_differences(F, name):
    """Central finite differences of the GPU forward pass itself, on random
    coordinates of every relation."""
    import torch
    inst = CASES[name]()
    plan = F.plan_from_instance(inst)
    vals = F.device_values(plan, inst)
    W = torch.as_tensor(_weighted(inst.n, 3), device="cuda")

    def loss(vs):
        return float((plan.r_factor(vs) * W).sum().item())

    vg = [v.clone().requires_grad_(True) for v in vals]
    R = F.figaro_r(plan, *vg)
    (R * W).sum().backward()
    rng = np.random.default_rng(0)
    num, ana = [], []
    for i in range(inst.r):
        for _ in range(6):
            c = int(rng.integers(0, vals[i].shape[0]))
            t = int(rng.integers(0, vals[i].shape[1]))
            h = 1e-6 * max(1.0, abs(float(vals[i][c, t])))
            vp = [v.clone() for v in vals]
            vm = [v.clone() for v in vals]
            vp[i][c, t] += h
            vm[i][c, t] -= h
            num.append((loss(vp) - loss(vm)) / (2 * h))
            ana.append(float(vg[i].grad[c, t]))
    num, ana = np.array(num), np.array(ana)
    err = np.linalg.norm(num - ana) / np.linalg.norm(ana)
    _say(f"[backward-fd] case={name} rel_err={err:.2e}")
    assert err <= 1e-6


@pytest.mark.parametrize("name", ["star_dim_root", "chain4", "star_wide_dimroot"])
def test_backward_fused_join_same_gradient(F, name):
    """R from a forward pass that reads the joined heads in place, and the
    gradients behind it, equal those of a plan that always stores them, bit
    for bit."""
    import torch
    inst = CASES[name]()
    W = torch.as_tensor(_weighted(inst.n, 11))
    _say(f"[backward-fused-join] case={name}")
    g1, R1, _ = gpu_grads(F, inst, lambda R: (R * W.to(R.device)).sum())
    g2, R2, _ = gpu_grads(F, inst, lambda R: (R * W.to(R.device)).sum(), separate_join=True)
    assert np.array_equal(R1, R2)
    for a, b in zip(g1, g2):
        assert np.array_equal(a, b)


def test_backward_split_tiles_same_gradient(F):
    import torch
    inst = CASES["two_rel_zipf"]()
    W = torch.as_tensor(_weighted(inst.n, 9))
    g0, _, _ = gpu_grads(F, inst, lambda R: (R * W.to(R.device)).sum())
    g1, _, _ = gpu_grads(F, inst, lambda R: (R * W.to(R.device)).sum(), tile_items=64, waves_per_task=5)
    assert max(_relf(a, b) for a, b in zip(g1, g0)) <= 1e-10


def test_backward_deterministic(F):
    import torch
    inst = CASES["star_pk"]()
    plan = F.plan_from_instance(inst)
    vals = F.device_values(plan, inst)
    R = plan.r_factor(vals)
    dR = torch.as_tensor(_weighted(inst.n, 1), device="cuda")
    a = [x.cpu().numpy() for x in plan.r_backward(vals, R, dR)]
    b = [x.cpu().numpy() for x in plan.r_backward(vals, R, dR)]
    assert all(np.array_equal(x, y) for x, y in zip(a, b))


def test_backward_dropped_rows_get_zero(F, oracle_lib):
    import torch
    inst = synth.two_relation(14, 500, 400, 3, 2, 40)
    inst.rels[0].keys[0, :25] = 1000 + np.arange(25)
    W = torch.as_tensor(_weighted(inst.n, 2))
    g, R, plan = gpu_grads(F, inst, lambda R: (R * W.to(R.device)).sum())
    assert np.all(g[0][:, :25] == 0.0)
    ref, _ = oracle_lib.grad_autograd(inst, lambda R: (R * W).sum())
    assert max(_relf(a, b) for a, b in zip(g, ref)) <= 1e-8


def test_backward_singular_status(F):
    import torch
    inst = synth.two_relation(15, 300, 200, 3, 2, 20)
    inst.rels[0].values[1, :] = 0.0          # a zero column: R has a zero diagonal entry
    plan = F.plan_from_instance(inst)
    vals = F.device_values(plan, inst)
    R = plan.r_factor(vals)
    plan.r_backward(vals, R, torch.eye(inst.n, device="cuda", dtype=torch.float64))
    assert plan.backward_status() == "ESINGULAR"
    inst2 = synth.two_relation(15, 300, 200, 3, 2, 20)
    plan2 = F.plan_from_instance(inst2)
    vals2 = F.device_values(plan2, inst2)
    plan2.r_backward(vals2, plan2.r_factor(vals2), torch.eye(inst2.n, device="cuda", dtype=torch.float64))
    assert plan2.backward_status() == "OK"


def _long_inverse_lists():
    """A 3-chain whose middle relation has ~3800 key groups that all join the
    last relation's single group: the join adjoint's list for that child
    group is longer than one chunk (1024 entries)."""
    inst = synth.random_chain(50, 3, 6000, 2, 5000)
    inst.rels[1].keys[1, :] = 0
    last = inst.rels[2]
    inst.rels[2] = synth.Rel(last.key_attrs, np.zeros((1, 3), np.int32), last.values[:, :3].copy(), last.parent,
                             last.name)
    return inst


def test_backward_long_inverse_lists(F, oracle_lib):
    """The join adjoint sums a long list of parent key groups in chunks (a
    partial per chunk and column, then the chunks in order): gradients match
    autograd through the materialised join, and the device-built plan gives
    bit for bit the gradients of the host-built one."""
    import torch
    inst = _long_inverse_lists()
    W = _weighted(inst.n, 11)
    Wt = torch.as_tensor(W)
    g, R, plan = gpu_grads(F, inst, lambda R: (R * Wt.to(R.device)).sum())
    assert plan.num_groups(1, 0) > 1024
    ref, Rref = oracle_lib.grad_autograd(inst, lambda R: (R * Wt).sum())
    errs = [_relf(a, b) for a, b in zip(g, ref)]
    _say(f"[backward] long inverse lists: groups={plan.num_groups(1, 0)} rel_errs={['%.2e' % e for e in errs]}")
    assert _relf(R, Rref) <= 1e-10
    assert max(errs) <= 1e-8
    g_host, _, _ = gpu_grads(F, inst, lambda R: (R * Wt.to(R.device)).sum(), host_plan=True)
    for a, b in zip(g, g_host):
        assert np.array_equal(a, b)

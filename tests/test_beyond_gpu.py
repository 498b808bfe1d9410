"""Q, SVD and PCA of the join from R (section "From R to Q, SVD and PCA"),
against the oracle's materialised join (needs an MI355X).

* The join-row enumeration: with M = I the rows of A M are the join's rows
  themselves; aligned by the tuple ids every row carries, they equal the
  oracle's materialised join bit for bit, and the ids are a bijection onto
  the oracle's join.
* Q = A R^-1 from the library's R, against the oracle's A times the inverse
  of the same R (the product alone), and against the oracle's Q.
* sigma, V from the SVD of R against LAPACK's SVD of the materialised join;
  U = A V Sigma^-1 and the PCA projection A V[:, :k] against the oracle's.
"""
import sys

import numpy as np
import pytest

import synth
from _parity import relf

pytestmark = pytest.mark.gpu


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


CASES = {
    "config1": lambda: synth.config1(),
    "config2_div1000": lambda: synth.config2(div=1000),
    "config3_div1000": lambda: synth.config3(div=1000),
    "paper_fig3_b": lambda: synth.paper_fig3(5, m=(40, 90, 30, 30), n=(3, 2, 4, 1), dom=3),
    "chain3": lambda: synth.random_chain(3, 3, 400, 3, 20),
    "star_pk": lambda: synth.random_star(5, 4, 3000, 50, 3),
    "star_dim_root_6": lambda: synth.random_star(23, 7, 2000, 30, 2, root=1),
    "cartesian": lambda: synth.cartesian_uniform(8, 300, 4, 200, 3),
    "chain4_wide_64": lambda: synth.random_chain(16, 4, 120, 16, 12),
}


def _align(ids_a, ids_b):
    """Row orders that sort both id arrays ((r, N) each) the same way; the
    two must hold the same rows."""
    oa = np.lexsort(ids_a[::-1])
    ob = np.lexsort(ids_b[::-1])
    assert np.array_equal(ids_a[:, oa], ids_b[:, ob])
    return oa, ob


def _setup(F, inst):
    import torch
    plan = F.plan_from_instance(inst)
    vals = F.device_values(plan, inst)
    R = plan.r_factor(vals)
    torch.cuda.synchronize()
    return plan, vals, R


@pytest.mark.parametrize("name", sorted(CASES))
def test_enumerated_rows_are_the_join(F, oracle_lib, name):
    import torch
    inst = CASES[name]()
    plan, vals, R = _setup(F, inst)
    rows, ids = plan.join_multiply(vals, torch.eye(inst.n, dtype=torch.float64, device="cuda"), with_ids=True)
    rows, ids = rows.cpu().numpy(), ids.cpu().numpy()
    A = oracle_lib.join(inst)
    ref_ids = oracle_lib.join_indices(inst)
    assert rows.shape == A.shape == (int(plan.join_rows), inst.n)
    oa, ob = _align(ids, ref_ids)
    assert np.array_equal(rows[oa], A[ob]), name
    _say(f"[enumerate] case={name} rows={rows.shape[0]} exact")


def test_row_slices_concatenate(F):
    """Rows taken in slices (row0, nrows) are the same as taken at once."""
    import torch
    inst = CASES["star_pk"]()
    plan, vals, R = _setup(F, inst)
    M = torch.randn((inst.n, 5), dtype=torch.float64, device="cuda")
    full = plan.join_multiply(vals, M)
    N = full.shape[0]
    cuts = [0, 1, 777, N // 2, N - 3, N]
    parts = [plan.join_multiply(vals, M, row0=a, nrows=b - a) for a, b in zip(cuts, cuts[1:])]
    assert torch.equal(torch.cat(parts), full)


@pytest.mark.parametrize("name", sorted(CASES))
def test_q_rows(F, oracle_lib, name):
    import torch
    inst = CASES[name]()
    plan, vals, R = _setup(F, inst)
    Q, ids = plan.join_multiply(vals, F.r_inverse(R), with_ids=True)
    Q, ids = Q.cpu().numpy(), ids.cpu().numpy()
    A = oracle_lib.join(inst)
    ref_ids = oracle_lib.join_indices(inst)
    oa, ob = _align(ids, ref_ids)
    Rh = R.cpu().numpy()
    # the product alone: the oracle's rows times the inverse of the same R
    import scipy.linalg
    Qs = scipy.linalg.solve_triangular(Rh, A.T, trans="T").T
    err_same = relf(Q[oa], Qs[ob])
    # against the oracle's Q (its own R), column by column
    Qref, _ = oracle_lib.q_of_join(inst)
    col = max(np.linalg.norm(Q[oa][:, j] - Qref[ob][:, j]) for j in range(inst.n))
    ortho = np.linalg.norm(Q.T @ Q - np.eye(inst.n))
    _say(f"[q] case={name} same-R rel={err_same:.2e} oracle max-col={col:.2e} |QtQ-I|={ortho:.2e}")
    assert err_same <= 1e-12
    assert col <= 1e-8
    assert ortho <= 1e-10


@pytest.mark.parametrize("n", [1, 2, 5, 17, 33, 64, 100, 128])
def test_svd_of_r_plain(F, n):
    import torch
    rng = np.random.default_rng(n)
    Rh = np.triu(rng.standard_normal((n, n)) * 10.0 ** rng.uniform(-2, 2, n))
    s, U, V = F.svd_of_r(torch.as_tensor(Rh).cuda())
    s, U, V = s.cpu().numpy(), U.cpu().numpy(), V.cpu().numpy()
    sref = np.linalg.svd(Rh, compute_uv=False)
    assert np.all(np.diff(s) <= 0)
    assert np.max(np.abs(s - sref)) <= 1e-12 * sref[0]
    assert np.linalg.norm(V.T @ V - np.eye(n)) <= 1e-13 * n
    assert np.linalg.norm(U.T @ U - np.eye(n)) <= 1e-13 * n
    assert np.linalg.norm((U * s) @ V.T - Rh) <= 1e-13 * np.linalg.norm(Rh)


@pytest.mark.parametrize("name", sorted(CASES))
def test_svd_and_pca_of_the_join(F, oracle_lib, name):
    import torch
    inst = CASES[name]()
    plan, vals, R = _setup(F, inst)
    s, UR, V = F.svd_of_r(R)
    Uref, sref, Vref, ref_ids = oracle_lib.svd_of_join(inst)
    sh, Vh = s.cpu().numpy(), V.cpu().numpy()
    # singular values: each within 1e-9 of itself plus 1e-12 of the largest
    assert np.all(np.abs(sh - sref) <= 1e-9 * sref + 1e-12 * sref[0]), name
    # right singular vectors (principal components) up to sign
    sign = np.sign(np.sum(Vh * Vref, axis=0))
    sign[sign == 0] = 1.0
    gaps = np.minimum(np.abs(np.diff(sref, prepend=np.inf)), np.abs(np.diff(sref, append=-np.inf)))
    distinct = gaps > 1e-6 * sref[0]
    verr = np.linalg.norm(Vh[:, distinct] * sign[distinct] - Vref[:, distinct])
    # left singular vectors U = A V Sigma^-1, and the PCA projection A V[:, :k]
    U, ids = plan.join_multiply(vals, V, col_scale=1.0 / s, with_ids=True)
    U, ids = U.cpu().numpy(), ids.cpu().numpy()
    oa, ob = _align(ids, ref_ids)
    uerr = np.linalg.norm(U[oa][:, distinct] * sign[distinct] - Uref[ob][:, distinct])
    k = min(3, inst.n)
    P = plan.join_multiply(vals, V[:, :k]).cpu().numpy()
    A = oracle_lib.join(inst)
    Pref = A @ Vref[:, :k]
    perr = relf(P[oa] * sign[:k], Pref[ob])
    _say(f"[svd] case={name} V err={verr:.2e} U err={uerr:.2e} PCA rel={perr:.2e}")
    assert verr <= 1e-8
    assert uerr <= 1e-8
    assert perr <= 1e-10

"""Pins for the CPU oracle (no GPU).  Each check compares the oracle against
something other than itself: values the paper prints or that follow from its
lemmas by hand (tests/golden), closed forms, invariants, brute force on tiny
inputs, an independent LAPACK factorisation, or a different oracle routine
that shares no arithmetic with the one under test."""
import json
import math
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _relf(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _lapack_r(A):
    R = np.linalg.qr(A, mode="r")
    return np.sign(np.where(np.diag(R) == 0, 1.0, np.diag(R)))[:, None] * R


# ---------------------------------------------------------------------------
# Householder, Givens, Gram, determinant
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,seed", [(1, 1, 0), (3, 3, 1), (7, 4, 2), (50, 6, 3), (200, 8, 4)])
def test_householder_matches_givens_and_lapack(oracle_lib, m, n, seed):
    rng = np.random.default_rng(seed)
    A = np.asfortranarray(rng.standard_normal((m, n)))
    R, zeros = oracle_lib.householder_r(A)
    assert zeros == 0
    assert np.all(np.diag(R) > 0)
    assert np.allclose(np.tril(R, -1), 0.0)
    Rg = oracle_lib.givens_r(A)
    assert _relf(R, Rg) <= 1e-13
    assert _relf(R, _lapack_r(A)) <= 1e-13


@pytest.mark.parametrize("m,n,seed", [(20, 3, 5), (120, 7, 6)])
def test_householder_gram_and_determinant(oracle_lib, m, n, seed):
    rng = np.random.default_rng(seed)
    A = np.asfortranarray(rng.standard_normal((m, n)) * 10.0 ** rng.uniform(-3, 3, n))
    R, _ = oracle_lib.householder_r(A)
    Ghi, Glo = oracle_lib.gram_ld(A)
    assert oracle_lib.gram_relerr(R, Ghi, Glo) <= 1e-14
    logdet = oracle_lib.logabsdet(Ghi, Glo)
    assert abs(2.0 * np.sum(np.log(np.diag(R))) - logdet) <= 1e-12 * max(1.0, abs(logdet))


def test_gram_ld_matches_integer_exact(oracle_lib):
    # integer matrix: A^T A is exact in integer arithmetic
    rng = np.random.default_rng(11)
    Ai = rng.integers(-50, 50, (40, 5))
    Ghi, Glo = oracle_lib.gram_ld(np.asfortranarray(Ai.astype(np.float64)))
    exact = Ai.T.astype(object) @ Ai.astype(object)
    assert np.array_equal(Ghi + Glo, np.array(exact, dtype=np.float64))


def test_householder_rank_deficient_flags(oracle_lib):
    rng = np.random.default_rng(12)
    A = rng.standard_normal((30, 3))
    A = np.asfortranarray(np.column_stack([A, A[:, 0]]))
    R, _ = oracle_lib.householder_r(A)
    # R^T R still equals A^T A although R is not unique
    Ghi, Glo = oracle_lib.gram_ld(A)
    assert oracle_lib.gram_relerr(R, Ghi, Glo) <= 1e-13
    assert abs(R[3, 3]) <= 1e-13 * np.abs(R).max()


def test_householder_triangular_input_is_fixed_point(oracle_lib):
    # R of an upper-triangular matrix with positive diagonal is itself
    rng = np.random.default_rng(13)
    U = np.triu(rng.standard_normal((6, 6)))
    U[np.diag_indices(6)] = np.abs(U[np.diag_indices(6)]) + 0.5
    R, _ = oracle_lib.householder_r(np.asfortranarray(U))
    assert _relf(R, U) <= 1e-15


# ---------------------------------------------------------------------------
# Joins
# ---------------------------------------------------------------------------

def _multiset(A):
    return sorted(map(tuple, np.round(A, 12).tolist()))


@pytest.mark.parametrize("maker", [
    lambda: synth.paper_fig3(1),
    lambda: synth.paper_fig3(2, m=(4, 7, 3, 3), dom=3),
    lambda: synth.random_chain(3, 3, 6, 2, 3),
    lambda: synth.random_star(4, 3, 8, 3, 2, pk_dims=False, dom=3),
    lambda: synth.cartesian_uniform(5, 3, 2, 4, 1),
])
def test_join_matches_brute_force(oracle_lib, maker):
    inst = maker()
    A = oracle_lib.join(inst)
    combos = oracle_lib.brute_join_rows(inst, list(range(inst.r)))
    assert A.shape[0] == len(combos)
    B = np.array([np.concatenate([inst.rels[i].values[:, c[i]] for i in range(inst.r)])
                  for c in combos]).reshape(len(combos), inst.n)
    assert _multiset(A) == _multiset(B)


@pytest.mark.parametrize("maker", [
    lambda: synth.paper_fig3(1),
    lambda: synth.paper_fig3(2, m=(4, 7, 3, 3), dom=3),
    lambda: synth.random_chain(3, 3, 6, 2, 3),
    lambda: synth.random_chain(7, 4, 5, 1, 2, dist="zipf"),
    lambda: synth.random_star(4, 3, 8, 3, 2, pk_dims=False, dom=3),
    lambda: synth.random_star(9, 3, 9, 3, 2, root=1),
    lambda: synth.cartesian_uniform(5, 3, 2, 4, 1),
    lambda: synth.two_relation(14, 12, 9, 2, 1, 5),
])
def test_join_indices_pinned(oracle_lib, maker):
    """join_indices against the definition of the natural join: its rows are
    exactly the combinations of tuples that agree on every shared attribute
    (brute force over all combinations), each once; and join() is the
    per-relation gather values_i[:, idx_i] of those rows, in the same order."""
    inst = maker()
    if inst.name == "two_relation_uniform":
        inst.rels[0].keys[0, :3] = 99      # dangling tuples take part in no row
    idx = oracle_lib.join_indices(inst)
    combos = oracle_lib.brute_join_rows(inst, list(range(inst.r)))
    assert idx.shape == (inst.r, len(combos))
    assert sorted(map(tuple, idx.T.tolist())) == sorted(combos)
    A = oracle_lib.join(inst)
    gathered = np.column_stack([inst.rels[i].values[:, idx[i]].T for i in range(inst.r)])
    assert np.array_equal(A, gathered)


def test_join_indices_planted_mistake_is_caught(oracle_lib):
    """Plausible indexing mistakes fail the definition check above: one join
    row repeated in place of another, or one relation's row index off by one
    in a single join row."""
    inst = synth.paper_fig3(2, m=(4, 7, 3, 3), dom=3)
    combos = sorted(oracle_lib.brute_join_rows(inst, list(range(inst.r))))
    idx = oracle_lib.join_indices(inst).copy()
    assert idx.shape[1] >= 2
    dup = idx.copy()
    dup[:, 1] = dup[:, 0]
    assert sorted(map(tuple, dup.T.tolist())) != combos
    off = idx.copy()
    off[1, 0] = (off[1, 0] + 1) % inst.rels[1].rows
    assert sorted(map(tuple, off.T.tolist())) != combos


def test_gram_relerr_exact_values(oracle_lib):
    """gram_relerr = ||R^T R - G||_F / ||G||_F against values computed exactly
    in integers: zero for G = R^T R, and the planted residual of a known
    integer perturbation E, also when E sits in the lo part of a hi + lo
    pair (2^-40 E, exactly representable in long double next to G)."""
    from fractions import Fraction
    rng = np.random.default_rng(31)
    n = 6
    Ri = np.triu(rng.integers(-9, 10, (n, n)))
    Ri[np.diag_indices(n)] = rng.integers(1, 10, n)
    Gi = Ri.T.astype(object) @ Ri.astype(object)
    R = Ri.astype(np.float64)
    G = np.array(Gi, dtype=np.float64)
    zero = np.zeros((n, n))
    assert oracle_lib.gram_relerr(R, G, zero) == 0.0
    E = np.zeros((n, n), dtype=np.int64)
    E[2, 4] = E[4, 2] = 3
    E[0, 0] = -5
    E[5, 1] = E[1, 5] = 7
    Gp = Gi + E.astype(object)
    expect = math.sqrt(Fraction(int(np.sum(E.astype(object) ** 2)), int(np.sum(Gp ** 2))))
    got = oracle_lib.gram_relerr(R, np.array(Gp, dtype=np.float64), zero)
    assert got > 0 and abs(got - expect) <= 1e-14 * expect
    lo = np.ldexp(E.astype(np.float64), -40)
    num = Fraction(int(np.sum(E.astype(object) ** 2)), 2 ** 80)
    den = sum((Fraction(int(g)) + Fraction(int(e), 2 ** 40)) ** 2 for g, e in zip(Gi.ravel(), E.ravel()))
    expect_lo = math.sqrt(num / den)
    got_lo = oracle_lib.gram_relerr(R, G, lo)
    assert abs(got_lo - expect_lo) <= 1e-12 * expect_lo
    # a wrong factor (the transpose) is far off
    assert oracle_lib.gram_relerr(R.T.copy(), G, zero) > 0.1


def test_join_two_relation_size_closed_form(oracle_lib):
    inst = synth.config1()
    ks = np.bincount(inst.rels[0].keys[0], minlength=100)
    kt = np.bincount(inst.rels[1].keys[0], minlength=100)
    assert oracle_lib.join_size(inst) == int(np.dot(ks, kt))


# ---------------------------------------------------------------------------
# The paper's worked values, Lemma 1, Lemma 2, Lemma 4, Definitions
# ---------------------------------------------------------------------------

def test_golden_intro_constant_column(oracle_lib):
    g = json.load(open(os.path.join(GOLDEN, "intro_constant_column.json")))
    s = g["s"]
    col = np.array([s, s, s])
    v = np.ones(3)
    # partial products of the rotation sequence of Lemma 1 (m = 3)
    for step in g["steps"]:
        k = step["after_rotation"] + 1
        Rk = oracle_lib.givens_matrix(3, 1, k, step["sin"], step["cos"])
        col = Rk @ col
        assert np.allclose(col, step["column"], rtol=0, atol=1e-14)
    G = oracle_lib.rotations_lemma(v)
    assert np.allclose(G @ np.array([s, s, s]), g["steps"][-1]["column"], atol=1e-14)
    # head of the constant column is sqrt(m) s, its tail is zero
    assert abs(oracle_lib.head(np.full((3, 1), s))[0] - math.sqrt(3) * s) <= 1e-14
    assert np.all(np.abs(oracle_lib.tail(np.full((3, 1), s))) <= 1e-15 * s)


def test_golden_lemma1_example(oracle_lib):
    g = json.load(open(os.path.join(GOLDEN, "lemma1_example.json")))
    S = np.array(g["S"])
    T = np.array(g["T"])
    m = T.shape[0]
    A = np.column_stack([np.repeat(S[None, :], m, axis=0), T])
    U = oracle_lib.rotations_lemma(np.ones(m)) @ A
    assert np.allclose(U, g["U"], atol=1e-14)
    assert np.allclose(oracle_lib.head(T), np.array(g["U"])[0, 1:], atol=1e-14)
    assert np.allclose(oracle_lib.tail(T), np.array(g["U"])[1:, 1:], atol=1e-14)


@pytest.mark.parametrize("m,n1,n2,seed", [(1, 1, 1, 0), (2, 2, 3, 1), (5, 1, 4, 2), (17, 3, 2, 3)])
def test_lemma1_rotations_equal_head_tail(oracle_lib, m, n1, n2, seed):
    rng = np.random.default_rng(seed)
    S = rng.standard_normal(n1)
    T = rng.standard_normal((m, n2))
    A = np.column_stack([np.repeat(S[None, :], m, axis=0), T])
    U = oracle_lib.rotations_lemma(np.ones(m)) @ A
    assert np.allclose(U[0, :n1], math.sqrt(m) * S, rtol=1e-14, atol=1e-14)
    assert np.allclose(U[1:, :n1], 0.0, atol=1e-13)
    assert np.allclose(U[0, n1:], oracle_lib.head(T), rtol=1e-13, atol=1e-13)
    assert np.allclose(U[1:, n1:], oracle_lib.tail(T), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("m,seed", [(2, 0), (6, 1), (23, 2)])
def test_lemma2_rotations_equal_generalized_head_tail(oracle_lib, m, seed):
    rng = np.random.default_rng(seed)
    v = rng.uniform(0.1, 5.0, m)
    S = rng.standard_normal(2)
    T = rng.standard_normal((m, 3))
    A = np.column_stack([v[:, None] * S[None, :], T])
    U = oracle_lib.rotations_lemma(v) @ A
    assert np.allclose(U[0, :2], np.linalg.norm(v) * S, rtol=1e-13)
    assert np.allclose(U[1:, :2], 0.0, atol=1e-12)
    assert np.allclose(U[0, 2:], oracle_lib.gen_head(T, v), rtol=1e-12, atol=1e-12)
    assert np.allclose(U[1:, 2:], oracle_lib.gen_tail(T, v), rtol=1e-12, atol=1e-12)


def test_generalized_reduces_to_plain_and_homogeneity(oracle_lib):
    rng = np.random.default_rng(7)
    A = rng.standard_normal((9, 4))
    v = rng.uniform(0.5, 2.0, 9)
    assert np.allclose(oracle_lib.gen_head(A, np.ones(9)), oracle_lib.head(A), rtol=1e-14)
    assert np.allclose(oracle_lib.gen_tail(A, np.ones(9)), oracle_lib.tail(A), rtol=1e-13, atol=1e-14)
    k, l = -2.5, 3.0   # Lemma 4
    assert np.allclose(oracle_lib.gen_head(k * A, l * v), k * oracle_lib.gen_head(A, v), rtol=1e-13)
    assert np.allclose(oracle_lib.gen_tail(k * A, l * v), k * oracle_lib.gen_tail(A, v), rtol=1e-12, atol=1e-13)


def test_tail_welford_form_and_gram(oracle_lib):
    # T_j = sqrt(j/(j+1)) (a_{j+1} - mean(a_1..a_j)); [H;T] has the Gram of A
    rng = np.random.default_rng(8)
    A = rng.standard_normal((12, 3))
    T = oracle_lib.tail(A)
    for j in range(1, 12):
        ref = math.sqrt(j / (j + 1)) * (A[j] - A[:j].mean(axis=0))
        assert np.allclose(T[j - 1], ref, rtol=1e-13, atol=1e-14)
    HT = np.vstack([oracle_lib.head(A), T])
    assert np.allclose(HT.T @ HT, A.T @ A, rtol=1e-13, atol=1e-13)


def test_planted_sign_mistake_is_caught(oracle_lib, monkeypatch):
    """A plausible mistake in the generalized tail (index shifted from v[j+1]
    to v[j]) must fail the Lemma 2 pin."""
    import oracle as O

    def wrong(A, v):
        A = np.asarray(A, float)
        out = np.zeros((A.shape[0] - 1, A.shape[1]))
        for j in range(1, A.shape[0]):
            nj = math.sqrt(np.sum(v[:j] ** 2))
            nj1 = math.sqrt(np.sum(v[:j + 1] ** 2))
            s = (v[:j, None] * A[:j]).sum(axis=0)
            out[j - 1] = (nj * A[j] - v[j - 1] * s / nj) / nj1
        return out
    rng = np.random.default_rng(9)
    v = rng.uniform(0.1, 5.0, 6)
    T = rng.standard_normal((6, 2))
    A = np.column_stack([v[:, None] * 1.0, T])
    U = O.rotations_lemma(v) @ A
    assert np.allclose(U[1:, 1:], O.gen_tail(T, v), atol=1e-12)
    assert not np.allclose(U[1:, 1:], wrong(T, v), atol=1e-6)


# ---------------------------------------------------------------------------
# Count queries (Fig. 4) by brute force
# ---------------------------------------------------------------------------

def test_counts_two_relation_closed_forms(oracle_lib):
    inst = synth.two_relation(21, 9, 7, 1, 1, 3)
    red, cnt = oracle_lib.brute_counts(inst)
    cs = {}
    ct = {}
    for t in range(red.rels[0].rows):
        cs[(int(red.rels[0].keys[0, t]),)] = cs.get((int(red.rels[0].keys[0, t]),), 0) + 1
    for t in range(red.rels[1].rows):
        ct[(int(red.rels[1].keys[0, t]),)] = ct.get((int(red.rels[1].keys[0, t]),), 0) + 1
    for k in cs:
        assert cnt[0]["phi_circ"][k] == ct[k]          # S's tuples each join c_T(k) rows
        assert cnt[0]["rows_per_key"][k] == cs[k]
        assert cnt[1]["phi_up"][k] == cs[k]
        assert cnt[1]["phi_down"][k] == ct[k]
        assert cnt[1]["phi_circ"][k] == cs[k]


@pytest.mark.parametrize("maker", [lambda: synth.paper_fig3(1), lambda: synth.random_chain(3, 4, 5, 1, 2),
                                   lambda: synth.random_star(4, 3, 8, 3, 1, pk_dims=False, dom=3)])
def test_counts_invariants(oracle_lib, maker):
    inst = maker()
    red, cnt = oracle_lib.brute_counts(inst)
    size = oracle_lib.join_size(red)
    assert size == oracle_lib.join_size(inst)
    for i, c in enumerate(cnt):
        # every join row contains exactly one tuple of S_i
        assert sum(c["rows_per_key"][x] * c["phi_circ"][x] for x in c["rows_per_key"]) == size
        if "phi_up" in c:
            assert sum(c["phi_up"][x] * c["phi_down"][x] for x in c["phi_up"]) == size
        if red.rels[i].parent < 0:
            assert sum(c["theta_down"].values()) == size


# ---------------------------------------------------------------------------
# Algorithm 3 (R0), Theorem 6, and the at-scale reference
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("maker", [
    lambda: synth.paper_fig3(1), lambda: synth.paper_fig3(5, m=(5, 8, 4, 6), dom=2),
    lambda: synth.random_chain(6, 3, 6, 2, 2), lambda: synth.random_chain(7, 4, 5, 1, 2),
    lambda: synth.random_star(8, 4, 9, 3, 2), lambda: synth.random_star(9, 3, 9, 3, 2, root=1),
    lambda: synth.cartesian_uniform(10, 4, 2, 5, 2), lambda: synth.two_relation(11, 9, 8, 2, 2, 3),
])
def test_alg3_theorem6(oracle_lib, maker):
    inst = maker()
    blocks, red = oracle_lib.figaro_alg3(inst)
    R0 = oracle_lib.stack_blocks(blocks)
    assert R0.shape[0] <= red.M                          # Theorem 6 (1)
    A = oracle_lib.join(inst)
    Ghi, Glo = oracle_lib.gram_ld(A)
    assert _relf(R0.T @ R0, Ghi + Glo) <= 1e-13          # Theorem 6 (2)
    R, _ = oracle_lib.householder_r(A)
    R0r, _ = oracle_lib.householder_r(np.asfortranarray(R0))
    assert _relf(R0r, R) <= 1e-12


def test_alg3_two_relation_closed_form(oracle_lib):
    """For S -> T on one key: heads [sqrt(c_T) H(S^k) | sqrt(c_S) H(T^k)],
    tails sqrt(c_T) T(S^k) | 0 and 0 | sqrt(c_S) T(T^k)."""
    inst = synth.two_relation(12, 7, 6, 2, 1, 2)
    blocks, red = oracle_lib.figaro_alg3(inst)
    S, T = red.rels
    for b in blocks:
        if b["kind"] == "root":
            root = b["rows"]
    keys = sorted(set(S.keys[0].tolist()))
    for idx, k in enumerate(keys):
        sk = S.values[:, S.keys[0] == k].T
        tk = T.values[:, T.keys[0] == k].T
        expect = np.concatenate([math.sqrt(tk.shape[0]) * oracle_lib.head(sk),
                                 math.sqrt(sk.shape[0]) * oracle_lib.head(tk)])
        assert np.allclose(root[idx], expect, rtol=1e-13)


def test_appendix_a_ground_truth(oracle_lib):
    inst, RS, m2 = synth.appendix_a(3, m1=6, n1=3, m2_root=3, n2=2)
    R = oracle_lib.r_of_join(inst)
    n1 = RS.shape[0]
    assert _relf(R[:n1, :n1], math.sqrt(m2) * RS) <= 1e-13
    blocks, _ = oracle_lib.figaro_alg3(inst)
    R0r, _ = oracle_lib.householder_r(np.asfortranarray(oracle_lib.stack_blocks(blocks)))
    assert _relf(R0r[:n1, :n1], math.sqrt(m2) * RS) <= 1e-13


@pytest.mark.parametrize("maker", [
    lambda: synth.config1(), lambda: synth.paper_fig3(2), lambda: synth.random_chain(3, 4, 30, 3, 5),
    lambda: synth.random_star(4, 4, 200, 20, 3), lambda: synth.config3(div=2000),
    lambda: synth.config2(div=2000), lambda: synth.cartesian_uniform(5, 20, 3, 30, 2),
])
def test_factorized_reference_matches_materialized(oracle_lib, maker):
    inst = maker()
    A = oracle_lib.join(inst)
    Ghi, Glo = oracle_lib.gram_ld(A)
    Fhi, Flo, rows = oracle_lib.factorized_gram(inst)
    assert rows == A.shape[0]
    assert _relf(Fhi + Flo, Ghi + Glo) <= 1e-15
    R, _ = oracle_lib.householder_r(A)
    Rf, _ = oracle_lib.factorized_r(inst)
    assert _relf(Rf, R) <= 1e-11


@pytest.mark.parametrize("maker", [lambda: synth.paper_fig3(3), lambda: synth.two_relation(4, 12, 9, 2, 3, 3),
                                   lambda: synth.random_star(5, 3, 15, 4, 2)])
def test_gradient_references_agree(oracle_lib, maker):
    """Autograd through the materialised QR equals the closed form
    d(sum log R_ii)/dA = A (A^T A)^{-1} pushed through the join's adjoint."""
    import torch
    inst = maker()
    g_auto, _ = oracle_lib.grad_autograd(inst, lambda R: torch.log(torch.diagonal(R)).sum())
    g_closed = oracle_lib.grad_logdet_closed_form(inst)
    for a, b in zip(g_auto, g_closed):
        assert _relf(a, b) <= 1e-10


# ---------------------------------------------------------------------------
# Q, SVD and PCA of the join (section "From R to Q, SVD and PCA")
# ---------------------------------------------------------------------------

BEYOND = [lambda: synth.config1(), lambda: synth.paper_fig3(5, m=(40, 90, 30, 30), n=(3, 2, 4, 1), dom=3),
          lambda: synth.random_chain(3, 3, 60, 2, 6), lambda: synth.random_star(4, 4, 80, 10, 2)]


@pytest.mark.parametrize("maker", BEYOND)
def test_q_of_join_is_orthonormal_and_reproduces_the_join(oracle_lib, maker):
    inst = maker()
    Q, ids = oracle_lib.q_of_join(inst)
    A = oracle_lib.join(inst)
    R = oracle_lib.r_of_join(inst)
    n = inst.n
    assert Q.shape == A.shape and ids.shape == (inst.r, A.shape[0])
    # rounding of sums over the join rows grows like their square root
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 1e-14 * np.sqrt(A.shape[0]) * n
    assert np.linalg.norm(Q @ R - A) <= 1e-13 * np.linalg.norm(A)


@pytest.mark.parametrize("maker", BEYOND)
def test_svd_of_join_matches_its_invariants(oracle_lib, maker):
    """U^T U = I, U diag(sigma) V^T = A, sigma decreasing, sigma^2 the
    eigenvalues of A^T A (long double Gram), and the singular values and
    right singular vectors of A those of R (the paper's second step)."""
    inst = maker()
    U, s, V, ids = oracle_lib.svd_of_join(inst)
    A = oracle_lib.join(inst)
    n = inst.n
    assert np.all(np.diff(s) <= 0)
    assert np.linalg.norm(U.T @ U - np.eye(n)) <= 1e-14 * np.sqrt(A.shape[0]) * n
    assert np.linalg.norm(V.T @ V - np.eye(n)) <= 1e-12
    assert np.linalg.norm((U * s) @ V.T - A) <= 1e-13 * np.linalg.norm(A)
    Ghi, Glo = oracle_lib.gram_ld(A)
    ev = np.sort(np.linalg.eigvalsh(Ghi + Glo))[::-1]
    assert np.max(np.abs(s ** 2 - ev)) <= 1e-12 * ev[0]
    R = oracle_lib.r_of_join(inst)
    sr = np.linalg.svd(R, compute_uv=False)
    assert np.max(np.abs(sr - s)) <= 1e-11 * s[0]

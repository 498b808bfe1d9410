"""CPU ORACLE -- test infrastructure only.

Plain, slow, obviously-correct CPU reference for the upper-triangular factor R
of the QR decomposition of an acyclic natural join (and for the intermediate
quantities the method defines).  Only `tests/`, the smoke check and the
`cpu_baseline` leg of the benchmark may import this package; the HIP library
never does, and the two share no code.  Inputs come from the `synth` package,
which holds no arithmetic of the method.

Contents, each following one passage of the paper:
  * join / r_of_join         natural join by index nested loops, textbook
                             Householder QR, non-negative diagonal (setup
                             section "Output": R is unique for full-rank A with
                             positive diagonal) -- C, figaro_oracle.c
  * givens_r                 brute-force Givens QR (Definition 1, Bindel's sign)
  * gram_ld, gram_relerr,
    logabsdet                A^T A and log det(A^T A) in long double
  * factorized_gram,
    factorized_r             A^T A summed over the join tree without
                             materialising it, Cholesky in __float128
  * head, tail               Definition "Head and Tail"
  * gen_head, gen_tail       Definition 2 (generalized head and tail)
  * rotations_lemma          the explicit rotation sequence of Lemmas 1 and 2
  * brute_counts             the count queries of Fig. 4 by brute force
  * q_of_join, svd_of_join   section "From R to Q, SVD and PCA": Q = A R^-1
                             of the materialised join (R from r_of_join),
                             the SVD of the materialised join by LAPACK
  * figaro_alg3              Algorithm 3 (heads_and_tails,
                             process_and_join_children,
                             project_away_join_attributes) in the paper's order

Parity status: every function above is pinned by tests in
tests/test_oracle.py against closed forms, brute force or identities that do
not reuse its own code.
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
import subprocess
from typing import Dict, List, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "figaro_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_figaro_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C part of the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lquadmath", "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _ORel(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("k", ctypes.c_int32),
                ("attrs", ctypes.POINTER(ctypes.c_int32)),
                ("keys", ctypes.POINTER(ctypes.c_int64)),
                ("n", ctypes.c_int32), ("vals", ctypes.POINTER(ctypes.c_double)),
                ("parent", ctypes.c_int32)]


def _load():
    global _lib
    if _lib is None:
        path = _LIB_PATH if os.path.exists(_LIB_PATH) else build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.or_join.restype = ctypes.c_int64
        lib.or_join.argtypes = [ctypes.c_int, ctypes.POINTER(_ORel), dp, ctypes.c_int64, ctypes.c_int64]
        lib.or_join_idx.restype = ctypes.c_int64
        lib.or_join_idx.argtypes = [ctypes.c_int, ctypes.POINTER(_ORel), ctypes.POINTER(ctypes.c_int64),
                                    ctypes.c_int64, ctypes.c_int64]
        lib.or_householder_r.restype = ctypes.c_int
        lib.or_householder_r.argtypes = [ctypes.c_int64, ctypes.c_int32, dp, ctypes.c_int64, dp]
        lib.or_givens_r.restype = ctypes.c_int
        lib.or_givens_r.argtypes = [ctypes.c_int64, ctypes.c_int32, dp, ctypes.c_int64, dp]
        lib.or_gram_ld.restype = None
        lib.or_gram_ld.argtypes = [ctypes.c_int64, ctypes.c_int32, dp, ctypes.c_int64, dp, dp]
        lib.or_gram_relerr.restype = ctypes.c_double
        lib.or_gram_relerr.argtypes = [ctypes.c_int32, dp, dp, dp]
        lib.or_logabsdet.restype = ctypes.c_double
        lib.or_logabsdet.argtypes = [ctypes.c_int32, dp, dp]
        lib.or_factorized_gram.restype = ctypes.c_int
        lib.or_factorized_gram.argtypes = [ctypes.c_int, ctypes.POINTER(_ORel), dp, dp, dp]
        lib.or_factorized_r.restype = ctypes.c_int
        lib.or_factorized_r.argtypes = [ctypes.c_int, ctypes.POINTER(_ORel), dp, dp]
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _orels(inst):
    """Marshal a synth.Instance into the C structs (keys widened to int64)."""
    keep = []
    arr = (_ORel * inst.r)()
    for i, rel in enumerate(inst.rels):
        attrs = np.ascontiguousarray(np.asarray(rel.key_attrs, dtype=np.int32))
        keys = np.ascontiguousarray(rel.keys.astype(np.int64)) if rel.keys.size else \
            np.zeros((0, rel.rows), np.int64)
        vals = np.ascontiguousarray(rel.values, dtype=np.float64)
        keep += [attrs, keys, vals]
        arr[i].m = rel.rows
        arr[i].k = len(rel.key_attrs)
        arr[i].attrs = attrs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        arr[i].keys = keys.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        arr[i].n = rel.ncols
        arr[i].vals = _dp(vals)
        arr[i].parent = rel.parent
    return arr, keep


# ---------------------------------------------------------------------------
# Join, Householder, Givens, checks (C)
# ---------------------------------------------------------------------------

def join_size(inst) -> int:
    lib = _load()
    arr, keep = _orels(inst)
    rows = lib.or_join(inst.r, arr, None, 0, 0)
    if rows < 0:
        raise ValueError("invalid join tree")
    return int(rows)


def join(inst, max_rows: int | None = None) -> np.ndarray:
    """Materialise the natural join's data columns as a Fortran-ordered
    (rows x n) float64 matrix; columns in relation order, then schema order."""
    lib = _load()
    rows = join_size(inst) if max_rows is None else max_rows
    arr, keep = _orels(inst)
    A = np.zeros((inst.n, max(rows, 1)), dtype=np.float64)   # [n][rows] == column-major
    got = lib.or_join(inst.r, arr, _dp(A), max(rows, 1), max(rows, 1))
    if got < 0:
        raise ValueError("join enumeration failed")
    return np.asfortranarray(A[:, :got].T)


def join_indices(inst) -> np.ndarray:
    """The join as tuple indices: (r, rows) array, entry [i, row] is the tuple
    of relation i in that join row (same row order as join())."""
    lib = _load()
    rows = join_size(inst)
    arr, keep = _orels(inst)
    idx = np.zeros((inst.r, max(rows, 1)), dtype=np.int64)
    got = lib.or_join_idx(inst.r, arr, idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), max(rows, 1),
                          max(rows, 1))
    if got < 0:
        raise ValueError("join enumeration failed")
    return idx[:, :got]


def householder_r(A: np.ndarray) -> Tuple[np.ndarray, int]:
    """Textbook Householder QR; returns (R with non-negative diagonal, number
    of zero diagonal entries)."""
    lib = _load()
    m, n = A.shape
    W = np.array(A, dtype=np.float64, order="F", copy=True)
    R = np.zeros((n, n), dtype=np.float64, order="F")
    z = lib.or_householder_r(m, n, _dp(W), max(m, 1), _dp(R))
    return R, int(z)


def givens_r(A: np.ndarray) -> np.ndarray:
    lib = _load()
    m, n = A.shape
    W = np.array(A, dtype=np.float64, order="F", copy=True)
    R = np.zeros((n, n), dtype=np.float64, order="F")
    lib.or_givens_r(m, n, _dp(W), max(m, 1), _dp(R))
    return R


def gram_ld(A: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    lib = _load()
    m, n = A.shape
    W = np.asfortranarray(A, dtype=np.float64)
    Ghi = np.zeros((n, n), order="F")
    Glo = np.zeros((n, n), order="F")
    lib.or_gram_ld(m, n, _dp(W), max(m, 1), _dp(Ghi), _dp(Glo))
    return Ghi, Glo


def gram_relerr(R: np.ndarray, Ghi: np.ndarray, Glo: np.ndarray) -> float:
    lib = _load()
    n = R.shape[0]
    Rf = np.asfortranarray(R, dtype=np.float64)
    return float(lib.or_gram_relerr(n, _dp(Rf), _dp(np.asfortranarray(Ghi)),
                                    _dp(np.asfortranarray(Glo))))


def logabsdet(Ghi: np.ndarray, Glo: np.ndarray) -> float:
    lib = _load()
    n = Ghi.shape[0]
    return float(lib.or_logabsdet(n, _dp(np.asfortranarray(Ghi)), _dp(np.asfortranarray(Glo))))


def factorized_gram(inst) -> Tuple[np.ndarray, np.ndarray, float]:
    """A^T A of the join summed by distributivity (never materialised), as
    hi + lo float64 pairs, and the join size."""
    lib = _load()
    arr, keep = _orels(inst)
    n = inst.n
    Ghi = np.zeros((n, n), order="F")
    Glo = np.zeros((n, n), order="F")
    rows = ctypes.c_double(0.0)
    st = lib.or_factorized_gram(inst.r, arr, _dp(Ghi), _dp(Glo), ctypes.byref(rows))
    if st != 0:
        raise ValueError("factorized_gram failed")
    return Ghi, Glo, rows.value


def factorized_r(inst) -> Tuple[np.ndarray, float]:
    """R = chol(A^T A) computed in __float128 from the factorised Gram matrix."""
    lib = _load()
    arr, keep = _orels(inst)
    n = inst.n
    R = np.zeros((n, n), order="F")
    rows = ctypes.c_double(0.0)
    st = lib.or_factorized_r(inst.r, arr, _dp(R), ctypes.byref(rows))
    if st < 0:
        raise ValueError("factorized_r failed")
    if st == 1:
        raise np.linalg.LinAlgError("join matrix is rank deficient")
    return R, rows.value


def r_of_join(inst) -> np.ndarray:
    """The plain definition: materialise the join, Householder QR, positive
    diagonal."""
    A = join(inst)
    R, zeros = householder_r(A)
    return R


# ---------------------------------------------------------------------------
# Heads and tails (definitions), explicit rotations (Lemmas 1 and 2)
# ---------------------------------------------------------------------------

def head(A: np.ndarray) -> np.ndarray:
    """H(A) = (1/sqrt(m)) sum_i A[i,:]   (Definition "Head and Tail")."""
    A = np.asarray(A, dtype=np.float64)
    m = A.shape[0]
    return A.sum(axis=0) / math.sqrt(m)


def tail(A: np.ndarray) -> np.ndarray:
    """T(A)[j,:] = (sqrt(j) A[j+1,:] - (sum_{i<=j} A[i,:]) / sqrt(j)) / sqrt(j+1),
    j = 1..m-1 (1-based), Definition "Head and Tail"."""
    A = np.asarray(A, dtype=np.float64)
    m = A.shape[0]
    out = np.zeros((max(m - 1, 0),) + A.shape[1:])
    csum = np.cumsum(A, axis=0)
    for j in range(1, m):
        out[j - 1] = (math.sqrt(j) * A[j] - csum[j - 1] / math.sqrt(j)) / math.sqrt(j + 1)
    return out


def gen_head(A: np.ndarray, v: np.ndarray) -> np.ndarray:
    """H(A, v) = (1/||v||) sum_i v[i] A[i,:]   (Definition 2)."""
    A = np.asarray(A, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    return (v[:, None] * A).sum(axis=0) / math.sqrt(float(np.sum(v * v)))


def gen_tail(A: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Definition 2, with the garbled alignment read as
    T(A,v)[j,:] = ( ||v[1..j]|| A[j+1,:] - v[j+1] (sum_{i<=j} v[i] A[i,:]) / ||v[1..j]|| )
                  / ||v[1..j+1]||,   j = 1..m-1."""
    A = np.asarray(A, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    m = A.shape[0]
    out = np.zeros((max(m - 1, 0),) + A.shape[1:])
    for j in range(1, m):
        nj = math.sqrt(float(np.sum(v[:j] ** 2)))
        nj1 = math.sqrt(float(np.sum(v[:j + 1] ** 2)))
        s = (v[:j, None] * A[:j]).sum(axis=0)
        out[j - 1] = (nj * A[j] - v[j] * s / nj) / nj1
    return out


def givens_matrix(d: int, i: int, j: int, sin: float, cos: float) -> np.ndarray:
    """Giv_d(i, j, sin, cos) of Definition 1 (1-based i, j)."""
    G = np.eye(d)
    G[i - 1, i - 1] = cos
    G[j - 1, j - 1] = cos
    G[i - 1, j - 1] = -sin
    G[j - 1, i - 1] = sin
    return G


def rotations_lemma(v: np.ndarray) -> np.ndarray:
    """G = R_m ... R_2 with R_i = Giv_m(1, i, -v_i/||v_1..i||, ||v_1..i-1||/||v_1..i||)
    (Lemma 2; with v = 1 this is Lemma 1)."""
    v = np.asarray(v, dtype=np.float64)
    m = v.shape[0]
    G = np.eye(m)
    for i in range(2, m + 1):
        ni = math.sqrt(float(np.sum(v[:i] ** 2)))
        ni1 = math.sqrt(float(np.sum(v[:i - 1] ** 2)))
        G = givens_matrix(m, 1, i, -v[i - 1] / ni, ni1 / ni) @ G
    return G


# ---------------------------------------------------------------------------
# Brute-force joins and the count queries of Fig. 4
# ---------------------------------------------------------------------------

def _tuples(rel):
    """Rows of a relation as (dict attr -> value, row index)."""
    out = []
    for t in range(rel.rows):
        out.append(({a: int(rel.keys[p, t]) for p, a in enumerate(rel.key_attrs)}, t))
    return out


def brute_join_rows(inst, subset: List[int]):
    """All combinations of tuples of the relations in `subset` that agree on
    every shared attribute (natural join by definition).  Each result is a
    tuple of row indices, one per relation of `subset`."""
    tuples = [_tuples(inst.rels[i]) for i in subset]
    res = []
    for combo in itertools.product(*tuples):
        asg = {}
        ok = True
        for (kv, _t) in combo:
            for a, x in kv.items():
                if asg.setdefault(a, x) != x:
                    ok = False
                    break
            if not ok:
                break
        if ok:
            res.append(tuple(t for (_kv, t) in combo))
    return res


def tree_children(inst, i):
    return [j for j, rel in enumerate(inst.rels) if rel.parent == i]


def subtree(inst, i):
    out = [i]
    for j in tree_children(inst, i):
        out += subtree(inst, j)
    return sorted(out)


def _key(rel, t, attrs):
    """Projection of row t of rel onto `attrs` (sorted attribute ids)."""
    pos = {a: p for p, a in enumerate(rel.key_attrs)}
    return tuple(int(rel.keys[pos[a], t]) for a in attrs)


def parent_attrs(inst, i):
    rel = inst.rels[i]
    if rel.parent < 0:
        return []
    return sorted(set(rel.key_attrs) & set(inst.rels[rel.parent].key_attrs))


def shared(inst, i, j):
    return sorted(set(inst.rels[i].key_attrs) & set(inst.rels[j].key_attrs))


def reduce_instance(inst):
    """Full reduction by definition: keep the tuples that occur in at least one
    row of the join (tiny inputs only).  Returns (reduced instance, kept row
    indices per relation)."""
    import copy
    rows = brute_join_rows(inst, list(range(inst.r)))
    kept = [sorted({combo[i] for combo in rows}) for i in range(inst.r)]
    red = copy.deepcopy(inst)
    for i, rel in enumerate(red.rels):
        idx = np.asarray(kept[i], dtype=np.int64)
        rel.keys = rel.keys[:, idx] if rel.keys.shape[0] else np.zeros((0, len(idx)), np.int32)
        rel.values = rel.values[:, idx]
    return red, kept


def brute_counts(inst):
    """Count queries of Fig. 4 and the per-key row counts, by brute force over
    the fully reduced relations.  Returns per relation a dict with
    'rows_per_key', 'phi_circ', 'theta_down' keyed by the projection onto X_i,
    and 'phi_up', 'phi_down' keyed by the projection onto X_p (attribute ids
    sorted)."""
    red, _ = reduce_instance(inst)
    r = red.r
    out = []
    for i in range(r):
        rel = red.rels[i]
        Xi = sorted(rel.key_attrs)
        Xp = parent_attrs(red, i)
        sub = subtree(red, i)
        others = [j for j in range(r) if j != i]
        upper = [j for j in range(r) if j not in sub]
        rpk: Dict[tuple, int] = {}
        for t in range(rel.rows):
            k = _key(rel, t, Xi)
            rpk[k] = rpk.get(k, 0) + 1

        def grouped(subset, attrs):
            cnt: Dict[tuple, int] = {}
            for combo in brute_join_rows(red, subset):
                asg = {}
                for pos, j in enumerate(subset):
                    rj = red.rels[j]
                    for p, a in enumerate(rj.key_attrs):
                        asg[a] = int(rj.keys[p, combo[pos]])
                k = tuple(asg[a] for a in attrs)
                cnt[k] = cnt.get(k, 0) + 1
            return cnt

        phi_circ = grouped(others, Xi) if others else {(): 1}
        theta = grouped(sub, Xi)
        d = {"rows_per_key": rpk,
             "phi_circ": {k: phi_circ.get(k, 0) for k in rpk},
             "theta_down": {k: theta.get(k, 0) for k in rpk}}
        if rel.parent >= 0:
            pk = {_key(rel, t, Xp) for t in range(rel.rows)}
            up = grouped(upper, Xp)
            down = grouped(sub, Xp)
            d["phi_up"] = {k: up.get(k, 0) for k in pk}
            d["phi_down"] = {k: down.get(k, 0) for k in pk}
        out.append(d)
    return red, out


# ---------------------------------------------------------------------------
# Algorithm 3, in the paper's order, for small inputs
# ---------------------------------------------------------------------------

def figaro_alg3(inst):
    """Algorithm 3 on the fully reduced instance, with the count queries taken
    from their definitions (brute_counts).  Readings: the products over j and
    j' range over the children of S_i; tails are scaled by the square roots
    of the counts.  Returns (R0 blocks, reduced instance); each block is a
    dict with keys 'rel', 'kind' ('tail', 'gen_tail' or 'root'), 'rows'
    (k x n array in global columns)."""
    red, counts = brute_counts(inst)
    r = red.r
    n = red.n
    col_off = np.cumsum([0] + [rel.ncols for rel in red.rels])
    blocks: List[dict] = []

    def cols_of(k):
        return slice(int(col_off[k]), int(col_off[k + 1]))

    def FiGaRo(i):
        rel = red.rels[i]
        Xi = sorted(rel.key_attrs)
        ch = tree_children(red, i)
        # heads_and_tails
        groups: Dict[tuple, List[int]] = {}
        for t in range(rel.rows):
            groups.setdefault(_key(rel, t, Xi), []).append(t)
        Data: Dict[tuple, np.ndarray] = {}
        scales: Dict[tuple, float] = {}
        for x in sorted(groups):
            A = rel.values[:, groups[x]].T
            T = tail(A) * math.sqrt(counts[i]["phi_circ"][x])
            rows = np.zeros((T.shape[0], n))
            rows[:, cols_of(i)] = T
            blocks.append({"rel": i, "kind": "tail", "rows": rows})
            d = np.zeros(n)
            d[cols_of(i)] = head(A)
            Data[x] = d
            scales[x] = math.sqrt(len(groups[x]))
        if ch:
            # process_and_join_children
            child = {j: FiGaRo(j) for j in ch}
            for x in list(Data):
                asg = dict(zip(Xi, x))
                xij = {j: tuple(asg[a] for a in shared(red, i, j)) for j in ch}
                new = Data[x].copy()
                for j in ch:
                    Dj, Sj = child[j]
                    f = scales[x]
                    for j2 in ch:
                        if j2 != j:
                            f *= child[j2][1][xij[j2]]
                    for k in subtree(red, j):
                        new[cols_of(k)] = Dj[xij[j]][cols_of(k)] * f
                prod = 1.0
                for j in ch:
                    prod *= child[j][1][xij[j]]
                new[cols_of(i)] = Data[x][cols_of(i)] * prod
                Data[x] = new
                scales[x] = scales[x] * prod
            if rel.parent >= 0:
                # project_away_join_attributes
                Xp = parent_attrs(red, i)
                pg: Dict[tuple, List[tuple]] = {}
                for x in sorted(Data):
                    asg = dict(zip(Xi, x))
                    pg.setdefault(tuple(asg[a] for a in Xp), []).append(x)
                sub_cols = np.concatenate([np.arange(col_off[k], col_off[k + 1])
                                           for k in subtree(red, i)])
                D2, S2 = {}, {}
                for xp in sorted(pg):
                    D = np.stack([Data[x] for x in pg[xp]])[:, sub_cols]
                    v = np.array([scales[x] for x in pg[xp]])
                    T = gen_tail(D, v) * math.sqrt(counts[i]["phi_up"][xp])
                    rows = np.zeros((T.shape[0], n))
                    rows[:, sub_cols] = T
                    blocks.append({"rel": i, "kind": "gen_tail", "rows": rows})
                    h = np.zeros(n)
                    h[sub_cols] = gen_head(D, v)
                    D2[xp] = h
                    S2[xp] = math.sqrt(counts[i]["phi_down"][xp])
                Data, scales = D2, S2
        if rel.parent < 0:
            rows = np.stack([Data[x] for x in sorted(Data)])
            blocks.append({"rel": i, "kind": "root", "rows": rows})
        return Data, scales

    root = [i for i in range(r) if red.rels[i].parent < 0][0]
    FiGaRo(root)
    return blocks, red


def stack_blocks(blocks) -> np.ndarray:
    rows = [b["rows"] for b in blocks if b["rows"].shape[0] > 0]
    return np.concatenate(rows, axis=0) if rows else np.zeros((0, 0))


# ---------------------------------------------------------------------------
# Gradients (the paper has no backward pass; these are plain references)
# ---------------------------------------------------------------------------

def grad_autograd(inst, loss_fn):
    """Gradients of loss_fn(R) with respect to every relation's values by
    autograd (PyTorch, CPU, FP64) through the QR of the materialised join:
    A = [values_i[:, idx_i]^T], R = qr(A).R with a non-negative diagonal.
    Returns (list of (n_i, m_i) arrays, R)."""
    import torch
    idx = join_indices(inst)
    vs = [torch.tensor(np.ascontiguousarray(rel.values), dtype=torch.float64, requires_grad=True)
          for rel in inst.rels]
    A = torch.cat([vs[i][:, torch.as_tensor(idx[i])].T for i in range(inst.r)], dim=1)
    R = torch.linalg.qr(A, mode="reduced")[1]
    d = torch.diagonal(R)
    R = torch.where(d < 0, -1.0, 1.0)[:, None] * R
    L = loss_fn(R)
    L.backward()
    return [v.grad.numpy().copy() for v in vs], R.detach().numpy()


def grad_logdet_closed_form(inst):
    """d/dvalues of sum_i log R_ii: since sum log R_ii = (1/2) log det(A^T A),
    dA = A (A^T A)^{-1}; the gradient of a tuple's values is the sum of dA
    over the join rows that contain the tuple (the join's adjoint)."""
    A = join(inst)
    idx = join_indices(inst)
    G = A.T @ A
    dA = A @ np.linalg.inv(G)
    out = []
    c0 = 0
    for i, rel in enumerate(inst.rels):
        g = np.zeros_like(rel.values)
        np.add.at(g.T, idx[i], dA[:, c0:c0 + rel.ncols])
        out.append(g)
        c0 += rel.ncols
    return out


def q_of_join(inst) -> Tuple[np.ndarray, np.ndarray]:
    """Q = A R^-1 by its definition (section "From R to Q, SVD and PCA"):
    the materialised join A, R from r_of_join, a triangular solve
    R^T Q^T = A^T.  Returns (Q, the join's tuple indices per row)."""
    import scipy.linalg
    A = join(inst)
    R = r_of_join(inst)
    Q = scipy.linalg.solve_triangular(R, A.T, trans="T", lower=False).T
    return Q, join_indices(inst)


def svd_of_join(inst) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    """The SVD A = U diag(sigma) V^T of the materialised join (LAPACK, thin),
    sigma decreasing.  Returns (U, sigma, V, the join's tuple indices)."""
    A = join(inst)
    U, s, Vt = np.linalg.svd(np.ascontiguousarray(A), full_matrices=False)
    return U, s, Vt.T, join_indices(inst)


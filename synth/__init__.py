"""Seeded synthetic join instances shared by the oracle side and the GPU side.

This module only draws inputs.  It contains none of the arithmetic of the
method (no heads, tails, counts, scale factors or factorizations): it returns
relations as plain arrays, and both the CPU oracle and the HIP library consume
the same arrays.

Data model (the paper's setup section): a database is a list of relations
S_1..S_r.  Relation i has key (join) attributes X_i, given as global attribute
ids, and n_i real-valued data columns Y_i.  A join tree is given by the parent
index of every relation (-1 for the root).  Two relations join on the
attributes whose ids they share (natural join).

Storage conventions used everywhere in this repository:
  * keys   : integer array of shape (k_i, m_i)   -- one row per key attribute
  * values : float64 array of shape (n_i, m_i)   -- column-major m_i x n_i matrix
             (values[c] is data column c, contiguous)

Draw order within one instance is fixed: instance-level parameters first, then
for every relation in index order its key columns (in attribute order) and then
its value columns.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction
from typing import List, Optional

import numpy as np

__all__ = [
    "Rel", "Instance", "config1", "config2", "config3", "config5_instance", "config5_params", "config5_sample",
    "config5", "cartesian_uniform", "appendix_a", "paper_fig3", "random_chain",
    "random_star", "two_relation", "zipf_probs",
]


@dataclass
class Rel:
    key_attrs: List[int]
    keys: np.ndarray          # (k, m) integer
    values: np.ndarray        # (n, m) float64, column-major matrix storage
    parent: int
    name: str = ""

    @property
    def rows(self) -> int:
        return int(self.values.shape[1]) if self.values.ndim == 2 else 0

    @property
    def ncols(self) -> int:
        return int(self.values.shape[0])


@dataclass
class Instance:
    name: str
    rels: List[Rel]
    meta: dict = field(default_factory=dict)

    @property
    def r(self) -> int:
        return len(self.rels)

    @property
    def n(self) -> int:
        return sum(rel.ncols for rel in self.rels)

    @property
    def M(self) -> int:
        return sum(rel.rows for rel in self.rels)


def zipf_probs(num_ids: int, s: float) -> np.ndarray:
    """Zipf(s) probabilities over ids 0..num_ids-1; id 0 is the most frequent."""
    w = 1.0 / np.arange(1, num_ids + 1, dtype=np.float64) ** s
    return w / w.sum()


def _normal(rng, n, m):
    return rng.standard_normal((n, m))


# ---------------------------------------------------------------------------
# The five workload configurations.
# ---------------------------------------------------------------------------

def config1(seed: int = 1001) -> Instance:
    """S(a, x1..x4) join T(a, y1..y3), 1000 tuples each, a uniform over 100 values.

    Root S, child T; values i.i.d. N(0, 1)."""
    rng = np.random.default_rng(seed)
    m = 1000
    ka = rng.integers(0, 100, m).astype(np.int32)
    vs = _normal(rng, 4, m)
    kb = rng.integers(0, 100, m).astype(np.int32)
    vt = _normal(rng, 3, m)
    rels = [Rel([0], ka[None, :], vs, -1, "S"), Rel([0], kb[None, :], vt, 0, "T")]
    return Instance("config1", rels, {"seed": seed})


def two_relation(seed: int, m_s: int, m_t: int, n_s: int, n_t: int,
                 num_keys: int, dist: str = "uniform", zipf_s: float = 1.1,
                 key_dtype=np.int32) -> Instance:
    """Generic S(a, Y_S) join T(a, Y_T) on one attribute, S the root."""
    rng = np.random.default_rng(seed)
    if dist == "zipf":
        p = zipf_probs(num_keys, zipf_s)
        ks = rng.choice(num_keys, size=m_s, p=p)
        vs = _normal(rng, n_s, m_s)
        kt = rng.choice(num_keys, size=m_t, p=p)
        vt = _normal(rng, n_t, m_t)
    else:
        ks = rng.integers(0, num_keys, m_s)
        vs = _normal(rng, n_s, m_s)
        kt = rng.integers(0, num_keys, m_t)
        vt = _normal(rng, n_t, m_t)
    rels = [Rel([0], ks.astype(key_dtype)[None, :], vs, -1, "S"),
            Rel([0], kt.astype(key_dtype)[None, :], vt, 0, "T")]
    return Instance(f"two_relation_{dist}", rels,
                    {"seed": seed, "num_keys": num_keys, "dist": dist})


def config2(seed: int = 1002, div: int = 1) -> Instance:
    """Two relations of 2,000,000 tuples each (divided by `div`), 16 N(0,1)
    columns each, join key Zipf(1.1) over the same 1000 ids in both relations
    (id 0 most frequent)."""
    m = 2_000_000 // div
    inst = two_relation(seed, m, m, 16, 16, 1000, "zipf", 1.1)
    inst.name = "config2" if div == 1 else f"config2_div{div}"
    inst.meta.update({"div": div})
    return inst


def config3(seed: int = 1003, div: int = 1) -> Instance:
    """Acyclic star: fact F(k1..k4, 8 cols) with 10^7 rows, four dimensions
    D_j(k_j, 8 cols) of 10^5 rows with a unique key each (both sizes divided by
    `div`); foreign keys uniform.  Values N(0,1) times a per-column scale
    10^U[-3,3] (40 scales, drawn first).  Relation order and join tree:
    0 = D1 (root), 1 = F (child of D1), 2..4 = D2..D4 (children of F)."""
    rng = np.random.default_rng(seed)
    nf = 10_000_000 // div
    nd = 100_000 // div
    scales = 10.0 ** rng.uniform(-3.0, 3.0, 40)
    rels: List[Rel] = []
    # D1
    k = rng.permutation(nd).astype(np.int32)
    v = _normal(rng, 8, nd) * scales[0:8, None]
    rels.append(Rel([0], k[None, :], v, -1, "D1"))
    # F
    kf = rng.integers(0, nd, (4, nf)).astype(np.int32)
    vf = _normal(rng, 8, nf) * scales[8:16, None]
    rels.append(Rel([0, 1, 2, 3], kf, vf, 0, "F"))
    for j in range(1, 4):
        k = rng.permutation(nd).astype(np.int32)
        v = _normal(rng, 8, nd) * scales[8 * (j + 1):8 * (j + 2), None]
        rels.append(Rel([j], k[None, :], v, 1, f"D{j + 1}"))
    name = "config3" if div == 1 else f"config3_div{div}"
    return Instance(name, rels, {"seed": seed, "div": div, "scales": scales})


def _config5_draw(i: int):
    """The instance-level draws of config5_instance(i), in its draw order;
    returns the generator positioned after them."""
    rng = np.random.default_rng(5000 + i)
    topology = "chain" if rng.random() < 0.5 else "star"
    r = int(rng.integers(2, 5))
    m = np.floor(10.0 ** rng.uniform(3.0, 6.0, r)).astype(np.int64)
    n = rng.integers(4, 33, r)
    dist = "zipf" if rng.random() < 0.5 else "uniform"
    return rng, topology, r, m, n, dist


def config5_params(i: int) -> dict:
    """Shape of instance i of the batched workload without drawing its keys
    and values: topology, key distribution, relation count, rows and columns
    per relation."""
    _, topology, r, m, n, dist = _config5_draw(i)
    return {"topology": topology, "dist": dist, "r": r, "rows": [int(x) for x in m],
            "cols": [int(x) for x in n], "n": int(n.sum())}


def config5_instance(i: int) -> Instance:
    """One instance of the batched workload (seed 5000+i).

    Chain or star (probability 1/2), r in {2,3,4}, m_j = floor(10^U[3,6]),
    n_j in {4..32}, keys uniform or Zipf(1.1).  Chains: relation j shares
    attribute e_j with relation j+1; the domain of e_j is max(10, max(m_j,
    m_{j+1}) // 10) for uniform keys, so the expected fan-out per edge is at
    most 10; with Zipf keys only edge e_0 is Zipf (1000 ids), which keeps the
    join size far below 2^53 by construction.  Stars: relation 0 is the fact
    table with one foreign key per dimension; dimension j has a unique key per
    row (a permutation of 0..m_j-1); the fact's foreign keys are uniform over
    the dimension's keys or Zipf over its first min(1000, m_j) keys."""
    rng, topology, r, m, n, dist = _config5_draw(i)
    rels: List[Rel] = []
    if topology == "chain":
        for j in range(r):
            attrs = []
            cols = []
            for e in (j - 1, j):
                if e < 0 or e >= r - 1:
                    continue
                attrs.append(e)
                if dist == "zipf" and e == 0:
                    cols.append(rng.choice(1000, size=int(m[j]), p=zipf_probs(1000, 1.1)))
                else:
                    dom = max(10, int(max(m[e], m[e + 1])) // 10)
                    cols.append(rng.integers(0, dom, int(m[j])))
            keys = np.stack(cols).astype(np.int32)
            vals = _normal(rng, int(n[j]), int(m[j]))
            rels.append(Rel(attrs, keys, vals, j - 1, f"C{j}"))
    else:
        # fact table first
        cols = []
        for j in range(1, r):
            if dist == "zipf":
                ids = min(1000, int(m[j]))
                cols.append(rng.choice(ids, size=int(m[0]), p=zipf_probs(ids, 1.1)))
            else:
                cols.append(rng.integers(0, int(m[j]), int(m[0])))
        keys = np.stack(cols).astype(np.int32)
        vals = _normal(rng, int(n[0]), int(m[0]))
        rels.append(Rel(list(range(r - 1)), keys, vals, -1, "F"))
        for j in range(1, r):
            k = rng.permutation(int(m[j])).astype(np.int32)
            vals = _normal(rng, int(n[j]), int(m[j]))
            rels.append(Rel([j - 1], k[None, :], vals, 0, f"D{j}"))
    return Instance(f"config5_{i}", rels,
                    {"seed": 5000 + i, "topology": topology, "dist": dist})


def config5_sample(per_cell: int = 3, seed: int = 2025):
    """Seeded stratified sample of the 512 instances of the batched workload:
    the instances are grouped by (topology, key distribution, number of
    relations, column bucket n <= 32 / <= 64 / <= 96 / > 96), and from every
    group up to `per_cell` ids are drawn without replacement with
    numpy.random.default_rng(seed)."""
    cells = {}
    for i in range(512):
        p = config5_params(i)
        nb = 0 if p["n"] <= 32 else 1 if p["n"] <= 64 else 2 if p["n"] <= 96 else 3
        cells.setdefault((p["topology"], p["dist"], p["r"], nb), []).append(i)
    rng = np.random.default_rng(seed)
    out = []
    for key in sorted(cells):
        ids = cells[key]
        out += rng.choice(ids, size=min(per_cell, len(ids)), replace=False).tolist()
    return sorted(int(i) for i in out)


def config5(count: int = 512, start: int = 0) -> List[Instance]:
    return [config5_instance(i) for i in range(start, start + count)]


# ---------------------------------------------------------------------------
# Small structured instances for tests.
# ---------------------------------------------------------------------------

def cartesian_uniform(seed: int, m_s: int, n_s: int, m_t: int, n_t: int) -> Instance:
    """Cartesian product S x T of two keyless relations with entries uniform in
    [-3, 3), as in the paper's synthetic experiments."""
    rng = np.random.default_rng(seed)
    vs = rng.uniform(-3.0, 3.0, (n_s, m_s))
    vt = rng.uniform(-3.0, 3.0, (n_t, m_t))
    empty = np.zeros((0, m_s), np.int32)
    rels = [Rel([], empty, vs, -1, "S"), Rel([], np.zeros((0, m_t), np.int32), vt, 0, "T")]
    return Instance("cartesian", rels, {"seed": seed})


def _rational_unit_vector(rng, m: int, den: int = 7) -> List[Fraction]:
    """A unit vector with rational entries (inverse stereographic projection of
    a random rational point); its first entry is never -1."""
    w = [Fraction(int(rng.integers(-den, den + 1)), den) for _ in range(m - 1)]
    s = sum(x * x for x in w)
    return [(1 - s) / (1 + s)] + [2 * x / (1 + s) for x in w]


def appendix_a(seed: int, m1: int, n1: int, m2_root: int, n2: int):
    """Cartesian-product instance with a known leading block of R.

    S = Qhat[:, :n1] R_S with Qhat = -I + (v + e1)(v + e1)^T / (1 + v1) for a
    rational unit vector v (an orthogonal matrix of rationals), R_S an upper
    triangular matrix with small integer entries and positive diagonal, and T an
    m2 x n2 matrix of natural numbers with m2 = m2_root^2.  S is formed exactly
    in rationals and rounded once to float64.

    Returns (instance, R_S as float64, m2)."""
    rng = np.random.default_rng(seed)
    v = _rational_unit_vector(rng, m1)
    u = list(v)
    u[0] = u[0] + 1
    d = 1 + v[0]
    RS = [[Fraction(0)] * n1 for _ in range(n1)]
    for i in range(n1):
        RS[i][i] = Fraction(int(rng.integers(1, 10)))
        for j in range(i + 1, n1):
            RS[i][j] = Fraction(int(rng.integers(-9, 10)))
    # Q[:, j] for j < n1
    S = np.zeros((n1, m1))
    for col in range(n1):
        acc = [Fraction(0)] * m1
        for k in range(col + 1):
            rk = RS[k][col]
            if rk == 0:
                continue
            # column k of Qhat: -e_k + u * u[k] / d
            for row in range(m1):
                q = u[row] * u[k] / d - (1 if row == k else 0)
                acc[row] += q * rk
        S[col, :] = [float(x) for x in acc]
    m2 = m2_root * m2_root
    T = rng.integers(0, 10, (n2, m2)).astype(np.float64)
    rels = [Rel([], np.zeros((0, m1), np.int32), S, -1, "S"),
            Rel([], np.zeros((0, m2), np.int32), T, 0, "T")]
    RSf = np.array([[float(x) for x in row] for row in RS])
    return Instance("appendix_a", rels, {"seed": seed}), RSf, m2


def paper_fig3(seed: int, m=(6, 9, 5, 5), n=(2, 2, 2, 2), dom=2) -> Instance:
    """The four-relation example of the paper's worked example section:
    S1(A, Y1), S2(A, B, C, Y2), S3(B, Y3), S4(C, Y4) with join tree
    S1 - S2 - {S3, S4}; attribute ids A=0, B=1, C=2."""
    rng = np.random.default_rng(seed)
    rels = []
    spec = [([0], -1), ([0, 1, 2], 0), ([1], 1), ([2], 1)]
    for i, (attrs, par) in enumerate(spec):
        keys = rng.integers(0, dom, (len(attrs), m[i])).astype(np.int32)
        vals = _normal(rng, n[i], m[i])
        rels.append(Rel(attrs, keys, vals, par, f"S{i + 1}"))
    return Instance("paper_fig3", rels, {"seed": seed})


def random_chain(seed: int, r: int, m: int, n: int, dom: int, dist="uniform") -> Instance:
    """A chain S_0 - S_1 - ... - S_{r-1}; S_j and S_{j+1} share attribute j."""
    rng = np.random.default_rng(seed)
    rels = []
    for j in range(r):
        attrs = [e for e in (j - 1, j) if 0 <= e < r - 1]
        if dist == "zipf":
            p = zipf_probs(dom, 1.1)
            keys = np.stack([rng.choice(dom, size=m, p=p) for _ in attrs]) if attrs \
                else np.zeros((0, m), np.int64)
        else:
            keys = rng.integers(0, dom, (len(attrs), m))
        vals = _normal(rng, n, m)
        rels.append(Rel(attrs, keys.astype(np.int32), vals, j - 1, f"C{j}"))
    return Instance("chain", rels, {"seed": seed})


def random_star(seed: int, r: int, m_fact: int, m_dim: int, n: int,
                pk_dims: bool = True, dom: Optional[int] = None,
                root: int = 0) -> Instance:
    """A star with fact table 0 and dimensions 1..r-1 (fact shares attribute
    j-1 with dimension j).  With pk_dims each dimension holds every key of its
    domain exactly once.  `root` selects which relation is the root of the
    join tree (0 = fact; j = dimension j, which then has the fact as child)."""
    rng = np.random.default_rng(seed)
    d = dom if dom is not None else m_dim
    keys = rng.integers(0, d, (r - 1, m_fact)).astype(np.int32)
    rels = [Rel(list(range(r - 1)), keys, _normal(rng, n, m_fact), -1, "F")]
    for j in range(1, r):
        if pk_dims:
            k = rng.permutation(d).astype(np.int32)
        else:
            k = rng.integers(0, d, m_dim).astype(np.int32)
        rels.append(Rel([j - 1], k[None, :], _normal(rng, n, k.shape[0]), 0, f"D{j}"))
    if root != 0:
        # re-hang the tree: the chosen dimension becomes the root, the fact its child
        for j in range(1, r):
            rels[j].parent = 0
        rels[root].parent = -1
        rels[0].parent = root
    return Instance("star", rels, {"seed": seed, "root": root})

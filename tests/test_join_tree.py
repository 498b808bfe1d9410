"""Join-tree selection (experiments section, "Effect of join trees"): the
chooser against brute force over every spanning tree and root of small
schemas, its counts against an analysis-only plan, and the cases the paper
names (a key/foreign-key star must not be rooted at its fact table; a cyclic
join has no join tree).  Host only: keys on the host."""
import itertools

import numpy as np
import pytest

import synth
import paper_2204_00525_amd as F


def _distinct(rel, attrs):
    if rel.rows == 0:
        return 0
    if not attrs:
        return 1
    pos = {a: p for p, a in enumerate(rel.key_attrs)}
    return len({tuple(int(rel.keys[pos[a], t]) for a in attrs) for t in range(rel.rows)})


def _valid(inst, edges):
    """Every attribute's relations form a connected part of the tree, and
    every key attribute is held by another relation too."""
    holders = {}
    for i, rel in enumerate(inst.rels):
        for a in rel.key_attrs:
            holders.setdefault(a, set()).add(i)
    for a, hs in holders.items():
        if len(hs) < 2:
            return False
        inner = sum(1 for i, j in edges if i in hs and j in hs)
        if inner != len(hs) - 1:
            return False
    return True


def _trees(r):
    """All spanning trees of the complete graph on r nodes (edge lists)."""
    pairs = [(i, j) for i in range(r) for j in range(i + 1, r)]
    for es in itertools.combinations(pairs, r - 1):
        comp = list(range(r))
        ok = True
        for i, j in es:
            a, b = comp[i], comp[j]
            if a == b:
                ok = False
                break
            comp = [a if c == b else c for c in comp]
        if ok:
            yield list(es)


def _score(inst, edges, root):
    r = inst.r
    adj = {i: [] for i in range(r)}
    for i, j in edges:
        adj[i].append(j)
        adj[j].append(i)
    parent = {root: -1}
    order = [root]
    for v in order:
        for w in adj[v]:
            if w not in parent:
                parent[w] = v
                order.append(w)
    nsub = {i: inst.rels[i].ncols for i in range(r)}
    for v in reversed(order):
        if parent[v] >= 0:
            nsub[parent[v]] += nsub[v]
    cost = 0.0
    for i, rel in enumerate(inst.rels):
        G = _distinct(rel, sorted(rel.key_attrs))
        cost += (rel.rows - G) * rel.ncols ** 2
        if parent[i] >= 0:
            shared = sorted(set(rel.key_attrs) & set(inst.rels[parent[i]].key_attrs))
            cost += (G - _distinct(rel, shared)) * nsub[i] ** 2
        else:
            cost += G * nsub[i] ** 2
    return cost, [parent[i] for i in range(r)]


SCHEMAS = [lambda: synth.paper_fig3(1), lambda: synth.paper_fig3(2, m=(4, 7, 3, 3), dom=3),
           lambda: synth.random_chain(3, 4, 6, 1, 2), lambda: synth.random_chain(4, 3, 9, 2, 3),
           lambda: synth.random_star(4, 4, 30, 3, 1, pk_dims=False, dom=3),
           lambda: synth.random_star(5, 4, 40, 5, 2, root=2),
           lambda: synth.two_relation(5, 9, 7, 1, 1, 3), lambda: synth.cartesian_uniform(6, 3, 1, 4, 1),
           lambda: synth.config3(div=100000)]


@pytest.mark.parametrize("maker", SCHEMAS)
def test_choice_is_the_brute_force_minimum(maker):
    inst = maker()
    best = None
    for edges in _trees(inst.r):
        if not _valid(inst, edges):
            continue
        for root in range(inst.r):
            c, par = _score(inst, edges, root)
            assert F.join_tree_cost(inst, par) == c, (edges, root)
            best = c if best is None else min(best, c)
    parents, cost = F.choose_join_tree(inst)
    assert cost == best
    assert F.join_tree_cost(inst, parents) == best
    assert parents.count(-1) == 1


def _kept(rel, rows):
    return synth.Rel(rel.key_attrs, rel.keys[:, rows], rel.values[:, rows], rel.parent, rel.name)


@pytest.mark.parametrize("maker", SCHEMAS[:7])
def test_counts_agree_with_the_plan(maker):
    """G_i and P_i of the score are the key groups and parent groups of the
    analysis-only plan, counted over the tuples the plan keeps (on a fully
    reduced database: all of them)."""
    inst = maker()
    plan = F.Plan(inst.rels, analyze_only=True)
    for i, rel in enumerate(inst.rels):
        kept = _kept(rel, plan.permutation(i)[:plan.rows(i)])
        assert plan.num_groups(i, 0) == _distinct(kept, sorted(rel.key_attrs))
        if rel.parent >= 0:
            shared = sorted(set(rel.key_attrs) & set(inst.rels[rel.parent].key_attrs))
            assert plan.num_groups(i, 1) == _distinct(kept, shared)


def test_star_is_not_rooted_at_the_fact_table():
    """Key/foreign-key star (fact 10^4 rows, four 10^2-row dimensions with
    primary keys): the chosen root is a dimension and the fact table sits
    right under it; rooting the star at the fact table scores higher."""
    inst = synth.config3(div=1000)
    parents, cost = F.choose_join_tree(inst)
    fact = [i for i, rel in enumerate(inst.rels) if rel.name == "F"][0]
    root = parents.index(-1)
    assert root != fact
    assert parents[fact] == root
    fact_rooted = [fact if i != fact else -1 for i in range(inst.r)]
    assert F.join_tree_cost(inst, fact_rooted) > cost


def test_cyclic_join_has_no_join_tree():
    rng = np.random.default_rng(0)
    rels = []
    for i, attrs in enumerate(([0, 1], [1, 2], [2, 0])):     # R(a,b), S(b,c), T(c,a)
        rels.append(synth.Rel(attrs, rng.integers(0, 3, (2, 6)).astype(np.int32), rng.standard_normal((1, 6)),
                              -1 if i == 0 else 0, f"R{i}"))
    inst = synth.Instance("triangle", rels)
    with pytest.raises(F.FigaroError) as e:
        F.choose_join_tree(inst)
    assert e.value.name == "ENOTTREE"
    with pytest.raises(F.FigaroError):
        F.join_tree_cost(inst, [-1, 0, 1])

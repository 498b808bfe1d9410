"""Host-side plan logic without a GPU (keys on the host, analysis only):
semi-join reduction, plan order, key groups and the count queries of
Algorithm 2, checked against the definitions of Fig. 4 by brute force."""
import numpy as np
import pytest

import synth
import paper_2204_00525_amd as F


def host_plan(inst, **kw):
    return F.Plan(inst.rels, analyze_only=True, **kw)


MAKERS = [lambda: synth.paper_fig3(1), lambda: synth.paper_fig3(2, m=(4, 7, 3, 3), dom=3),
          lambda: synth.random_chain(3, 4, 6, 1, 2), lambda: synth.random_chain(4, 3, 7, 1, 3),
          lambda: synth.random_star(4, 3, 9, 3, 1, pk_dims=False, dom=3),
          lambda: synth.random_star(5, 4, 8, 3, 1, root=2),
          lambda: synth.two_relation(5, 9, 7, 1, 1, 3), lambda: synth.cartesian_uniform(6, 3, 1, 4, 1)]


@pytest.mark.parametrize("maker", MAKERS)
def test_counts_match_definitions(oracle_lib, maker):
    inst = maker()
    plan = host_plan(inst)
    red, cnt = oracle_lib.brute_counts(inst)
    assert plan.join_rows == oracle_lib.join_size(inst)
    for i, rel in enumerate(inst.rels):
        assert plan.rows(i) == red.rels[i].rows
        Xi = sorted(rel.key_attrs)
        pos = {a: p for p, a in enumerate(rel.key_attrs)}
        first = plan.group_first_rows(i, 0)
        keys = [tuple(int(rel.keys[pos[a], t]) for a in Xi) for t in first]
        assert len(set(keys)) == len(keys)
        for kind in ("rows_per_key", "phi_circ", "theta_down"):
            got = plan.counts(i, kind)
            assert [cnt[i][kind][k] for k in keys] == got.tolist(), (i, kind)
        if rel.parent >= 0:
            Xp = oracle_lib.parent_attrs(inst, i)
            firstp = plan.group_first_rows(i, 1)
            pk = [tuple(int(rel.keys[pos[a], t]) for a in Xp) for t in firstp]
            for kind in ("phi_up", "phi_down"):
                got = plan.counts(i, kind)
                assert [cnt[i][kind][k] for k in pk] == got.tolist(), (i, kind)


@pytest.mark.parametrize("maker", MAKERS + [lambda: synth.config1(), lambda: synth.config3(div=1000)])
def test_plan_order_is_a_sorted_permutation(oracle_lib, maker):
    inst = maker()
    plan = host_plan(inst)
    for i, rel in enumerate(inst.rels):
        perm = plan.permutation(i)
        m = plan.rows(i)
        assert sorted(perm.tolist()) == list(range(rel.rows))
        if rel.keys.shape[0] == 0:
            continue
        xp = oracle_lib.parent_attrs(inst, i)
        rest = sorted(set(rel.key_attrs) - set(xp))
        pos = {a: p for p, a in enumerate(rel.key_attrs)}
        kt = [tuple(int(rel.keys[pos[a], t]) for a in xp + rest) + (int(t),) for t in perm[:m]]
        assert kt == sorted(kt)
        # groups: number of distinct key tuples among kept rows
        assert plan.num_groups(i, 0) == len({k[:-1] for k in kt})


def test_reduction_drops_dangling(oracle_lib):
    inst = synth.two_relation(14, 500, 400, 3, 2, 40)
    inst.rels[0].keys[0, :25] = 1000 + np.arange(25)
    plan = host_plan(inst)
    assert plan.dropped_rows(0) == 25
    assert set(plan.permutation(0)[plan.rows(0):].tolist()) == set(range(25))
    assert plan.join_rows == oracle_lib.join_size(inst)


def test_empty_join():
    inst = synth.two_relation(15, 50, 40, 2, 2, 5)
    inst.rels[1].keys[0, :] = 999
    with pytest.raises(F.FigaroError) as e:
        host_plan(inst)
    assert e.value.name == "EEMPTY_JOIN"


def test_count_overflow_is_detected():
    # a 4-chain where every tuple shares one key: |A| = (2^14)^4 = 2^56 >= 2^53
    m = 1 << 14
    rng = np.random.default_rng(0)
    rels = []
    for j in range(4):
        attrs = [e for e in (j - 1, j) if 0 <= e < 3]
        rels.append(synth.Rel(attrs, np.zeros((len(attrs), m), np.int32), rng.standard_normal((1, m)), j - 1))
    with pytest.raises(F.FigaroError) as e:
        host_plan(synth.Instance("big", rels))
    assert e.value.name == "EOVERFLOW"


def test_config2_join_size_exact(oracle_lib):
    inst = synth.config2(div=20)
    plan = host_plan(inst)
    ks = np.bincount(inst.rels[0].keys[0], minlength=1000).astype(object)
    kt = np.bincount(inst.rels[1].keys[0], minlength=1000).astype(object)
    assert plan.join_rows == float(sum(ks * kt))


def test_config5_sample_covers_every_stratum():
    """The parity sample of the batched workload has at least 64 instances and
    contains every topology, key distribution, relation count and column
    bucket of the 512."""
    ids = synth.config5_sample()
    assert len(ids) >= 64 and len(set(ids)) == len(ids)
    def strata(i):
        p = synth.config5_params(i)
        nb = 0 if p["n"] <= 32 else 1 if p["n"] <= 64 else 2 if p["n"] <= 96 else 3
        return p["topology"], p["dist"], p["r"], nb
    everything = {strata(i) for i in range(512)}
    got = {strata(i) for i in ids}
    assert got == everything
    # the draws of the shape parameters are those of the full instance
    for i in ids[:5]:
        inst = synth.config5_instance(i)
        p = synth.config5_params(i)
        assert [rel.rows for rel in inst.rels] == p["rows"] and inst.n == p["n"]


def test_column_limits():
    """Plans take up to 16384 data columns in total (above 128 the stack is
    reduced by the blocked QR); more are refused before any work."""
    inst = synth.cartesian_uniform(7, 3, 150, 4, 100)
    p = host_plan(inst)
    assert p.n == 250
    wide = synth.cartesian_uniform(8, 2, 16384, 2, 1)
    with pytest.raises(F.FigaroError) as e:
        host_plan(wide)
    assert e.value.name == "EUNSUPPORTED"

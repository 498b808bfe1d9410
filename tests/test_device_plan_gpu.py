"""The plan built on the device (dictionary encoding, semi-join reduction,
radix sort, key and parent groups, child indices, the count queries of
Algorithm 2, the first level of every head/tail task) against the plan the
host builds from the same keys: every permutation, group boundary and count
array equal, and R and the gradients bit for bit equal, which holds only if
the per-item coefficients, piece ids and join multipliers are identical too
(needs an MI355X)."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

KINDS = ("rows_per_key", "theta_down", "phi_circ", "phi_up", "phi_down")


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


def _with_duplicates_and_dangling():
    inst = synth.two_relation(41, 3000, 2500, 3, 2, 40)
    s = inst.rels[0]
    s.keys = np.concatenate([s.keys, s.keys[:, :50], np.full((1, 30), 777, np.int32)], axis=1)
    s.values = np.concatenate([s.values, s.values[:, :50], np.ones((s.values.shape[0], 30))], axis=1)
    return inst


def _wide_keys():
    """int64 keys spread over most of the 64-bit range, negative ones too
    (a key range far beyond any direct table: 62 bits to sort on)."""
    inst = synth.two_relation(12, 4000, 3000, 2, 2, 5000, key_dtype=np.int64)
    for rel in inst.rels:
        rel.keys = (rel.keys.astype(np.int64) * 1_000_000_000_000_003 - 2_500_000_000_000_000_000).astype(np.int64)
    return inst


CASES = {
    "config1": lambda: synth.config1(),
    "config2_div1000": lambda: synth.config2(div=1000),
    "config3_div1000": lambda: synth.config3(div=1000),
    "paper_fig3": lambda: synth.paper_fig3(1),
    "paper_fig3_b": lambda: synth.paper_fig3(5, m=(40, 90, 30, 30), n=(3, 2, 4, 1), dom=3),
    "chain4_zipf": lambda: synth.random_chain(4, 4, 300, 2, 30, dist="zipf"),
    "star_nonpk": lambda: synth.random_star(6, 3, 500, 60, 2, pk_dims=False, dom=12),
    "star_dim_root_6": lambda: synth.random_star(23, 7, 2000, 30, 2, root=1),
    "cartesian": lambda: synth.cartesian_uniform(8, 300, 4, 200, 3),
    "two_rel_int64": lambda: synth.two_relation(11, 3000, 2000, 3, 4, 50, key_dtype=np.int64),
    "wide_keys_int64": lambda: _wide_keys(),
    "chain4_wide_64": lambda: synth.random_chain(16, 4, 120, 16, 12),
    "duplicates_and_dangling": _with_duplicates_and_dangling,
    "config5_3": lambda: synth.config5_instance(3),
    "config5_18": lambda: synth.config5_instance(18),
}


def compare_plans(F, inst, label, tile_items=0):
    import torch
    dev = F.plan_from_instance(inst, tile_items=tile_items)
    host = F.plan_from_instance(inst, tile_items=tile_items, host_plan=True)
    assert dev.join_rows == host.join_rows, label
    for i, rel in enumerate(inst.rels):
        assert dev.rows(i) == host.rows(i), (label, i)
        assert np.array_equal(dev.permutation(i), host.permutation(i)), (label, i)
        for which in (0, 1):
            if which == 1 and rel.parent < 0:
                continue
            assert np.array_equal(dev.group_first_rows(i, which), host.group_first_rows(i, which)), (label, i, which)
        for kind in KINDS:
            if rel.parent < 0 and kind in ("phi_up", "phi_down"):
                continue
            assert np.array_equal(dev.counts(i, kind), host.counts(i, kind)), (label, i, kind)
    vals_d = F.device_values(dev, inst)
    vals_h = F.device_values(host, inst)
    Rd = dev.r_factor(vals_d)
    Rh = host.r_factor(vals_h)
    torch.cuda.synchronize()
    assert torch.equal(Rd, Rh), label
    return dev, host, vals_d, vals_h, Rd


@pytest.mark.parametrize("name", sorted(CASES))
def test_device_plan_equals_host_plan(F, name):
    import torch
    inst = CASES[name]()
    _say(f"[device-plan] case={name} r={inst.r} M={inst.M}")
    dev, host, vd, vh, R = compare_plans(F, inst, name)
    # the backward pass reads the inverse child indices and the stored join
    d = torch.diagonal(R)
    dR = torch.diag(1.0 / d)
    gd = dev.r_backward(vd, R, dR)
    gh = host.r_backward(vh, R, dR)
    torch.cuda.synchronize()
    for a, b in zip(gd, gh):
        assert torch.equal(a, b), name
    dev.close()
    host.close()


@pytest.mark.parametrize("tile", [8, 64])
@pytest.mark.parametrize("name", ["config3_div1000", "chain4_zipf", "paper_fig3_b", "config1"])
def test_device_plan_small_tiles(F, name, tile):
    """Small chunks split key groups over several upper levels (built on the
    host from the device's first level)."""
    dev, host, *_ = compare_plans(F, CASES[name](), f"{name}/tile{tile}", tile_items=tile)
    dev.close()
    host.close()


def test_device_plan_empty_join(F):
    inst = synth.two_relation(3, 50, 40, 1, 1, 10)
    inst.rels[1].keys[:] = 1000
    for host_plan in (False, True):
        with pytest.raises(F.FigaroError) as e:
            F.plan_from_instance(inst, host_plan=host_plan)
        assert e.value.name == "EEMPTY_JOIN"


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", ["config2", "config3"])
def test_device_plan_full_size(F, name):
    """The two-relation join (2 x 2*10^6 tuples) and the star join (10^7 fact
    rows) at full size."""
    inst = getattr(synth, name)()
    dev, host, *_ = compare_plans(F, inst, name)
    dev.close()
    host.close()

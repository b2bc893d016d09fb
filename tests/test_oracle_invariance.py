"""Invariance and structure pins of the oracle (slot map, tours, plan cost).

Readings: the cost of a plan depends only on the multiset of (aisle, depth)
points per tour, so relabellings that keep every picked SKU's point leave the
distance unchanged; tours depend on the order sequence only (next-fit, the
picking-list sequence of section 5, Subproblem 5, and section 6).
"""
import numpy as np
import pytest

import oracle
import synth
from synth import Instance
from tests.whelpers import tiny_geometry


@pytest.fixture(scope="module")
def tiny():
    return synth.workload("tiny", n_plans=16)


def _clone(inst, **kw):
    d = dict(n_aisles=inst.n_aisles, slots_per_side=inst.slots_per_side, pitch_dm=inst.pitch_dm,
             spacing_dm=inst.spacing_dm, capacity=inst.capacity, n_categories=inst.n_categories,
             sku_category=inst.sku_category, order_offsets=inst.order_offsets,
             order_skus=inst.order_skus)
    d.update(kw)
    return Instance(**d)


def test_category_relabelling(tiny):
    inst, Z, S = tiny
    rng = np.random.default_rng(7)
    C = inst.n_categories
    relabel = rng.permutation(C)          # new id of old category c
    inst2 = _clone(inst, sku_category=relabel[inst.sku_category].astype(np.int32))
    for p in range(8):
        z2 = Z[p].copy()
        z2[relabel] = Z[p][:C]            # the new id keeps the old zone
        assert oracle.eval_plan(inst, Z[p], S[p]) == oracle.eval_plan(inst2, z2, S[p])


def test_order_relabelling(tiny):
    inst, Z, S = tiny
    rng = np.random.default_rng(8)
    n = inst.n_orders
    newid = rng.permutation(n)            # order o becomes newid[o]
    old_of_new = np.argsort(newid)
    lens = np.diff(inst.order_offsets)
    off = np.zeros(n + 1, dtype=np.int32)
    off[1:] = np.cumsum(lens[old_of_new])
    skus = np.concatenate([inst.order_skus[inst.order_offsets[o]:inst.order_offsets[o + 1]]
                           for o in old_of_new]).astype(np.int32)
    inst2 = _clone(inst, order_offsets=off, order_skus=skus)
    for p in range(8):
        s2 = newid[S[p]].astype(np.uint16)
        assert oracle.eval_plan(inst, Z[p], S[p]) == oracle.eval_plan(inst2, Z[p], s2)


def test_side_mirroring(tiny):
    inst, Z, S = tiny
    for p in range(4):
        loc = oracle.locations(inst, Z[p])
        tf = oracle.tours(inst, S[p])
        for t in range(len(tf) - 1):
            locs = []
            for i in range(tf[t], tf[t + 1]):
                o = S[p][i]
                locs += [int(loc[s]) for s in inst.order_skus[inst.order_offsets[o]:inst.order_offsets[o + 1]]]
            mirrored = [l ^ 1 for l in locs]
            assert oracle.sshape_cost(inst, locs) == oracle.sshape_cost(inst, mirrored)


def test_tours_do_not_depend_on_zones(tiny):
    inst, Z, S = tiny
    # tours are a function of the sequence and the order sizes only
    for p in range(4):
        tf = oracle.tours(inst, S[p])
        inst2 = _clone(inst, order_skus=np.zeros_like(inst.order_skus))
        assert np.array_equal(tf, oracle.tours(inst2, S[p]))


def test_swap_of_unpicked_equal_zones():
    # categories 3 and 7 (equal size 50) hold no ordered SKU: exchanging their
    # zones moves nothing that is picked
    orders = [[0, 130], [599], [61, 62, 300], [401, 402], [20]]
    inst = tiny_geometry(orders, capacity=4)
    rng = np.random.default_rng(3)
    for _ in range(5):
        z = np.full(64, 0xFF, dtype=np.uint8)
        z[:12] = rng.permutation(12)
        z2 = z.copy()
        z2[3], z2[7] = z[7], z[3]
        seq = rng.permutation(len(orders)).astype(np.uint16)
        assert oracle.eval_plan(inst, z, seq) == oracle.eval_plan(inst, z2, seq)


@pytest.mark.parametrize("seed", range(20))
def test_next_fit_properties(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 300))
    Q = int(rng.integers(1, 33))
    lens = 1 + rng.poisson(rng.uniform(0.2, 6.0), size=n)
    orders = [[0] * int(k) for k in lens]
    inst = tiny_geometry(orders, capacity=Q)
    seq = rng.permutation(n).astype(np.uint16)
    tf = oracle.tours(inst, seq)
    items = lens[seq]
    loads = [int(items[tf[t]:tf[t + 1]].sum()) for t in range(len(tf) - 1)]
    assert tf[0] == 0 and tf[-1] == n and np.all(np.diff(tf) >= 1)
    assert sum(loads) == int(lens.sum())                       # items conserved
    for t in range(len(loads)):
        assert loads[t] <= Q or tf[t + 1] - tf[t] == 1          # capacity, or one big order
        if t + 1 < len(loads):
            assert loads[t] + items[tf[t + 1]] > Q              # maximality (next-fit)
    assert len(loads) >= -(-int(lens.sum()) // Q)              # at least ceil(I / Q) tours


@pytest.mark.parametrize("seed", range(20))
def test_next_fit_prefix_sum_formulation(seed):
    # independent formulation: a tour starting at position i ends at the
    # first position whose cumulative item count passes P[i] + Q
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 400))
    Q = int(rng.integers(1, 33))
    lens = 1 + rng.poisson(2.0, size=n)
    inst = tiny_geometry([[0] * int(k) for k in lens], capacity=Q)
    seq = rng.permutation(n).astype(np.uint16)
    P = np.concatenate([[0], np.cumsum(lens[seq])])
    starts = [0]
    while starts[-1] < n:
        i = starts[-1]
        e = int(np.searchsorted(P, P[i] + Q, side="right")) - 1
        starts.append(max(e, i + 1))
    assert np.array_equal(oracle.tours(inst, seq), np.asarray(starts))


def test_slot_map_structure(tiny):
    inst, Z, _ = tiny
    sizes = inst.category_sizes()
    for p in range(8):
        loc = oracle.locations(inst, Z[p])
        assert np.array_equal(np.sort(loc), np.arange(inst.n_skus))   # bijection onto [0, sum sizes)
        for c in range(inst.n_categories):
            skus = np.flatnonzero(inst.sku_category == c)
            l = loc[skus]
            assert np.array_equal(l, l[0] + np.arange(len(skus)))        # contiguous, ascending SKU id
            before = sizes[[cc for cc in range(inst.n_categories) if Z[p][cc] < Z[p][c]]].sum()
            assert l[0] == before                                        # zones in zone order


def test_slot_map_dirichlet_tail_empty():
    inst, Z, _ = synth.workload("paper", n_plans=2)
    loc = oracle.locations(inst, Z[0])
    assert loc.max() == inst.n_skus - 1 < inst.n_locations              # unused locations at the tail


def test_rejects_bad_plans(tiny):
    inst, Z, S = tiny
    z = Z[0].copy()
    z[1] = z[0]
    with pytest.raises(ValueError):
        oracle.eval_plan(inst, z, S[0])
    s = S[0].copy()
    s[0] = inst.n_orders
    with pytest.raises(ValueError):
        oracle.eval_plan(inst, Z[0], s)


def test_threads_agree(tiny):
    inst, Z, S = tiny
    d1, t1 = oracle.eval_plans(inst, Z, S, n_threads=1)
    d4, t4 = oracle.eval_plans(inst, Z, S, n_threads=4)
    assert np.array_equal(d1, d4) and np.array_equal(t1, t4)
    for p in range(len(Z)):
        _, d, t = oracle.eval_plan(inst, Z[p], S[p])
        assert d == d1[p] and t == t1[p]

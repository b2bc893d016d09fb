"""Pins of the oracle's seed order batching (oracle/wo_oracle.c,
orc_tours_seed): tours built one at a time from the earliest unbatched order
of the sequence, each then taking, while any fits, the order that adds the
fewest aisles the tour does not visit yet (ties: earlier in the sequence).

* A hand-worked plan where seed batching groups orders by aisle and first fit
  does not, with both distances derived by hand.
* The tie rule, by hand.
* A warehouse of one aisle: every order adds no aisle, so the tie rule makes
  each tour take, in sequence, every order that still fits -- first fit's
  assignment tour by tour (by induction over the tours: the first order that
  did not fit tour t is the earliest unbatched one, so it seeds tour t + 1, and
  the later orders that fit join in sequence exactly as first fit places
  them).  Seed batching then equals first fit, partition and distance.
* Properties of the assignment on random plans: every tour but an oversize
  seed's respects the capacity; a tour's first order is the earliest order
  not in an earlier tour; when a tour is closed no order outside the tours so
  far fits it; every order is in exactly one tour.
* Invariance: the slotting moves aisles, so the tours change with it; but
  relabelling categories (zones permuted along) keeps every location and the
  whole result.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from tests.whelpers import identity_zones, tiny_geometry


def _seed(inst):
    return dataclasses.replace(inst, batching=2)


def test_hand_example_groups_orders_by_aisle():
    # tiny geometry: 10 aisles x 2 x 30 slots, pitch 10 dm, spacing 30 dm,
    # identity zones, so SKU s sits at location s, aisle s // 60, depth index
    # (s % 60) // 2.  Capacity 3.
    #   A = {180, 181}: aisle 3, y = 5      (2 items)
    #   B = {420}:      aisle 7, y = 5      (1 item)
    #   C = {200}:      aisle 3, y = 105    (1 item)
    #   D = {430, 431}: aisle 7, y = 55     (2 items)
    # seed: A seeds tour 0; B and D would add aisle 7, C adds none: C joins
    # (load 3, full).  B seeds tour 1; D adds no aisle and fits: {B, D}.
    #   {A, C}: one aisle (3), odd: 2*30*3 + 2*105 = 390
    #   {B, D}: one aisle (7), odd: 2*30*7 + 2*55 = 530            -> 920
    # first fit: {A, B} (load 3), {C, D}: each visits aisles 3 and 7, even:
    #   2*30*7 + 2*300 = 1020 each                                  -> 2040
    inst = tiny_geometry([[180, 181], [420], [200], [430, 431]], capacity=3)
    Z = identity_zones(12)[None, :]
    S = np.arange(4, dtype=np.uint16)[None, :]
    assert oracle.tours_seed(_seed(inst), Z[0], S[0]).tolist() == [0, 1, 0, 1]
    d_seed, _ = oracle.eval_plans(_seed(inst), Z, S)
    d_ff, _ = oracle.eval_plans(dataclasses.replace(inst, batching=1), Z, S)
    assert d_seed.tolist() == [920] and d_ff.tolist() == [2040]


def test_ties_go_to_the_earlier_order():
    # capacity 3; A (1 item, aisle 3) seeds; C and B (2 items each, both in
    # aisle 5) add one aisle each and only one of them fits: the one earlier
    # in the sequence joins, the other seeds the next tour
    A, B, C = [180], [300, 301], [310, 311]
    inst = _seed(tiny_geometry([A, B, C], capacity=3))
    z = identity_zones(12)
    assert oracle.tours_seed(inst, z, np.array([0, 2, 1], np.uint16)).tolist() == [0, 0, 1]   # C earlier
    assert oracle.tours_seed(inst, z, np.array([0, 1, 2], np.uint16)).tolist() == [0, 0, 1]   # B earlier
    # tour membership by order: with C earlier, {A, C}; with B earlier, {A, B}
    t = oracle.tours_seed(inst, z, np.array([0, 2, 1], np.uint16))
    assert t[1] == t[0]            # position 1 holds C


def test_fewer_new_aisles_beat_the_sequence():
    # A seeds (aisle 3); B comes first but adds aisle 8; C adds nothing: C
    # joins before B although B is earlier in the sequence
    A, B, C = [180], [480], [182]
    inst = _seed(tiny_geometry([A, B, C], capacity=2))
    assert oracle.tours_seed(inst, identity_zones(12), np.arange(3, dtype=np.uint16)).tolist() == [0, 1, 0]


@pytest.mark.parametrize("seed", range(6))
def test_one_aisle_equals_first_fit(seed):
    rng = np.random.default_rng(seed)
    inst = synth.make_instance(n_aisles=1, slots_per_side=60, pitch_dm=10, spacing_dm=30,
                               capacity=int(rng.integers(3, 20)), n_categories=6, n_skus=100,
                               category_mode="dirichlet", n_orders=150, lines_lambda=2.0, zipf_s=1.0,
                               seed=seed)
    Z, S = synth.make_plans(inst, 4, seed=seed)
    for z, s in zip(Z, S):
        t_seed = oracle.tours_seed(_seed(inst), z, s)
        t_ff = oracle.tours_first_fit(inst, s)
        # the same partition of the positions (tour numbers may differ when
        # an oversize order seeds a tour later than first fit opens it)
        part = lambda t: sorted(tuple(np.flatnonzero(t == k)) for k in range(t.max() + 1))
        assert part(t_seed) == part(t_ff)
    d_seed, _ = oracle.eval_plans(_seed(inst), Z, S)
    d_ff, _ = oracle.eval_plans(dataclasses.replace(inst, batching=1), Z, S)
    assert np.array_equal(d_seed, d_ff)


@pytest.mark.parametrize("seed", range(5))
def test_assignment_properties(seed):
    rng = np.random.default_rng(100 + seed)
    inst = synth.make_instance(n_aisles=int(rng.integers(3, 40)), slots_per_side=20, pitch_dm=10, spacing_dm=30,
                               capacity=int(rng.integers(2, 16)), n_categories=12, n_skus=300,
                               category_mode="dirichlet", n_orders=200, lines_lambda=2.0, zipf_s=1.0, seed=seed)
    sizes = np.diff(inst.order_offsets)
    Q = inst.capacity
    Z, S = synth.make_plans(inst, 3, seed=seed)
    for z, s in zip(Z, S):
        t = oracle.tours_seed(_seed(inst), z, s)
        T = t.max() + 1
        assert (t >= 0).all() and sorted(set(t.tolist())) == list(range(T))
        sz = sizes[s.astype(np.int64)]
        placed = np.zeros(len(s), bool)
        for k in range(T):
            members = np.flatnonzero(t == k)
            first = int(np.flatnonzero(~placed)[0])
            assert members[0] == first                      # the seed: earliest order in no earlier tour
            load = int(sz[members].sum())
            assert load <= Q or (members.size == 1 and sz[first] > Q)
            placed[members] = True
            rest = ~placed
            assert not (rest & (load + sz <= Q)).any()      # nothing left fits the closed tour


def test_category_relabelling_keeps_the_result():
    inst, Z, S = synth.workload("tiny", n_plans=6)
    inst = _seed(inst)
    rng = np.random.default_rng(4)
    perm = rng.permutation(inst.n_categories)
    # category c becomes perm[c]; its zone goes along
    inst2 = dataclasses.replace(inst, sku_category=perm[inst.sku_category].astype(np.int32))
    Z2 = Z.copy()
    Z2[:, perm] = Z[:, :inst.n_categories]
    assert np.array_equal(oracle.eval_plans(inst, Z, S)[0], oracle.eval_plans(inst2, Z2, S)[0])
    for z, z2, s in zip(Z, Z2, S):
        assert np.array_equal(oracle.tours_seed(inst, z, s), oracle.tours_seed(inst2, z2, s))


def test_distance_is_the_sum_over_its_tours():
    inst, Z, S = synth.workload("tiny", n_plans=4)
    inst = _seed(inst)
    d, _ = oracle.eval_plans(inst, Z, S)
    for k in range(4):
        loc = oracle.locations(inst, Z[k])
        t = oracle.tours_seed(inst, Z[k], S[k])
        total = 0
        for tour in range(t.max() + 1):
            picks = [int(loc[inst.order_skus[l]]) for i in np.flatnonzero(t == tour)
                     for l in range(inst.order_offsets[S[k][i]], inst.order_offsets[S[k][i] + 1])]
            total += oracle.sshape_cost(inst, np.asarray(picks, np.int32))
        assert total == d[k]


def test_an_orders_aisles_count_once():
    # A (aisle 3) seeds, capacity 3.  Y = {300, 420} comes first and adds two
    # aisles (5 and 7); X = {480, 490} adds one aisle (8) with both its lines:
    # X has fewer new aisles and joins although Y is earlier.  Counting X's
    # two lines in aisle 8 twice would tie the two and let Y in.
    A, Y, X = [180], [300, 420], [480, 490]
    inst = _seed(tiny_geometry([A, Y, X], capacity=3))
    assert oracle.tours_seed(inst, identity_zones(12), np.arange(3, dtype=np.uint16)).tolist() == [0, 1, 0]

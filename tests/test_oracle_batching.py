"""Pins of the oracle's first-fit order batching.

* A hand-worked example where first fit and next fit differ.
* A checker of the rule's defining property, run over the assignment the
  oracle returns: each order sits in the earliest-opened tour that had room
  for it at its turn, and a tour is opened only when no open tour had room.
* Special cases: single-item orders (first fit = next fit = consecutive groups
  of Q) and orders larger than the capacity (a tour of their own).
* First fit never opens more tours than next fit.  Proof: cut the sequence
  into next fit's tours; while first fit places the orders of one of them it
  opens at most one tour, since a tour opened then holds only orders of that
  group, whose items all fit one tour, so every later order of the group fits
  into it.
* A plan's distance under first fit is the sum of the route costs of its
  tours, each tour's picks gathered by hand from the assignment.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from tests.whelpers import identity_zones, tiny_geometry


def _sizes(inst):
    return np.diff(inst.order_offsets)


def _ff(inst):
    return dataclasses.replace(inst, batching=1)


def test_hand_example():
    # capacity 10, order sizes 6, 5, 4, 3, 2 in sequence:
    # first fit: 6 -> t0, 5 -> t1, 4 -> t0 (10), 3 -> t1 (8), 2 -> t1 (10): 2 tours
    # next fit:  [6], [5, 4], [3, 2]: 3 tours
    orders = [list(range(10 * i, 10 * i + n)) for i, n in enumerate([6, 5, 4, 3, 2])]
    inst = tiny_geometry(orders, capacity=10)
    seq = np.arange(5, dtype=np.uint16)
    assert oracle.tours_first_fit(inst, seq).tolist() == [0, 1, 0, 1, 1]
    assert oracle.tours(inst, seq).tolist() == [0, 1, 3, 5]
    # sequence 4, 3, 2, 1, 0 (sizes 2, 3, 4, 5, 6): 2+3+4 = 9, then 5 and 6 open tours
    assert oracle.tours_first_fit(inst, seq[::-1].copy()).tolist() == [0, 0, 0, 1, 2]


def _check_first_fit(sizes, Q, seq, tour_of):
    loads = []
    for i, o in enumerate(seq):
        s = int(sizes[o])
        t = int(tour_of[i])
        room = [u for u, l in enumerate(loads) if l + s <= Q]
        if room:
            assert t == room[0], (i, t, room[0])
            loads[t] += s
        else:
            assert t == len(loads), (i, t, len(loads))
            loads.append(s)
    return len(loads)


@pytest.mark.parametrize("seed", range(20))
def test_first_fit_property_and_not_above_next_fit(seed):
    rng = np.random.default_rng(100 + seed)
    Q = int(rng.integers(1, 33))
    inst = synth.make_instance(n_aisles=20, slots_per_side=30, pitch_dm=10, spacing_dm=30,
                               capacity=Q, n_categories=8, n_skus=800, category_mode="dirichlet",
                               n_orders=int(rng.integers(1, 400)),
                               lines_lambda=float(rng.uniform(0, 4)), zipf_s=1.0,
                               seed=int(rng.integers(1 << 30)))
    seq = rng.permutation(inst.n_orders).astype(np.uint16)
    tour_of = oracle.tours_first_fit(inst, seq)
    n_ff = _check_first_fit(_sizes(inst), Q, seq, tour_of)
    n_nf = len(oracle.tours(inst, seq)) - 1
    assert n_ff <= n_nf


def test_single_item_orders_group_consecutively():
    inst = tiny_geometry([[i] for i in range(47)], capacity=5)
    seq = np.random.default_rng(3).permutation(47).astype(np.uint16)
    assert oracle.tours_first_fit(inst, seq).tolist() == [i // 5 for i in range(47)]


def test_oversize_orders_ride_alone():
    # capacity 3; orders of 5 and 4 lines open tours nothing joins
    inst = tiny_geometry([[0, 1, 2, 3, 4], [5], [6, 7, 8, 9], [10, 11], [12]], capacity=3)
    seq = np.arange(5, dtype=np.uint16)
    # 5 -> t0 (alone), 1 -> t1, 4 -> t2 (alone), 2 -> t1 (3), 1 -> t3
    assert oracle.tours_first_fit(inst, seq).tolist() == [0, 1, 2, 1, 3]


@pytest.mark.parametrize("routing", [0, 1, 2, 3])
def test_plan_distance_is_sum_over_first_fit_tours(routing):
    inst, Z, S = synth.workload("tiny", n_plans=6)
    inst = dataclasses.replace(inst, routing=routing)
    differs = False
    for p in range(6):
        tour_of = oracle.tours_first_fit(inst, S[p])
        loc = oracle.locations(inst, Z[p])
        total = 0
        for t in range(int(tour_of.max()) + 1):
            picks = [int(loc[inst.order_skus[l]]) for i in np.flatnonzero(tour_of == t)
                     for l in range(inst.order_offsets[S[p][i]], inst.order_offsets[S[p][i] + 1])]
            total += oracle.tour_cost(inst, picks)
        assert oracle.eval_plan(_ff(inst), Z[p], S[p])[0] == total
        differs |= oracle.eval_plan(inst, Z[p], S[p])[0] != total
    assert differs                  # the rule matters on these plans


def test_first_fit_worked_plan():
    # capacity 3; orders A = {61, 62} (aisle 1, y 5 and 15), B = {598, 599}
    # (aisle 9, y 295 on both sides), C = {0} (aisle 0, y 5), picked A, B, C.
    # next fit: [A], [B, C]: 2*30*1 + 2*15 = 90, plus 2*30*9 + 2*300 = 1140
    # first fit: [A, C], [B]: 2*30*1 + 2*300 = 660, plus 2*30*9 + 2*295 = 1130
    inst = tiny_geometry([[61, 62], [598, 599], [0]], capacity=3)
    Z = identity_zones(12)
    seq = np.arange(3, dtype=np.uint16)
    assert oracle.tours_first_fit(inst, seq).tolist() == [0, 1, 0]
    assert oracle.eval_plan(inst, Z, seq)[0] == 90 + 1140
    assert oracle.eval_plan(_ff(inst), Z, seq)[0] == 660 + 1130

"""Pins of the oracle against hand-derived closed forms and a worked plan.

The route objective is the sum of per-tour distances and the picking rate is
a function of that distance (arXiv 2110.13693, section 5, Subproblem 2,
Eq. (2)); the per-tour distance is the S-shape route.  Values are in
tests/golden/worked_examples.json with their derivations.
"""
import json
import os

import numpy as np
import pytest

import oracle
from tests.whelpers import identity_zones, tiny_geometry

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")))


@pytest.fixture(scope="module")
def geo():
    return tiny_geometry([[0]])


@pytest.mark.parametrize("case", GOLD["single_pick"], ids=lambda c: "loc%d" % c["loc"])
def test_single_pick(geo, case):
    assert oracle.sshape_cost(geo, [case["loc"]]) == case["cost"]


@pytest.mark.parametrize("case", GOLD["multi_pick"], ids=lambda c: str(c["cost"]))
def test_multi_pick(geo, case):
    assert oracle.sshape_cost(geo, case["locs"]) == case["cost"]


def _every_aisle(n_aisles, far_y_index):
    inst = tiny_geometry([[0]], n_aisles=n_aisles)
    locs = [a * 60 for a in range(n_aisles)]
    locs[-1] = (n_aisles - 1) * 60 + 2 * far_y_index  # farthest pick of the last aisle
    return inst, locs


@pytest.mark.parametrize("n_aisles", [2, 4, 10])
def test_every_aisle_even(n_aisles):
    inst, locs = _every_aisle(n_aisles, 17)
    L, w = 300, 30
    assert oracle.sshape_cost(inst, locs) == n_aisles * L + 2 * w * (n_aisles - 1)


@pytest.mark.parametrize("n_aisles,j", [(1, 0), (3, 29), (9, 11)])
def test_every_aisle_odd(n_aisles, j):
    inst, locs = _every_aisle(n_aisles, j)
    L, w = 300, 30
    y_far = 10 * j + 5
    assert oracle.sshape_cost(inst, locs) == (n_aisles - 1) * L + 2 * y_far + 2 * w * (n_aisles - 1)


def test_sides_share_depth(geo):
    # both sides of a slot are the same point of the centre line
    for a in range(10):
        for j in range(30):
            l0 = a * 60 + 2 * j
            assert oracle.sshape_cost(geo, [l0]) == oracle.sshape_cost(geo, [l0 + 1])


def test_repeated_location_adds_nothing(geo):
    assert oracle.sshape_cost(geo, [130, 130, 130]) == oracle.sshape_cost(geo, [130])


def _worked_instance(orders, capacity):
    return tiny_geometry(orders, capacity=capacity)


@pytest.mark.parametrize("case", GOLD["worked_plan"]["cases"], ids=lambda c: str(c["D"]))
def test_worked_plan(case):
    wp = GOLD["worked_plan"]
    inst = _worked_instance(wp["orders"], wp["capacity"])
    z = identity_zones(12)
    if case["zone_swap"]:
        a, b = case["zone_swap"]
        z[a], z[b] = z[b], z[a]
    seq = np.asarray(case["seq"], dtype=np.uint16)
    # slot map: the tours' locations as listed
    loc = oracle.locations(inst, z)
    tf = oracle.tours(inst, seq)
    got_tours = []
    for t in range(len(tf) - 1):
        ls = []
        for i in range(tf[t], tf[t + 1]):
            o = seq[i]
            ls += [int(loc[s]) for s in wp["orders"][o]]
        got_tours.append(ls)
    assert got_tours == case["tours"]
    assert [oracle.sshape_cost(inst, t) for t in got_tours] == case["tour_costs"]
    de, d, thr = oracle.eval_plan(inst, z, seq)
    assert de == d == case["D"]


def test_throughput_closed_form():
    g = GOLD["throughput"]
    inst = _worked_instance(GOLD["worked_plan"]["orders"], 3)
    assert inst.n_items == g["items"] and inst.n_orders == g["n_orders"]
    de, d, thr = oracle.eval_plan(inst, identity_zones(12), np.arange(3, dtype=np.uint16))
    assert de == g["D"]
    assert thr == np.float32(g["orders_per_window"])
    # exact rational check of the expected value itself
    assert abs(g["orders_per_window"] - 1036800 / 3350) < 1e-12


def test_saturation_of_int32_output():
    # every order is its own tour (capacity 1) and the aisle spacing is huge,
    # so the exact sum passes INT32_MAX while the int32 output saturates
    n_orders = 60000
    big = tiny_geometry([[599]] * n_orders, capacity=1, spacing=40000)
    de, d, _ = oracle.eval_plan(big, identity_zones(12), np.arange(n_orders, dtype=np.uint16))
    assert de == n_orders * (2 * 40000 * 9 + 2 * 295) and de > 2**31 - 1
    assert d == 2**31 - 1

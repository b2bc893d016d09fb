"""Pins of the aisle-width design oracle (oracle/aisles.py; section 5,
Subproblem 1, Eq. (1)): the utilisation closed form, the rate it couples
through, the route distance as a function of the spacing, and the design as
the narrowest feasible width."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import aisles as A
from tests.whelpers import identity_zones, tiny_geometry


def test_utilisation_closed_form():
    # racks of depth 10 on both sides of a 30 dm aisle, 300 dm long, cross
    # aisles of 20 dm: 2*10*300 / ((30 + 20) (300 + 40)) = 6000 / 17000
    assert A.utilization(30, 10, 300, 20) == pytest.approx(6000 / 17000, rel=1e-15)
    # paper-sized racks: 2*12*2500 / ((25 + 24) (2500 + 60)) = 60000 / 125440
    assert A.utilization(25, 12, 2500, 30) == pytest.approx(60000 / 125440, rel=1e-15)
    # no cross aisles and no corridor: the racks cover the floor
    assert A.utilization(0, 7, 100, 0) == pytest.approx(1.0, rel=1e-15)
    u = [A.utilization(a, 10, 300, 20) for a in range(1, 200)]
    assert all(x > y for x, y in zip(u, u[1:]))


def test_rate_is_the_evaluators_rate():
    # the double rate, rounded once to float, is the oracle's float32 rate
    inst, Z, S = synth.workload("tiny", n_plans=6)
    for z, s in zip(Z, S):
        _, D, thr = oracle.eval_plan(inst, z, s)
        assert np.float32(A.orders_per_window(inst, D)) == np.float32(thr)
    # the worked value of the golden file: 3 orders, 6 items, D = 2630
    inst = tiny_geometry([[0, 130], [599], [61, 62, 300]], capacity=3)
    assert A.orders_per_window(inst, 2630) == pytest.approx(1036800 / 3350, rel=1e-15)


def test_worked_plan_distance_is_affine_in_the_spacing():
    # the worked plan's tours are {0, 130, 599} (aisles 0, 2, 9) and
    # {61, 62, 300} (aisles 1, 5); S-shape crosses 2 w a_max horizontally,
    # so D(w) = 2 w (9 + 5) + 1790, the rest of the worked D = 2630 at w = 30
    inst = tiny_geometry([[0, 130], [599], [61, 62, 300]], capacity=3)
    z, s = identity_zones(12), np.array([0, 1, 2], np.uint16)
    for w in (0, 1, 30, 40, 77):
        assert A.distance_at(inst, z, s, w) == 28 * w + 1790


def test_sshape_slope_is_twice_the_farthest_aisles():
    # D(w) = (2 sum over tours of the farthest aisle) w + const, the slope
    # taken from the oracle's own tours and locations
    inst, Z, S = synth.workload("tiny", n_plans=3)
    for z, s in zip(Z, S):
        loc = oracle.locations(inst, z)
        bounds = oracle.tours(inst, s)
        slope = 0
        for t in range(len(bounds) - 1):
            orders = s[bounds[t]:bounds[t + 1]]
            picks = [loc[inst.order_skus[l]] for o in orders
                     for l in range(inst.order_offsets[o], inst.order_offsets[o + 1])]
            slope += 2 * max(p // (2 * inst.slots_per_side) for p in picks)
        d = [A.distance_at(inst, z, s, w) for w in range(10, 60, 7)]
        assert all(d[i + 1] - d[i] == 7 * slope for i in range(len(d) - 1))


@pytest.mark.parametrize("route", [0, 1, 2, 3, 4])
def test_distance_grows_and_rate_falls_with_the_spacing(route):
    inst, Z, S = synth.workload("tiny", n_plans=2)
    inst = dataclasses.replace(inst, routing=route)
    for z, s in zip(Z, S):
        d = [A.distance_at(inst, z, s, w) for w in range(4, 80, 3)]
        assert all(x <= y for x, y in zip(d, d[1:]))
        r = [A.orders_per_window(inst, D) for D in d]
        assert all(x >= y for x, y in zip(r, r[1:]))


def _quadratic_design(inst, z, s, r, k, a_min, a_max):
    """The S-shape design from the affine distance D = m (a + 2 r) + b: the
    constraint k n W / ((m (a + 2 r) + b) / v + t I) <= a is a quadratic in
    a; its positive root, rounded up and checked one step either side."""
    d0 = A.distance_at(inst, z, s, 0)
    m = A.distance_at(inst, z, s, 1) - d0
    b = d0
    v, t, I = inst.walk_dm_per_s, inst.seconds_per_item, inst.n_items
    nW = inst.n_orders * inst.window_s
    # a (m (a + 2r) + b) / v + a t I - k nW >= 0  <=>  qa a^2 + qb a + qc >= 0
    qa = m / v
    qb = (2 * r * m + b) / v + t * I
    qc = -k * nW
    root = (-qb + math.sqrt(qb * qb - 4 * qa * qc)) / (2 * qa) if qa > 0 else -qc / qb
    a = max(a_min, math.ceil(root))

    def ok(x):
        return k * A.orders_per_window(inst, m * (x + 2 * r) + b) <= x
    while a > a_min and ok(a - 1):
        a -= 1
    while a <= a_max and not ok(a):
        a += 1
    return a if a <= a_max else None


@pytest.mark.parametrize("k", [0.0, 0.01, 0.05, 0.08])
def test_design_is_the_narrowest_feasible_width(k):
    inst, Z, S = synth.workload("tiny", n_plans=2)
    for z, s in zip(Z, S):
        res = A.design_width(inst, z, s, rack_depth=10, cross_aisle=20, k=k, a_min=8, a_max=60)
        assert len(res["dist"]) == 53
        want = _quadratic_design(inst, z, s, 10, k, 8, 60)
        if want is None:
            assert not res["feasible"] and res["width_dm"] == 60
        else:
            assert res["feasible"] and res["width_dm"] == want
            a = res["width_dm"]
            assert k * res["orders_per_window"] <= a
            if a > 8:
                prev = A.orders_per_window(inst, res["dist"][a - 1 - 8])
                assert k * prev > a - 1
        assert res["utilization"] == A.utilization(res["width_dm"], 10, 300, 20)
    if k == 0.0:
        assert res["width_dm"] == 8


def test_design_without_a_feasible_width():
    inst, Z, S = synth.workload("tiny", n_plans=1)
    res = A.design_width(inst, Z[0], S[0], rack_depth=10, cross_aisle=20, k=10.0, a_min=8, a_max=20)
    assert not res["feasible"] and res["width_dm"] == 20 and res["spacing_dm"] == 40

"""GPU aisle-width design (wo_aisle_width; section 5, Subproblem 1, Eq. (1))
against the oracle's plain sweep: the distance at every width bit-exact, the
same design, rate and utilisation."""
import dataclasses

import numpy as np
import pytest

import synth
from oracle import aisles as A

pytestmark = pytest.mark.gpu


def _run(inst, z, s, r, c, k, a_min, a_max):
    import torch
    from paper_2110_13693_amd import wo
    wh = wo.wo_load_warehouse([inst])
    zd = torch.from_numpy(np.ascontiguousarray(z, np.uint8)).cuda()
    sd = torch.from_numpy(np.ascontiguousarray(s, np.uint16).view(np.int16)).cuda()
    res, dist = wo.wo_aisle_width(wh, zd, sd, r, c, k, a_min, a_max)
    wh.free()
    return res, dist


def _compare(inst, z, s, r=10, c=20, k=0.05, a_min=8, a_max=60):
    res, dist = _run(inst, z, s, r, c, k, a_min, a_max)
    ref = A.design_width(inst, z, s, r, c, k, a_min, a_max)
    assert np.array_equal(dist, np.asarray(ref["dist"], np.int32))
    assert res["width_dm"] == ref["width_dm"] and bool(res["feasible"]) == ref["feasible"]
    assert res["spacing_dm"] == ref["spacing_dm"] and res["distance"] == ref["distance"]
    assert res["widths_evaluated"] == a_max - a_min + 1
    assert res["orders_per_window"] == ref["orders_per_window"]
    assert res["utilization"] == pytest.approx(ref["utilization"], rel=1e-15)
    return res


@pytest.mark.parametrize("k", [0.0, 0.05, 0.08, 10.0])
def test_tiny_plan(k):
    inst, Z, S = synth.workload("tiny", n_plans=2)
    for z, s in zip(Z, S):
        print("tiny k", k, flush=True)
        _compare(inst, z, s, k=k)


@pytest.mark.parametrize("route,batching", [(1, 0), (2, 0), (3, 0), (4, 0), (0, 1), (3, 1)])
def test_other_routes_and_first_fit(route, batching):
    inst, Z, S = synth.workload("tiny", n_plans=1)
    inst = dataclasses.replace(inst, routing=route, batching=batching)
    print("route", route, "batching", batching, flush=True)
    _compare(inst, Z[0], S[0], k=0.05)


def test_paper_plan_many_widths():
    # the paper-scale warehouse: 400 widths in one launch, an interior optimum
    inst, Z, S = synth.workload("paper", n_plans=1)
    print("paper 400 widths", flush=True)
    res = _compare(inst, Z[0], S[0], r=12, c=30, k=0.5, a_min=5, a_max=404)
    assert res["feasible"] and 5 < res["width_dm"] < 404


def test_single_width_and_odd_order_count():
    # a range of one width; an odd number of orders (sequence rows that do
    # not fill whole 32-bit words)
    rng = np.random.default_rng(4)
    inst = synth.make_instance(n_aisles=20, slots_per_side=40, pitch_dm=10, spacing_dm=30, capacity=20,
                               n_categories=16, n_skus=1200, category_mode="dirichlet", n_orders=301,
                               lines_lambda=1.5, zipf_s=1.0, seed=int(rng.integers(1 << 30)))
    Z, S = synth.make_plans(inst, 1, seed=3)
    print("odd order count", flush=True)
    _compare(inst, Z[0], S[0], k=0.05, a_min=17, a_max=17)
    _compare(inst, Z[0], S[0], k=0.05, a_min=3, a_max=90)

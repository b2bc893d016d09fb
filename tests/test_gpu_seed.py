"""GPU parity of seed order batching (WO_BATCH_SEED), under every route,
against the CPU oracle (through the C ABI): distances bit-exact, the rate to
1e-6 relative."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import gpu_eval
from tests.test_gpu_eval import THR_RTOL, _random_instance, _wo

pytestmark = pytest.mark.gpu

ROUTES = [0, 1, 2, 3, 4]


def _sd(inst, routing=None):
    inst = dataclasses.replace(inst, batching=2)
    return inst if routing is None else dataclasses.replace(inst, routing=routing)


def _compare(inst, Z, S):
    wo = _wo()
    wh = wo.wo_load_warehouse([inst])
    d_ref, t_ref = oracle.eval_plans(inst, Z, S, n_threads=8)
    d_gpu, t_gpu = gpu_eval(wh, Z, S)
    wh.free()
    bad = np.flatnonzero(d_gpu != d_ref)
    assert bad.size == 0, "plans %s: gpu %s oracle %s" % (bad[:5], d_gpu[bad[:5]], d_ref[bad[:5]])
    np.testing.assert_allclose(t_gpu, t_ref, rtol=THR_RTOL, atol=0)
    return d_gpu


@pytest.mark.parametrize("routing", ROUTES)
def test_tiny_all_plans(routing):
    inst, Z, S = synth.workload("tiny")
    print("tiny seed", routing, flush=True)
    d = _compare(_sd(inst, routing), Z, S)
    d_ff, _ = oracle.eval_plans(dataclasses.replace(inst, routing=routing, batching=1), Z, S)
    assert (d != d_ff).any()


@pytest.mark.parametrize("routing", [0, 3])
def test_paper_scale_sample(routing):
    inst, Z, S = synth.workload("paper", n_plans=16)
    print("paper seed", routing, flush=True)
    _compare(_sd(inst, routing), Z, S)


def test_worked_plan_on_gpu():
    # the hand-worked plan of the oracle pins: {A, C}, {B, D} -> 390 + 530
    from tests.whelpers import identity_zones, tiny_geometry
    inst = _sd(tiny_geometry([[180, 181], [420], [200], [430, 431]], capacity=3))
    wo = _wo()
    wh = wo.wo_load_warehouse([inst])
    d, _ = gpu_eval(wh, identity_zones(12)[None, :], np.arange(4, dtype=np.uint16)[None, :])
    wh.free()
    assert d.tolist() == [920]


SEED_CASES = [
    # (aisles, slots, orders, capacity, categories, lambda)
    (1, 1, 1, 1, 1, 0.0),          # one location, one order
    (1, 5, 7, 1, 3, 2.0),          # capacity 1: every order a tour, most oversize
    (1, 60, 300, 12, 6, 2.0),      # one aisle: first fit's tours
    (3, 4, 50, 2, 5, 3.0),         # many oversize orders
    (33, 7, 300, 32, 64, 1.5),     # capacity 32, two aisle words
    (64, 3, 129, 5, 17, 0.5),      # a multiple of 32 aisles
    (400, 250, 3000, 7, 64, 4.0),  # large orders, capacity 7
    (100, 250, 12000, 30, 8, 1.5), # 12,000 orders: most of the LDS
    (2000, 20, 3000, 30, 64, 1.5), # 2,000 aisles
    (10, 30, 1, 20, 12, 1.5),      # a single order
]


@pytest.mark.parametrize("case", SEED_CASES, ids=lambda c: "N%d_S%d_n%d_Q%d_C%d" % c[:5])
def test_edge_cases(case):
    rng = np.random.default_rng(abs(hash(case)) % (1 << 31))
    inst = _sd(_random_instance(rng, *case))
    Z, S = synth.make_plans(inst, 9, seed=int(rng.integers(1 << 30)))
    print("case", case, flush=True)
    _compare(inst, Z, S)


@pytest.mark.parametrize("routing", [1, 2, 4])
def test_routed_edge_cases(routing):
    rng = np.random.default_rng(61)
    for case in [(3, 4, 50, 2, 5, 3.0), (33, 7, 300, 32, 64, 1.5), (60, 2, 500, 12, 16, 1.5)]:
        inst = _sd(_random_instance(rng, *case), routing)
        Z, S = synth.make_plans(inst, 7, seed=int(rng.integers(1 << 30)))
        print("case", case, routing, flush=True)
        _compare(inst, Z, S)


def test_batched_instances_match_single():
    wo = _wo()
    rng = np.random.default_rng(67)
    insts = [_sd(_random_instance(rng, a, 250, o, 30, 64)) for a, o in [(8, 50), (400, 4000), (37, 700), (120, 61)]]
    per = [5, 3, 6, 2]
    Zs, Ss, offs = [], [], [0]
    for inst, k in zip(insts, per):
        Z, S = synth.make_plans(inst, k, seed=int(rng.integers(1 << 30)))
        Zs.append(Z)
        Ss.append(S.reshape(-1))
        offs.append(offs[-1] + k)
    wh = wo.wo_load_warehouse(insts)
    d, t = gpu_eval(wh, np.concatenate(Zs), np.concatenate(Ss), plan_offsets=offs)
    wh.free()
    for i, inst in enumerate(insts):
        dr, tr = oracle.eval_plans(inst, Zs[i], Ss[i].reshape(per[i], -1))
        assert np.array_equal(d[offs[i]:offs[i + 1]], dr)
        np.testing.assert_allclose(t[offs[i]:offs[i + 1]], tr, rtol=THR_RTOL)


def test_too_large_for_lds_is_refused():
    wo = _wo()
    rng = np.random.default_rng(71)
    inst = _sd(_random_instance(rng, 100, 250, 40000, 30, 8, lam=0.0))
    with pytest.raises(wo.WoError) as e:
        wo.wo_load_warehouse([inst])
    assert e.value.status == wo.WO_E_UNSUPPORTED


def test_malformed_sequence_stays_in_bounds(monkeypatch):
    wo = _wo()
    inst, Z, S = synth.workload("tiny", n_plans=8)
    wh = wo.wo_load_warehouse([_sd(inst)])
    S2 = S.copy()
    S2[0, 0] = 60000                    # out of range id
    S2[1, :50] = S2[1, 0]               # one order fifty times
    d, _ = gpu_eval(wh, Z, S2)
    assert d.shape == (8,)
    d_ref, _ = oracle.eval_plans(_sd(inst), Z[2:], S[2:])
    assert np.array_equal(d[2:], d_ref)  # the well-formed plans of the same call
    monkeypatch.setenv("WO_VALIDATE", "1")
    with pytest.raises(wo.WoError):
        gpu_eval(wh, Z, S2)
    wh.free()


def test_orders_over_many_aisles_are_refused():
    # an order of 1,100 lines in a warehouse of 2,000 aisles could visit more
    # than the 1,023 aisles a state word counts
    from tests.whelpers import tiny_geometry
    wo = _wo()
    inst = _sd(tiny_geometry([list(range(0, 4400, 4))[:1100], [5]], capacity=32, n_aisles=2000, slots=2,
                             n_cat=1, cat_size=8000))
    with pytest.raises(wo.WoError) as e:
        wo.wo_load_warehouse([inst])
    assert e.value.status == wo.WO_E_UNSUPPORTED

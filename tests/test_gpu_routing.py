"""GPU parity of the return, largest-gap, optimal and combined routes against the CPU
oracle (through the C ABI).  Distances must match bit-exactly; the throughput to
1e-6 relative, as for the S-shape route."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_eval import _compare, _random_instance, _structured_sequences, _wo

pytestmark = pytest.mark.gpu

ROUTES = [1, 2, 3, 4]    # return, largest gap, optimal, combined


def _routed(inst, routing):
    return dataclasses.replace(inst, routing=routing)


@pytest.mark.parametrize("routing", ROUTES)
def test_tiny_all_plans(routing):
    inst, Z, S = synth.workload("tiny")
    print("tiny", routing, flush=True)
    _compare(_routed(inst, routing), Z, S)


@pytest.mark.parametrize("routing", ROUTES)
def test_paper_scale_sample(routing):
    inst, Z, S = synth.workload("paper", n_plans=64)
    print("paper", routing, flush=True)
    _compare(_routed(inst, routing), Z, S)


def test_optimal_route_near_its_32_bit_bound():
    # slots 2,000 dm apart: L = 500,000 dm and 4 L (N + 1) + 4 w (N + 2) = 8.0e8 dm,
    # close to the 2^30 the load allows; the programme's sums stay exact
    import synth as sy
    inst = sy.make_instance(n_aisles=400, slots_per_side=250, pitch_dm=2000, spacing_dm=30, capacity=30,
                            n_categories=64, n_skus=150000, category_mode="dirichlet", n_orders=4000,
                            lines_lambda=1.5, zipf_s=1.1, seed=17)
    Z, S = sy.make_plans(inst, 24, seed=18)
    for routing in (3, 4):
        print("large geometry", routing, flush=True)
        _compare(_routed(inst, routing), Z, S)


ROUTE_CASES = [
    # (aisles, slots, orders, capacity, categories, lambda)
    (1, 5, 7, 3, 3, 2.0),          # one aisle: every tour is a return route
    (3, 4, 50, 2, 5, 3.0),         # oversize orders, their own tours
    (33, 7, 300, 32, 64, 1.5),     # capacity 32: rows of 32 picks
    (400, 250, 4000, 1, 64, 0.3),  # ~4,000 tours: several tour tiles
    (400, 250, 6000, 30, 64, 1.5), # sequence in memory
    (60, 2, 500, 12, 16, 1.5),     # aisles 20 dm long, 30 dm apart: loops over empty aisles pay
    (300, 1, 400, 8, 8, 1.0),      # aisles 10 dm long, long runs without picks
    (2000, 100, 2000, 30, 64, 1.5),   # 2,000 aisles: long runs between aisles with picks
]


@pytest.mark.parametrize("routing", ROUTES)
@pytest.mark.parametrize("case", ROUTE_CASES, ids=lambda c: "N%d_S%d_n%d_Q%d_C%d" % c[:5])
def test_route_edge_cases(case, routing):
    rng = np.random.default_rng(abs(hash(case)) % (1 << 31))
    inst = _routed(_random_instance(rng, *case), routing)
    Z, S = synth.make_plans(inst, 23, seed=int(rng.integers(1 << 30)))
    print("case", case, routing, flush=True)
    _compare(inst, Z, S)


@pytest.mark.parametrize("routing", ROUTES)
def test_structured_sequences_routed(routing):
    rng = np.random.default_rng(29)
    inst = _routed(_random_instance(rng, 400, 250, 4000, 30, 64, lam=1.5), routing)
    S = _structured_sequences(inst, rng)
    Z = synth.generators.random_zone_perms(rng, S.shape[0], inst.n_categories)
    _compare(inst, Z, S)


@pytest.mark.parametrize("routing", [2, 3, 4])
def test_batched_routed_instances_match_single(routing):
    import torch
    wo = _wo()
    rng = np.random.default_rng(31)
    # orders up to 1,024, up to 2,048 and beyond: all three launch classes
    insts = [_routed(_random_instance(rng, n_a, 40, n_o, 20, 16), routing)
             for n_a, n_o in ((8, 60), (30, 500), (12, 200), (60, 1500), (100, 3000))]
    plans = [synth.make_plans(i, 16, seed=k) for k, i in enumerate(insts)]
    wh = wo.wo_load_warehouse(insts)
    Z = np.concatenate([p[0] for p in plans])
    S = np.concatenate([p[1].reshape(-1) for p in plans])
    n = 16 * len(insts)
    offs = np.arange(0, n + 1, 16, dtype=np.int64)
    z = torch.from_numpy(Z).cuda()
    s = torch.from_numpy(S.view(np.int16)).cuda()
    d = torch.empty(n, dtype=torch.int32, device="cuda")
    t = torch.empty(n, dtype=torch.float32, device="cuda")
    wo.wo_eval_plans(wh, z, s, d, t, plan_offsets=offs)
    torch.cuda.synchronize()
    for k, (inst, (Zi, Si)) in enumerate(zip(insts, plans)):
        d_ref, _ = oracle.eval_plans(inst, Zi, Si)
        assert np.array_equal(d.cpu().numpy()[16 * k:16 * (k + 1)], d_ref)
    wh.free()


def _with_long_orders(rng, base, long_sizes):
    """`base` with some orders replaced by longer ones (the routes keep 32
    picks per tour row; longer orders are tours of their own, routed apart)."""
    sizes = np.diff(base.order_offsets).copy()
    idx = rng.choice(len(sizes), size=len(long_sizes), replace=False)
    sizes[idx] = long_sizes
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    skus = rng.integers(0, base.n_skus, size=int(offs[-1]), dtype=np.int32)
    return dataclasses.replace(base, order_offsets=offs, order_skus=skus)


@pytest.mark.parametrize("batching", [0, 1, 2])
@pytest.mark.parametrize("routing", ROUTES)
def test_orders_longer_than_a_pick_row(routing, batching):
    # orders of 33 .. 700 lines among ordinary ones (capacity 20): each is a
    # tour of its own, sorted and walked apart from the pick rows, under
    # next fit, first fit and seed batching
    rng = np.random.default_rng(41 + routing)
    base = _random_instance(rng, 120, 40, 400, 20, 16, lam=1.5)
    inst = _with_long_orders(rng, base, [33, 40, 64, 65, 200, 700])
    inst = dataclasses.replace(inst, routing=routing, batching=batching)
    Z, S = synth.make_plans(inst, 19, seed=int(rng.integers(1 << 30)))
    print("long orders", routing, batching, flush=True)
    _compare(inst, Z, S, line_passes=(0,))


def test_longest_routed_order_and_beyond():
    # an order of WO_MAX_ROUTED_ORDER_LINES lines is evaluated (its sort
    # fills 32 KB of LDS); one line more is refused at load
    wo = _wo()
    rng = np.random.default_rng(37)
    base = _random_instance(rng, 400, 250, 60, 30, 64, lam=1.0)
    inst = dataclasses.replace(_with_long_orders(rng, base, [8192, 100]), routing=3)
    Z, S = synth.make_plans(inst, 6, seed=5)
    print("order of 8,192 lines", flush=True)
    _compare(inst, Z, S, line_passes=(0,))
    inst = dataclasses.replace(_with_long_orders(rng, base, [8193]), routing=1)
    with pytest.raises(wo.WoError) as e:
        wo.wo_load_warehouse([inst])
    assert "lines" in str(e.value)
    # the S-shape route has no such limit
    wh = wo.wo_load_warehouse([dataclasses.replace(inst, routing=0)])
    wh.free()


@pytest.mark.parametrize("routing", [1, 3])
def test_batched_instances_with_long_orders(routing):
    # long orders in every launch class (64-, 128- and 256-thread workgroups)
    import torch
    wo = _wo()
    rng = np.random.default_rng(43)
    insts = []
    for n_a, n_o in ((20, 300), (60, 1500), (100, 3000)):
        base = _random_instance(rng, n_a, 40, n_o, 20, 16)
        insts.append(dataclasses.replace(_with_long_orders(rng, base, [35, 150]), routing=routing))
    plans = [synth.make_plans(i, 12, seed=k) for k, i in enumerate(insts)]
    wh = wo.wo_load_warehouse(insts)
    Z = np.concatenate([p[0] for p in plans])
    S = np.concatenate([p[1].reshape(-1) for p in plans])
    n = 12 * len(insts)
    offs = np.arange(0, n + 1, 12, dtype=np.int64)
    d = torch.empty(n, dtype=torch.int32, device="cuda")
    wo.wo_eval_plans(wh, torch.from_numpy(Z).cuda(), torch.from_numpy(S.view(np.int16)).cuda(), d,
                     plan_offsets=offs)
    torch.cuda.synchronize()
    for k, (inst, (Zi, Si)) in enumerate(zip(insts, plans)):
        d_ref, _ = oracle.eval_plans(inst, Zi, Si)
        assert np.array_equal(d.cpu().numpy()[12 * k:12 * (k + 1)], d_ref), k
    wh.free()

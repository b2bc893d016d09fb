"""GPU parity of first-fit order batching, under every route, against the CPU
oracle (through the C ABI).  Distances must match bit-exactly; the throughput to 1e-6 relative,
as for next fit."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import gpu_eval
from tests.test_gpu_eval import THR_RTOL, _random_instance, _structured_sequences, _wo

pytestmark = pytest.mark.gpu


ROUTES = [0, 1, 2, 3, 4]    # S-shape, return, largest gap, optimal, combined


def _ff(inst, routing=None):
    inst = dataclasses.replace(inst, batching=1)
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
    print("tiny first fit", routing, flush=True)
    d_ff = _compare(_ff(inst, routing), Z, S)
    d_nf, _ = oracle.eval_plans(dataclasses.replace(inst, routing=routing), Z, S)
    assert (d_ff != d_nf).any()          # the rule changes the tours


@pytest.mark.parametrize("routing", ROUTES)
def test_paper_scale_sample(routing):
    inst, Z, S = synth.workload("paper", n_plans=64)
    print("paper first fit", routing, flush=True)
    _compare(_ff(inst, routing), Z, S)


def test_worked_plan_on_gpu():
    # A = {61, 62}, B = {598, 599}, C = {0}, capacity 3: first fit [A, C], [B]
    from tests.whelpers import identity_zones, tiny_geometry
    inst = _ff(tiny_geometry([[61, 62], [598, 599], [0]], capacity=3))
    Z = identity_zones(12)[None, :]
    S = np.arange(3, dtype=np.uint16)[None, :]
    wo = _wo()
    wh = wo.wo_load_warehouse([inst])
    d, _ = gpu_eval(wh, Z, S)
    wh.free()
    assert d.tolist() == [660 + 1130]


FF_CASES = [
    # (aisles, slots, orders, capacity, categories, lambda)
    (1, 1, 1, 1, 1, 0.0),          # one location, one order
    (1, 5, 7, 1, 3, 2.0),          # capacity 1: every order a tour, most oversize
    (3, 4, 50, 2, 5, 3.0),         # many oversize orders
    (33, 7, 300, 32, 64, 1.5),     # capacity 32, two aisle words
    (64, 3, 129, 5, 17, 0.5),      # a multiple of 32 aisles
    (400, 250, 4096, 1, 64, 0.0),  # 4,096 single-item orders at capacity 1: 4,096 tours, 22 S-shape tiles
    (400, 250, 4096, 30, 64, 1.5), # 4,096 orders
    (400, 250, 9000, 30, 64, 1.5), # more orders than tours a wave could keep room for in registers
    (100, 250, 20000, 2, 8, 0.5),  # 20,000 orders, about 13,000 tours
    (100, 250, 4000, 3, 8, 1.5),   # oversize orders among small ones
    (10, 30, 1, 20, 12, 1.5),      # a single order
    (400, 250, 3000, 7, 64, 4.0),  # large orders, capacity 7
]


@pytest.mark.parametrize("case", FF_CASES, ids=lambda c: "N%d_S%d_n%d_Q%d_C%d" % c[:5])
def test_edge_cases(case):
    rng = np.random.default_rng(abs(hash(case)) % (1 << 31))
    inst = _ff(_random_instance(rng, *case))
    Z, S = synth.make_plans(inst, 29, seed=int(rng.integers(1 << 30)))
    print("case", case, flush=True)
    _compare(inst, Z, S)


ROUTED_CASES = [
    (1, 5, 7, 3, 3, 2.0),          # one aisle
    (3, 4, 50, 2, 5, 3.0),         # oversize orders ride alone
    (33, 7, 300, 32, 64, 1.5),     # rows of 32 picks
    (400, 250, 4096, 1, 64, 0.0),  # 4,096 tours, 64 tiles of 64
    (60, 2, 500, 12, 16, 1.5),     # short aisles: loops over empty aisles pay (optimal)
]


@pytest.mark.parametrize("routing", [1, 2, 3, 4])
@pytest.mark.parametrize("case", ROUTED_CASES, ids=lambda c: "N%d_S%d_n%d_Q%d_C%d" % c[:5])
def test_routed_edge_cases(case, routing):
    rng = np.random.default_rng(abs(hash(case)) % (1 << 31))
    inst = _ff(_random_instance(rng, *case), routing)
    Z, S = synth.make_plans(inst, 17, seed=int(rng.integers(1 << 30)))
    print("case", case, routing, flush=True)
    _compare(inst, Z, S)


def _sized_orders(sizes, capacity, seed):
    """An instance of the tiny geometry whose orders have the given line
    counts (SKUs drawn uniformly, repeats allowed)."""
    from tests.whelpers import tiny_geometry
    rng = np.random.default_rng(seed)
    return _ff(tiny_geometry([list(rng.integers(0, 600, int(k))) for k in sizes], capacity=capacity))


@pytest.mark.parametrize("routing", [0, 1])
def test_open_tours_beyond_the_lanes(routing):
    # 150 orders of 16 items each leave a tour with room 14 (capacity 30), so
    # 150 tours are open at once: 64 in the lanes and 86 queued; the one- to
    # three-item orders that follow fill them in opening order, the lanes
    # refilling from the queue, and orders that fit no tour in the lanes find
    # theirs in the queue.  The plans shuffle this order too.
    rng = np.random.default_rng(53)
    sizes = [16] * 150 + list(rng.integers(1, 4, 600)) + [15] * 40 + list(rng.integers(1, 3, 200))
    inst = dataclasses.replace(_sized_orders(sizes, 30, 5), routing=routing)
    n = len(sizes)
    S = np.stack([np.arange(n, dtype=np.uint16)] + [rng.permutation(n).astype(np.uint16) for _ in range(7)])
    Z = synth.generators.random_zone_perms(rng, S.shape[0], inst.n_categories)
    # the queue is in use: first fit leaves more than 64 tours open at once
    lens = np.diff(inst.order_offsets)
    rooms, most = [], 0
    for o in S[0]:
        k = next((i for i, r in enumerate(rooms) if r >= lens[o]), None)
        if k is None:
            rooms.append(30 - lens[o])
        else:
            rooms[k] -= lens[o]
        most = max(most, sum(r >= 1 for r in rooms))
    assert most > 64
    _compare(inst, Z, S)


@pytest.mark.parametrize("routing", [0, 2])
def test_rooms_no_order_fits_are_dropped(routing):
    # every order has at least 9 items at capacity 20: a room below 9 is never
    # used again (no order fits it), so those tours leave the open list
    rng = np.random.default_rng(59)
    sizes = list(rng.integers(9, 21, 700))
    inst = dataclasses.replace(_sized_orders(sizes, 20, 6), routing=routing)
    Z, S = synth.make_plans(inst, 9, seed=3)
    _compare(inst, Z, S)


def test_structured_sequences():
    # sequences sorted by order size, both ways, and blocked: first fit packs
    # the small orders of a run into the room the large ones left
    rng = np.random.default_rng(41)
    inst = _ff(_random_instance(rng, 400, 250, 4000, 30, 64, lam=1.5))
    S = _structured_sequences(inst, rng)
    Z = synth.generators.random_zone_perms(rng, S.shape[0], inst.n_categories)
    _compare(inst, Z, S)


@pytest.mark.parametrize("routing", [0, 3])
def test_batched_instances_match_single(routing):
    import torch
    wo = _wo()
    rng = np.random.default_rng(43)
    insts = [_ff(_random_instance(rng, a, 250, o, 30, 64), routing)
             for a, o in [(8, 50), (400, 4000), (37, 700), (120, 61)]]
    per = [5, 3, 8, 2]
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
    del torch


def test_validation_mode(monkeypatch):
    wo = _wo()
    inst, Z, S = synth.workload("tiny", n_plans=8)
    wh = wo.wo_load_warehouse([_ff(inst)])
    monkeypatch.setenv("WO_VALIDATE", "1")
    gpu_eval(wh, Z, S)                  # valid plans pass
    S2 = S.copy()
    S2[3, 5] = S2[3, 6]                 # duplicate order id
    with pytest.raises(wo.WoError) as ei:
        gpu_eval(wh, Z, S2)
    assert ei.value.status == wo.WO_E_INVAL
    Z2 = Z.copy()
    Z2[1, 0] = Z2[1, 1]                 # duplicate zone
    with pytest.raises(wo.WoError):
        gpu_eval(wh, Z2, S)
    monkeypatch.delenv("WO_VALIDATE")
    S3 = S.copy()
    S3[0, 0] = 60000                    # out of range id without validation: defined, in bounds
    d, _ = gpu_eval(wh, Z, S3)
    assert d.shape == (8,)
    wh.free()


def test_repeat_calls_deterministic():
    wo = _wo()
    inst, Z, S = synth.workload("paper", n_plans=256)
    wh = wo.wo_load_warehouse([_ff(inst)])
    d1, t1 = gpu_eval(wh, Z, S)
    d2, t2 = gpu_eval(wh, Z, S)
    wh.free()
    assert np.array_equal(d1, d2) and np.array_equal(t1, t2)


def test_graph_capture_replays():
    # first fit allocates nothing per call: a captured evaluation replays exactly
    import torch
    wo = _wo()
    rng = np.random.default_rng(47)
    insts = [_ff(_random_instance(rng, a, 250, o, 30, 64)) for a, o in [(8, 50), (400, 4000), (37, 700)]]
    per = 6
    Zs, Ss = [], []
    for inst in insts:
        Z, S = synth.make_plans(inst, per, seed=int(rng.integers(1 << 30)))
        Zs.append(Z)
        Ss.append(S.reshape(-1))
    offs = np.arange(len(insts) + 1, dtype=np.int64) * per
    wh = wo.wo_load_warehouse(insts)
    z = torch.from_numpy(np.concatenate(Zs)).cuda()
    s = torch.from_numpy(np.concatenate(Ss).view(np.int16)).cuda()
    n = z.shape[0]
    d_eager, t_eager = gpu_eval(wh, np.concatenate(Zs), np.concatenate(Ss), plan_offsets=offs)
    d = torch.zeros(n, dtype=torch.int32, device="cuda")
    t = torch.zeros(n, dtype=torch.float32, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        wo.wo_eval_plans(wh, z, s, d, t, plan_offsets=offs)   # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        wo.wo_eval_plans(wh, z, s, d, t, plan_offsets=offs)
    for rep in range(4):
        d.zero_()
        t.zero_()
        d2, _ = gpu_eval(wh, np.concatenate(Zs), np.concatenate(Ss), plan_offsets=offs)   # eager work between
        assert np.array_equal(d2, d_eager)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(d.cpu().numpy(), d_eager), rep
        assert np.array_equal(t.cpu().numpy(), t_eager), rep
    del g
    wh.free()


def test_autotune_times_first_fit_once():
    import torch
    wo = _wo()
    inst, Z, S = synth.workload("paper", n_plans=256)
    wh = wo.wo_load_warehouse([_ff(inst)])
    z = torch.from_numpy(Z).cuda()
    s = torch.from_numpy(S.view(np.int16)).cuda().reshape(-1)
    d = torch.empty(256, dtype=torch.int32, device="cuda")
    best, all_cfgs = wo.wo_autotune_eval(wh, z, s, d, reps=2)
    assert len(all_cfgs) == 1 and best["ms"] > 0
    d_gpu, _ = gpu_eval(wh, Z, S)
    wh.free()
    assert np.array_equal(d_gpu, oracle.eval_plans(_ff(inst), Z, S)[0])

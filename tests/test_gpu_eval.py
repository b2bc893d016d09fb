"""GPU parity of exact plan evaluation against the CPU oracle (through the C ABI).

Distances must match bit-exactly (integer decimetres); the time-window
throughput is computed in IEEE double on both sides and must agree to 1e-6
relative (it is expected to be identical)."""
import os

import numpy as np
import pytest

import oracle
import synth
from synth import Instance
from tests.gpu_util import gpu_eval

pytestmark = pytest.mark.gpu

THR_RTOL = 1e-6


def _wo():
    import torch
    from paper_2110_13693_amd import wo
    assert torch.cuda.is_available()
    return wo


def _compare(inst, Z, S, wh=None, n_threads=8, line_passes=(1, 2, 0)):
    wo = _wo()
    own = wh is None
    if own:
        wh = wo.wo_load_warehouse([inst])
    d_ref, t_ref = oracle.eval_plans(inst, Z, S, n_threads=n_threads)
    for lp in line_passes:           # every mapping of the aisle-set pass
        wo.wo_set_eval_config(wh, 256, 0, 0, lp)
        d_gpu, t_gpu = gpu_eval(wh, Z, S)
        bad = np.flatnonzero(d_gpu != d_ref)
        assert bad.size == 0, "line pass %d, plans %s: gpu %s oracle %s" % (
            lp, bad[:5], d_gpu[bad[:5]], d_ref[bad[:5]])
        np.testing.assert_allclose(t_gpu, t_ref, rtol=THR_RTOL, atol=0)
    if own:
        wh.free()


def test_tiny_all_plans():
    inst, Z, S = synth.workload("tiny")
    print("case tiny 256 plans", flush=True)
    _compare(inst, Z, S)


def test_paper_scale_all_plans():
    # the benchmarked configuration: 4,096 plans on the 400-aisle warehouse
    inst, Z, S = synth.workload("paper")
    print("case paper 4096 plans", flush=True)
    _compare(inst, Z, S)


def test_worked_plan_on_gpu():
    from tests.whelpers import identity_zones, tiny_geometry
    inst = tiny_geometry([[0, 130], [599], [61, 62, 300]], capacity=3)
    Z = np.stack([identity_zones(12)] * 3)
    Z[2][0], Z[2][11] = 11, 0
    S = np.asarray([[0, 1, 2], [1, 2, 0], [0, 1, 2]], dtype=np.uint16)
    wo = _wo()
    wh = wo.wo_load_warehouse([inst])
    d, _ = gpu_eval(wh, Z, S)
    wh.free()
    assert d.tolist() == [2630, 2750, 2150]


def _random_instance(rng, n_aisles, slots, n_orders, capacity, n_cat, lam=1.5, zipf=1.0, fill=0.8):
    n_sku = max(n_cat, int(2 * n_aisles * slots * fill))
    return synth.make_instance(n_aisles=n_aisles, slots_per_side=slots, pitch_dm=10, spacing_dm=30,
                               capacity=capacity, n_categories=n_cat, n_skus=n_sku,
                               category_mode="dirichlet", n_orders=n_orders, lines_lambda=lam,
                               zipf_s=zipf, seed=int(rng.integers(1 << 30)))


EDGE_CASES = [
    # (aisles, slots, orders, capacity, categories, lambda)
    (1, 1, 1, 1, 1, 0.0),        # one location, one order
    (1, 5, 7, 1, 3, 2.0),        # capacity 1: every order a tour, most oversize
    (3, 4, 50, 2, 5, 3.0),       # many oversize orders
    (33, 7, 300, 32, 64, 1.5),   # 64 categories, capacity at the limit, 2 aisle words
    (64, 3, 129, 5, 17, 0.5),    # aisle count a multiple of 32
    (65, 250, 1000, 30, 64, 1.5),
    (400, 250, 4000, 1, 64, 0.3),  # ~4,000 tours: several tour tiles
    (10, 30, 1, 20, 12, 1.5),    # a single order
    (400, 250, 6000, 30, 64, 1.5),    # more orders than one block keeps in registers
    (400, 250, 12000, 3, 64, 1.5),    # oversize orders (serial chain), several tiles, sequence in memory
    (100, 250, 40000, 30, 8, 0.0),    # 40,000 single-line orders: near the LDS limit, tiles halved
    (100, 250, 6000, 2, 8, 0.0),      # single-line orders at capacity 2: 64 chase segments
    (2000, 100, 2000, 30, 64, 1.5),   # 2,000 aisles: 63-word aisle sets
    (4096, 512, 3000, 20, 64, 1.5),   # the most locations a warehouse may have (2^22)
]


@pytest.mark.parametrize("case", EDGE_CASES, ids=lambda c: "N%d_S%d_n%d_Q%d_C%d" % c[:5])
def test_edge_cases(case):
    rng = np.random.default_rng(abs(hash(case)) % (1 << 31))
    inst = _random_instance(rng, *case)
    Z, S = synth.make_plans(inst, 37, seed=int(rng.integers(1 << 30)))
    print("case", case, flush=True)
    _compare(inst, Z, S)


def _structured_sequences(inst, rng):
    """Order sequences that defeat the sizing of the parallel next-fit: runs
    of small orders put more candidate entries in a segment than its chase
    lanes hold, and runs of large ones more openings than a chase record list
    holds, so such plans fall back to the serial chain."""
    sizes = np.diff(inst.order_offsets)
    asc = np.argsort(sizes, kind="stable")
    half = len(asc) // 2
    small, large = asc[:half], asc[half:][::-1]
    blocks = []
    for i in range(0, half, 100):
        blocks += [small[i:i + 100], large[i:i + 100]]
    blocked = np.concatenate(blocks + [asc[2 * half:]])
    middle = np.concatenate([large[: half // 2], small, large[half // 2:], asc[2 * half:]])
    seqs = [asc, asc[::-1], blocked, middle, rng.permutation(len(asc))]
    for s in seqs:
        assert np.array_equal(np.sort(s), np.arange(len(asc)))
    return np.stack(seqs).astype(np.uint16)


def _bimodal_instance(rng, n_orders, capacity, small, large, p_small=0.5):
    """Orders of `small` lines (fraction p_small) or `large` lines on a
    400-aisle warehouse."""
    import dataclasses
    base = _random_instance(rng, 400, 250, n_orders, capacity, 64, lam=0.0)
    sizes = np.where(rng.random(n_orders) < p_small, small, large).astype(np.int32)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    skus = rng.integers(0, base.n_skus, size=int(offs[-1]), dtype=np.int32)
    return dataclasses.replace(base, order_offsets=offs, order_skus=skus)


@pytest.mark.parametrize("kind", ["paper", "bimodal", "skewed", "oversize"])
def test_structured_sequences(kind):
    rng = np.random.default_rng(23)
    if kind == "paper":
        inst = _random_instance(rng, 400, 250, 4000, 30, 64, lam=1.5)
    elif kind == "bimodal":
        inst = _bimodal_instance(rng, 2000, 30, 1, 16)
    elif kind == "skewed":       # sorted runs of the rare 16-line orders overflow the chase records
        inst = _bimodal_instance(rng, 4000, 30, 1, 16, p_small=0.9)
    else:                        # orders larger than the capacity: the serial chain
        inst = _random_instance(rng, 400, 250, 2000, 8, 64, lam=1.5)
    S = _structured_sequences(inst, rng)
    Z = synth.generators.random_zone_perms(rng, S.shape[0], inst.n_categories)
    print("structured sequences", kind, flush=True)
    _compare(inst, Z, S)


def test_instance_beyond_lds_is_rejected():
    # 65,535 orders need more LDS than a CU has: the load fails cleanly
    wo = _wo()
    rng = np.random.default_rng(11)
    inst = _random_instance(rng, 200, 250, 65535, 30, 8, lam=0.0)
    with pytest.raises(wo.WoError) as e:
        wo.wo_load_warehouse([inst])
    assert "LDS" in str(e.value)


def test_zero_plans_is_noop():
    import torch
    wo = _wo()
    inst, Z, S = synth.workload("tiny", n_plans=1)
    wh = wo.wo_load_warehouse([inst])
    z = torch.zeros((0, 64), dtype=torch.uint8, device="cuda")
    s = torch.zeros((0,), dtype=torch.int16, device="cuda")
    d = torch.zeros((0,), dtype=torch.int32, device="cuda")
    wo.wo_eval_plans(wh, z, s, d)
    wh.free()


def test_batched_instances_match_single():
    rng = np.random.default_rng(11)
    insts = [_random_instance(rng, int(a), 250, int(o), 30, 64)
             for a, o in [(8, 50), (400, 4000), (37, 700), (120, 61), (9, 3999)]]
    per = [5, 3, 8, 1, 6]
    Zs, Ss, offs = [], [], [0]
    for inst, k in zip(insts, per):
        Z, S = synth.make_plans(inst, k, seed=int(rng.integers(1 << 30)))
        Zs.append(Z)
        Ss.append(S.reshape(-1))
        offs.append(offs[-1] + k)
    wo = _wo()
    wh = wo.wo_load_warehouse(insts)
    d, t = gpu_eval(wh, np.concatenate(Zs), np.concatenate(Ss), plan_offsets=offs)
    wh.free()
    for i, inst in enumerate(insts):
        dr, tr = oracle.eval_plans(inst, Zs[i], Ss[i].reshape(per[i], -1))
        assert np.array_equal(d[offs[i]:offs[i + 1]], dr)
        np.testing.assert_allclose(t[offs[i]:offs[i + 1]], tr, rtol=THR_RTOL)


def test_validation_mode(monkeypatch):
    wo = _wo()
    inst, Z, S = synth.workload("tiny", n_plans=8)
    wh = wo.wo_load_warehouse([inst])
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
    import torch
    wo = _wo()
    inst, Z, S = synth.workload("paper", n_plans=512)
    wh = wo.wo_load_warehouse([inst])
    d1, t1 = gpu_eval(wh, Z, S)
    d2, t2 = gpu_eval(wh, Z, S)
    wh.free()
    assert np.array_equal(d1, d2) and np.array_equal(t1, t2)


def test_layout_change_on_another_stream_while_busy_is_refused():
    # The plan map and the tables built from it are shared by every call on
    # a handle, and a call uploads them in its own stream.  While the
    # previous call (first stream) may still run, a call on a second stream
    # is refused when either call rewrites that state; two calls that only
    # read it may overlap; once the first stream has drained, the new layout
    # is accepted too.  Results are checked against the oracle.
    import torch
    wo = _wo()
    rng = np.random.default_rng(5)
    insts = [_random_instance(rng, 12, 250, 300, 30, 64), _random_instance(rng, 20, 250, 500, 30, 64)]

    def layout(per):
        Zs, Ss = [], []
        for inst, k in zip(insts, per):
            Z, S = synth.make_plans(inst, k, seed=int(rng.integers(1 << 30)))
            Zs.append(Z)
            Ss.append(S.reshape(-1))
        return Zs, Ss, [0, per[0], per[0] + per[1]]

    Z1, S1, off1 = layout((8, 8))
    Z2, S2, off2 = layout((4, 12))
    wh = wo.wo_load_warehouse(insts)

    def dev(Zs, Ss):
        z = torch.from_numpy(np.concatenate(Zs)).cuda()
        s = torch.from_numpy(np.concatenate(Ss).view(np.int16)).cuda()
        return z, s, torch.full((z.shape[0],), -1, dtype=torch.int32, device="cuda")

    z1, s1, d0 = dev(Z1, S1)
    z2, s2, d2 = dev(Z2, S2)
    _, _, d1 = dev(Z1, S1)
    _, _, d3 = dev(Z1, S1)
    # the first layout's tables are uploaded and in place before the streams
    wo.wo_eval_plans(wh, z1, s1, d0, plan_offsets=off1)
    torch.cuda.synchronize()
    a, b = torch.cuda.Stream(), torch.cuda.Stream()
    x = torch.randn(4096, 4096, device="cuda")
    w = torch.randn(4096, 4096, device="cuda") / 64.0
    torch.cuda.synchronize()
    with torch.cuda.stream(a):
        for _ in range(40):          # tens of milliseconds of work ahead of the call
            x = x @ w
        wo.wo_eval_plans(wh, z1, s1, d1, plan_offsets=off1, stream=a)
    print("stream a busy; a new layout on stream b", flush=True)
    with pytest.raises(wo.WoError) as e:
        wo.wo_eval_plans(wh, z2, s2, d2, plan_offsets=off2, stream=b)
    assert e.value.status == wo.WO_E_STATE
    # the same layout only reads the shared tables
    wo.wo_eval_plans(wh, z1, s1, d3, plan_offsets=off1, stream=b)
    torch.cuda.synchronize()
    wo.wo_eval_plans(wh, z2, s2, d2, plan_offsets=off2, stream=b)
    torch.cuda.synchronize()
    for (Zs, Ss, off), d in (((Z1, S1, off1), d0), ((Z1, S1, off1), d1), ((Z1, S1, off1), d3),
                             ((Z2, S2, off2), d2)):
        got = d.cpu().numpy()
        for i, inst in enumerate(insts):
            ref, _ = oracle.eval_plans(inst, Zs[i], Ss[i].reshape(off[i + 1] - off[i], -1))
            assert np.array_equal(got[off[i]:off[i + 1]], ref)
    wh.free()

"""GPU genetic search: one generation must equal the CPU re-implementation
(oracle/search.py) bit-exactly -- same parents, mutations, children,
distances and replacement -- for the plain and the screened arm."""
import numpy as np
import pytest

import oracle
import synth
from oracle import search as G

pytestmark = pytest.mark.gpu


def _wo():
    import torch
    from paper_2110_13693_amd import wo
    assert torch.cuda.is_available()
    return wo


def _init(inst, P, seed):
    rng = np.random.default_rng([seed, synth.generators.STREAM_SEARCH_INIT])
    Z = synth.generators.random_zone_perms(rng, P, inst.n_categories)
    S = synth.generators.random_order_perms(rng, P, inst.n_orders)
    return Z, S


def _population(wo, s, P, n, keep=0):
    import torch
    z = torch.empty((P, 64), dtype=torch.uint8, device="cuda")
    q = torch.empty((P * n,), dtype=torch.int16, device="cuda")
    d = torch.empty(P, dtype=torch.int32, device="cuda")
    k = torch.empty(keep, dtype=torch.int32, device="cuda") if keep else None
    wo.wo_search_population(s, z, q, d, k)
    torch.cuda.synchronize()
    out = (z.cpu().numpy(), q.cpu().numpy().view(np.uint16).reshape(P, n), d.cpu().numpy())
    return out + ((k.cpu().numpy(),) if keep else ())


@pytest.mark.parametrize("workload,P,variant", [("tiny", 64, {}), ("paper", 16, {}),
                                                ("tiny", 64, {"batching": 1}), ("tiny", 64, {"routing": 3}),
                                                ("paper", 16, {"batching": 1, "routing": 2})])
def test_plain_generations_match_cpu(workload, P, variant):
    import dataclasses
    import torch
    wo = _wo()
    inst, _, _ = synth.workload(workload, n_plans=1)
    inst = dataclasses.replace(inst, **variant)     # the search evaluates under the load's rules
    Z, S = _init(inst, P, 3)
    wh = wo.wo_load_warehouse([inst])
    seed = 1234
    s = wo.wo_search_create(wh, 0, torch.from_numpy(Z).cuda(),
                            torch.from_numpy(S.view(np.int16)).cuda().reshape(-1), P, seed=seed)
    D, _ = oracle.eval_plans(inst, Z, S)
    z0, q0, d0 = _population(wo, s, P, inst.n_orders)
    assert np.array_equal(d0, D)
    for gen in range(2):
        wo.wo_search_step(wh, s, None, 1)
        Z, S, D = G.plain_generation(inst, Z, S, D, seed=seed, gen=gen)
        zg, qg, dg = _population(wo, s, P, inst.n_orders)
        assert np.array_equal(zg, Z), gen
        assert np.array_equal(qg, S), gen
        assert np.array_equal(dg, D), gen
    zb, qb, db, g = wo.wo_search_best(s)
    assert g == 2 and db == D.min()
    s.free()
    wh.free()


def test_screened_generation_matches_cpu():
    import torch
    wo = _wo()
    inst, _, _ = synth.workload("tiny", n_plans=1)
    P, K, keep, seed = 64, 512, 20, 77
    Z, S = _init(inst, P, 4)
    wh = wo.wo_load_warehouse([inst])
    sur = wo.wo_sur_create(inst.n_categories, None, seed=5)
    wo.wo_sur_set_scale(sur, 7.5e4, 2e3)
    s = wo.wo_search_create(wh, 0, torch.from_numpy(Z).cuda(),
                            torch.from_numpy(S.view(np.int16)).cuda().reshape(-1), P,
                            candidates=K, keep=keep, seed=seed)
    D, _ = oracle.eval_plans(inst, Z, S)
    wo.wo_search_step(wh, s, sur, 1)
    zg, qg, dg, kept = _population(wo, s, P, inst.n_orders, keep)
    assert len(set(kept.tolist())) == keep and kept.min() >= 0 and kept.max() < K
    Z2, S2, D2 = G.screened_generation(inst, Z, S, D, seed=seed, gen=0, kept_ids=kept)
    assert np.array_equal(zg, Z2) and np.array_equal(qg, S2) and np.array_equal(dg, D2)
    s.free()
    sur.free()
    wh.free()


def test_search_keeps_best_and_improves():
    import torch
    wo = _wo()
    inst, _, _ = synth.workload("paper", n_plans=1)
    P = 512
    Z, S = _init(inst, P, 5)
    wh = wo.wo_load_warehouse([inst])
    s = wo.wo_search_create(wh, 0, torch.from_numpy(Z).cuda(),
                            torch.from_numpy(S.view(np.int16)).cuda().reshape(-1), P, seed=9)
    best = []
    for _ in range(6):
        best.append(wo.wo_search_best(s)[2])
        wo.wo_search_step(wh, s, None, 2)
    best.append(wo.wo_search_best(s)[2])
    assert all(b2 <= b1 for b1, b2 in zip(best, best[1:]))
    assert best[-1] < best[0]
    # the reported best is a real plan with that exact distance
    zb, qb, db, _ = wo.wo_search_best(s)
    _, d, _ = oracle.eval_plan(inst, zb, qb)
    assert d == db
    s.free()
    wh.free()


def test_checkpoint_resumes_bit_exactly(tmp_path):
    import torch
    wo = _wo()
    inst, _, _ = synth.workload("tiny", n_plans=1)
    P = 64
    Z, S = _init(inst, P, 5)
    wh = wo.wo_load_warehouse([inst])
    s = wo.wo_search_create(wh, 0, torch.from_numpy(Z).cuda(),
                            torch.from_numpy(S.view(np.int16)).cuda().reshape(-1), P, seed=77)
    wo.wo_search_step(wh, s, None, 3)
    path = str(tmp_path / "search.bin")
    wo.wo_search_save(s, path)
    r = wo.wo_search_load(wh, 0, path)
    assert wo.wo_search_best(r)[3] == 3                       # the generation counter travels
    wo.wo_search_step(wh, s, None, 4)
    wo.wo_search_step(wh, r, None, 4)
    a = _population(wo, s, P, inst.n_orders)
    b = _population(wo, r, P, inst.n_orders)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert wo.wo_search_best(s)[2:] == wo.wo_search_best(r)[2:]
    # a different instance with the same sizes gives other distances: refused
    other = synth.workload("tiny", seed=9, n_plans=1)[0]
    assert other.n_orders == inst.n_orders and other.n_categories == inst.n_categories
    wh2 = wo.wo_load_warehouse([other])
    with pytest.raises(wo.WoError):
        wo.wo_search_load(wh2, 0, path)
    wh2.free()
    r.free()
    s.free()
    wh.free()

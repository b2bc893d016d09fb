"""Batched evaluation of uneven instances: one launch over many warehouses
(aisles and orders log-uniform), grid-stride and cost-ordered queue
distributions, graph capture and replay, and the autotuner."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _wo():
    import torch
    from paper_2110_13693_amd import wo
    assert torch.cuda.is_available()
    return wo


def _batch(n_inst, per, seed=0):
    insts = synth.make_batched_instances(n_inst, seed=seed)
    Z, S, _ = synth.generators.pack_batched_plans(insts, per, seed=seed)
    offs = np.arange(n_inst + 1, dtype=np.int64) * per
    return insts, Z, S, offs


def _dev(Z, S):
    import torch
    return (torch.from_numpy(Z).cuda(), torch.from_numpy(S.view(np.int16)).cuda())


def _run(wo, wh, z, s, offs):
    import torch
    n = z.shape[0]
    d = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    t = torch.full((n,), -1.0, dtype=torch.float32, device="cuda")
    wo.wo_eval_plans(wh, z, s, d, t, plan_offsets=offs)
    torch.cuda.synchronize()
    return d.cpu().numpy(), t.cpu().numpy()


def _check_sample(insts, Z, S, offs, d, t, per, picks):
    base = 0
    rows = {}
    for i, inst in enumerate(insts):
        rows[i] = (base, inst.n_orders)
        base += per * inst.n_orders
    for p in picks:
        i = int(np.searchsorted(offs, p, side="right") - 1)
        b, n = rows[i]
        r = p - offs[i]
        seq = S[b + r * n: b + (r + 1) * n]
        _, dr, tr = oracle.eval_plan(insts[i], Z[p], seq)
        assert d[p] == dr, (p, i)
        assert abs(t[p] - tr) <= 1e-6 * abs(tr)


@pytest.mark.parametrize("queue", [0, 1])
def test_uneven_batch_all_plans(queue):
    wo = _wo()
    insts, Z, S, offs = _batch(48, 8, seed=1)
    wh = wo.wo_load_warehouse(insts)
    wo.wo_set_eval_config(wh, 256, 0, queue)
    z, s = _dev(Z, S)
    d, t = _run(wo, wh, z, s, offs)
    _check_sample(insts, Z, S, offs, d, t, 8, range(len(d)))
    wh.free()


def test_full_batched_configuration_sampled():
    # 512 instances x 256 plans in one launch; 300 sampled plans checked one by one
    wo = _wo()
    insts, Z, S, offs = _batch(512, 256, seed=0)
    wh = wo.wo_load_warehouse(insts)
    z, s = _dev(Z, S)
    d0, t0 = _run(wo, wh, z, s, offs)
    wo.wo_set_eval_config(wh, 256, 0, 1)
    d1, t1 = _run(wo, wh, z, s, offs)
    assert np.array_equal(d0, d1) and np.array_equal(t0, t1)
    picks = np.random.default_rng(3).choice(len(d0), 300, replace=False)
    _check_sample(insts, Z, S, offs, d1, t1, 256, sorted(picks.tolist()))
    wh.free()


@pytest.mark.parametrize("block,queue", [(128, 0), (512, 1)])
def test_block_sizes_agree(block, queue):
    wo = _wo()
    insts, Z, S, offs = _batch(24, 6, seed=2)
    wh = wo.wo_load_warehouse(insts)
    z, s = _dev(Z, S)
    d_ref, t_ref = _run(wo, wh, z, s, offs)
    wo.wo_set_eval_config(wh, block, 2, queue)
    d, t = _run(wo, wh, z, s, offs)
    assert np.array_equal(d, d_ref) and np.array_equal(t, t_ref)
    _check_sample(insts, Z, S, offs, d, t, 6, range(0, len(d), 7))
    wh.free()


@pytest.mark.parametrize("queue", [0, 1])
def test_small_instance_launch_matches_single_launch(queue):
    # instances of up to 1,024 orders go to a launch of 64-thread workgroups;
    # switching that off (small_orders = 0) must not change any result
    wo = _wo()
    insts, Z, S, offs = _batch(40, 6, seed=6)
    assert any(i.n_orders <= 1024 for i in insts) and any(i.n_orders > 1024 for i in insts)
    wh = wo.wo_load_warehouse(insts)
    z, s = _dev(Z, S)
    wo.wo_set_eval_config(wh, 256, 0, queue, 0, 1024)
    d_split, t_split = _run(wo, wh, z, s, offs)
    wo.wo_set_eval_config(wh, 256, 0, queue, 0, 0)
    d_one, t_one = _run(wo, wh, z, s, offs)
    assert np.array_equal(d_split, d_one) and np.array_equal(t_split, t_one)
    _check_sample(insts, Z, S, offs, d_split, t_split, 6, range(0, len(d_split), 5))
    wh.free()


@pytest.mark.parametrize("line_pass", [1, 2])
def test_line_passes_agree_on_uneven_batch(line_pass):
    # the aisle-set pass by order per lane (1) and in sequence order (2), in
    # every launch class (64-, 128- and 256-thread workgroups), against the
    # default mapping and the oracle
    wo = _wo()
    insts, Z, S, offs = _batch(40, 6, seed=8)
    wh = wo.wo_load_warehouse(insts)
    z, s = _dev(Z, S)
    d_ref, t_ref = _run(wo, wh, z, s, offs)
    wo.wo_set_eval_config(wh, 256, 0, 1, line_pass, 1024)
    d, t = _run(wo, wh, z, s, offs)
    assert np.array_equal(d, d_ref) and np.array_equal(t, t_ref)
    _check_sample(insts, Z, S, offs, d, t, 6, range(0, len(d), 9))
    wh.free()


def test_64_thread_workgroups_all_instances():
    # every instance in 64-thread workgroups, including those with more orders
    # than one wave keeps in registers
    wo = _wo()
    insts, Z, S, offs = _batch(24, 6, seed=7)
    wh = wo.wo_load_warehouse(insts)
    z, s = _dev(Z, S)
    d_ref, t_ref = _run(wo, wh, z, s, offs)
    wo.wo_set_eval_config(wh, 64, 0, 1, 0, 0)
    d, t = _run(wo, wh, z, s, offs)
    assert np.array_equal(d, d_ref) and np.array_equal(t, t_ref)
    _check_sample(insts, Z, S, offs, d, t, 6, range(0, len(d), 7))
    wh.free()


@pytest.mark.parametrize("queue", [0, 1])
def test_graph_capture_replays(queue):
    import torch
    wo = _wo()
    insts, Z, S, offs = _batch(32, 8, seed=4)
    wh = wo.wo_load_warehouse(insts)
    wo.wo_set_eval_config(wh, 256, 0, queue)
    z, s = _dev(Z, S)
    n = z.shape[0]
    d_eager, t_eager = _run(wo, wh, z, s, offs)        # also uploads the plan map / work list
    d = torch.zeros(n, dtype=torch.int32, device="cuda")
    t = torch.zeros(n, dtype=torch.float32, device="cuda")
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        wo.wo_eval_plans(wh, z, s, d, t, plan_offsets=offs)   # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        wo.wo_eval_plans(wh, z, s, d, t, plan_offsets=offs)
    for rep in range(4):
        d.zero_()
        t.zero_()
        d2, _ = _run(wo, wh, z, s, offs)                 # eager work between replays
        assert np.array_equal(d2, d_eager)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(d.cpu().numpy(), d_eager), rep
        assert np.array_equal(t.cpu().numpy(), t_eager), rep
    del g
    wh.free()


def test_autotuner_picks_a_valid_config_and_keeps_results():
    wo = _wo()
    insts, Z, S, offs = _batch(64, 16, seed=5)
    wh = wo.wo_load_warehouse(insts)
    z, s = _dev(Z, S)
    d_ref, t_ref = _run(wo, wh, z, s, offs)
    import torch
    dist = torch.empty(z.shape[0], dtype=torch.int32, device="cuda")
    best, timings = wo.wo_autotune_eval(wh, z, s, dist, plan_offsets=offs, reps=2)
    assert best["block_threads"] in (128, 256, 512) and best["queue"] in (0, 1)
    assert len(timings) >= 6 and best["ms"] == min(x["ms"] for x in timings)
    assert wo.wo_get_eval_config(wh)["block_threads"] == best["block_threads"]
    d, t = _run(wo, wh, z, s, offs)
    assert np.array_equal(d, d_ref) and np.array_equal(t, t_ref)
    wh.free()

"""GPU K-means class-based storage against the exact CPU oracle (through the
C ABI): categories, categories used and assignment count must be identical."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from oracle import kmeans
from tests.gpu_util import gpu_eval

pytestmark = pytest.mark.gpu


def _gpu(order_skus, n_skus, k, max_iter=100):
    import torch
    from paper_2110_13693_amd import wo
    skus = torch.from_numpy(np.ascontiguousarray(order_skus, dtype=np.int32)).cuda()
    cat = torch.full((n_skus,), -1, dtype=torch.int32, device="cuda")
    used, iters = wo.wo_kmeans_categories(skus, n_skus, k, cat, max_iter=max_iter)
    return cat.cpu().numpy(), used, iters


def _compare(order_skus, n_skus, k, max_iter=100):
    freq = kmeans.pick_frequency(n_skus, order_skus)
    ref = kmeans.kmeans_categories(freq, k, max_iter=max_iter)
    got = _gpu(order_skus, n_skus, k, max_iter)
    assert got[1:] == ref[1:], (got[1:], ref[1:])
    assert np.array_equal(got[0], ref[0])
    return got


@pytest.mark.parametrize("k", [1, 2, 8, 16, 64])
def test_paper_order_history(k):
    inst, _, _ = synth.workload("paper", n_plans=1)
    print("paper k", k, flush=True)
    _compare(inst.order_skus, inst.n_skus, k)


@pytest.mark.parametrize("seed", range(5))
def test_random_histories(seed):
    rng = np.random.default_rng(seed)
    n_skus = int(rng.integers(1, 5000))
    n_lines = int(rng.integers(1, 200000))
    skus = np.minimum(rng.zipf(1.2 + 0.2 * seed, size=n_lines) - 1, n_skus - 1)
    print("random", seed, n_skus, n_lines, flush=True)
    _compare(skus, n_skus, int(rng.integers(1, 65)))


def test_largest_history():
    # 2^24 lines (the most a call takes) over 2^22 SKUs: 16,777,217 histogram
    # bins, centroid sums near 2^24 and counts near 2^22, so the distance
    # products reach 2^68 and need the 128-bit comparison
    rng = np.random.default_rng(9)
    n_skus = 1 << 22
    skus = (rng.zipf(1.3, size=1 << 24) - 1) % n_skus
    print("largest history", flush=True)
    _compare(skus, n_skus, 64, max_iter=40)


def test_max_iter_stops_early():
    rng = np.random.default_rng(7)
    skus = rng.integers(0, 3000, size=100000) ** 2 // 3000
    for it in (1, 2, 3, 9):
        _, _, n = _compare(skus, 3000, 40, max_iter=it)
        assert n <= it


def test_out_of_range_sku_is_rejected():
    from paper_2110_13693_amd import wo
    with pytest.raises(wo.WoError) as e:
        _gpu(np.array([0, 1, 5]), 3, 2)
    assert e.value.status == wo.WO_E_INVAL


def test_categories_feed_the_evaluator():
    # the K-means classes as the instance's categories: plans evaluate as the oracle says
    inst, _, _ = synth.workload("paper", n_plans=1)
    cat, used, _ = _gpu(inst.order_skus, inst.n_skus, 16)
    inst2 = dataclasses.replace(inst, sku_category=cat, n_categories=used)
    Z, S = synth.make_plans(inst2, 32, seed=5)
    from paper_2110_13693_amd import wo
    wh = wo.wo_load_warehouse([inst2])
    d, t = gpu_eval(wh, Z, S)
    wh.free()
    d_ref, _ = oracle.eval_plans(inst2, Z, S)
    assert np.array_equal(d, d_ref)

"""The allocation-free K-means entry point (wo_kmeans_categories_noalloc)
against wo_kmeans_categories through the C ABI: identical categories,
categories used and assignment counts on two calls in a row, the second
with a smaller input, so that the static scratch still holds the first
call's contents when the second one starts."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _wo():
    import torch
    from paper_2110_13693_amd import wo
    assert torch.cuda.is_available()
    return wo


def _both(wo, skus, n_skus, k, max_iter):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(skus, dtype=np.int32)).cuda()
    cat_a = torch.full((n_skus,), -7, dtype=torch.int32, device="cuda")
    used_a, iters_a = wo.wo_kmeans_categories(t, n_skus, k, cat_a, max_iter=max_iter)
    cat_b = torch.full((n_skus,), -7, dtype=torch.int32, device="cuda")
    used_b = torch.full((1,), -9, dtype=torch.int32, device="cuda")
    iters_b = torch.full((1,), -9, dtype=torch.int32, device="cuda")
    wo.wo_kmeans_categories_noalloc(t, n_skus, k, cat_b, used_b, iters_b, max_iter=max_iter)
    torch.cuda.synchronize()
    return (cat_a.cpu().numpy(), used_a, iters_a), (cat_b.cpu().numpy(), int(used_b.item()), int(iters_b.item()))


def test_noalloc_matches_allocating_entry_point():
    wo = _wo()
    inst, _, _ = synth.workload("paper", n_plans=1)
    rng = np.random.default_rng(3)
    small = np.minimum(rng.zipf(1.3, size=20000) - 1, 2999)
    cases = [("paper order history, k 16", inst.order_skus, inst.n_skus, 16, 100),
             ("smaller history, k 5", small, 3000, 5, 60)]
    for name, skus, n_skus, k, it in cases:
        print("case", name, flush=True)
        (ca, ua, ia), (cb, ub, ib) = _both(wo, skus, n_skus, k, it)
        assert (ub, ib) == (ua, ia), (name, (ub, ib), (ua, ia))
        assert np.array_equal(cb, ca), name
        assert ca.min() >= 0 and ca.max() < ua


def test_noalloc_flags_out_of_range_sku():
    import torch
    wo = _wo()
    skus = torch.tensor([0, 1, 5, 2], dtype=torch.int32, device="cuda")
    cat = torch.empty(4, dtype=torch.int32, device="cuda")
    used = torch.zeros(1, dtype=torch.int32, device="cuda")
    wo.wo_kmeans_categories_noalloc(skus, 4, 2, cat, used, None, max_iter=10)
    torch.cuda.synchronize()
    assert int(used.item()) == -1

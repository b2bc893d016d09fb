"""Seeded input generators: shapes, value ranges and determinism of the
synthetic workloads that stand in for the paper's proprietary case-study data
(section 1 gives the magnitudes: ~4,000 orders, ~10,000 items, ~200,000
locations per day)."""
import numpy as np

import synth


def test_tiny_workload_shape():
    inst, Z, S = synth.workload("tiny")
    assert inst.n_locations == 600 and inst.n_skus == 600 and inst.n_orders == 200
    assert np.all(inst.category_sizes() == 50)
    lens = np.diff(inst.order_offsets)
    assert lens.min() >= 1 and lens.max() <= 8
    assert Z.shape == (256, 64) and S.shape == (256, 200)
    assert np.all(Z[:, 12:] == 0xFF)
    assert all(sorted(z[:12]) == list(range(12)) for z in Z)
    assert all(sorted(s) == list(range(200)) for s in S[:16])


def test_paper_workload_magnitudes():
    inst, Z, S = synth.workload("paper", n_plans=8)
    sizes = inst.category_sizes()
    assert inst.n_locations == 200_000 and inst.n_skus == 150_000 and sizes.sum() == 150_000
    assert sizes.min() >= 1 and inst.n_categories == 64
    assert 9_500 < inst.n_items < 10_500 and inst.n_orders == 4000
    assert inst.capacity == 30


def test_generators_are_deterministic():
    a = synth.workload("paper", n_plans=4)
    b = synth.workload("paper", n_plans=4)
    assert np.array_equal(a[0].order_skus, b[0].order_skus)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    c = synth.workload("paper", seed=1, n_plans=4)
    assert not np.array_equal(a[0].order_skus, c[0].order_skus)


def test_zipf_popularity_ordering():
    inst, _, _ = synth.workload("paper", n_plans=1)
    counts = np.bincount(inst.order_skus, minlength=inst.n_skus)
    assert counts[:10].sum() > counts[1000:1010].sum()        # rank 0 is the most popular


def test_batched_shapes_log_uniform():
    insts = synth.make_batched_instances(64, seed=0)
    aisles = np.array([i.n_aisles for i in insts])
    orders = np.array([i.n_orders for i in insts])
    assert aisles.min() >= 8 and aisles.max() <= 400 and orders.min() >= 50 and orders.max() <= 4000
    assert np.median(aisles) < 150 and np.median(orders) < 1200          # log-uniform, not uniform
    for i in insts:
        assert i.n_skus == (3 * i.n_locations) // 4 and i.n_categories == 64

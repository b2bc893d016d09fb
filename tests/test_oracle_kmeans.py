"""Pins of the K-means class-based storage oracle.

* scikit-learn's Lloyd K-means from the same starting centroids reaches the
  same partition on data without ties or empty clusters (a library routine
  the 1-D case reduces to);
* the result is a fixed point, checked in exact fractions independently of
  the oracle's cross-multiplied comparisons: every SKU sits in a nearest
  centroid's cluster and every non-empty centroid is its members' mean;
* the within-cluster sum of squares never increases from one assignment to
  the next;
* well-separated groups are recovered, numbered fastest first; one cluster,
  equal frequencies and more clusters than distinct values degenerate as
  they must.
"""
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import kmeans


def _partition(labels):
    groups = {}
    for i, c in enumerate(labels):
        groups.setdefault(int(c), []).append(i)
    return sorted(tuple(g) for g in groups.values())


@pytest.mark.parametrize("seed", range(6))
def test_matches_sklearn_lloyd(seed):
    from sklearn.cluster import KMeans
    rng = np.random.default_rng(seed)
    k = int(rng.integers(2, 7))
    freq = rng.choice(np.arange(0, 5000), size=300, replace=False)   # distinct values: no ties
    _, values, _, _, _, n_iter, _ = kmeans.kmeans_trace(freq, k, max_iter=300)
    D = len(values)
    seeds = np.array([values[(2 * c + 1) * D // (2 * k)] for c in range(k)], dtype=np.float64)
    km = KMeans(n_clusters=k, init=seeds.reshape(-1, 1), n_init=1, algorithm="lloyd", tol=0.0,
                max_iter=300).fit(freq.astype(np.float64).reshape(-1, 1))
    cat, used, _ = kmeans.kmeans_categories(freq, k, max_iter=300)
    assert used == k
    assert _partition(cat) == _partition(km.labels_)


@pytest.mark.parametrize("seed", range(6))
def test_fixed_point_in_fractions(seed):
    rng = np.random.default_rng(100 + seed)
    freq = np.minimum(rng.zipf(1.6, size=4000), 3000)
    k = int(rng.integers(2, 20))
    labels, values, mults, S, N, n_iter, _ = kmeans.kmeans_trace(freq, k, max_iter=500)
    assert n_iter < 500                                     # converged
    cent = [Fraction(s, n) for s, n in zip(S, N)]
    sums, cnts = [0] * k, [0] * k
    for v, m, c in zip(values, mults, labels):
        sums[c] += v * m
        cnts[c] += m
    for c in range(k):
        if cnts[c]:
            assert cent[c] == Fraction(sums[c], cnts[c])
    for v, c in zip(values, labels):
        d = [abs(Fraction(v) - x) for x in cent]
        assert d[c] == min(d) and c == d.index(min(d))      # nearest, lowest index on a tie


@pytest.mark.parametrize("seed", range(4))
def test_inertia_never_increases(seed):
    rng = np.random.default_rng(200 + seed)
    freq = rng.integers(0, 1000, size=2000) ** 2 // 1000
    *_, inertia = kmeans.kmeans_trace(freq, 12, max_iter=200)
    assert all(b <= a for a, b in zip(inertia, inertia[1:]))


def test_separated_groups_fastest_first():
    freq = np.array([9, 10, 11] * 5 + [100, 101] * 7 + [1000, 1002, 998])
    cat, used, _ = kmeans.kmeans_categories(freq, 3)
    assert used == 3
    assert set(cat[freq >= 998]) == {0} and set(cat[(freq >= 100) & (freq <= 101)]) == {1}
    assert set(cat[freq <= 11]) == {2}


def test_degenerate_cases():
    freq = np.array([3, 0, 7, 7, 1, 0])
    cat, used, _ = kmeans.kmeans_categories(freq, 1)
    assert used == 1 and not cat.any()
    cat, used, _ = kmeans.kmeans_categories(np.full(50, 4), 8)
    assert used == 1 and not cat.any()
    # more clusters than distinct values: one class per value, fastest first
    cat, used, _ = kmeans.kmeans_categories(freq, 64)
    assert used == 4
    assert cat.tolist() == [1, 3, 0, 0, 2, 3]
    # one assignment only: the starting centroids decide
    _, _, n_iter = kmeans.kmeans_categories(np.arange(100), 5, max_iter=1)
    assert n_iter == 1


def test_pick_frequency_counts_lines():
    inst, _, _ = synth.workload("tiny", n_plans=1)
    f = kmeans.pick_frequency(inst.n_skus, inst.order_skus)
    assert f.sum() == inst.n_items
    assert f[int(inst.order_skus[0])] == int((inst.order_skus == inst.order_skus[0]).sum())

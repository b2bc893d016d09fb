"""Class-based storage by K-means on pick frequency -- TEST INFRASTRUCTURE ONLY.

Section 5, Subproblem 3: products are placed by how often they are picked,
and an unsupervised classification such as K-means (MacQueen 1967) can decide
the placement.  Reading: the feature of a SKU is its pick frequency, the
number of order lines naming it; the SKUs are clustered into k classes by
Lloyd's iteration of K-means, and the classes become the categories that the
zones hold (class 0 the fastest movers).

Every step is exact:
  * a centroid is the rational S / N (sum and count of its members'
    frequencies); a SKU of frequency f is nearer to centroid j than to k iff
    |f N_j - S_j| N_k < |f N_k - S_k| N_j, in Python integers; a tie goes to
    the lower index;
  * start: with v_0 < v_1 < ... < v_{D-1} the distinct frequencies, centroid
    c is v_i for i = floor((2c + 1) D / (2k)): spread over the distinct
    values rather than over the SKUs, since most SKUs share the few lowest
    frequencies (with D < k some centroids coincide and their clusters stay
    empty);
  * one step assigns every SKU, then moves every non-empty cluster's centroid
    to its members' mean (an empty cluster keeps its centroid); the iteration
    stops at the first assignment equal to the previous one, or after
    max_iter assignments;
  * the non-empty clusters are numbered by descending mean frequency (equal
    means: lower cluster index first).

SKUs of equal frequency always share a cluster, so the iteration runs over
the distinct frequencies with their multiplicities.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np


def pick_frequency(n_skus: int, order_skus) -> np.ndarray:
    """Order lines naming each SKU."""
    return np.bincount(np.asarray(order_skus, dtype=np.int64), minlength=n_skus).astype(np.int64)


def _nearer(f: int, Sj: int, Nj: int, Sk: int, Nk: int) -> bool:
    """Is f strictly nearer to Sj / Nj than to Sk / Nk?"""
    return abs(f * Nj - Sj) * Nk < abs(f * Nk - Sk) * Nj


def _assign(values: List[int], S: List[int], N: List[int]) -> List[int]:
    out = []
    for f in values:
        best = 0
        for c in range(1, len(S)):
            if _nearer(f, S[c], N[c], S[best], N[best]):
                best = c
        out.append(best)
    return out


def kmeans_trace(freq, k: int, max_iter: int = 100):
    """Run the iteration and return (labels per distinct value, values,
    multiplicities, S, N, n_iter, inertia after each assignment)."""
    freq = np.asarray(freq, dtype=np.int64)
    if freq.size < 1 or not (1 <= k <= 64) or max_iter < 1:
        raise ValueError("need SKUs, 1 <= k <= 64 and max_iter >= 1")
    vals, mult = np.unique(freq, return_counts=True)
    values = [int(v) for v in vals]
    mults = [int(m) for m in mult]
    D = len(values)
    S = [values[(2 * c + 1) * D // (2 * k)] for c in range(k)]
    N = [1] * k
    labels = None
    inertia = []
    n_iter = max_iter
    for it in range(1, max_iter + 1):
        new = _assign(values, S, N)
        inertia.append(_inertia(values, mults, new, k))
        if labels is not None and new == labels:
            n_iter = it
            break
        labels = new
        sums, cnts = [0] * k, [0] * k
        for v, m, c in zip(values, mults, labels):
            sums[c] += v * m
            cnts[c] += m
        for c in range(k):
            if cnts[c]:
                S[c], N[c] = sums[c], cnts[c]
    return labels, values, mults, S, N, n_iter, inertia


def _inertia(values, mults, labels, k):
    """Within-cluster sum of squares (exact, as a fraction numerator / denominator pair
    reduced to a float only for reporting)."""
    from fractions import Fraction
    sums, cnts = [0] * k, [0] * k
    for v, m, c in zip(values, mults, labels):
        sums[c] += v * m
        cnts[c] += m
    tot = Fraction(0)
    for v, m, c in zip(values, mults, labels):
        tot += m * (Fraction(v) - Fraction(sums[c], cnts[c])) ** 2
    return tot


def kmeans_categories(freq, k: int, max_iter: int = 100) -> Tuple[np.ndarray, int, int]:
    """(category of every SKU, categories used, assignments performed)."""
    labels, values, mults, S, N, n_iter, _ = kmeans_trace(freq, k, max_iter)
    cnt = [0] * k
    for m, c in zip(mults, labels):
        cnt[c] += m
    used = [c for c in range(k) if cnt[c]]
    # descending mean S/N, then lower index: a before b iff S_a N_b > S_b N_a
    rank = {}
    for c in used:
        rank[c] = sum(1 for d in used if S[d] * N[c] > S[c] * N[d] or (S[d] * N[c] == S[c] * N[d] and d < c))
    by_value = {v: rank[c] for v, c in zip(values, labels)}
    freq = np.asarray(freq, dtype=np.int64)
    cat = np.fromiter((by_value[int(f)] for f in freq), dtype=np.int32, count=freq.size)
    return cat, len(used), n_iter

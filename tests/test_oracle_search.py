"""Pins of the CPU genetic-search reference (oracle/search.py)."""
import numpy as np
import pytest

import synth
from oracle import search as G


def test_splitmix64_published_vectors():
    # SplitMix64 started from state 0 (Steele, Lea & Flood 2014): the first
    # outputs are the generator's published reference values
    assert G.splitmix64(0) == 0xE220A8397B1DCDAF
    assert G.splitmix64(0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4
    assert G.splitmix64((2 * 0x9E3779B97F4A7C15) & G.MASK64) == 0x06C45D188009454F


def test_bernoulli_threshold_and_rate():
    assert G.P_MUT == int(0.02 * 2**32)
    hits = sum(G.draw(1, G.STREAM_INSERT_COIN, 0, c, i) < G.P_MUT for c in range(20) for i in range(1000))
    assert abs(hits / 20000 - 0.02) < 0.004


def test_uniform_multiply_shift_range():
    for m in (1, 2, 7, 63, 4000):
        vals = [G.uniform(G.draw(3, 9, 0, 0, k), m) for k in range(2000)]
        assert min(vals) >= 0 and max(vals) < m
        if m > 1:
            assert len(set(vals)) > min(m, 2000) * 0.5


def test_mutations_keep_permutations():
    rng = np.random.default_rng(0)
    for child in range(30):
        z = np.full(64, 0xFF, np.uint8)
        z[:12] = rng.permutation(12)
        z2 = G.mutate_zones(z, 12, 5, 3, child)
        assert sorted(z2[:12]) == list(range(12)) and np.all(z2[12:] == 0xFF)
        s = rng.permutation(200).astype(np.uint16)
        s2 = G.mutate_sequence(s, 5, 3, child)
        assert sorted(s2) == list(range(200))


def test_insert_move_semantics():
    # with every coin forced to one outcome the move is remove-then-insert
    seq = [10, 11, 12, 13, 14]
    v = seq.pop(1)
    seq.insert(3, v)
    assert seq == [10, 12, 13, 11, 14]


def test_tournament_picks_minimum_of_draws():
    rng = np.random.default_rng(1)
    dist = rng.integers(0, 50, 64)
    for child in range(50):
        idx = [G.uniform(G.draw(9, G.STREAM_TOURNAMENT, 2, child, k), 64) for k in range(4)]
        w = G.tournament(dist, 9, 2, child)
        assert w in idx and all((dist[w], w) <= (dist[i], i) for i in idx)


def test_plain_generation_keeps_best_and_never_worsens():
    inst, Z, S = synth.workload("tiny", n_plans=32)
    import oracle
    D, _ = oracle.eval_plans(inst, Z, S)
    best0 = D.min()
    for g in range(3):
        Z, S, D = G.plain_generation(inst, Z, S, D, seed=11, gen=g)
        assert D[0] <= best0
        best0 = D.min()

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


class ScriptedDraws:
    """Stands in for the counter generator: (stream, child, position) -> r32
    from a table; every other draw is 0xFFFFFFFF (a coin that never fires,
    a uniform integer of m - 1)."""

    def __init__(self, table):
        self.table = dict(table)

    def __call__(self, seed, stream, gen, child, pos):
        return self.table.get((stream, child, pos), 0xFFFFFFFF)


def r32_for(j, m):
    """A 32-bit draw whose multiply-shift uniform integer in [0, m) is j."""
    r = ((j << 32) + m - 1) // m
    assert (r * m) >> 32 == j
    return r


FIRE = 0   # a coin draw below the threshold


def test_zone_swap_partner_skips_its_own_position(monkeypatch):
    # 5 categories, the coin fires at position c = 2 only.  The partner is a
    # uniform draw over the 4 other positions: 0, 1 stand for themselves,
    # 2, 3 for positions 3, 4 (the own position is skipped).
    z0 = np.array([40, 41, 42, 43, 44] + [0xFF] * 59, np.uint8)
    want = {0: [42, 41, 40, 43, 44], 1: [40, 42, 41, 43, 44],
            2: [40, 41, 43, 42, 44], 3: [40, 41, 44, 43, 42]}
    for j, row in want.items():
        monkeypatch.setattr(G, "draw", ScriptedDraws({(G.STREAM_ZONE_COIN, 7, 2): FIRE,
                                                       (G.STREAM_ZONE_PARTNER, 7, 2): r32_for(j, 4)}))
        got = G.mutate_zones(z0, 5, 0, 0, 7)
        assert list(got[:5]) == row, (j, list(got[:5]))
        assert np.all(got[5:] == 0xFF)


def test_zone_swaps_apply_in_position_order(monkeypatch):
    # coins at positions 0 and 3; position 0 swaps with position 3 (draw 2 of
    # 0..3 -> 3), then position 3 -- now holding zone 40 -- swaps with
    # position 1 (draw 1 -> 1)
    z0 = np.array([40, 41, 42, 43, 44] + [0xFF] * 59, np.uint8)
    monkeypatch.setattr(G, "draw", ScriptedDraws({
        (G.STREAM_ZONE_COIN, 1, 0): FIRE, (G.STREAM_ZONE_PARTNER, 1, 0): r32_for(2, 4),
        (G.STREAM_ZONE_COIN, 1, 3): FIRE, (G.STREAM_ZONE_PARTNER, 1, 3): r32_for(1, 4)}))
    got = G.mutate_zones(z0, 5, 0, 0, 1)
    # after the first swap: 43 41 42 40 44; after the second: 43 40 42 41 44
    assert list(got[:5]) == [43, 40, 42, 41, 44]


def test_insert_move_semantics(monkeypatch):
    # one coin at position 1 with target 3: the element at 1 is removed and
    # inserted so that it ends at position 3
    s0 = np.array([10, 11, 12, 13, 14], np.uint16)
    monkeypatch.setattr(G, "draw", ScriptedDraws({(G.STREAM_INSERT_COIN, 4, 1): FIRE,
                                                   (G.STREAM_INSERT_TARGET, 4, 1): r32_for(3, 5)}))
    assert list(G.mutate_sequence(s0, 0, 0, 4)) == [10, 12, 13, 11, 14]
    # a move towards the front: position 3 to position 0
    monkeypatch.setattr(G, "draw", ScriptedDraws({(G.STREAM_INSERT_COIN, 4, 3): FIRE,
                                                   (G.STREAM_INSERT_TARGET, 4, 3): r32_for(0, 5)}))
    assert list(G.mutate_sequence(s0, 0, 0, 4)) == [13, 10, 11, 12, 14]


def test_insert_moves_apply_to_the_current_sequence(monkeypatch):
    # coins at positions 0 (target 2), 2 (target 4) and 4 (target 0), in
    # turn, each moving whatever element sits at that position by then:
    #   start        10 11 12 13 14
    #   i=0 -> 2     11 12 10 13 14   (10 moved)
    #   i=2 -> 4     11 12 13 14 10   (10 again: it sits at position 2 now)
    #   i=4 -> 0     10 11 12 13 14   (and once more)
    s0 = np.array([10, 11, 12, 13, 14], np.uint16)
    T = G.STREAM_INSERT_TARGET
    monkeypatch.setattr(G, "draw", ScriptedDraws({
        (G.STREAM_INSERT_COIN, 2, 0): FIRE, (T, 2, 0): r32_for(2, 5),
        (G.STREAM_INSERT_COIN, 2, 2): FIRE, (T, 2, 2): r32_for(4, 5),
        (G.STREAM_INSERT_COIN, 2, 4): FIRE, (T, 2, 4): r32_for(0, 5)}))
    assert list(G.mutate_sequence(s0, 0, 0, 2)) == [10, 11, 12, 13, 14]
    # the same with the last move absent
    monkeypatch.setattr(G, "draw", ScriptedDraws({
        (G.STREAM_INSERT_COIN, 2, 0): FIRE, (T, 2, 0): r32_for(2, 5),
        (G.STREAM_INSERT_COIN, 2, 2): FIRE, (T, 2, 2): r32_for(4, 5)}))
    assert list(G.mutate_sequence(s0, 0, 0, 2)) == [11, 12, 13, 14, 10]


def test_worst_individuals_order_and_ties():
    dist = [5, 9, 9, 3, 9, 1, 7]
    # largest distance first; equal distances by smaller index
    assert G.worst_individuals(dist, 3) == [1, 2, 4]
    assert G.worst_individuals(dist, 5) == [1, 2, 4, 6, 0]
    assert G.worst_individuals(dist, 7) == [1, 2, 4, 6, 0, 3, 5]


def test_screened_generation_replaces_worst_in_rank_order(monkeypatch):
    # a population of 4 tiny plans; no mutation fires, and the scripted
    # tournaments pick parent 3 for candidate 5 and parent 0 for candidate 2.
    # The kept candidates, in rank order (5, 2), replace the worst and the
    # second worst individual, so individual 1 (worst) becomes a copy of
    # plan 3 and individual 2 (second worst) a copy of plan 0.
    import oracle
    inst, Z, S = synth.workload("tiny", n_plans=4)
    D, _ = oracle.eval_plans(inst, Z, S)
    dist = np.array([D[0], 10 ** 9, 10 ** 8, D[3]], np.int64)
    TS = G.STREAM_TOURNAMENT
    monkeypatch.setattr(G, "draw", ScriptedDraws({
        (TS, 5, 0): r32_for(3, 4), (TS, 5, 1): r32_for(3, 4), (TS, 5, 2): r32_for(3, 4), (TS, 5, 3): r32_for(3, 4),
        (TS, 2, 0): r32_for(0, 4), (TS, 2, 1): r32_for(1, 4), (TS, 2, 2): r32_for(0, 4), (TS, 2, 3): r32_for(2, 4)}))
    Z2, S2, D2 = G.screened_generation(inst, Z, S, dist, seed=0, gen=0, kept_ids=[5, 2])
    assert np.array_equal(Z2[1], Z[3]) and np.array_equal(S2[1], S[3]) and D2[1] == D[3]
    assert np.array_equal(Z2[2], Z[0]) and np.array_equal(S2[2], S[0]) and D2[2] == D[0]
    # the rest of the population is untouched
    for i in (0, 3):
        assert np.array_equal(Z2[i], Z[i]) and np.array_equal(S2[i], S[i]) and D2[i] == dist[i]


def test_plain_generation_children(monkeypatch):
    # child 0 is the best individual unchanged; child b is its tournament
    # winner (scripted: parent 2 for child 1, parent 0 for child 2, parent 1
    # for child 3) with the mutations (none fire here)
    import oracle
    inst, Z, S = synth.workload("tiny", n_plans=4)
    D, _ = oracle.eval_plans(inst, Z, S)
    best = int(np.lexsort((np.arange(4), D))[0])
    TS = G.STREAM_TOURNAMENT
    table = {}
    for child, par in ((1, 2), (2, 0), (3, 1)):
        for k in range(4):
            table[(TS, child, k)] = r32_for(par, 4)
    monkeypatch.setattr(G, "draw", ScriptedDraws(table))
    Z2, S2, D2 = G.plain_generation(inst, Z, S, D, seed=0, gen=0)
    for child, par in ((0, best), (1, 2), (2, 0), (3, 1)):
        assert np.array_equal(Z2[child], Z[par]) and np.array_equal(S2[child], S[par]) and D2[child] == D[par]


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

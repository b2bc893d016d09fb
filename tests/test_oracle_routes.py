"""Pins of the oracle's route distances (S-shape, return, largest gap)
against independent route geometry.

* Dijkstra on the explicit aisle graph (the paper computes distances between
  pick positions with Dijkstra's algorithm, section 5, Subproblem 2) equals
  the single-block point-to-point closed form.
* Brute force over all visiting orders (the paper's "permutations of picking
  sequences", same passage) gives the optimal tour; S-shape is never shorter.
* An explicit waypoint walk of the S-shape route reproduces the oracle's cost
  and passes every pick.
"""
import numpy as np
import pytest

import oracle
from tests.whelpers import (aisle_graph_dijkstra, largest_gap_walk, optimal_tour_length, point,
                            return_walk, sshape_walk, tiny_geometry)


def closed_form_distance(inst, p, q):
    L = inst.slots_per_side * inst.pitch_dm
    (a1, y1), (a2, y2) = p, q
    if a1 == a2:
        return abs(y1 - y2)
    return inst.spacing_dm * abs(a1 - a2) + min(y1 + y2, 2 * L - y1 - y2)


@pytest.mark.parametrize("seed", range(6))
def test_dijkstra_matches_closed_form(seed):
    inst = tiny_geometry([[0]], n_aisles=6)
    rng = np.random.default_rng(seed)
    locs = rng.integers(0, inst.n_locations, size=5)
    pts = [point(inst, int(l)) for l in locs]
    m = aisle_graph_dijkstra(inst, pts)
    allp = [(0, 0)] + pts
    for i in range(len(allp)):
        for j in range(len(allp)):
            assert m[i, j] == closed_form_distance(inst, allp[i], allp[j])


def _random_tour(rng, inst, n):
    return [int(x) for x in rng.integers(0, inst.n_locations, size=n)]


@pytest.mark.parametrize("seed", range(40))
def test_sshape_at_least_optimum(seed):
    inst = tiny_geometry([[0]], n_aisles=10)
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 7))
    locs = _random_tour(rng, inst, n)
    pts = sorted({point(inst, l) for l in locs})
    opt = optimal_tour_length(aisle_graph_dijkstra(inst, pts))
    s = oracle.sshape_cost(inst, locs)
    assert s >= opt


def test_sshape_equals_optimum_cases():
    inst = tiny_geometry([[0]], n_aisles=10)
    # any set of picks in one aisle: S-shape goes in and back out, which is optimal
    for locs in ([0], [59], [194], [180, 200, 238], [540, 599]):
        pts = sorted({point(inst, l) for l in locs})
        assert oracle.sshape_cost(inst, locs) == optimal_tour_length(aisle_graph_dijkstra(inst, pts))
    # two aisles, far pick at the back of the first: 840 = optimum
    pts = [point(inst, 119), point(inst, 240)]
    assert oracle.sshape_cost(inst, [119, 240]) == 840 == optimal_tour_length(aisle_graph_dijkstra(inst, pts))


def test_sshape_strictly_worse_examples():
    inst = tiny_geometry([[0]], n_aisles=10)
    # {(1,5),(2,5)}: S-shape 720, optimum 140
    locs = [60, 120]
    pts = [point(inst, l) for l in locs]
    assert oracle.sshape_cost(inst, locs) == 720
    assert optimal_tour_length(aisle_graph_dijkstra(inst, pts)) == 140
    # {(0,5),(2,55),(9,295)}: S-shape 1730, optimum 1150
    locs = [0, 130, 599]
    pts = [point(inst, l) for l in locs]
    assert oracle.sshape_cost(inst, locs) == 1730
    assert optimal_tour_length(aisle_graph_dijkstra(inst, pts)) == 1150


@pytest.mark.parametrize("seed", range(200))
def test_route_walk_matches(seed):
    rng = np.random.default_rng(seed)
    n_aisles = int(rng.integers(1, 25))
    slots = int(rng.integers(1, 40))
    pitch = 2 * int(rng.integers(1, 8))
    spacing = int(rng.integers(0, 60))
    inst = tiny_geometry([[0]], n_aisles=n_aisles, slots=slots, pitch=pitch, spacing=spacing)
    n = int(rng.integers(1, 40))
    locs = _random_tour(rng, inst, n)
    pts = [point(inst, l) for l in locs]
    length, covered = sshape_walk(inst, pts)
    assert all(covered)
    assert oracle.sshape_cost(inst, locs) == length


@pytest.mark.parametrize("seed", range(50))
def test_adding_a_pick_never_decreases(seed):
    rng = np.random.default_rng(5000 + seed)
    inst = tiny_geometry([[0]], n_aisles=int(rng.integers(1, 15)))
    locs = _random_tour(rng, inst, int(rng.integers(1, 20)))
    base = oracle.sshape_cost(inst, locs)
    extra = _random_tour(rng, inst, 1)
    assert oracle.sshape_cost(inst, locs + extra) >= base
    # lower bound: reach the farthest aisle and back, plus the far depth there
    a = [point(inst, l) for l in locs]
    a_max = max(x for x, _ in a)
    y_far = max(y for x, y in a if x == a_max)
    assert base >= 2 * inst.spacing_dm * a_max + 2 * y_far


# ------------------------------------------------ return and largest gap
def test_return_and_largest_gap_hand_examples():
    inst = tiny_geometry([[0]], n_aisles=10)       # L = 300 dm, aisles 30 dm apart
    # (1,5),(2,5): return goes up 5 dm in each aisle: 2*30*2 + 2*5 + 2*5 = 140 (the
    # optimum); largest gap crosses both aisles: 2*30*2 + 2*300 = 720
    assert oracle.return_cost(inst, [60, 120]) == 140
    assert oracle.largest_gap_cost(inst, [60, 120]) == 720
    # (0,5),(2,55),(9,295): return 2*30*9 + 2*(5 + 55 + 295) = 1250; largest gap
    # crosses aisles 0 and 9 (2*30*9 + 2*300) and dips 55 dm into aisle 2 from
    # the front (its largest gap is the 245 dm behind the pick): 1250
    assert oracle.return_cost(inst, [0, 130, 599]) == 1250
    assert oracle.largest_gap_cost(inst, [0, 130, 599]) == 1250
    # three picks in the inner aisle 3 at y = 15, 155, 285: gaps 15, 140, 130, 15;
    # the 140 dm gap is skipped: 2*30*5 + 2*300 + 2*(300 - 140) = 1220
    locs = [0, 3 * 60 + 2, 3 * 60 + 30, 3 * 60 + 56, 5 * 60]
    assert oracle.largest_gap_cost(inst, locs) == 1220


@pytest.mark.parametrize("seed", range(40))
def test_return_and_largest_gap_walks(seed):
    # the closed forms equal an explicit walk of each route, which passes every pick
    inst = tiny_geometry([[0]], n_aisles=12)
    rng = np.random.default_rng(3000 + seed)
    locs = _random_tour(rng, inst, int(rng.integers(1, 12)))
    pts = [point(inst, l) for l in locs]
    for cost, walk in ((oracle.return_cost, return_walk), (oracle.largest_gap_cost, largest_gap_walk)):
        length, covered = walk(inst, pts)
        assert all(covered)
        assert cost(inst, locs) == length


@pytest.mark.parametrize("seed", range(40))
def test_return_and_largest_gap_at_least_optimum(seed):
    inst = tiny_geometry([[0]], n_aisles=10)
    rng = np.random.default_rng(2000 + seed)
    locs = _random_tour(rng, inst, int(rng.integers(1, 7)))
    pts = sorted({point(inst, l) for l in locs})
    opt = optimal_tour_length(aisle_graph_dijkstra(inst, pts))
    assert oracle.return_cost(inst, locs) >= opt
    assert oracle.largest_gap_cost(inst, locs) >= opt


def test_single_aisle_routes_agree_and_are_optimal():
    # with one aisle holding picks every policy goes in to the farthest pick and back
    inst = tiny_geometry([[0]], n_aisles=10)
    for locs in ([0], [59], [194], [180, 200, 238], [540, 599]):
        pts = sorted({point(inst, l) for l in locs})
        opt = optimal_tour_length(aisle_graph_dijkstra(inst, pts))
        assert oracle.sshape_cost(inst, locs) == oracle.return_cost(inst, locs) == \
            oracle.largest_gap_cost(inst, locs) == opt


def test_routing_field_selects_the_tour_cost():
    import dataclasses
    base = tiny_geometry([[0]], n_aisles=10)
    locs = [0, 130, 599]
    for routing, f in ((0, oracle.sshape_cost), (1, oracle.return_cost), (2, oracle.largest_gap_cost)):
        inst = dataclasses.replace(base, routing=routing)
        assert oracle.tour_cost(inst, locs) == f(base, locs)

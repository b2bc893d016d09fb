"""Pins of the oracle's route distances (S-shape, return, largest gap,
optimal) against independent route geometry.

* Dijkstra on the explicit aisle graph (the paper computes distances between
  pick positions with Dijkstra's algorithm, section 5, Subproblem 2) equals
  the single-block point-to-point closed form.
* Brute force over all visiting orders (the paper's "permutations of picking
  sequences", same passage) gives the optimal tour; S-shape is never shorter.
* An explicit waypoint walk of the S-shape route reproduces the oracle's cost
  and passes every pick.
* The optimal route's dynamic programme equals that brute-force optimum
  exactly, and is never longer than any of the heuristic routes.
"""
import numpy as np
import pytest

import oracle
from tests.whelpers import (aisle_graph_dijkstra, combined_walks, largest_gap_walk, optimal_tour_length,
                            point, return_walk, sshape_walk, tiny_geometry)


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
    for routing, f in ((0, oracle.sshape_cost), (1, oracle.return_cost), (2, oracle.largest_gap_cost),
                       (3, oracle.optimal_cost), (4, oracle.combined_cost)):
        inst = dataclasses.replace(base, routing=routing)
        assert oracle.tour_cost(inst, locs) == f(base, locs)


# ------------------------------------------------------------ optimal route
OPT_GEOMETRIES = [
    dict(n_aisles=10),                         # L = 300 dm, aisles 30 dm apart
    dict(n_aisles=7, slots=3, spacing=30),     # short aisles: L = 30 dm, as long as a step across
    dict(n_aisles=8, slots=2, spacing=50),     # aisles shorter than a step across
    dict(n_aisles=5, slots=30, spacing=4),     # long aisles close together
    dict(n_aisles=12, slots=5, pitch=4, spacing=9),
]


@pytest.mark.parametrize("geom", range(len(OPT_GEOMETRIES)))
@pytest.mark.parametrize("seed", range(12))
def test_optimal_equals_brute_force(geom, seed):
    # the dynamic programme against Dijkstra distances and every visiting order
    inst = tiny_geometry([[0]], **OPT_GEOMETRIES[geom])
    rng = np.random.default_rng(7000 + 100 * geom + seed)
    for _ in range(6):
        locs = _random_tour(rng, inst, int(rng.integers(1, 8)))
        pts = sorted({point(inst, l) for l in locs})
        assert oracle.optimal_cost(inst, locs) == optimal_tour_length(aisle_graph_dijkstra(inst, pts)), locs


def test_optimal_hand_examples():
    inst = tiny_geometry([[0]], n_aisles=10)
    assert oracle.optimal_cost(inst, [60, 120]) == 140       # the return route
    assert oracle.optimal_cost(inst, [0, 130, 599]) == 1150
    # picks at y = 5 and y = 295 in aisle 5 only: in from the front to the deep
    # pick and back (2*5*30 + 2*295 = 890) beats the loop up the empty aisle 0,
    # along the back and down aisle 5 (2*300 + 2*5*30 = 900)
    assert oracle.optimal_cost(inst, [5 * 60, 5 * 60 + 59]) == 890
    # aisles 30 dm long and 50 dm apart, picks at y = 25 in aisles 2 and 5:
    # front to aisle 2, across it, along the back to aisle 5, down it and back
    # along the front: 2*50 + 30 + 3*50 + 30 + 5*50 = 560, against 600 for
    # going in from the front twice
    short = tiny_geometry([[0]], n_aisles=8, slots=3, spacing=50)
    locs = [2 * 6 + 4, 5 * 6 + 4]
    pts = sorted({point(short, l) for l in locs})
    assert oracle.optimal_cost(short, locs) == optimal_tour_length(aisle_graph_dijkstra(short, pts)) == 560


@pytest.mark.parametrize("seed", range(30))
def test_optimal_not_above_heuristics(seed):
    # paper-like aisles (250 slots, 400 aisles) and tours of up to 30 picks
    rng = np.random.default_rng(8000 + seed)
    inst = tiny_geometry([[0]], n_aisles=400, slots=250, n_cat=1, cat_size=1)
    locs = _random_tour(rng, inst, int(rng.integers(1, 31)))
    opt = oracle.optimal_cost(inst, locs)
    assert opt <= min(oracle.sshape_cost(inst, locs), oracle.return_cost(inst, locs),
                      oracle.largest_gap_cost(inst, locs))
    pts = [point(inst, l) for l in locs]
    a_max = max(a for a, _ in pts)
    # at least the walk to the farthest aisle and back, and twice the
    # depot distance of any pick
    L = inst.slots_per_side * inst.pitch_dm
    assert opt >= 2 * inst.spacing_dm * a_max
    assert opt >= max(2 * (inst.spacing_dm * a + min(y, 2 * L - y)) for a, y in pts)


@pytest.mark.parametrize("seed", range(10))
def test_optimal_invariant_under_pick_order_and_duplicates(seed):
    rng = np.random.default_rng(9000 + seed)
    inst = tiny_geometry([[0]], n_aisles=40, slots=50)
    locs = _random_tour(rng, inst, 20)
    base = oracle.optimal_cost(inst, locs)
    assert oracle.optimal_cost(inst, list(rng.permutation(locs))) == base
    assert oracle.optimal_cost(inst, locs + locs[:5]) == base
    # a pick on the other side of the same aisle position is the same point
    twin = [l ^ 1 for l in locs]
    assert oracle.optimal_cost(inst, twin) == base


# ----------------------------------------------------------- combined route
@pytest.mark.parametrize("geom", range(len(OPT_GEOMETRIES)))
@pytest.mark.parametrize("seed", range(10))
def test_combined_equals_best_enumerated_walk(geom, seed):
    # the two-state programme against every crossing choice walked out
    inst = tiny_geometry([[0]], **OPT_GEOMETRIES[geom])
    rng = np.random.default_rng(11000 + 100 * geom + seed)
    for _ in range(5):
        locs = _random_tour(rng, inst, int(rng.integers(1, 12)))
        pts = [point(inst, l) for l in locs]
        walks = combined_walks(inst, pts)
        assert all(ok for _, ok in walks)
        assert oracle.combined_cost(inst, locs) == min(length for length, _ in walks), locs


@pytest.mark.parametrize("seed", range(30))
def test_combined_between_optimum_and_sshape_return(seed):
    rng = np.random.default_rng(12000 + seed)
    inst = tiny_geometry([[0]], n_aisles=400, slots=250, n_cat=1, cat_size=1)
    locs = _random_tour(rng, inst, int(rng.integers(1, 31)))
    c = oracle.combined_cost(inst, locs)
    assert c <= min(oracle.sshape_cost(inst, locs), oracle.return_cost(inst, locs))
    assert c >= oracle.optimal_cost(inst, locs)


def test_combined_hand_example():
    inst = tiny_geometry([[0]], n_aisles=10)       # L = 300 dm, aisles 30 dm apart
    # (0,5),(2,55),(9,295): return everywhere is 2*30*9 + 2*(5 + 55 + 295) = 1250; crossing
    # aisles 0 and 9 and returning in aisle 2 from the back costs 2*30*9 + 2*300 + 2*(300 - 55)
    # = 1630; crossing 2 and 9 and returning in 0: 540 + 10 + 600 = 1150 -- the best
    assert oracle.combined_cost(inst, [0, 130, 599]) == 1150

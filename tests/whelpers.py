"""Small helpers shared by the tests: hand-made instances and route geometry.

Nothing here computes a plan cost; the route-geometry helpers below are an
independent restatement used to pin the oracle (point-to-point distances on
the aisle graph, and an explicit walk of the S-shape route).
"""
import heapq
import itertools

import numpy as np

from synth import Instance


def tiny_geometry(orders, capacity=20, n_aisles=10, slots=30, pitch=10, spacing=30,
                  n_cat=12, cat_size=50):
    """Instance with unshuffled categories (category c = SKUs c*size..), given orders."""
    n_sku = n_cat * cat_size
    cat = (np.arange(n_sku) // cat_size).astype(np.int32)
    off = np.zeros(len(orders) + 1, dtype=np.int32)
    off[1:] = np.cumsum([len(o) for o in orders])
    skus = np.asarray([s for o in orders for s in o], dtype=np.int32)
    return Instance(n_aisles=n_aisles, slots_per_side=slots, pitch_dm=pitch,
                    spacing_dm=spacing, capacity=capacity, n_categories=n_cat,
                    sku_category=cat, order_offsets=off, order_skus=skus)


def identity_zones(n_cat):
    z = np.full(64, 0xFF, dtype=np.uint8)
    z[:n_cat] = np.arange(n_cat)
    return z


def loc_of(aisle, j, side, slots):
    return aisle * 2 * slots + 2 * j + side


def point(inst, loc):
    """(aisle, y) of a location, restated from the geometry."""
    per = 2 * inst.slots_per_side
    a = loc // per
    j = (loc % per) // 2
    return a, j * inst.pitch_dm + inst.pitch_dm // 2


# ---------------------------------------------------------------- Dijkstra
def aisle_graph_dijkstra(inst, points):
    """All-pairs shortest paths between ``points`` (list of (aisle, y)) and the
    depot (index 0 of the result) on the explicit single-block aisle graph:
    vertical edges along each aisle, horizontal edges along the front (y=0)
    and back (y=L) cross aisles.  Plain Dijkstra with a binary heap."""
    L = inst.slots_per_side * inst.pitch_dm
    w = inst.spacing_dm
    pts = [(0, 0)] + list(points)
    nodes = set()
    for a in range(inst.n_aisles):
        nodes.add((a, 0))
        nodes.add((a, L))
    for p in pts:
        nodes.add(p)
    adj = {n: [] for n in nodes}
    for a in range(inst.n_aisles):
        ys = sorted(y for (aa, y) in nodes if aa == a)
        for y0, y1 in zip(ys, ys[1:]):
            adj[(a, y0)].append(((a, y1), y1 - y0))
            adj[(a, y1)].append(((a, y0), y1 - y0))
        if a + 1 < inst.n_aisles:
            for y in (0, L):
                adj[(a, y)].append(((a + 1, y), w))
                adj[(a + 1, y)].append(((a, y), w))

    def sssp(src):
        dist = {src: 0}
        pq = [(0, src)]
        while pq:
            d, u = heapq.heappop(pq)
            if d > dist[u]:
                continue
            for v, c in adj[u]:
                nd = d + c
                if nd < dist.get(v, 1 << 60):
                    dist[v] = nd
                    heapq.heappush(pq, (nd, v))
        return dist

    n = len(pts)
    m = np.zeros((n, n), dtype=np.int64)
    for i in range(n):
        di = sssp(pts[i])
        for j in range(n):
            m[i, j] = di[pts[j]]
    return m


def optimal_tour_length(dmat):
    """Brute force: shortest closed walk depot -> all points -> depot."""
    n = dmat.shape[0] - 1
    best = None
    for perm in itertools.permutations(range(1, n + 1)):
        d = dmat[0, perm[0]] + dmat[perm[-1], 0]
        for a, b in zip(perm, perm[1:]):
            d += dmat[a, b]
        best = d if best is None else min(best, d)
    return 0 if best is None else int(best)


# ------------------------------------------------------- S-shape route walk
def sshape_walk(inst, points):
    """Walk the S-shape route waypoint by waypoint and return (length, visited).

    The picker starts at the depot (front of aisle 0), goes along the current
    cross aisle to each aisle holding a pick (ascending), crosses it entirely
    -- except, when the number of such aisles is odd, the last one, which is
    entered from the front up to its farthest pick and left the same way --
    and finally returns to the depot along the cross aisle it is on.  Returns
    the length and, for every point, whether the route passed it."""
    L = inst.slots_per_side * inst.pitch_dm
    w = inst.spacing_dm
    aisles = sorted({a for a, _ in points})
    k = len(aisles)
    x, y, length = 0, 0, 0
    covered = [False] * len(points)
    for idx, a in enumerate(aisles):
        length += abs(a * w - x)
        x = a * w
        last = idx == k - 1
        if last and k % 2 == 1:
            assert y == 0, "odd S-shape must enter its last aisle from the front"
            far = max(py for pa, py in points if pa == a)
            length += 2 * far
            for i, (pa, py) in enumerate(points):
                if pa == a and py <= far:
                    covered[i] = True
        else:
            length += L
            y = L - y
            for i, (pa, _) in enumerate(points):
                if pa == a:
                    covered[i] = True
    length += x  # back to the depot along the cross aisle
    if k:
        assert y == 0, "route must end on the front cross aisle"
    return length, covered


# ------------------------------------------- return and largest-gap walks
def return_walk(inst, points):
    """Walk the return route and return (length, visited): along the front
    cross aisle to each aisle holding a pick (ascending), up that aisle to its
    farthest pick and back down, and finally back to the depot."""
    w = inst.spacing_dm
    x, length = 0, 0
    covered = [False] * len(points)
    for a in sorted({a for a, _ in points}):
        length += abs(a * w - x)
        x = a * w
        far = max(py for pa, py in points if pa == a)
        length += 2 * far
        for i, (pa, py) in enumerate(points):
            if pa == a and py <= far:
                covered[i] = True
    return length + x, covered


def largest_gap_walk(inst, points):
    """Walk the largest-gap route and return (length, visited).

    One aisle with picks: the return route.  Otherwise the picker goes along
    the front to the first such aisle, crosses it to the back, goes along the
    back to the last one (dipping into every aisle in between from the back
    down to the upper end of its largest gap and back up), crosses the last
    aisle to the front and returns along the front (dipping into every aisle
    in between from the front up to the lower end of its largest gap)."""
    L = inst.slots_per_side * inst.pitch_dm
    w = inst.spacing_dm
    aisles = sorted({a for a, _ in points})
    if len(aisles) <= 1:
        return return_walk(inst, points)
    covered = [False] * len(points)

    def gap(a):
        ys = [0] + sorted(py for pa, py in points if pa == a) + [L]
        best = max(range(len(ys) - 1), key=lambda i: ys[i + 1] - ys[i])
        return ys[best], ys[best + 1]          # lower and upper end

    def cover(a, lo, hi):
        for i, (pa, py) in enumerate(points):
            if pa == a and lo <= py <= hi:
                covered[i] = True

    a_lo, a_hi = aisles[0], aisles[-1]
    length = a_lo * w + L                      # depot -> first aisle, across it
    cover(a_lo, 0, L)
    x = a_lo
    for a in aisles[1:-1]:                     # along the back
        length += (a - x) * w
        x = a
        _, up = gap(a)
        length += 2 * (L - up)
        cover(a, up, L)
    length += (a_hi - x) * w + L               # to the last aisle, across it
    cover(a_hi, 0, L)
    x = a_hi
    for a in reversed(aisles[1:-1]):           # along the front, back to the depot
        length += (x - a) * w
        x = a
        lo, _ = gap(a)
        length += 2 * lo
        cover(a, 0, lo)
    return length + x * w, covered


def combined_walks(inst, points):
    """Every walk of the combined policy, by brute force over the crossing
    choices: aisles holding picks are visited in ascending order along the
    cross aisle the picker is on; each is crossed, or entered from that cross
    aisle to its farthest pick (from the front: the deepest; from the back:
    the shallowest) and left the same way; from the back the picker ends by
    crossing the last aisle, then walks home along the front.  Returns the
    list of (length, every pick passed) over all 2^k choices."""
    import itertools as it
    L = inst.slots_per_side * inst.pitch_dm
    w = inst.spacing_dm
    aisles = sorted({a for a, _ in points})
    out = []
    for choice in it.product((0, 1), repeat=len(aisles)):   # 1: cross
        x, back, length = 0, False, 0
        covered = [False] * len(points)
        for a, cross in zip(aisles, choice):
            length += abs(a * w - x)
            x = a * w
            ys = [py for pa, py in points if pa == a]
            if cross:
                length += L
                back = not back
                lo, hi = 0, L
            elif not back:
                length += 2 * max(ys)
                lo, hi = 0, max(ys)
            else:
                length += 2 * (L - min(ys))
                lo, hi = min(ys), L
            for i, (pa, py) in enumerate(points):
                if pa == a and lo <= py <= hi:
                    covered[i] = True
        if back:
            length += L
        out.append((length + x, all(covered)))
    return out

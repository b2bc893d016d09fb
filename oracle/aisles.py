"""Aisle-width design by a plain sweep -- TEST INFRASTRUCTURE ONLY.

Section 5, Subproblem 1, Eq. (1): maximise A_ind / A_max, the share of the
warehouse floor the racks take, with the width a between racks as the design
variable, subject to k * delta - a <= 0, where delta is the picking
frequency Subproblem 2 returns (Eq. (2): delta = f(d)).

Reading (the paper gives no geometry for Eq. (1)):
  * each aisle of the single block is a corridor of width a between two rack
    faces of depth r (racks of neighbouring aisles stand back to back), so the
    aisles are a + 2 r apart centre to centre; racks are L = S * pitch long;
    a cross aisle of width c runs along the front and along the back;
  * A_ind = N * 2 r L (the racks), A_max = N (a + 2 r) (L + 2 c) (the floor):
    A_ind / A_max = 2 r L / ((a + 2 r) (L + 2 c));
  * delta is the evaluator's rate for the plan, n_orders * window /
    (D / walk + t_item * items), computed in IEEE double from the integer
    total distance D at spacing a + 2 r;
  * widths are whole decimetres in [a_min, a_max]; the design is the
    narrowest width that meets k * delta(a) <= a (none: a_max, infeasible).

The sweep evaluates the plan at every width with the C oracle and takes the
first feasible one: no search, no shortcut.
"""
from __future__ import annotations

import dataclasses

import oracle


def utilization(a: float, r: float, L: float, c: float) -> float:
    """A_ind / A_max of the single block at aisle width a."""
    return (2.0 * r * L) / ((a + 2.0 * r) * (L + 2.0 * c))


def orders_per_window(inst, D: int) -> float:
    """delta = n_orders * window / (D / walk + t_item * items), IEEE double,
    one operation at a time."""
    q = float(D) / float(inst.walk_dm_per_s)
    u = float(inst.seconds_per_item) * float(inst.n_items)
    T = q + u
    num = float(inst.n_orders) * float(inst.window_s)
    return num / T


def distance_at(inst, zone_of, seq, spacing_dm: int) -> int:
    """The plan's int32 total distance with aisles spacing_dm apart."""
    w = dataclasses.replace(inst, spacing_dm=int(spacing_dm))
    _, d32, _ = oracle.eval_plan(w, zone_of, seq)
    return d32


def design_width(inst, zone_of, seq, rack_depth: int, cross_aisle: int, k: float, a_min: int, a_max: int):
    """The narrowest width in [a_min, a_max] with k * delta(a) <= a, and the
    distance at every width of the range."""
    dist = []
    pick = None
    for a in range(a_min, a_max + 1):
        D = distance_at(inst, zone_of, seq, a + 2 * rack_depth)
        dist.append(D)
        if pick is None and k * orders_per_window(inst, D) <= float(a):
            pick = a
    feasible = pick is not None
    a = pick if feasible else a_max
    D = dist[a - a_min]
    L = inst.slots_per_side * inst.pitch_dm
    return {"width_dm": a, "spacing_dm": a + 2 * rack_depth, "feasible": feasible, "distance": D,
            "orders_per_window": orders_per_window(inst, D),
            "utilization": utilization(a, rack_depth, L, cross_aisle), "dist": dist}

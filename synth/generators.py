"""Seeded generators for warehouse instances and candidate picking plans.

The paper's case-study data (company A, section 6) is proprietary, so these
generators stand in for it with the workload magnitudes the paper quotes in
section 1: about 4,000 orders, about 10,000 items and about 200,000 locations
per day.  Everything is drawn from numpy's PCG64 with ``default_rng([seed,
stream])`` so each kind of draw has its own stream:

    0  SKU -> category assignment        3  batched instance shapes
    1  order history                      4  surrogate training plans
    2  candidate plans                    5  surrogate held-out plans
                                          6  search initial population

Recipe:

* Category sizes are equal (``n_skus / C`` each) or Dirichlet(alpha) scaled to
  ``n_skus`` by largest remainder with every size >= 1.
* SKU ids are popularity ranks (0 = most popular).  A seeded permutation of
  the SKU ids is split contiguously by the category sizes.
* Lines per order are ``1 + Poisson(lam)``, optionally capped; every line is
  one item, and a SKU is drawn per line from a finite Zipf(s) law over ranks
  by inverse CDF (``searchsorted(cdf, u, 'right')``).
* A plan is a category->zone permutation (``uint8[64]``, 0xFF padding) and an
  order permutation (``uint16[n_orders]``).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

MAX_CATEGORIES = 64
ZONE_PAD = 0xFF

STREAM_SKU_CATEGORY = 0
STREAM_ORDERS = 1
STREAM_PLANS = 2
STREAM_BATCH_SHAPES = 3
STREAM_SURROGATE_TRAIN = 4
STREAM_SURROGATE_HELDOUT = 5
STREAM_SEARCH_INIT = 6
STREAM_ORDER_TYPES = 7


@dataclasses.dataclass
class Instance:
    """One single-block parallel-aisle warehouse with its order history.

    Geometry is in integer decimetres: ``n_aisles`` aisles, two sides of
    ``slots_per_side`` slots each, slot pitch ``pitch_dm`` (even) and aisle
    centre spacing ``spacing_dm``.  Orders are a CSR list of SKU ids.
    """

    n_aisles: int
    slots_per_side: int
    pitch_dm: int
    spacing_dm: int
    capacity: int
    n_categories: int
    sku_category: np.ndarray  # int32 [n_skus]
    order_offsets: np.ndarray  # int32 [n_orders + 1]
    order_skus: np.ndarray  # int32 [order_offsets[-1]]
    walk_dm_per_s: float = 12.0
    seconds_per_item: float = 10.0
    window_s: float = 28800.0
    routing: int = 0          # 0 S-shape, 1 return, 2 largest gap, 3 optimal, 4 combined
    batching: int = 0         # 0 next fit, 1 first fit, 2 seed

    @property
    def n_skus(self) -> int:
        return int(self.sku_category.shape[0])

    @property
    def n_orders(self) -> int:
        return int(self.order_offsets.shape[0] - 1)

    @property
    def n_items(self) -> int:
        return int(self.order_offsets[-1])

    @property
    def n_locations(self) -> int:
        return 2 * self.n_aisles * self.slots_per_side

    def category_sizes(self) -> np.ndarray:
        return np.bincount(self.sku_category, minlength=self.n_categories).astype(np.int64)


# --------------------------------------------------------------------------
# primitive draws
# --------------------------------------------------------------------------

def _category_sizes(rng: np.random.Generator, n_skus: int, n_cat: int,
                    mode: str, alpha: float) -> np.ndarray:
    if mode == "equal":
        if n_skus % n_cat:
            raise ValueError("equal categories need n_skus divisible by n_categories")
        return np.full(n_cat, n_skus // n_cat, dtype=np.int64)
    if mode != "dirichlet":
        raise ValueError(mode)
    if n_skus < n_cat:
        raise ValueError("need at least one SKU per category")
    p = rng.dirichlet(np.full(n_cat, alpha))
    raw = p * n_skus
    sizes = np.floor(raw).astype(np.int64)
    rem = n_skus - int(sizes.sum())
    order = np.argsort(-(raw - sizes), kind="stable")
    sizes[order[:rem]] += 1
    # every category holds at least one SKU: take from the largest ones
    while (sizes < 1).any():
        i = int(np.argmin(sizes))
        j = int(np.argmax(sizes))
        sizes[i] += 1
        sizes[j] -= 1
    assert int(sizes.sum()) == n_skus
    return sizes


def _zipf_cdf(n: int, s: float) -> np.ndarray:
    w = np.arange(1, n + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    return cdf / cdf[-1]


def make_instance(*, n_aisles: int, slots_per_side: int, pitch_dm: int,
                  spacing_dm: int, capacity: int, n_categories: int,
                  n_skus: int, category_mode: str, dirichlet_alpha: float = 2.0,
                  n_orders: int, lines_lambda: float = 1.5,
                  line_cap: Optional[int] = None, zipf_s: float = 1.0,
                  seed: int = 0, sub_stream: Optional[int] = None,
                  walk_dm_per_s: float = 12.0, seconds_per_item: float = 10.0,
                  window_s: float = 28800.0) -> Instance:
    """Draw one warehouse instance (categories, SKU assignment, orders)."""

    def rng(stream: int) -> np.random.Generator:
        key = [seed, stream] if sub_stream is None else [seed, stream, sub_stream]
        return np.random.default_rng(key)

    r_cat = rng(STREAM_SKU_CATEGORY)
    sizes = _category_sizes(r_cat, n_skus, n_categories, category_mode, dirichlet_alpha)
    perm = r_cat.permutation(n_skus)
    sku_category = np.empty(n_skus, dtype=np.int32)
    start = 0
    for c, sz in enumerate(sizes):
        sku_category[perm[start:start + sz]] = c
        start += int(sz)

    r_ord = rng(STREAM_ORDERS)
    lines = 1 + r_ord.poisson(lines_lambda, size=n_orders)
    if line_cap is not None:
        lines = np.minimum(lines, line_cap)
    offsets = np.zeros(n_orders + 1, dtype=np.int64)
    np.cumsum(lines, out=offsets[1:])
    total = int(offsets[-1])
    cdf = _zipf_cdf(n_skus, zipf_s)
    u = r_ord.random(total)
    skus = np.searchsorted(cdf, u, side="right")
    skus = np.minimum(skus, n_skus - 1).astype(np.int32)

    return Instance(n_aisles=n_aisles, slots_per_side=slots_per_side,
                    pitch_dm=pitch_dm, spacing_dm=spacing_dm, capacity=capacity,
                    n_categories=n_categories, sku_category=sku_category,
                    order_offsets=offsets.astype(np.int32), order_skus=skus,
                    walk_dm_per_s=walk_dm_per_s,
                    seconds_per_item=seconds_per_item, window_s=window_s)


def random_zone_perms(rng: np.random.Generator, n_plans: int, n_cat: int) -> np.ndarray:
    """``uint8[n_plans, 64]``: row p maps category c -> zone, 0xFF padded."""
    z = np.full((n_plans, MAX_CATEGORIES), ZONE_PAD, dtype=np.uint8)
    base = np.tile(np.arange(n_cat, dtype=np.uint8), (n_plans, 1))
    z[:, :n_cat] = rng.permuted(base, axis=1)
    return z


def random_order_perms(rng: np.random.Generator, n_plans: int, n_orders: int) -> np.ndarray:
    """``uint16[n_plans, n_orders]``: each row a permutation of order ids."""
    if n_orders > 65535:
        raise ValueError("order ids are 16-bit")
    base = np.tile(np.arange(n_orders, dtype=np.uint16), (n_plans, 1))
    return rng.permuted(base, axis=1)


def make_plans(inst: Instance, n_plans: int, seed: int = 0,
               stream: int = STREAM_PLANS, fixed_sequence: bool = False):
    """Draw ``n_plans`` candidate plans for ``inst``.

    Returns ``(zone_of uint8[n_plans, 64], order_seq uint16[n_plans, n_orders])``.
    With ``fixed_sequence`` every plan uses the identity order sequence (the
    orders are i.i.d., so the identity is itself a random sequence).
    """
    rng = np.random.default_rng([seed, stream])
    zone_of = random_zone_perms(rng, n_plans, inst.n_categories)
    if fixed_sequence:
        seq = np.tile(np.arange(inst.n_orders, dtype=np.uint16), (n_plans, 1))
    else:
        seq = random_order_perms(rng, n_plans, inst.n_orders)
    return zone_of, seq


def _log_uniform_ints(rng: np.random.Generator, lo: int, hi: int, n: int) -> np.ndarray:
    x = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n))
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


def make_batched_instances(n_instances: int = 512, seed: int = 0,
                           aisles=(8, 400), orders=(50, 4000),
                           slots_per_side: int = 250) -> List[Instance]:
    """Uneven instances for one batched launch (aisles and orders log-uniform).

    Per instance: 64 Dirichlet(2) categories over 75% of its locations, Zipf
    1.1, capacity 30, lines 1 + Poisson(1.5) uncapped, the paper-scale
    geometry otherwise.
    """
    r = np.random.default_rng([seed, STREAM_BATCH_SHAPES])
    na = _log_uniform_ints(r, aisles[0], aisles[1], n_instances)
    no = _log_uniform_ints(r, orders[0], orders[1], n_instances)
    out = []
    for i in range(n_instances):
        n_loc = 2 * int(na[i]) * slots_per_side
        out.append(make_instance(
            n_aisles=int(na[i]), slots_per_side=slots_per_side, pitch_dm=10,
            spacing_dm=30, capacity=30, n_categories=64,
            n_skus=(3 * n_loc) // 4, category_mode="dirichlet",
            dirichlet_alpha=2.0, n_orders=int(no[i]), lines_lambda=1.5,
            line_cap=None, zipf_s=1.1, seed=seed, sub_stream=i))
    return out


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def _tiny(seed: int = 0) -> Instance:
    return make_instance(n_aisles=10, slots_per_side=30, pitch_dm=10, spacing_dm=30,
                         capacity=20, n_categories=12, n_skus=600,
                         category_mode="equal", n_orders=200, lines_lambda=1.5,
                         line_cap=8, zipf_s=1.0, seed=seed)


def _paper(seed: int = 0) -> Instance:
    return make_instance(n_aisles=400, slots_per_side=250, pitch_dm=10, spacing_dm=30,
                         capacity=30, n_categories=64, n_skus=150_000,
                         category_mode="dirichlet", dirichlet_alpha=2.0,
                         n_orders=4000, lines_lambda=1.5, line_cap=None,
                         zipf_s=1.1, seed=seed)


WORKLOADS: Dict[str, dict] = {
    # 10 aisles x 2 x 30 slots, 12 x 50 SKUs, 200 orders (cap 8), Q = 20, 256 plans
    "tiny": dict(make=_tiny, n_plans=256),
    # 400 aisles x 2 x 250 slots, 150k SKUs in 64 Dirichlet(2) categories,
    # 4,000 orders (~10k items), Q = 30, 4,096 plans per call
    "paper": dict(make=_paper, n_plans=4096),
}


def workload(name: str, seed: int = 0, n_plans: Optional[int] = None):
    """``(instance, zone_of, order_seq)`` for a named single-instance workload."""
    w = WORKLOADS[name]
    inst = w["make"](seed)
    zone_of, seq = make_plans(inst, n_plans or w["n_plans"], seed=seed)
    return inst, zone_of, seq


def pack_batched_plans(insts: Sequence[Instance], plans_per_instance: int, seed: int = 0):
    """Plans for a batch: zone_of ``uint8[sum, 64]`` and the packed sequences.

    Plan rows of instance i occupy ``plans_per_instance`` consecutive rows;
    the order sequences are concatenated row after row (instance-major), so
    the rows of instance i start at ``seq_base[i]`` elements.
    """
    zones, seqs, bases = [], [], []
    base = 0
    for i, inst in enumerate(insts):
        rng = np.random.default_rng([seed, STREAM_PLANS, i])
        zones.append(random_zone_perms(rng, plans_per_instance, inst.n_categories))
        s = random_order_perms(rng, plans_per_instance, inst.n_orders)
        seqs.append(s.reshape(-1))
        bases.append(base)
        base += s.size
    return np.concatenate(zones), np.concatenate(seqs), np.asarray(bases, dtype=np.int64)


def make_typed_orders(n_orders: int, n_types: int, sku_category: np.ndarray, n_categories: int, *,
                      lines_lambda: float = 1.5, concentration: float = 0.3, drift: float = 0.0,
                      seed: int = 0, chunk: int = 65536):
    """Orders that each belong to one of ``n_types`` order types, the labels
    of the order-category learning (no labelled order history exists).

    Type t prefers categories by a Dirichlet(``concentration``) weight vector
    that moves linearly, over the order index, from one draw to a second one
    as far as ``drift`` (0: fixed types, 1: the whole way), so that older
    orders describe the types less well than recent ones.  An order draws its
    type uniformly, 1 + Poisson(``lines_lambda``) lines, each line's category
    from its type's weights and the SKU uniformly within the category.
    Returns ``(order_offsets int32 [n + 1], order_skus int32, types int32 [n])``.
    """
    rng = np.random.default_rng([seed, STREAM_ORDER_TYPES])
    C = int(n_categories)
    pref0 = rng.dirichlet(np.full(C, concentration), size=n_types)
    pref1 = rng.dirichlet(np.full(C, concentration), size=n_types)
    cat = np.asarray(sku_category, np.int64)
    order = np.argsort(cat, kind="stable")
    counts = np.bincount(cat, minlength=C)
    first = np.concatenate([[0], np.cumsum(counts)[:-1]])
    types = rng.integers(0, n_types, n_orders).astype(np.int32)
    lens = (1 + rng.poisson(lines_lambda, n_orders)).astype(np.int64)
    off = np.zeros(n_orders + 1, np.int64)
    off[1:] = np.cumsum(lens)
    skus = np.empty(int(off[-1]), np.int32)
    for o0 in range(0, n_orders, chunk):
        o1 = min(n_orders, o0 + chunk)
        line_order = np.repeat(np.arange(o0, o1), lens[o0:o1])
        s = drift * line_order / max(1, n_orders - 1)
        t = types[line_order]
        p = (1.0 - s)[:, None] * pref0[t] + s[:, None] * pref1[t]
        cdf = np.cumsum(p, axis=1)
        u = rng.random(line_order.size) * cdf[:, -1]
        c = np.minimum((cdf < u[:, None]).sum(axis=1), C - 1)
        c = np.where(counts[c] > 0, c, np.argmax(counts))   # an empty category gives way to the largest
        k = (rng.random(line_order.size) * counts[c]).astype(np.int64)
        skus[off[o0]:off[o1]] = order[first[c] + np.minimum(k, counts[c] - 1)]
    return off.astype(np.int32), skus, types

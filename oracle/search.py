"""CPU re-implementation of one generation of the genetic plan search --
TEST INFRASTRUCTURE ONLY.

The paper puts a top-level optimiser on the CPU that organises the subsystem
searches (section 5, the paragraph on Figure 10) and optimises clustering and
order sequence together (section 6).  The search here is a genetic algorithm
over plans (category -> zone permutation, order sequence):

  * random numbers come from a counter-based generator: the SplitMix64
    finaliser (Steele, Lea & Flood 2014) applied to (seed, stream,
    generation, child, position), so any draw can be recomputed anywhere;
  * tournament selection: 4 uniform draws with replacement from the
    population, the winner is the smallest (distance, index);
  * zone-swap mutation: for each category position c in turn, with
    probability 0.02 (integer test r32 < floor(0.02 * 2^32)), swap its zone
    with that of a uniformly chosen other position;
  * insert mutation: for each sequence position i = 0 .. n-1 in turn, with
    probability 0.02, move the element currently at i so that it ends at a
    uniform position j (remove, then insert);
  * uniform integers in [0, m) take the high 32 bits r32 and compute
    (r32 * m) >> 32 (Lemire's multiply-shift).

Plain arm (one generation): child 0 is the best individual, unchanged; every
other child is a tournament winner with both mutations; the children replace
the population.
"""
from __future__ import annotations

import numpy as np

import oracle

MASK64 = (1 << 64) - 1
P_MUT = 85899345  # floor(0.02 * 2^32)

STREAM_TOURNAMENT = 1
STREAM_ZONE_COIN = 2
STREAM_ZONE_PARTNER = 3
STREAM_INSERT_COIN = 4
STREAM_INSERT_TARGET = 5


def splitmix64(x: int) -> int:
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def draw(seed: int, stream: int, gen: int, child: int, pos: int) -> int:
    """32-bit draw for (seed, stream, generation, child, position)."""
    h = splitmix64((seed + stream) & MASK64)
    h = splitmix64(h ^ (((gen & 0xFFFFFFFF) << 32) | (child & 0xFFFFFFFF)))
    h = splitmix64(h ^ (pos & 0xFFFFFFFF))
    return h >> 32


def uniform(r32: int, m: int) -> int:
    return (r32 * m) >> 32


def tournament(dist, seed, gen, child, size=4, stream=STREAM_TOURNAMENT) -> int:
    best = None
    for k in range(size):
        i = uniform(draw(seed, stream, gen, child, k), len(dist))
        key = (int(dist[i]), i)
        if best is None or key < best:
            best = key
    return best[1]


def mutate_zones(z: np.ndarray, n_cat: int, seed, gen, child) -> np.ndarray:
    z = z.copy()
    if n_cat < 2:
        return z
    for c in range(n_cat):
        if draw(seed, STREAM_ZONE_COIN, gen, child, c) < P_MUT:
            j = uniform(draw(seed, STREAM_ZONE_PARTNER, gen, child, c), n_cat - 1)
            j = j if j < c else j + 1
            z[c], z[j] = z[j], z[c]
    return z


def mutate_sequence(s: np.ndarray, seed, gen, child) -> np.ndarray:
    seq = [int(v) for v in s]
    n = len(seq)
    for i in range(n):
        if draw(seed, STREAM_INSERT_COIN, gen, child, i) < P_MUT:
            j = uniform(draw(seed, STREAM_INSERT_TARGET, gen, child, i), n)
            v = seq.pop(i)
            seq.insert(j, v)
    return np.asarray(seq, dtype=s.dtype)


def plain_generation(inst, zone_of, seq, dist, seed: int, gen: int):
    """One generation of the plain (exact-evaluation) arm.

    Returns the new population ``(zone_of, seq, dist)``."""
    P = zone_of.shape[0]
    best = min(range(P), key=lambda i: (int(dist[i]), i))
    Z = np.empty_like(zone_of)
    Sq = np.empty_like(seq)
    Z[0], Sq[0] = zone_of[best], seq[best]
    for b in range(1, P):
        par = tournament(dist, seed, gen, b)
        Z[b] = mutate_zones(zone_of[par], inst.n_categories, seed, gen, b)
        Sq[b] = mutate_sequence(seq[par], seed, gen, b)
    D, _ = oracle.eval_plans(inst, Z, Sq)
    return Z, Sq, D


def worst_individuals(dist, k):
    """The k worst individuals: largest distance first, ties by smaller index."""
    return sorted(range(len(dist)), key=lambda i: (-int(dist[i]), i))[:k]


def screened_generation(inst, zone_of, seq, dist, seed: int, gen: int, kept_ids):
    """One generation of the screened arm, given the candidate ids the
    surrogate kept (in rank order).

    Candidate b is a tournament winner (child id b) with the zone swap; each
    kept candidate takes its parent's sequence with the order insert (child
    id = candidate id), is evaluated exactly and replaces the next of the
    worst individuals.  Returns the new population ``(zone_of, seq, dist)``."""
    Z, Sq, D = zone_of.copy(), seq.copy(), np.asarray(dist).copy()
    kids_z, kids_s = [], []
    for cid in kept_ids:
        cid = int(cid)
        par = tournament(dist, seed, gen, cid)
        kids_z.append(mutate_zones(zone_of[par], inst.n_categories, seed, gen, cid))
        kids_s.append(mutate_sequence(seq[par], seed, gen, cid))
    kz, ks = np.stack(kids_z), np.stack(kids_s)
    kd, _ = oracle.eval_plans(inst, kz, ks)
    for r, slot in enumerate(worst_individuals(dist, len(kept_ids))):
        Z[slot], Sq[slot], D[slot] = kz[r], ks[r], kd[r]
    return Z, Sq, D

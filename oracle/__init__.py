"""CPU oracle for the warehouse plan evaluator -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding) never does, and this package never imports the product path.

``svm.c`` holds the order categories by linear SVM (features, training,
prediction; wrapped by ``svm.py``);
``wo_oracle.c`` is the plain sequential evaluator (slot map, next-fit tours,
S-shape, return, largest-gap, combined or optimal route distance, time-window throughput);
``surrogate.py`` is the float64
reference of the surrogate network; ``search.py`` re-implements one step of the
genetic search on the CPU; ``kmeans.py`` is the exact K-means class-based
storage.  Each cites the passage of arXiv 2110.13693 it
follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wo_oracle.c")
_SRC_SVM = os.path.join(_HERE, "svm.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


class _Inst(ctypes.Structure):
    _fields_ = [
        ("n_aisles", ctypes.c_int32), ("slots_per_side", ctypes.c_int32),
        ("pitch_dm", ctypes.c_int32), ("spacing_dm", ctypes.c_int32),
        ("capacity", ctypes.c_int32), ("n_categories", ctypes.c_int32),
        ("n_skus", ctypes.c_int32), ("sku_category", ctypes.c_void_p),
        ("n_orders", ctypes.c_int32), ("order_offsets", ctypes.c_void_p),
        ("order_skus", ctypes.c_void_p),
        ("walk_dm_per_s", ctypes.c_double), ("seconds_per_item", ctypes.c_double),
        ("window_s", ctypes.c_double), ("routing", ctypes.c_int32), ("batching", ctypes.c_int32),
    ]

ROUTE_SSHAPE, ROUTE_RETURN, ROUTE_LARGEST_GAP, ROUTE_OPTIMAL, ROUTE_COMBINED = 0, 1, 2, 3, 4
BATCH_NEXT_FIT, BATCH_FIRST_FIT, BATCH_SEED = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (plain -O2, no vectorisation flags)."""
    with _lock:
        if force or not os.path.exists(_LIB):
            tmp = _LIB + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=200809L",
                                   "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-Wextra",
                                   "-o", tmp, _SRC, _SRC_SVM, "-lpthread"])
            os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC),
                                                                      os.path.getmtime(_SRC_SVM)):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        lib.orc_locations.argtypes = [P(_Inst), ctypes.c_void_p, ctypes.c_void_p]
        lib.orc_tours.argtypes = [P(_Inst), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.orc_tours_first_fit.argtypes = [P(_Inst), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.orc_tours_seed.argtypes = [P(_Inst), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]
        lib.orc_sshape_cost.argtypes = [P(_Inst), ctypes.c_void_p, ctypes.c_int32]
        lib.orc_sshape_cost.restype = ctypes.c_int64
        for f in (lib.orc_return_cost, lib.orc_largest_gap_cost, lib.orc_optimal_cost, lib.orc_combined_cost,
                  lib.orc_tour_cost):
            f.argtypes = [P(_Inst), ctypes.c_void_p, ctypes.c_int32]
            f.restype = ctypes.c_int64
        lib.orc_eval_plan.argtypes = [P(_Inst), ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.orc_int_ops.argtypes = [ctypes.c_int64, ctypes.c_uint32, P(ctypes.c_uint32)]
        lib.orc_order_features.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
        lib.orc_svm_train.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_double, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_void_p]
        lib.orc_svm_predict.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]
        lib.orc_int_ops.restype = ctypes.c_int64
        lib.orc_eval_plans.argtypes = [P(_Inst), ctypes.c_int64, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int]
        _lib = lib
    return _lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class _Bound:
    """Keeps the numpy arrays alive while the C struct points at them."""

    def __init__(self, inst):
        self.cat = _c(inst.sku_category, np.int32)
        self.off = _c(inst.order_offsets, np.int32)
        self.sku = _c(inst.order_skus, np.int32)
        self.s = _Inst(inst.n_aisles, inst.slots_per_side, inst.pitch_dm, inst.spacing_dm,
                       inst.capacity, inst.n_categories, self.cat.size,
                       self.cat.ctypes.data, self.off.size - 1, self.off.ctypes.data,
                       self.sku.ctypes.data, float(inst.walk_dm_per_s),
                       float(inst.seconds_per_item), float(inst.window_s),
                       int(getattr(inst, "routing", ROUTE_SSHAPE)),
                       int(getattr(inst, "batching", BATCH_NEXT_FIT)))
        self.n_orders = self.off.size - 1

    def ref(self):
        return ctypes.byref(self.s)


def _check(rc):
    if rc != 0:
        raise ValueError("oracle rejected the input (code %d)" % rc)


def locations(inst, zone_of) -> np.ndarray:
    """Location of every SKU under one zone assignment (slot map)."""
    b = _Bound(inst)
    z = _c(zone_of, np.uint8)
    out = np.empty(b.cat.size, dtype=np.int32)
    _check(_load().orc_locations(b.ref(), z.ctypes.data, out.ctypes.data))
    return out


def tours(inst, seq) -> np.ndarray:
    """Next-fit tour boundaries: positions in ``seq`` where tours start, plus n_orders."""
    b = _Bound(inst)
    s = _c(seq, np.uint16)
    out = np.empty(b.n_orders + 1, dtype=np.int32)
    n = ctypes.c_int32(0)
    _check(_load().orc_tours(b.ref(), s.ctypes.data, out.ctypes.data, ctypes.byref(n)))
    return out[: n.value + 1].copy()


def tours_first_fit(inst, seq) -> np.ndarray:
    """First-fit tour of every sequence position, tours numbered in opening order."""
    b = _Bound(inst)
    s = _c(seq, np.uint16)
    out = np.empty(b.n_orders, dtype=np.int32)
    n = ctypes.c_int32(0)
    _check(_load().orc_tours_first_fit(b.ref(), s.ctypes.data, out.ctypes.data, ctypes.byref(n)))
    assert n.value == int(out.max()) + 1
    return out


def tours_seed(inst, zone_of, seq) -> np.ndarray:
    """Seed-batching tour of every sequence position under slotting
    ``zone_of``, tours numbered in the order they are built."""
    b = _Bound(inst)
    loc = locations(inst, zone_of)
    s = _c(seq, np.uint16)
    out = np.empty(b.n_orders, dtype=np.int32)
    n = ctypes.c_int32(0)
    _check(_load().orc_tours_seed(b.ref(), loc.ctypes.data, s.ctypes.data, out.ctypes.data, ctypes.byref(n)))
    assert n.value == int(out.max()) + 1
    return out


def sshape_cost(inst, locs) -> int:
    """S-shape route length (dm) of one tour given its pick locations."""
    b = _Bound(inst)
    l = _c(locs, np.int32)
    return int(_load().orc_sshape_cost(b.ref(), l.ctypes.data, l.size))


def return_cost(inst, locs) -> int:
    """Return-route length (dm) of one tour given its pick locations."""
    b = _Bound(inst)
    l = _c(locs, np.int32)
    return int(_load().orc_return_cost(b.ref(), l.ctypes.data, l.size))


def largest_gap_cost(inst, locs) -> int:
    """Largest-gap route length (dm) of one tour given its pick locations."""
    b = _Bound(inst)
    l = _c(locs, np.int32)
    return int(_load().orc_largest_gap_cost(b.ref(), l.ctypes.data, l.size))


def optimal_cost(inst, locs) -> int:
    """Shortest closed walk (dm) from the depot through every pick of one tour."""
    b = _Bound(inst)
    l = _c(locs, np.int32)
    return int(_load().orc_optimal_cost(b.ref(), l.ctypes.data, l.size))


def combined_cost(inst, locs) -> int:
    """Combined-route length (dm) of one tour given its pick locations."""
    b = _Bound(inst)
    l = _c(locs, np.int32)
    return int(_load().orc_combined_cost(b.ref(), l.ctypes.data, l.size))


def tour_cost(inst, locs) -> int:
    """Route length (dm) of one tour under the instance's routing policy."""
    b = _Bound(inst)
    l = _c(locs, np.int32)
    return int(_load().orc_tour_cost(b.ref(), l.ctypes.data, l.size))


def eval_plan(inst, zone_of, seq) -> Tuple[int, int, float]:
    """``(D exact int, D int32 saturated, orders per window float32)`` for one plan."""
    b = _Bound(inst)
    z = _c(zone_of, np.uint8)
    s = _c(seq, np.uint16)
    de = ctypes.c_int64(0)
    d = ctypes.c_int32(0)
    t = ctypes.c_float(0)
    _check(_load().orc_eval_plan(b.ref(), z.ctypes.data, s.ctypes.data,
                                 ctypes.byref(de), ctypes.byref(d), ctypes.byref(t)))
    return int(de.value), int(d.value), float(np.float32(t.value))


def eval_plans(inst, zone_of, seq, n_threads: int = 1):
    """Distances (int32) and throughputs (float32) for many plans."""
    b = _Bound(inst)
    z = _c(zone_of, np.uint8)
    s = _c(seq, np.uint16)
    n = z.shape[0]
    if z.shape != (n, 64) or s.shape != (n, b.n_orders):
        raise ValueError("plan arrays have the wrong shape")
    dist = np.empty(n, dtype=np.int32)
    thr = np.empty(n, dtype=np.float32)
    _check(_load().orc_eval_plans(b.ref(), n, z.ctypes.data, s.ctypes.data,
                                  dist.ctypes.data, thr.ctypes.data, int(n_threads)))
    return dist, thr


def int_ops_per_second(min_s: float = 0.3) -> float:
    """Measured scalar integer operations per second of one core (eight
    independent add/xor chains), for the CPU roofline of the baseline timing."""
    import time
    lib = _load()
    sink = ctypes.c_uint32(0)
    steps = 1 << 20
    while True:
        t0 = time.perf_counter()
        ops = lib.orc_int_ops(steps, 12345, ctypes.byref(sink))
        dt = time.perf_counter() - t0
        if dt >= min_s:
            return ops / dt
        steps *= 2

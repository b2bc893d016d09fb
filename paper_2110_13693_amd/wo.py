"""Thin ctypes binding of ``libwo.so`` (names follow ``include/wo.h``).

Only argument marshalling happens here: every step of plan evaluation runs in
the library's kernels.  Tensors must already live on the GPU; the library is
required -- there is no CPU fallback, and a missing library raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# WO_LIBRARY selects another build of the library (e.g. the host-sanitizer build)
LIB_PATH = os.environ.get("WO_LIBRARY") or os.path.join(_HERE, "libwo.so")

WO_OK, WO_E_INVAL, WO_E_RANGE, WO_E_NOMEM, WO_E_DEVICE, WO_E_STATE, WO_E_UNSUPPORTED = range(7)
WO_MAX_CATEGORIES = 64
WO_MAX_ORDERS = 65535
WO_MAX_CAPACITY = 32
WO_MAX_LOCATIONS = 1 << 22
WO_MAX_LINES = 1 << 24

# every symbol include/wo.h declares
EXPORTS = sorted([
    "wo_status_str", "wo_last_error", "wo_load_warehouse", "wo_free_warehouse",
    "wo_instance_info", "wo_eval_plans",
    "wo_sur_create", "wo_sur_free", "wo_sur_set_scale", "wo_sur_get_scale", "wo_sur_get_params",
    "wo_sur_gradients", "wo_sur_train", "wo_sur_predict", "wo_sur_save", "wo_sur_load",
    "wo_screen_plans",
    "wo_search_create", "wo_search_free", "wo_search_step", "wo_search_best", "wo_search_population",
    "wo_search_save", "wo_search_load",
    "wo_set_eval_config", "wo_get_eval_config", "wo_autotune_eval", "wo_tune_cache_store", "wo_tune_cache_lookup",
    "wo_kmeans_categories", "wo_kmeans_categories_noalloc", "wo_measure_int_peak", "wo_measure_peaks",
    "wo_aisle_width",
    "wo_order_features", "wo_svm_create", "wo_svm_free", "wo_svm_push", "wo_svm_train", "wo_svm_predict",
    "wo_svm_get_weights",
])
WO_SUR_PARAMS = 4457985
WO_SCREEN_MAX_KEEP = 4096


class WoError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (_status_name(status), message))
        self.status = status


class wo_eval_config(ctypes.Structure):
    _fields_ = [("block_threads", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("queue", ctypes.c_int32), ("line_pass", ctypes.c_int32), ("small_orders", ctypes.c_int32),
                ("ms", ctypes.c_float)]


class wo_search_params(ctypes.Structure):
    _fields_ = [("population", ctypes.c_int32), ("tournament", ctypes.c_int32),
                ("mutation_threshold", ctypes.c_uint32), ("candidates", ctypes.c_int32),
                ("keep", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class wo_aisle_params(ctypes.Structure):
    _fields_ = [("rack_depth_dm", ctypes.c_int32), ("cross_aisle_dm", ctypes.c_int32),
                ("min_width_dm", ctypes.c_int32), ("max_width_dm", ctypes.c_int32), ("k_dm", ctypes.c_double)]


class wo_peaks(ctypes.Structure):
    _fields_ = [("int_ops_per_s", ctypes.c_double), ("lds_bytes_per_s", ctypes.c_double),
                ("hbm_read_bytes_per_s", ctypes.c_double), ("bf16_flops_per_s", ctypes.c_double),
                ("l2_read_bytes_per_s", ctypes.c_double)]


class wo_aisle_result(ctypes.Structure):
    _fields_ = [("width_dm", ctypes.c_int32), ("spacing_dm", ctypes.c_int32), ("feasible", ctypes.c_int32),
                ("widths_evaluated", ctypes.c_int32), ("distance", ctypes.c_int32),
                ("orders_per_window", ctypes.c_double), ("utilization", ctypes.c_double)]


class wo_instance_desc(ctypes.Structure):
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


WO_ROUTE_SSHAPE, WO_ROUTE_RETURN, WO_ROUTE_LARGEST_GAP, WO_ROUTE_OPTIMAL, WO_ROUTE_COMBINED = 0, 1, 2, 3, 4
WO_BATCH_NEXT_FIT, WO_BATCH_FIRST_FIT, WO_BATCH_SEED = 0, 1, 2

_lib = None


def lib():
    """Load ``libwo.so``; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libwo.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        V, P, I32, I64 = ctypes.c_void_p, ctypes.POINTER, ctypes.c_int32, ctypes.c_int64
        L.wo_status_str.argtypes = [ctypes.c_int]
        L.wo_status_str.restype = ctypes.c_char_p
        L.wo_last_error.argtypes = []
        L.wo_last_error.restype = ctypes.c_char_p
        L.wo_load_warehouse.argtypes = [P(wo_instance_desc), I32, V, P(V)]
        L.wo_free_warehouse.argtypes = [V]
        L.wo_instance_info.argtypes = [V, I32, P(I32), P(I32), P(I32)]
        L.wo_eval_plans.argtypes = [V, V, I64, V, V, V, V, V]
        F32, F64, U64 = ctypes.c_float, ctypes.c_double, ctypes.c_uint64
        L.wo_sur_create.argtypes = [I32, V, U64, V, P(V)]
        L.wo_sur_free.argtypes = [V]
        L.wo_sur_set_scale.argtypes = [V, F64, F64]
        L.wo_sur_get_scale.argtypes = [V, P(F64), P(F64)]
        L.wo_sur_get_params.argtypes = [V, V]
        L.wo_sur_gradients.argtypes = [V, I32, V, V, V, P(F32), V]
        L.wo_sur_train.argtypes = [V, I64, V, V, I32, I32, F32, U64, P(F32), V]
        L.wo_sur_predict.argtypes = [V, I64, V, V, V]
        L.wo_sur_save.argtypes = [V, ctypes.c_char_p]
        L.wo_sur_load.argtypes = [ctypes.c_char_p, V, P(V)]
        L.wo_screen_plans.argtypes = [V, I32, V, I64, V, V, I64, V, V]
        L.wo_set_eval_config.argtypes = [V, P(wo_eval_config)]
        L.wo_get_eval_config.argtypes = [V, P(wo_eval_config)]
        L.wo_autotune_eval.argtypes = [V, V, I64, V, V, V, I32, V, P(wo_eval_config), V, P(I32)]
        L.wo_tune_cache_store.argtypes = [V, ctypes.c_char_p, I64, V]
        L.wo_tune_cache_lookup.argtypes = [V, ctypes.c_char_p, I64, P(I32)]
        L.wo_search_create.argtypes = [V, I32, P(wo_search_params), V, V, V, P(V)]
        L.wo_search_free.argtypes = [V]
        L.wo_search_step.argtypes = [V, V, V, I32, V]
        L.wo_search_best.argtypes = [V, V, V, P(I32), P(I32), V]
        L.wo_search_population.argtypes = [V, V, V, V, V, V]
        L.wo_search_save.argtypes = [V, ctypes.c_char_p, V]
        L.wo_search_load.argtypes = [V, I32, ctypes.c_char_p, V, P(V)]
        L.wo_kmeans_categories.argtypes = [V, I64, I32, I32, I32, V, P(I32), P(I32), V]
        L.wo_kmeans_categories_noalloc.argtypes = [V, I64, I32, I32, I32, V, V, V, V]
        L.wo_measure_int_peak.argtypes = [I32, P(F64), V]
        L.wo_measure_peaks.argtypes = [I32, P(wo_peaks), V]
        L.wo_aisle_width.argtypes = [V, I32, V, V, P(wo_aisle_params), V, V, P(wo_aisle_result)]
        L.wo_order_features.argtypes = [V, V, I32, I64, V, I32, I32, V, V]
        L.wo_svm_create.argtypes = [I32, I32, I32, F64, V, P(V)]
        L.wo_svm_free.argtypes = [V]
        L.wo_svm_push.argtypes = [V, I64, V, V, V]
        L.wo_svm_train.argtypes = [V, I32, V]
        L.wo_svm_predict.argtypes = [V, I64, V, V, V]
        L.wo_svm_get_weights.argtypes = [V, V, P(I64), P(I64), V]
        for name in EXPORTS:
            getattr(L, name).restype = getattr(L, name).restype if name in (
                "wo_status_str", "wo_last_error") else ctypes.c_int
        _lib = L
    return _lib


def _status_name(s: int) -> str:
    try:
        return lib().wo_status_str(int(s)).decode()
    except ImportError:
        return "status %d" % s


def _check(status: int):
    if status != WO_OK:
        raise WoError(status, lib().wo_last_error().decode())


def wo_status_str(s: int) -> str:
    return lib().wo_status_str(int(s)).decode()


def wo_last_error() -> str:
    return lib().wo_last_error().decode()


def _stream_handle(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(getattr(stream, "cuda_stream", stream))


def _ptr(t, dtype_size: int, name: str) -> int:
    if t is None:
        return 0
    if not getattr(t, "is_cuda", False):
        raise ValueError("%s must be a GPU tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.element_size() != dtype_size:
        raise ValueError("%s must have %d-byte elements" % (name, dtype_size))
    return t.data_ptr()


class Warehouse:
    """Owns a ``wo_wh*`` handle (one or more loaded instances)."""

    def __init__(self, handle: int, instances):
        self.handle = ctypes.c_void_p(handle)
        self.n_orders = [int(i.n_orders) for i in instances]
        self.n_items = [int(i.n_items) for i in instances]
        self.n_instances = len(self.n_orders)

    def free(self):
        if self.handle:
            _check(lib().wo_free_warehouse(self.handle))
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def make_desc(inst, keep: list) -> wo_instance_desc:
    """Descriptor of a :class:`synth.Instance`-like object (arrays kept alive in ``keep``)."""
    cat = np.ascontiguousarray(inst.sku_category, dtype=np.int32)
    off = np.ascontiguousarray(inst.order_offsets, dtype=np.int32)
    sku = np.ascontiguousarray(inst.order_skus, dtype=np.int32)
    keep += [cat, off, sku]
    return wo_instance_desc(int(inst.n_aisles), int(inst.slots_per_side), int(inst.pitch_dm),
                            int(inst.spacing_dm), int(inst.capacity), int(inst.n_categories),
                            cat.size, cat.ctypes.data, off.size - 1, off.ctypes.data,
                            sku.ctypes.data, float(inst.walk_dm_per_s),
                            float(inst.seconds_per_item), float(inst.window_s),
                            int(getattr(inst, "routing", WO_ROUTE_SSHAPE)),
                            int(getattr(inst, "batching", WO_BATCH_NEXT_FIT)))


def wo_load_warehouse(instances: Sequence, stream=None) -> Warehouse:
    """Load one or more instances onto the current device (synchronous)."""
    keep: list = []
    arr = (wo_instance_desc * len(instances))(*[make_desc(i, keep) for i in instances])
    out = ctypes.c_void_p(0)
    _check(lib().wo_load_warehouse(arr, len(instances), ctypes.c_void_p(_stream_handle(stream)),
                                   ctypes.byref(out)))
    return Warehouse(out.value, instances)


def wo_free_warehouse(wh: Warehouse):
    wh.free()


def wo_eval_plans(wh: Warehouse, zone_of, order_seq, dist, orders_per_window=None,
                  plan_offsets: Optional[Sequence[int]] = None, stream=None):
    """Enqueue exact evaluation of ``zone_of.shape[0]`` plans (async on ``stream``).

    ``zone_of``: uint8 [n, 64]; ``order_seq``: 2-byte elements, rows packed
    instance after instance; ``dist``: int32 [n]; ``orders_per_window``:
    float32 [n] or None.
    """
    n = int(zone_of.shape[0])
    if zone_of.dim() != 2 or zone_of.shape[1] != 64:
        raise ValueError("zone_of must be [n_plans, 64]")
    if dist.numel() != n or (orders_per_window is not None and orders_per_window.numel() != n):
        raise ValueError("output length must equal the number of plans")
    offs = None
    if plan_offsets is not None:
        offs = np.ascontiguousarray(plan_offsets, dtype=np.int64)
        need = int(sum((offs[i + 1] - offs[i]) * wh.n_orders[i] for i in range(wh.n_instances)))
    else:
        need = n * wh.n_orders[0]
    if order_seq.numel() != need:
        raise ValueError("order_seq holds %d entries, the plans need %d" % (order_seq.numel(), need))
    _check(lib().wo_eval_plans(
        wh.handle, None if offs is None else offs.ctypes.data, n,
        _ptr(zone_of, 1, "zone_of"), _ptr(order_seq, 2, "order_seq"), _ptr(dist, 4, "dist"),
        _ptr(orders_per_window, 4, "orders_per_window"),
        ctypes.c_void_p(_stream_handle(stream))))
    return dist, orders_per_window


# ---------------------------------------------------------------------------
# surrogate and screening
# ---------------------------------------------------------------------------

class Surrogate:
    """Owns a ``wo_sur*`` handle."""

    def __init__(self, handle: int):
        self.handle = ctypes.c_void_p(handle)

    def free(self):
        if self.handle:
            _check(lib().wo_sur_free(self.handle))
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def wo_sur_create(n_categories: int, init: Optional[np.ndarray] = None, seed: int = 0,
                  stream=None) -> Surrogate:
    """New surrogate; ``init`` float32[WO_SUR_PARAMS] in the host layout or None."""
    buf = None
    if init is not None:
        buf = np.ascontiguousarray(init, dtype=np.float32).reshape(-1)
        if buf.size != WO_SUR_PARAMS:
            raise ValueError("init must hold %d values" % WO_SUR_PARAMS)
    out = ctypes.c_void_p(0)
    _check(lib().wo_sur_create(int(n_categories), None if buf is None else buf.ctypes.data,
                               int(seed) & ((1 << 64) - 1),
                               ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(out)))
    return Surrogate(out.value)


def wo_sur_free(s: Surrogate):
    s.free()


def wo_sur_set_scale(s: Surrogate, mean: float, std: float):
    _check(lib().wo_sur_set_scale(s.handle, float(mean), float(std)))


def wo_sur_get_scale(s: Surrogate):
    m, d = ctypes.c_double(0), ctypes.c_double(0)
    _check(lib().wo_sur_get_scale(s.handle, ctypes.byref(m), ctypes.byref(d)))
    return m.value, d.value


def wo_sur_get_params(s: Surrogate) -> np.ndarray:
    out = np.empty(WO_SUR_PARAMS, dtype=np.float32)
    _check(lib().wo_sur_get_params(s.handle, out.ctypes.data))
    return out


def wo_sur_gradients(s: Surrogate, zone_of, target, stream=None):
    """``(grad float32[WO_SUR_PARAMS] host layout, loss)`` of one batch."""
    n = int(zone_of.shape[0])
    grad = np.empty(WO_SUR_PARAMS, dtype=np.float32)
    loss = ctypes.c_float(0)
    _check(lib().wo_sur_gradients(s.handle, n, _ptr(zone_of, 1, "zone_of"), _ptr(target, 4, "target"),
                                  grad.ctypes.data, ctypes.byref(loss),
                                  ctypes.c_void_p(_stream_handle(stream))))
    return grad, loss.value


def wo_sur_train(s: Surrogate, zone_of, dist, epochs: int = 1, batch: int = 1024, lr: float = 1e-3,
                 seed: int = 0, stream=None) -> float:
    """Train on (plan, exact distance) pairs; returns the last epoch's mean batch loss."""
    n = int(zone_of.shape[0])
    if dist.numel() != n:
        raise ValueError("one distance per plan")
    loss = ctypes.c_float(0)
    _check(lib().wo_sur_train(s.handle, n, _ptr(zone_of, 1, "zone_of"), _ptr(dist, 4, "dist"),
                              int(epochs), int(batch), float(lr), int(seed) & ((1 << 64) - 1),
                              ctypes.byref(loss), ctypes.c_void_p(_stream_handle(stream))))
    return loss.value


def wo_sur_predict(s: Surrogate, zone_of, pred, stream=None):
    n = int(zone_of.shape[0])
    if pred.numel() != n:
        raise ValueError("one prediction per plan")
    _check(lib().wo_sur_predict(s.handle, n, _ptr(zone_of, 1, "zone_of"), _ptr(pred, 4, "pred"),
                                ctypes.c_void_p(_stream_handle(stream))))
    return pred


def wo_sur_save(s: Surrogate, path: str):
    _check(lib().wo_sur_save(s.handle, os.fsencode(path)))


def wo_sur_load(path: str, stream=None) -> Surrogate:
    out = ctypes.c_void_p(0)
    _check(lib().wo_sur_load(os.fsencode(path), ctypes.c_void_p(_stream_handle(stream)),
                             ctypes.byref(out)))
    return Surrogate(out.value)


def wo_screen_plans(wh: Warehouse, inst: int, s: Surrogate, zone_of, keep: int, keep_idx,
                    pred=None, stream=None):
    """Indices of the ``keep`` best predicted plans, ordered by (prediction, index)."""
    n = int(zone_of.shape[0])
    if keep_idx.numel() != keep:
        raise ValueError("keep_idx must hold `keep` entries")
    if pred is not None and pred.numel() != n:
        raise ValueError("pred must hold one value per plan")
    _check(lib().wo_screen_plans(wh.handle, int(inst), s.handle, n, _ptr(zone_of, 1, "zone_of"),
                                 _ptr(pred, 4, "pred"), int(keep), _ptr(keep_idx, 4, "keep_idx"),
                                 ctypes.c_void_p(_stream_handle(stream))))
    return keep_idx


# ---------------------------------------------------------------------------
# class-based storage
# ---------------------------------------------------------------------------

def wo_kmeans_categories(order_skus, n_skus: int, k: int, category, max_iter: int = 100, stream=None):
    """K-means categories of the SKUs by pick frequency into ``category``
    (int32 GPU tensor of n_skus); returns (categories used, assignments)."""
    if category.numel() != n_skus:
        raise ValueError("category must hold one entry per SKU")
    used, iters = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().wo_kmeans_categories(_ptr(order_skus, 4, "order_skus"), int(order_skus.numel()), int(n_skus),
                                      int(k), int(max_iter), _ptr(category, 4, "category"), ctypes.byref(used),
                                      ctypes.byref(iters), ctypes.c_void_p(_stream_handle(stream))))
    return used.value, iters.value


def wo_kmeans_categories_noalloc(order_skus, n_skus: int, k: int, category, k_used=None, n_iter=None,
                                 max_iter: int = 100, stream=None):
    """The allocation-free K-means (asynchronous): categories into
    ``category`` (int32 GPU tensor of n_skus), categories used and
    assignments into the one-element int32 GPU tensors ``k_used`` and
    ``n_iter`` (each may be None)."""
    if category.numel() != n_skus:
        raise ValueError("category must hold one entry per SKU")
    _check(lib().wo_kmeans_categories_noalloc(
        _ptr(order_skus, 4, "order_skus"), int(order_skus.numel()), int(n_skus), int(k), int(max_iter),
        _ptr(category, 4, "category"), _ptr(k_used, 4, "k_used") if k_used is not None else None,
        _ptr(n_iter, 4, "n_iter") if n_iter is not None else None, ctypes.c_void_p(_stream_handle(stream))))


def wo_aisle_width(wh: Warehouse, zone_of, order_seq, rack_depth_dm: int, cross_aisle_dm: int, k_dm: float,
                   min_width_dm: int, max_width_dm: int, inst: int = 0, stream=None):
    """Aisle width design for one plan (zone row of 64 bytes and sequence of
    n_orders uint16 on the GPU): returns (result dict, distance at every
    width of the range as a numpy array)."""
    import numpy as np
    prm = wo_aisle_params(int(rack_depth_dm), int(cross_aisle_dm), int(min_width_dm), int(max_width_dm), float(k_dm))
    n_w = max(0, int(max_width_dm) - int(min_width_dm) + 1)
    dist = np.zeros(max(n_w, 1), dtype=np.int32)
    out = wo_aisle_result()
    _check(lib().wo_aisle_width(wh.handle, int(inst), _ptr(zone_of, 1, "zone_of"), _ptr(order_seq, 2, "order_seq"),
                                ctypes.byref(prm), dist.ctypes.data, ctypes.c_void_p(_stream_handle(stream)),
                                ctypes.byref(out)))
    res = {f: getattr(out, f) for f, _ in wo_aisle_result._fields_}
    return res, dist[:n_w]


def wo_order_features(order_offsets, order_skus, sku_category, n_features: int, features, stream=None):
    """Shares of each order's lines per category into ``features`` (float64
    GPU tensor [n_orders, n_features]); inputs are int32 GPU tensors."""
    n = int(order_offsets.numel()) - 1
    if features.shape[0] != n or features.shape[1] != n_features:
        raise ValueError("features must be [n_orders, n_features]")
    _check(lib().wo_order_features(_ptr(order_offsets, 4, "order_offsets"), _ptr(order_skus, 4, "order_skus"), n,
                                   int(order_skus.numel()), _ptr(sku_category, 4, "sku_category"),
                                   int(sku_category.numel()), int(n_features), _ptr(features, 8, "features"),
                                   ctypes.c_void_p(_stream_handle(stream))))


class Svm:
    def __init__(self, handle: int, n_features: int, n_classes: int):
        self.handle = handle
        self.n_features = n_features
        self.n_classes = n_classes

    def free(self):
        if self.handle:
            lib().wo_svm_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def wo_svm_create(n_features: int, n_classes: int, window: int, lam: float, stream=None) -> Svm:
    out = ctypes.c_void_p(0)
    _check(lib().wo_svm_create(int(n_features), int(n_classes), int(window), float(lam),
                               ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(out)))
    return Svm(out.value, n_features, n_classes)


def wo_svm_push(s: Svm, features, labels, stream=None):
    n = int(labels.numel())
    _check(lib().wo_svm_push(s.handle, n, _ptr(features, 8, "features"), _ptr(labels, 4, "labels"),
                             ctypes.c_void_p(_stream_handle(stream))))


def wo_svm_train(s: Svm, iterations: int, stream=None):
    _check(lib().wo_svm_train(s.handle, int(iterations), ctypes.c_void_p(_stream_handle(stream))))


def wo_svm_predict(s: Svm, features, out, stream=None):
    _check(lib().wo_svm_predict(s.handle, int(out.numel()), _ptr(features, 8, "features"), _ptr(out, 4, "class"),
                                ctypes.c_void_p(_stream_handle(stream))))


def wo_svm_get_weights(s: Svm, stream=None):
    """(weights numpy [n_classes, n_features + 1], steps, samples in the window)."""
    import numpy as np
    w = np.zeros((s.n_classes, s.n_features + 1), np.float64)
    steps, cnt = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().wo_svm_get_weights(s.handle, w.ctypes.data, ctypes.byref(steps), ctypes.byref(cnt),
                                    ctypes.c_void_p(_stream_handle(stream))))
    return w, steps.value, cnt.value


def wo_measure_peaks(reps: int = 3, stream=None) -> dict:
    """Measured peaks of the device: integer VALU ops/s, LDS read bytes/s,
    HBM read bytes/s and dense BF16 MFMA FLOP/s."""
    p = wo_peaks()
    _check(lib().wo_measure_peaks(int(reps), ctypes.byref(p), ctypes.c_void_p(_stream_handle(stream))))
    return {"int_ops_per_s": p.int_ops_per_s, "lds_bytes_per_s": p.lds_bytes_per_s,
            "hbm_read_bytes_per_s": p.hbm_read_bytes_per_s, "bf16_flops_per_s": p.bf16_flops_per_s,
            "l2_read_bytes_per_s": p.l2_read_bytes_per_s}


def wo_measure_int_peak(reps: int = 5, stream=None) -> float:
    """Measured 32-bit integer VALU operations per second of the device."""
    v = ctypes.c_double(0.0)
    _check(lib().wo_measure_int_peak(int(reps), ctypes.byref(v), ctypes.c_void_p(_stream_handle(stream))))
    return v.value


# ---------------------------------------------------------------------------
# genetic search
# ---------------------------------------------------------------------------

MUTATION_2PCT = 85899345   # floor(0.02 * 2^32)


class Search:
    """Owns a ``wo_search*`` handle."""

    def __init__(self, handle: int, n_orders: int, population: int, keep: int):
        self.handle = ctypes.c_void_p(handle)
        self.n_orders = n_orders
        self.population = population
        self.keep = keep

    def free(self):
        if self.handle:
            _check(lib().wo_search_free(self.handle))
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def wo_search_create(wh: Warehouse, inst: int, init_zone_of, init_seq, population: int,
                     tournament: int = 4, mutation_threshold: int = MUTATION_2PCT, candidates: int = 0,
                     keep: int = 0, seed: int = 0, stream=None) -> Search:
    prm = wo_search_params(int(population), int(tournament), int(mutation_threshold), int(candidates),
                           int(keep), int(seed) & ((1 << 64) - 1))
    n = wh.n_orders[inst]
    if init_zone_of.shape[0] != population or init_seq.numel() != population * n:
        raise ValueError("initial population has the wrong shape")
    out = ctypes.c_void_p(0)
    _check(lib().wo_search_create(wh.handle, int(inst), ctypes.byref(prm), _ptr(init_zone_of, 1, "zone_of"),
                                  _ptr(init_seq, 2, "seq"), ctypes.c_void_p(_stream_handle(stream)),
                                  ctypes.byref(out)))
    return Search(out.value, n, population, keep)


def wo_search_save(s: Search, path: str, stream=None):
    """Checkpoint the search to ``path`` (synchronous)."""
    _check(lib().wo_search_save(s.handle, os.fsencode(path), ctypes.c_void_p(_stream_handle(stream))))


def wo_search_load(wh: Warehouse, inst: int, path: str, stream=None) -> Search:
    """Resume a checkpointed search on instance ``inst`` of ``wh``."""
    import struct
    out = ctypes.c_void_p(0)
    _check(lib().wo_search_load(wh.handle, int(inst), os.fsencode(path), ctypes.c_void_p(_stream_handle(stream)),
                                ctypes.byref(out)))
    with open(path, "rb") as f:                 # population and keep, for the Python-side shapes
        head = f.read(8 + 16 + ctypes.sizeof(wo_search_params))
    population = struct.unpack_from("<i", head, 16)[0]
    prm = wo_search_params.from_buffer_copy(head[24:24 + ctypes.sizeof(wo_search_params)])
    return Search(out.value, wh.n_orders[inst], population, prm.keep)


def wo_search_free(s: Search):
    s.free()


def wo_search_step(wh: Warehouse, s: Search, sur: Optional[Surrogate], n_generations: int = 1, stream=None):
    _check(lib().wo_search_step(wh.handle, s.handle, None if sur is None else sur.handle,
                                int(n_generations), ctypes.c_void_p(_stream_handle(stream))))


def wo_search_best(s: Search, stream=None):
    """``(zone_of uint8[64], seq uint16[n], dist, generation)`` of the best individual."""
    z = np.empty(64, dtype=np.uint8)
    q = np.empty(s.n_orders, dtype=np.uint16)
    d = ctypes.c_int32(0)
    g = ctypes.c_int32(0)
    _check(lib().wo_search_best(s.handle, z.ctypes.data, q.ctypes.data, ctypes.byref(d), ctypes.byref(g),
                                ctypes.c_void_p(_stream_handle(stream))))
    return z, q, d.value, g.value


def wo_search_population(s: Search, zone_of=None, seq=None, dist=None, last_kept=None, stream=None):
    _check(lib().wo_search_population(s.handle, _ptr(zone_of, 1, "zone_of"), _ptr(seq, 2, "seq"),
                                      _ptr(dist, 4, "dist"), _ptr(last_kept, 4, "last_kept"),
                                      ctypes.c_void_p(_stream_handle(stream))))


# ---------------------------------------------------------------------------
# launch configuration and autotuning
# ---------------------------------------------------------------------------

def wo_set_eval_config(wh: Warehouse, block_threads: int, blocks_per_cu: int = 0, queue: int = 0,
                       line_pass: int = 0, small_orders: int = 1024):
    cfg = wo_eval_config(int(block_threads), int(blocks_per_cu), int(queue), int(line_pass), int(small_orders),
                         0.0)
    _check(lib().wo_set_eval_config(wh.handle, ctypes.byref(cfg)))


def wo_get_eval_config(wh: Warehouse) -> dict:
    cfg = wo_eval_config()
    _check(lib().wo_get_eval_config(wh.handle, ctypes.byref(cfg)))
    return {"block_threads": cfg.block_threads, "blocks_per_cu": cfg.blocks_per_cu, "queue": cfg.queue,
            "line_pass": cfg.line_pass, "small_orders": cfg.small_orders}


def wo_tune_cache_store(wh: Warehouse, path: str, n_plans: int, cfg: Optional[dict] = None):
    """Store ``cfg`` (None: the handle's configuration) as the cache entry of
    the handle's key for ``n_plans`` plans."""
    c = None
    if cfg is not None:
        c = wo_eval_config(int(cfg["block_threads"]), int(cfg["blocks_per_cu"]), int(cfg["queue"]),
                           int(cfg["line_pass"]), int(cfg["small_orders"]), float(cfg.get("ms", 0.0)))
    _check(lib().wo_tune_cache_store(wh.handle, os.fsencode(path), int(n_plans),
                                     None if c is None else ctypes.byref(c)))


def wo_tune_cache_lookup(wh: Warehouse, path: str, n_plans: int) -> bool:
    """Apply the cache entry of the handle's key for ``n_plans`` plans; True if found."""
    found = ctypes.c_int32(0)
    _check(lib().wo_tune_cache_lookup(wh.handle, os.fsencode(path), int(n_plans), ctypes.byref(found)))
    return bool(found.value)


def wo_autotune_eval(wh: Warehouse, zone_of, order_seq, dist, plan_offsets=None, reps: int = 3, stream=None):
    """Time every launch configuration; keep and return the fastest (plus all timings)."""
    n = int(zone_of.shape[0])
    offs = None if plan_offsets is None else np.ascontiguousarray(plan_offsets, dtype=np.int64)
    best = wo_eval_config()
    allc = (wo_eval_config * 256)()
    cnt = ctypes.c_int32(256)
    _check(lib().wo_autotune_eval(wh.handle, None if offs is None else offs.ctypes.data, n,
                                  _ptr(zone_of, 1, "zone_of"), _ptr(order_seq, 2, "order_seq"),
                                  _ptr(dist, 4, "dist"), int(reps), ctypes.c_void_p(_stream_handle(stream)),
                                  ctypes.byref(best), allc, ctypes.byref(cnt)))
    conv = lambda c: {"block_threads": c.block_threads, "blocks_per_cu": c.blocks_per_cu, "queue": c.queue,
                      "line_pass": c.line_pass, "small_orders": c.small_orders, "ms": c.ms}
    return conv(best), [conv(allc[i]) for i in range(min(cnt.value, 256))]

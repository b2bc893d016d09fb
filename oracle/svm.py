"""Order categories by linear SVM (section 5, subroutine 5) -- TEST
INFRASTRUCTURE ONLY.  Python side of oracle/svm.c (readings there): order
features, training by full-batch subgradient steps, prediction, and the
sliding window of the most recent orders the SVM is refreshed from."""
from __future__ import annotations

import numpy as np

import oracle


def order_features(order_offsets, order_skus, sku_category, n_features: int) -> np.ndarray:
    """``[n_orders, n_features]`` shares of each order's lines per category."""
    off = np.ascontiguousarray(order_offsets, np.int32)
    sk = np.ascontiguousarray(order_skus, np.int32)
    cat = np.ascontiguousarray(sku_category, np.int32)
    n = off.size - 1
    x = np.empty((n, n_features), np.float64)
    oracle._load().orc_order_features(n, off.ctypes.data, sk.ctypes.data, cat.ctypes.data, cat.size,
                                      int(n_features), x.ctypes.data)
    return x


def train(x, labels, n_classes: int, lam: float, iters: int, w=None, t0: int = 0) -> np.ndarray:
    """``iters`` steps from weights ``w`` ([K, F + 1], zeros if None), steps
    numbered from t0 + 1; returns the new weights."""
    x = np.ascontiguousarray(x, np.float64)
    lab = np.ascontiguousarray(labels, np.int32)
    n, F = x.shape
    w = np.zeros((n_classes, F + 1), np.float64) if w is None else np.array(w, np.float64, copy=True)
    rc = oracle._load().orc_svm_train(n, F, int(n_classes), x.ctypes.data, lab.ctypes.data, float(lam), int(t0),
                                      int(iters), w.ctypes.data)
    if rc != 0:
        raise MemoryError("oracle SVM training ran out of memory")
    return w


def predict(x, w) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float64)
    w = np.ascontiguousarray(w, np.float64)
    n, F = x.shape
    out = np.empty(n, np.int32)
    oracle._load().orc_svm_predict(n, F, w.shape[0], x.ctypes.data, w.ctypes.data, out.ctypes.data)
    return out


class Window:
    """The most recent ``capacity`` samples, oldest first: pushing more
    drops the oldest (newer data replaces the previous)."""

    def __init__(self, capacity: int, n_features: int):
        self.capacity = capacity
        self.x = np.zeros((0, n_features), np.float64)
        self.y = np.zeros(0, np.int32)

    def push(self, x, y):
        self.x = np.concatenate([self.x, np.asarray(x, np.float64)])[-self.capacity:]
        self.y = np.concatenate([self.y, np.asarray(y, np.int32)])[-self.capacity:]

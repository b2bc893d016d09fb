"""Pins of the order-category SVM oracle (oracle/svm.c, oracle/svm.py;
section 5, subroutine 5): the features by hand, two subgradient steps by
hand, the trained objective against scikit-learn's liblinear solution of the
same problem, the sliding window, and what refreshing from recent orders
gains when the order types drift."""
import numpy as np
import pytest

import synth
from oracle import svm


def test_features_by_hand():
    # SKU categories 0 0 1 3 2; orders {0, 1, 3}, {2}, {4, 4, 9 (no such SKU)}
    cat = np.array([0, 0, 1, 3, 2], np.int32)
    off = np.array([0, 3, 4, 7], np.int32)
    skus = np.array([0, 1, 3, 2, 4, 4, 9], np.int32)
    x = svm.order_features(off, skus, cat, 4)
    np.testing.assert_array_equal(x[0], [2 / 3, 0, 0, 1 / 3])
    np.testing.assert_array_equal(x[1], [0, 1, 0, 0])
    np.testing.assert_array_equal(x[2], [0, 0, 2 / 3, 0])     # the unknown SKU counts in the length only
    # categories beyond the feature count are left out the same way
    np.testing.assert_array_equal(svm.order_features(off, skus, cat, 2)[0], [2 / 3, 0])


def test_two_steps_by_hand():
    # two samples x = 1 (category 0) and x = 0 (category 1), lambda 1/2.
    # Step 1 (eta = 2): every score is 0, so both samples are inside both
    # margins: w0 = -2 (0 - (1*1 - 1*0) / 2) = 1, w1 = -1, biases 0.
    # Step 2 (eta = 1): sample 0 sits on both margins (y s = 1), sample 1 is
    # inside them: w0 = 1 - (1/2 - 0) = 1/2, b0 = -(0 + 1/2) = -1/2,
    # w1 = -1 - (-1/2 - 0) = -1/2, b1 = 1/2.
    x = np.array([[1.0], [0.0]])
    y = np.array([0, 1], np.int32)
    w1 = svm.train(x, y, 2, 0.5, 1)
    np.testing.assert_array_equal(w1, [[1.0, 0.0], [-1.0, 0.0]])
    w2 = svm.train(x, y, 2, 0.5, 1, w=w1, t0=1)
    np.testing.assert_array_equal(w2, [[0.5, -0.5], [-0.5, 0.5]])
    np.testing.assert_array_equal(svm.train(x, y, 2, 0.5, 2), w2)
    # x = 1 scores 0 in both classes: the tie goes to the lower class
    np.testing.assert_array_equal(svm.predict(x, w2), [0, 1])


def _objective(w, x, y, k, lam):
    yy = np.where(y == k, 1.0, -1.0)
    s = x @ w[:-1] + w[-1]
    return lam / 2 * (w @ w) + np.mean(np.maximum(0.0, 1.0 - yy * s))


def test_objective_reaches_liblinears_minimum():
    # the same problem per category (hinge loss, the bias a regularised
    # weight of a constant 1): liblinear minimises |w|^2 / 2 + C sum hinge,
    # which is the oracle's objective divided by lambda with C = 1 / (lambda n)
    from sklearn.svm import LinearSVC
    rng = np.random.default_rng(0)
    n, F, K, lam = 300, 4, 3, 0.05
    centers = rng.normal(0, 1, (K, F))
    y = rng.integers(0, K, n).astype(np.int32)
    x = centers[y] + rng.normal(0, 0.6, (n, F))
    w = svm.train(x, y, K, lam, 1000)
    for k in range(K):
        yy = np.where(y == k, 1, -1)
        clf = LinearSVC(C=1.0 / (lam * n), loss="hinge", dual=True, fit_intercept=True, intercept_scaling=1.0,
                        tol=1e-10, max_iter=200000).fit(x, yy)
        opt = _objective(np.concatenate([clf.coef_[0], clf.intercept_]), x, y, k, lam)
        got = _objective(w[k], x, y, k, lam)
        assert got >= opt * (1 - 1e-6)
        assert got <= opt * (1 + 1e-3), (k, got, opt)


def test_separable_classes_are_learned():
    rng = np.random.default_rng(1)
    y = rng.integers(0, 4, 400).astype(np.int32)
    x = np.eye(4)[y] * 0.8 + rng.random((400, 4)) * 0.1
    w = svm.train(x, y, 4, 1e-3, 200)
    assert np.array_equal(svm.predict(x, w), y)


def test_window_keeps_the_most_recent_samples():
    win = svm.Window(12, 2)
    a = np.arange(20, dtype=np.float64).reshape(10, 2)
    win.push(a, np.arange(10))
    assert win.x.shape == (10, 2)
    b = 100 + np.arange(14, dtype=np.float64).reshape(7, 2)
    win.push(b, np.arange(10, 17))
    np.testing.assert_array_equal(win.y, np.arange(5, 17))
    np.testing.assert_array_equal(win.x[:5], a[5:])
    np.testing.assert_array_equal(win.x[5:], b)
    win.push(np.zeros((30, 2)), np.full(30, 7))
    assert win.x.shape == (12, 2) and np.all(win.y == 7)


def test_recent_window_predicts_drifting_orders_better():
    # order types drift over time: an SVM refreshed from the most recent
    # orders categorises the next ones better than one kept on the oldest
    inst, _, _ = synth.workload("paper", n_plans=1)
    off, skus, ty = synth.make_typed_orders(40000, 8, inst.sku_category, inst.n_categories, drift=1.0, seed=2)
    x = svm.order_features(off, skus, inst.sku_category, 64)
    old = svm.train(x[:8000], ty[:8000], 8, 1e-3, 150)
    new = svm.train(x[28000:36000], ty[28000:36000], 8, 1e-3, 150)
    test_x, test_y = x[36000:], ty[36000:]
    acc_old = np.mean(svm.predict(test_x, old) == test_y)
    acc_new = np.mean(svm.predict(test_x, new) == test_y)
    assert acc_new > acc_old + 0.05, (acc_old, acc_new)
    assert acc_new > 2.0 / 8

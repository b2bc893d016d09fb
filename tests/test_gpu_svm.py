"""GPU order categories (section 5, subroutine 5) against the oracle: order
features, SVM weights after training on a sliding window that wraps around,
and predicted categories -- all bit-exact (IEEE double, one operation at a
time and every sum in the same order on both sides)."""
import numpy as np
import pytest

import synth
from oracle import svm as O

pytestmark = pytest.mark.gpu


def _wo():
    import torch
    from paper_2110_13693_amd import wo
    assert torch.cuda.is_available()
    return wo


def _t(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def _features(wo, off, skus, cat, F):
    import torch
    x = torch.empty((off.size - 1, F), dtype=torch.float64, device="cuda")
    wo.wo_order_features(_t(off, np.int32), _t(skus, np.int32), _t(cat, np.int32), F, x)
    torch.cuda.synchronize()
    return x


@pytest.fixture(scope="module")
def typed():
    inst, _, _ = synth.workload("paper", n_plans=1)
    off, skus, ty = synth.make_typed_orders(6000, 8, inst.sku_category, inst.n_categories, drift=0.5, seed=3)
    return inst, off, skus, ty


def test_order_features(typed):
    wo = _wo()
    inst, off, skus, ty = typed
    print("features 6000 orders", flush=True)
    got = _features(wo, off, skus, inst.sku_category, 64).cpu().numpy()
    assert np.array_equal(got, O.order_features(off, skus, inst.sku_category, 64))
    # fewer features than categories, and SKUs outside the category table
    skus2 = skus.copy()
    skus2[::7] = inst.n_skus + 5
    got = _features(wo, off, skus2, inst.sku_category, 20).cpu().numpy()
    assert np.array_equal(got, O.order_features(off, skus2, inst.sku_category, 20))


def test_training_on_a_wrapping_window(typed):
    import torch
    wo = _wo()
    inst, off, skus, ty = typed
    x = _features(wo, off, skus, inst.sku_category, 64)
    xh = x.cpu().numpy()
    lam, W, K = 1e-3, 2500, 8
    s = wo.wo_svm_create(64, K, W, lam)
    win = O.Window(W, 64)
    w_ref, t0 = None, 0
    # pushes of 1,700, 1,300 (wraps), 4 and 3,000 (more than the window)
    bounds = [(0, 1700), (1700, 3000), (3000, 3004), (3004, 6000)]
    for i, (a, b) in enumerate(bounds):
        print("push", a, b, flush=True)
        wo.wo_svm_push(s, x[a:b], _t(ty[a:b], np.int32))
        win.push(xh[a:b], ty[a:b])
        it = 7 + 3 * i
        wo.wo_svm_train(s, it)
        w_ref = O.train(win.x, win.y, K, lam, it, w=w_ref, t0=t0)
        t0 += it
        w_gpu, steps, cnt = wo.wo_svm_get_weights(s)
        assert steps == t0 and cnt == len(win.y)
        assert np.array_equal(w_gpu, w_ref), i
    # categories of every order under the trained weights
    cls = torch.empty(6000, dtype=torch.int32, device="cuda")
    wo.wo_svm_predict(s, x, cls)
    torch.cuda.synchronize()
    pred = cls.cpu().numpy()
    assert np.array_equal(pred, O.predict(xh, w_ref))
    assert np.mean(pred[3000:] == ty[3000:]) > 2.0 / K     # well above chance
    s.free()


def test_small_and_degenerate():
    import torch
    wo = _wo()
    rng = np.random.default_rng(7)
    x = rng.random((50, 3))
    y = rng.integers(-1, 4, 50).astype(np.int32)          # labels outside [0, 3) are negatives everywhere
    s = wo.wo_svm_create(3, 3, 1, 0.25)                  # a window of one sample
    wo.wo_svm_push(s, _t(x, np.float64), _t(y, np.int32))
    wo.wo_svm_train(s, 5)
    w_gpu, steps, cnt = wo.wo_svm_get_weights(s)
    assert cnt == 1 and steps == 5
    assert np.array_equal(w_gpu, O.train(x[-1:], y[-1:], 3, 0.25, 5))
    s.free()
    s = wo.wo_svm_create(3, 3, 64, 0.25)
    with pytest.raises(wo.WoError) as e:
        wo.wo_svm_train(s, 1)                            # nothing pushed yet
    assert e.value.status == wo.WO_E_STATE
    wo.wo_svm_push(s, _t(x, np.float64), _t(y, np.int32))
    wo.wo_svm_train(s, 40)
    w_gpu, _, _ = wo.wo_svm_get_weights(s)
    assert np.array_equal(w_gpu, O.train(x, y, 3, 0.25, 40))
    cls = torch.empty(50, dtype=torch.int32, device="cuda")
    wo.wo_svm_predict(s, _t(x, np.float64), cls)
    torch.cuda.synchronize()
    assert np.array_equal(cls.cpu().numpy(), O.predict(x, w_gpu))
    s.free()


@pytest.mark.parametrize("F,K,n", [(64, 64, 200), (63, 64, 131), (64, 8, 1000), (1, 2, 65), (17, 5, 64)])
def test_prediction_shapes(F, K, n):
    # the largest model (64 classes over 64 features), odd feature counts,
    # a ragged last wave of orders and a wave of exactly 64
    import torch
    wo = _wo()
    rng = np.random.default_rng(F * 1000 + K)
    x = rng.normal(size=(n, F))
    y = rng.integers(0, K, n).astype(np.int32)
    s = wo.wo_svm_create(F, K, n, 0.05)
    wo.wo_svm_push(s, _t(x, np.float64), _t(y, np.int32))
    wo.wo_svm_train(s, 3)
    w_gpu, _, _ = wo.wo_svm_get_weights(s)
    assert np.array_equal(w_gpu, O.train(x, y, K, 0.05, 3))
    cls = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    wo.wo_svm_predict(s, _t(x, np.float64), cls)
    torch.cuda.synchronize()
    assert np.array_equal(cls.cpu().numpy(), O.predict(x, w_gpu))
    s.free()

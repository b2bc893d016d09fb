"""GPU surrogate (MFMA forward/backward, training, screening) against the
float64 reference of oracle/surrogate.py on identical bf16-rounded weights.

Tolerances (bf16 keeps 8 significant bits, so activations and the backward
products carry ~0.4% rounding per element): forward relative L2 <= 1e-2,
gradients relative L2 <= 2e-2 per parameter block."""
import os
import tempfile

import numpy as np
import pytest

import synth
from oracle import surrogate as S

pytestmark = pytest.mark.gpu

SHAPES = [("W1", (S.N_IN, S.N_H1)), ("b1", (S.N_H1,)), ("W2", (S.N_H1, S.N_H2)), ("b2", (S.N_H2,)),
          ("W3", (S.N_H2, 1)), ("b3", (1,))]


def _wo():
    import torch
    from paper_2110_13693_amd import wo
    assert torch.cuda.is_available()
    return wo


def flat(p):
    return np.concatenate([np.asarray(p[k], np.float32).reshape(-1) for k, _ in SHAPES])


def unflat(v):
    out, o = {}, 0
    for k, sh in SHAPES:
        n = int(np.prod(sh))
        out[k] = v[o:o + n].reshape(sh)
        o += n
    return out


def _params(seed=0):
    p = S.init_params(seed)
    rng = np.random.default_rng(seed + 50)
    p["b1"] = rng.normal(0, 0.05, S.N_H1).astype(np.float32)
    p["b2"] = rng.normal(0, 0.05, S.N_H2).astype(np.float32)
    p["b3"] = np.array([0.1], np.float32)
    return p


def _ref_params(p):
    """The GPU multiplies with bf16 copies of W1 and W2; the rest stays fp32."""
    q = dict(p)
    q["W1"] = S.bf16_round(p["W1"])
    q["W2"] = S.bf16_round(p["W2"])
    return q


def _zones(n, seed, n_cat=64):
    rng = np.random.default_rng(seed)
    return synth.generators.random_zone_perms(rng, n, n_cat)


def _rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(1e-30, np.linalg.norm(b)))


@pytest.mark.parametrize("n_cat", [64, 12])
def test_forward_matches_reference(n_cat):
    import torch
    wo = _wo()
    p = _params(1)
    s = wo.wo_sur_create(n_cat, flat(p))
    wo.wo_sur_set_scale(s, 0.0, 1.0)
    Z = _zones(300, 2, n_cat)              # 300 rows: a ragged last tile
    z = torch.from_numpy(Z).cuda()
    pred = torch.empty(300, dtype=torch.float32, device="cuda")
    wo.wo_sur_predict(s, z, pred)
    torch.cuda.synchronize()
    y, _ = S.forward(_ref_params(p), S.one_hot(Z, n_cat))
    assert _rel_l2(pred.cpu().numpy(), y) <= 1e-2
    # de-standardisation
    wo.wo_sur_set_scale(s, 1000.0, 50.0)
    wo.wo_sur_predict(s, z, pred)
    torch.cuda.synchronize()
    np.testing.assert_allclose(pred.cpu().numpy(), y * 50.0 + 1000.0, rtol=2e-3, atol=1.0)
    s.free()


def test_large_screen_matches_reference_on_samples():
    # 70,000 candidates: one full 65,536-row pass and a ragged second one;
    # sampled rows of both against the reference forward
    import torch
    wo = _wo()
    p = _params(6)
    s = wo.wo_sur_create(64, flat(p))
    wo.wo_sur_set_scale(s, 0.0, 1.0)
    n = 70000
    Z = _zones(n, 7)
    z = torch.from_numpy(Z).cuda()
    pred = torch.empty(n, dtype=torch.float32, device="cuda")
    wo.wo_sur_predict(s, z, pred)
    torch.cuda.synchronize()
    rows = np.concatenate([np.arange(0, 64), np.arange(65472, 65600), np.arange(n - 64, n)])
    y, _ = S.forward(_ref_params(p), S.one_hot(Z[rows], 64))
    assert _rel_l2(pred.cpu().numpy()[rows], y) <= 1e-2
    s.free()


def test_padding_bytes_are_ignored():
    import torch
    wo = _wo()
    s = wo.wo_sur_create(12, flat(_params(4)))
    wo.wo_sur_set_scale(s, 0.0, 1.0)
    Z = _zones(128, 5, 12)
    Z2 = Z.copy()
    Z2[:, 12:] = np.random.default_rng(1).integers(0, 64, size=(128, 52))
    out = []
    for zz in (Z, Z2):
        pr = torch.empty(128, dtype=torch.float32, device="cuda")
        wo.wo_sur_predict(s, torch.from_numpy(zz).cuda(), pr)
        torch.cuda.synchronize()
        out.append(pr.cpu().numpy())
    assert np.array_equal(out[0], out[1])
    s.free()


@pytest.mark.parametrize("n", [128, 384])
def test_gradients_match_reference(n):
    import torch
    wo = _wo()
    p = _params(2)
    s = wo.wo_sur_create(64, flat(p))
    Z = _zones(n, 3)
    t = np.random.default_rng(4).normal(0, 1, n).astype(np.float32)
    g, loss = wo.wo_sur_gradients(s, torch.from_numpy(Z).cuda(), torch.from_numpy(t).cuda())
    q = _ref_params(p)
    y, cache = S.forward(q, S.one_hot(Z, 64))
    ref = S.backward(q, cache, y, t.astype(np.float64))
    got = unflat(g)
    for k, _ in SHAPES:
        err = _rel_l2(got[k], ref[k])
        assert err <= 2e-2, (k, err)
    assert abs(loss - np.mean((y - t) ** 2)) <= 1e-2 * np.mean((y - t) ** 2)
    s.free()


def test_screen_orders_by_prediction_then_index():
    import torch
    wo = _wo()
    inst, _, _ = synth.workload("paper", n_plans=1)
    wh = wo.wo_load_warehouse([inst])
    s = wo.wo_sur_create(64, flat(_params(5)))
    wo.wo_sur_set_scale(s, 2.3e7, 3e5)
    n, k = 20000, 1000
    Z = _zones(n, 6)
    z = torch.from_numpy(Z).cuda()
    pred = torch.empty(n, dtype=torch.float32, device="cuda")
    idx = torch.empty(k, dtype=torch.int32, device="cuda")
    wo.wo_screen_plans(wh, 0, s, z, k, idx, pred=pred)
    torch.cuda.synchronize()
    pr = pred.cpu().numpy()
    want = np.lexsort((np.arange(n), pr))[:k]
    assert np.array_equal(idx.cpu().numpy(), want)
    # all predictions equal: ties broken by index
    p0 = _params(5)
    p0["W3"][:] = 0
    s2 = wo.wo_sur_create(64, flat(p0))
    wo.wo_screen_plans(wh, 0, s2, z, k, idx)
    torch.cuda.synchronize()
    assert np.array_equal(idx.cpu().numpy(), np.arange(k))
    s.free()
    s2.free()
    wh.free()


def test_checkpoint_roundtrip():
    import torch
    wo = _wo()
    s = wo.wo_sur_create(64, None, seed=9)
    wo.wo_sur_set_scale(s, 10.0, 2.0)
    Z = _zones(256, 7)
    z = torch.from_numpy(Z).cuda()
    d = torch.from_numpy(np.random.default_rng(8).integers(1000, 2000, 256).astype(np.int32)).cuda()
    wo.wo_sur_train(s, z, d, epochs=1, batch=128, lr=1e-3, seed=1)
    with tempfile.TemporaryDirectory() as tdir:
        path = os.path.join(tdir, "sur.bin")
        wo.wo_sur_save(s, path)
        s2 = wo.wo_sur_load(path)
    assert np.array_equal(wo.wo_sur_get_params(s), wo.wo_sur_get_params(s2))
    assert wo.wo_sur_get_scale(s) == wo.wo_sur_get_scale(s2)
    # one more identical training step on both: bit-identical (Adam state restored)
    wo.wo_sur_train(s, z, d, epochs=1, batch=128, lr=1e-3, seed=2)
    wo.wo_sur_train(s2, z, d, epochs=1, batch=128, lr=1e-3, seed=2)
    assert np.array_equal(wo.wo_sur_get_params(s), wo.wo_sur_get_params(s2))
    s.free()
    s2.free()


def test_training_step_matches_reference_adam():
    import torch
    wo = _wo()
    p = _params(6)
    s = wo.wo_sur_create(64, flat(p))
    wo.wo_sur_set_scale(s, 0.0, 1.0)
    n = 256
    Z = _zones(n, 9)
    d = np.random.default_rng(10).integers(-2, 3, n).astype(np.int32)
    wo.wo_sur_train(s, torch.from_numpy(Z).cuda(), torch.from_numpy(d).cuda(), epochs=1, batch=n, lr=1e-3,
                    seed=3)
    got = unflat(wo.wo_sur_get_params(s))
    # reference: one Adam step from the same start on the same (full) batch
    q = _ref_params(p)
    y, cache = S.forward(q, S.one_hot(Z, 64))
    g = S.backward(q, cache, y, d.astype(np.float64))
    ref = {k: np.asarray(v, np.float64) for k, v in p.items()}
    m = {k: np.zeros_like(v) for k, v in ref.items()}
    v = {k: np.zeros_like(v) for k, v in ref.items()}
    S.adam_step(ref, g, m, v, 1)
    for k, _ in SHAPES:
        delta_ref = ref[k] - p[k]
        delta_got = got[k] - p[k]
        # the first Adam step is ~lr * sign(g); compare the update directions
        mask = np.abs(g[k]) > 1e-3 * np.abs(g[k]).max()
        agree = np.mean(np.sign(delta_ref[mask]) == np.sign(delta_got[mask]))
        assert agree > 0.97, (k, agree)
    s.free()

"""The persistent autotune cache (include/wo.h): the autotuner's winner is
stored under the key (architecture, compute units, route, batching, buckets
of instances, orders and plans) and found again by a new handle of the same
shape, explicitly or on its first evaluation."""
import json

import numpy as np
import pytest

import synth
from tests.gpu_util import gpu_eval

pytestmark = pytest.mark.gpu


def _wo():
    import torch
    from paper_2110_13693_amd import wo
    assert torch.cuda.is_available()
    return wo


def _cfg(c):
    return {k: c[k] for k in ("block_threads", "blocks_per_cu", "queue", "line_pass", "small_orders")}


def _tensors(Z, S):
    import torch
    z = torch.from_numpy(Z).cuda()
    s = torch.from_numpy(S.reshape(-1).view(np.int16)).cuda()
    d = torch.empty(Z.shape[0], dtype=torch.int32, device="cuda")
    return z, s, d


def test_autotune_stores_and_a_new_handle_finds(tmp_path, monkeypatch):
    wo = _wo()
    path = str(tmp_path / "tune.json")
    monkeypatch.setenv("WO_TUNE_CACHE", path)
    inst, Z, S = synth.workload("tiny", n_plans=256)
    wh = wo.wo_load_warehouse([inst])
    best, _ = wo.wo_autotune_eval(wh, *_tensors(Z, S), reps=1)
    wh.free()
    doc = json.load(open(path))
    assert len(doc["entries"]) == 1
    e = doc["entries"][0]
    assert e["arch"].startswith("gfx") and e["cus"] > 0
    assert (e["route"], e["batching"], e["instances"], e["plans"]) == (0, 0, 0, 8)   # 256 plans: bucket 8
    assert e["orders"] == int(np.ceil(np.log2(inst.n_orders)))
    assert _cfg(e) == _cfg(best)
    # a new handle of the same shape takes the entry on its first call
    wh = wo.wo_load_warehouse([inst])
    d_ref, _ = gpu_eval(wh, Z, S)
    assert _cfg(wo.wo_get_eval_config(wh)) == _cfg(best)
    wh.free()
    # ... and another plan-count bucket falls back to the defaults
    wh = wo.wo_load_warehouse([inst])
    gpu_eval(wh, Z[:100], S[:100])
    assert _cfg(wo.wo_get_eval_config(wh)) == {"block_threads": 256, "blocks_per_cu": 0, "queue": 0,
                                               "line_pass": 0, "small_orders": 1024}
    wh.free()


def test_explicit_store_and_lookup(tmp_path):
    wo = _wo()
    path = str(tmp_path / "tune.json")
    inst, Z, S = synth.workload("tiny", n_plans=64)
    wh = wo.wo_load_warehouse([inst])
    assert not wo.wo_tune_cache_lookup(wh, path, 64)          # no file: an empty cache
    cfg = {"block_threads": 128, "blocks_per_cu": 3, "queue": 1, "line_pass": 1, "small_orders": 0, "ms": 0.5}
    wo.wo_tune_cache_store(wh, path, 64, cfg)
    wo.wo_tune_cache_store(wh, path, 4096, None)              # the handle's (default) configuration
    cfg2 = dict(cfg, blocks_per_cu=2)
    wo.wo_tune_cache_store(wh, path, 60, cfg2)                # same bucket as 64: replaces the entry
    assert len(json.load(open(path))["entries"]) == 2
    assert wo.wo_tune_cache_lookup(wh, path, 33)              # 33 .. 64 share a bucket
    assert _cfg(wo.wo_get_eval_config(wh)) == _cfg(cfg2)
    d, _ = gpu_eval(wh, Z, S)                                 # the configuration evaluates the same
    wh2 = wo.wo_load_warehouse([inst])
    d2, _ = gpu_eval(wh2, Z, S)
    assert np.array_equal(d, d2)
    assert not wo.wo_tune_cache_lookup(wh, path, 200)         # bucket 8: no entry, configuration kept
    assert _cfg(wo.wo_get_eval_config(wh)) == _cfg(cfg2)
    # an entry whose configuration is not one the evaluator takes
    doc = json.load(open(path))
    bad = [e for e in doc["entries"] if e["plans"] == 6][0]
    bad["block_threads"] = 100
    json.dump(doc, open(path, "w"))
    with pytest.raises(wo.WoError) as err:
        wo.wo_tune_cache_lookup(wh2, path, 64)
    assert err.value.status == wo.WO_E_INVAL
    bad["block_threads"] = 128
    json.dump(doc, open(path, "w"))
    # an entry of another device does not match
    doc = json.load(open(path))
    for e in doc["entries"]:
        e["cus"] += 1
    json.dump(doc, open(path, "w"))
    assert not wo.wo_tune_cache_lookup(wh2, path, 64)
    wh.free()
    wh2.free()


@pytest.mark.parametrize("text", ['{"entries": [{"arch": "gfx950"}]}', "not json", '{"entries": [{"arch": 3',
                                  '{"entries": [{"arch": "gfx950", "cus": "many"}]}'])
def test_malformed_cache(tmp_path, monkeypatch, text):
    wo = _wo()
    path = str(tmp_path / "bad.json")
    open(path, "w").write(text)
    inst, Z, S = synth.workload("tiny", n_plans=8)
    wh = wo.wo_load_warehouse([inst])
    with pytest.raises(wo.WoError) as e:
        wo.wo_tune_cache_lookup(wh, path, 8)
    assert e.value.status == wo.WO_E_INVAL
    # evaluation through the environment variable ignores the file
    monkeypatch.setenv("WO_TUNE_CACHE", path)
    d, _ = gpu_eval(wh, Z, S)
    assert d.shape == (8,)
    wh.free()

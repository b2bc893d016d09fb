"""What the trained surrogate gains over the method without it.

On the paper-scale warehouse with a fixed order sequence, a surrogate trained
on (plan, exact distance) pairs produced by the GPU evaluator screens 65,536
fresh candidate slottings and keeps the best 5% (3,277); the exact evaluator
re-scores them.  At the same exact-evaluation budget, plain random search
scores 3,277 random candidates.  The screened best must beat the random best.
The surrogate's error against the exact evaluator is reported as numbers."""
import numpy as np
import pytest

import synth
from oracle import surrogate as S

pytestmark = pytest.mark.gpu


def test_screening_beats_random_at_equal_budget():
    import torch
    from paper_2110_13693_amd import wo
    inst = synth.WORKLOADS["paper"]["make"](0)
    n = inst.n_orders
    wh = wo.wo_load_warehouse([inst])

    def exact(Z):
        m = Z.shape[0]
        z = torch.from_numpy(Z).cuda()
        seq = torch.arange(n, dtype=torch.int16, device="cuda").repeat(m)   # identity sequence
        d = torch.empty(m, dtype=torch.int32, device="cuda")
        wo.wo_eval_plans(wh, z, seq, d)
        torch.cuda.synchronize()
        return z, d

    n_train, n_cand, keep = 65536, 65536, 3277
    rng_tr = np.random.default_rng([0, synth.generators.STREAM_SURROGATE_TRAIN])
    rng_ho = np.random.default_rng([0, synth.generators.STREAM_SURROGATE_HELDOUT])
    Ztr = synth.generators.random_zone_perms(rng_tr, n_train, inst.n_categories)
    Zho = synth.generators.random_zone_perms(rng_ho, n_cand, inst.n_categories)
    ztr, dtr = exact(Ztr)
    s = wo.wo_sur_create(inst.n_categories, None, seed=1)
    loss = wo.wo_sur_train(s, ztr, dtr, epochs=4, batch=1024, lr=1e-3, seed=2)
    zho, dho = exact(Zho)
    pred = torch.empty(n_cand, dtype=torch.float32, device="cuda")
    idx = torch.empty(keep, dtype=torch.int32, device="cuda")
    wo.wo_screen_plans(wh, 0, s, zho, keep, idx, pred=pred)
    torch.cuda.synchronize()
    exact_all = dho.cpu().numpy().astype(np.float64)
    p = pred.cpu().numpy().astype(np.float64)
    kept = idx.cpu().numpy()
    best_screened = exact_all[kept].min()
    best_random = exact_all[:keep].min()          # held-out plans are random: equal budget
    rel_mae = float(np.mean(np.abs(p - exact_all) / exact_all))
    rho = S.spearman(p, exact_all)
    print("surrogate: last-epoch loss %.4f, rel-MAE %.5f, Spearman %.3f; best screened %d vs random %d"
          % (loss, rel_mae, rho, best_screened, best_random))
    assert np.all(np.isfinite(p))
    assert rho > 0.3
    assert best_screened < best_random
    s.free()
    wh.free()

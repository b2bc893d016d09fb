"""Helpers for GPU tests: move plans to the device and run the C-ABI path."""
import numpy as np


def to_dev(zone_of, seq):
    import torch
    z = torch.from_numpy(np.ascontiguousarray(zone_of, dtype=np.uint8)).cuda()
    s = torch.from_numpy(np.ascontiguousarray(seq, dtype=np.uint16).view(np.int16)).cuda()
    return z, s


def gpu_eval(wh, zone_of, seq, plan_offsets=None):
    import torch
    from paper_2110_13693_amd import wo
    z, s = to_dev(zone_of, seq)
    n = z.shape[0]
    dist = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    thr = torch.full((n,), -1.0, dtype=torch.float32, device="cuda")
    wo.wo_eval_plans(wh, z, s.reshape(-1), dist, thr, plan_offsets=plan_offsets)
    torch.cuda.synchronize()
    return dist.cpu().numpy(), thr.cpu().numpy()

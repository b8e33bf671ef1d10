"""Helpers for the device tests: move a workload to the GPU, run a mode, fetch
results.  Everything goes through the C ABI (paper_1208_0277_amd)."""

from __future__ import annotations

import numpy as np

import paper_1208_0277_amd as sccg


def device_workload(A, B, pa, pb):
    import torch
    dev = torch.device("cuda:0")
    dA = sccg.DevicePolys.from_host(A.off, A.xy, dev)
    dB = sccg.DevicePolys.from_host(B.off, B.xy, dev)
    tpa = torch.from_numpy(np.ascontiguousarray(pa, np.int32)).to(dev)
    tpb = torch.from_numpy(np.ascontiguousarray(pb, np.int32)).to(dev)
    return dA, dB, tpa, tpb


def run(ctx, dev_wl, mode):
    dA, dB, tpa, tpb = dev_wl
    I, U = ctx.area_pairs(dA, dB, tpa, tpb, mode=mode)
    ctx.sync()
    return I.cpu().numpy(), U.cpu().numpy()


def first_diff(got_i, got_u, exp_i, exp_u, k=5):
    bad = np.nonzero((got_i != exp_i) | (got_u != exp_u))[0]
    return [(int(i), int(got_i[i]), int(exp_i[i]), int(got_u[i]), int(exp_u[i])) for i in bad[:k]], len(bad)


def assert_exact(got_i, got_u, exp_i, exp_u, what=""):
    diffs, n = first_diff(got_i, got_u, exp_i, exp_u)
    assert n == 0, f"{what}: {n} pairs differ; first (pair, I, I_exp, U, U_exp): {diffs}"

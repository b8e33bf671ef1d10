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


def graph_context(**params):
    """A context on its own (non-null) stream: BATCHED calls are captured once
    into a HIP graph and replayed (unless SCCG_F_NO_GRAPH is set)."""
    import torch
    return sccg.Context(0, stream=torch.cuda.Stream(), **params)


def run_graph(ctx, dev_wl, mode=sccg.SCCG_BATCHED, expect_graph=True, out=None):
    """Run one call on ctx's stream (inputs made on the default stream are
    complete first) and return host counts; with expect_graph, check that the
    call went through the context's captured graph.  `out` = (I, U) device
    tensors to write (the graph is keyed on them; new ones otherwise)."""
    import torch
    dA, dB, tpa, tpb = dev_wl
    n = int(tpa.shape[0])
    if out is None:
        out = (torch.empty(n, dtype=torch.int64, device=tpa.device),
               torch.empty(n, dtype=torch.int64, device=tpa.device))
    I, U = out
    I.fill_(-1)
    U.fill_(-1)
    torch.cuda.synchronize()
    before = ctx.graph_launches()
    with torch.cuda.stream(ctx.stream):
        ctx.area_pairs(dA, dB, tpa, tpb, out_inter=I, out_union=U, mode=mode)
    ctx.sync()
    if expect_graph and mode == sccg.SCCG_BATCHED and n > 0:
        assert ctx.graph_launches() == before + 1, "the call did not replay the captured graph"
    return I.cpu().numpy(), U.cpu().numpy()


def first_diff(got_i, got_u, exp_i, exp_u, k=5):
    bad = np.nonzero((got_i != exp_i) | (got_u != exp_u))[0]
    return [(int(i), int(got_i[i]), int(exp_i[i]), int(got_u[i]), int(exp_u[i])) for i in bad[:k]], len(bad)


def assert_exact(got_i, got_u, exp_i, exp_u, what=""):
    diffs, n = first_diff(got_i, got_u, exp_i, exp_u)
    assert n == 0, f"{what}: {n} pairs differ; first (pair, I, I_exp, U, U_exp): {diffs}"

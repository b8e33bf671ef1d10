"""The no-allocation entry point (sccg_area_pairs_noalloc) against BATCHED
sccg_area_pairs: identical counts on the same inputs, on calls in a row that
share the device's one scratch array (the second smaller than the first),
under another queue layout, at the pair limit, and the rejection above it.
All calls go through the C ABI."""

import numpy as np
import pytest

import paper_1208_0277_amd as sccg
import sccg_gen
from tests.gpu_util import assert_exact, device_workload

pytestmark = pytest.mark.gpu

LIMIT = 1 << 18  # most pairs per call


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.nodeid}", flush=True)


@pytest.fixture(scope="module")
def wl3():
    # the heavy-tailed mix, cut to the limit: small, medium and heavy pairs
    return sccg_gen.pairs(3, n_pairs=LIMIT)


def _both(ctx, dev_wl, n):
    """Counts of the first n pairs from BATCHED sccg_area_pairs and from the
    no-allocation entry point (outputs prefilled with -1)."""
    import torch
    dA, dB, tpa, tpb = dev_wl
    pa, pb = tpa[:n].contiguous(), tpb[:n].contiguous()
    rI, rU = ctx.area_pairs(dA, dB, pa, pb, mode=sccg.SCCG_BATCHED)
    nI = torch.full((n,), -1, dtype=torch.int64, device=pa.device)
    nU = torch.full((n,), -1, dtype=torch.int64, device=pa.device)
    ctx.area_pairs_noalloc(dA, dB, pa, pb, nI, nU)
    ctx.sync()
    return rI.cpu().numpy(), rU.cpu().numpy(), nI.cpu().numpy(), nU.cpu().numpy()


def test_two_calls_in_a_row_second_smaller(wl3):
    ctx = sccg.Context(0)
    try:
        dev = device_workload(wl3.A, wl3.B, wl3.pa, wl3.pb)
        for n in (200_000, 30_001):
            rI, rU, nI, nU = _both(ctx, dev, n)
            assert_exact(nI, nU, rI, rU, f"no-allocation entry point, {n} pairs")
    finally:
        ctx.close()


def test_at_the_limit_then_another_queue_layout(wl3):
    dev = device_workload(wl3.A, wl3.B, wl3.pa, wl3.pb)
    ctx = sccg.Context(0)
    try:
        rI, rU, nI, nU = _both(ctx, dev, LIMIT)
        assert_exact(nI, nU, rI, rU, "no-allocation entry point at the pair limit")
    finally:
        ctx.close()
    # two small queues that overflow often: the slots of the previous layout
    # are cleared before the first call in this one
    small = sccg.Context(0, n_queues=2, queue_cap=64, min_queue_cells=1, heavy_verts=64)
    try:
        for n in (100_000, 5_000):
            rI, rU, nI, nU = _both(small, dev, n)
            assert_exact(nI, nU, rI, rU, f"no-allocation entry point, 2 queues of 64 slots, {n} pairs")
    finally:
        small.close()


def test_above_the_limit_is_rejected(wl3):
    import torch
    ctx = sccg.Context(0)
    try:
        dA, dB, tpa, tpb = device_workload(wl3.A, wl3.B, wl3.pa, wl3.pb)
        pa = torch.cat([tpa, tpa[:1]])
        pb = torch.cat([tpb, tpb[:1]])
        out = torch.zeros(LIMIT + 1, dtype=torch.int64, device=pa.device)
        with pytest.raises(sccg.SccgError) as e:
            ctx.area_pairs_noalloc(dA, dB, pa, pb, out, out.clone())
        assert e.value.code == sccg.SCCG_E_ARG and "limit" in str(e.value)
        # the context stays usable
        rI, rU, nI, nU = _both(ctx, (dA, dB, tpa, tpb), 1000)
        assert_exact(nI, nU, rI, rU, "no-allocation entry point after a rejected call")
    finally:
        ctx.close()

"""Device parity: every count of both kernels equals the oracle (or a closed
form) exactly, across workloads, tuning parameters and edge cases.  All calls
go through the C ABI."""

import numpy as np
import pytest

import oracle
import paper_1208_0277_amd as sccg
import sccg_gen
from sccg_gen import Polys, concat
from tests.gpu_util import assert_exact, device_workload, graph_context, run, run_graph
from tests.shapes import (band_rects, band_ring, comb_pairs, limit_cases, random_bands, rect_ring, rects_area,
                          rects_inter, staircase, transform)

pytestmark = pytest.mark.gpu

MODES = [sccg.SCCG_PLAIN, sccg.SCCG_BATCHED]


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.nodeid}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = sccg.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def wl1():
    wl = sccg_gen.pairs(1)
    I, U = oracle.area_pairs(wl.A, wl.B, wl.pa, wl.pb)
    return wl, I, U


@pytest.mark.parametrize("mode", MODES)
def test_config1_full(ctx, wl1, mode):
    wl, eI, eU = wl1
    gI, gU = run(ctx, device_workload(wl.A, wl.B, wl.pa, wl.pb), mode)
    assert_exact(gI, gU, eI, eU, f"workload 1 mode {mode}")


@pytest.mark.parametrize("mode", MODES)
def test_band_polygons_closed_form(ctx, mode):
    rng = np.random.default_rng(5)
    ra, rb, expect = [], [], []
    for t in range(2000):
        nb = int(rng.integers(1, 14))
        ring_a, rects_a = random_bands(rng, nb, span=int(rng.integers(8, 200)), hmax=int(rng.integers(1, 30)))
        ring_b, rects_b = random_bands(rng, int(rng.integers(1, 14)), x0=int(rng.integers(-20, 20)),
                                       y0=int(rng.integers(-20, 60)), span=int(rng.integers(8, 200)),
                                       hmax=int(rng.integers(1, 30)))
        sx, sy = (1 if rng.random() < 0.5 else -1), (1 if rng.random() < 0.5 else -1)
        sw = bool(rng.random() < 0.5)
        k = int(rng.choice([1, 1, 1, 2, 7]))
        dx, dy = (int(v) for v in rng.integers(-100000, 100000, 2))
        ring_a, rects_a = transform(ring_a, rects_a, sx, sy, sw, dx, dy, k)
        ring_b, rects_b = transform(ring_b, rects_b, sx, sy, sw, dx, dy, k)
        ra.append(ring_a)
        rb.append(ring_b)
        i = rects_inter(rects_a, rects_b)
        expect.append((i, rects_area(rects_a) + rects_area(rects_b) - i))
    A, B = concat(ra), concat(rb)
    idx = np.arange(len(ra), dtype=np.int32)
    gI, gU = run(ctx, device_workload(A, B, idx, idx), mode)
    eI = np.array([e[0] for e in expect], np.int64)
    eU = np.array([e[1] for e in expect], np.int64)
    assert_exact(gI, gU, eI, eU, f"band polygons mode {mode}")


@pytest.mark.parametrize("k", [40, 300, 1000])
@pytest.mark.parametrize("mode", MODES)
def test_scaled_shapes_k_squared(ctx, wl1, k, mode):
    """Workload-1 shapes scaled by k (pair boxes up to ~32000 px, so 1-3 split
    levels): every count is k^2 times the oracle's unscaled count."""
    wl, eI, eU = wl1
    sel = np.arange(0, wl.n_pairs, 4 if k < 1000 else 25)
    As = Polys(wl.A.off, wl.A.xy * k)
    Bs = Polys(wl.B.off, wl.B.xy * k)
    # spread the pairs so that coordinates stay below 2^30
    pa, pb = wl.pa[sel], wl.pb[sel]
    if mode == sccg.SCCG_PLAIN and k >= 300:
        sel = sel[:20]  # the plain kernel tests every pixel of every leaf: keep it short
        pa, pb = pa[:20], pb[:20]
    gI, gU = run(ctx, device_workload(As, Bs, pa, pb), mode)
    assert_exact(gI, gU, k * k * eI[sel], k * k * eU[sel], f"scale {k} mode {mode}")


@pytest.fixture(scope="module")
def tiny():
    from tests.test_oracle import _bits, _valid_4x4_masks
    masks = _valid_4x4_masks()
    rings = [sccg_gen.trace_mask(_bits(m)) for m in masks]
    rng = np.random.default_rng(9)
    n = 40000
    ia = rng.integers(0, len(masks), n)
    ib = rng.integers(0, len(masks), n)
    sh = rng.integers(-4, 5, (n, 2)).astype(np.int32)
    A = concat(rings)
    B = concat([rings[j] + sh[t] for t, j in enumerate(ib)])
    pa = ia.astype(np.int32)
    pb = np.arange(n, dtype=np.int32)
    I, U = oracle.area_pairs(A, B, pa, pb)
    return A, B, pa, pb, I, U


@pytest.mark.parametrize("mode", MODES)
def test_tiny_grid_pairs(ctx, tiny, mode):
    A, B, pa, pb, eI, eU = tiny
    gI, gU = run(ctx, device_workload(A, B, pa, pb), mode)
    assert_exact(gI, gU, eI, eU, f"tiny grid mode {mode}")


@pytest.fixture(scope="module")
def wl3s():
    wl = sccg_gen.pairs(3, 60000)
    I, U = oracle.area_pairs(wl.A, wl.B, wl.pa, wl.pb, form=oracle.ROWS)
    return wl, I, U


@pytest.mark.parametrize("mode", MODES)
def test_config3_subset(ctx, wl3s, mode):
    wl, eI, eU = wl3s
    gI, gU = run(ctx, device_workload(wl.A, wl.B, wl.pa, wl.pb), mode)
    assert_exact(gI, gU, eI, eU, f"heavy-tailed mix (60k pairs) mode {mode}")


def test_config3_full_size():
    """The whole 2,000,000-pair heavy-tailed mix in one persistent launch with
    the parameters of the committed headline profile, through the captured
    HIP graph: every pair's counts equal the oracle's (row-bucketed form, all
    host threads)."""
    import json
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    import bench
    with open(os.path.join(root, "profiles", bench.PROFILE_STEMS[3] + ".json")) as f:
        params = json.load(f)["params"]
    wl = sccg_gen.pairs(3, 2_000_000)
    print(f"[gpu] generated {len(wl.pa)} pairs, params {params}", flush=True)
    c = graph_context(**params)
    try:
        gI, gU = run_graph(c, device_workload(wl.A, wl.B, wl.pa, wl.pb))
    finally:
        c.close()
    eI, eU = oracle.area_pairs(wl.A, wl.B, wl.pa, wl.pb, form=oracle.ROWS, threads=min(os.cpu_count() or 1, 16))
    assert_exact(gI, gU, eI, eU, "heavy-tailed mix, 2,000,000 pairs, headline parameters")


@pytest.mark.parametrize("mode", MODES)
def test_config2_full_size(ctx, mode):
    """The whole 200,000-pair uniform workload (the plain kernel's baseline
    set) in both modes: every pair equals the oracle.  BATCHED runs through
    the captured graph, PLAIN on the null stream."""
    import os
    wl = sccg_gen.pairs(2, 200_000)
    dwl = device_workload(wl.A, wl.B, wl.pa, wl.pb)
    if mode == sccg.SCCG_BATCHED:
        c = graph_context()
        try:
            gI, gU = run_graph(c, dwl)
        finally:
            c.close()
    else:
        gI, gU = run(ctx, dwl, mode)
    eI, eU = oracle.area_pairs(wl.A, wl.B, wl.pa, wl.pb, form=oracle.ROWS, threads=min(os.cpu_count() or 1, 16))
    assert_exact(gI, gU, eI, eU, f"uniform workload, 200,000 pairs, mode {mode}")


def test_config4_full_size():
    """Workload 4 at its full size (64 tiles of 8192 x 8192, the grid-join
    candidates in one launch through the captured graph), with the union
    sweep leaving pair boxes to the medium sweep and counting them itself:
    every pair and every tile's sums, J and J' equal the oracle."""
    import os
    import torch
    wl = sccg_gen.sets(n_tiles=64, tile_side=8192, cell=64)
    print(f"[gpu] generated {wl.n_pairs} pairs in {len(wl.set_off) - 1} tiles", flush=True)
    dwl = device_workload(wl.A, wl.B, wl.pa, wl.pb)
    so = torch.from_numpy(wl.set_off).cuda()
    got = []
    for spb in (1, 2):
        c = graph_context(sweep_pair_box=spb)
        try:
            gI, gU = run_graph(c, dwl)
            I, U = torch.from_numpy(gI).cuda(), torch.from_numpy(gU).cuda()
            torch.cuda.synchronize()
            with torch.cuda.stream(c.stream):
                sets = c.jaccard_sets(so, I, U)
            c.sync()
            got.append((spb, gI, gU, [t.cpu().numpy() for t in sets]))
        finally:
            c.close()
    eI, eU = oracle.area_pairs(wl.A, wl.B, wl.pa, wl.pb, form=oracle.ROWS, threads=min(os.cpu_count() or 1, 16))
    osi, osu, onn, oj, ojp = oracle.jaccard_sets(wl.set_off, eI, eU)
    for spb, gI, gU, (si, su, nn, j, jp) in got:
        assert_exact(gI, gU, eI, eU, f"set workload, 64 tiles, sweep_pair_box {spb}")
        assert np.array_equal(si, osi) and np.array_equal(su, osu)
        assert np.array_equal(nn, onn)
        assert np.array_equal(j, oj) and np.array_equal(jp, ojp)


PLAIN_TUNINGS = [
    dict(box_threshold=64), dict(box_threshold=512), dict(box_threshold=8192), dict(box_threshold=2),
    dict(wg_size=128), dict(wg_size=256), dict(wg_size=256, box_threshold=100000),
    dict(split_gx=16, split_gy=4), dict(lds_vertex_cap=1), dict(grid=7),
]


@pytest.mark.parametrize("params", PLAIN_TUNINGS, ids=[str(p) for p in PLAIN_TUNINGS])
def test_plain_tuning_invariance(wl3s, params):
    wl, eI, eU = wl3s
    sel = np.concatenate([np.nonzero(wl.blob)[0][:40], np.arange(0, wl.n_pairs, 97)])
    c = sccg.Context(0, **params)
    gI, gU = run(c, device_workload(wl.A, wl.B, wl.pa[sel], wl.pb[sel]), sccg.SCCG_PLAIN)
    c.close()
    assert_exact(gI, gU, eI[sel], eU[sel], f"plain {params}")


def with_pair_box_sweep(ctx, mode):
    """ctx, then for BATCHED a context whose union sweep also counts pair
    boxes (closed when the caller's loop ends)."""
    yield ctx
    if mode == sccg.SCCG_BATCHED:
        c = sccg.Context(0, sweep_pair_box=2)
        try:
            yield c
        finally:
            c.close()


BATCH_TUNINGS = [
    dict(queue_cap=1), dict(queue_cap=3, min_queue_cells=1), dict(min_queue_cells=1), dict(min_queue_cells=65),
    dict(flags=sccg.SCCG_F_NO_SPLIT_QUEUE), dict(flags=sccg.SCCG_F_NO_KNOWN_INSIDE),
    dict(flags=sccg.SCCG_F_NO_LPT), dict(flags=sccg.SCCG_F_NO_GRAPH), dict(queue_chunk=1), dict(queue_chunk=64), dict(queue_chunk=37),
    dict(waves_per_wg=1), dict(waves_per_wg=8), dict(n_queues=1), dict(grid=3), dict(heavy_verts=1),
    dict(heavy_verts=1, min_queue_cells=1, queue_cap=50), dict(heavy_verts=100000),
    dict(min_classify_cells=1), dict(min_classify_cells=65), dict(flags=sccg.SCCG_F_NO_UNION_TILE), dict(min_classify_cells=65, heavy_verts=1, min_queue_cells=1),
    dict(flags=sccg.SCCG_F_NO_SEP), dict(flags=sccg.SCCG_F_PIXEL_ONLY),
    dict(flags=sccg.SCCG_F_NO_SEP, heavy_verts=1, min_queue_cells=1),
    dict(flags=sccg.SCCG_F_PIXEL_ONLY | sccg.SCCG_F_NO_KNOWN_INSIDE, heavy_verts=1, min_queue_cells=1),
    dict(sweep_pair_box=2), dict(sweep_pair_box=2, flags=sccg.SCCG_F_NO_UNION_TILE),
    dict(sweep_pair_box=2, queue_chunk=1, flags=sccg.SCCG_F_NO_GRAPH), dict(sweep_pair_box=2, flags=sccg.SCCG_F_NO_SEP),
    dict(sweep_pair_box=2, flags=sccg.SCCG_F_PIXEL_ONLY),
]


@pytest.mark.parametrize("params", BATCH_TUNINGS, ids=[str(p) for p in BATCH_TUNINGS])
def test_batched_tuning_invariance(wl3s, params):
    """Every tuning of BATCHED mode gives the oracle's counts, through the
    captured graph (eager launches with SCCG_F_NO_GRAPH)."""
    wl, eI, eU = wl3s
    c = graph_context(**params)
    try:
        graph = not (params.get("flags", 0) & sccg.SCCG_F_NO_GRAPH)
        gI, gU = run_graph(c, device_workload(wl.A, wl.B, wl.pa, wl.pb), expect_graph=graph)
        if not graph:
            assert c.graph_launches() == 0
    finally:
        c.close()
    assert_exact(gI, gU, eI, eU, f"batched {params}")


def test_reserve_after_capture_recaptures(wl3s):
    """Growing the scratch after a graph was captured frees the buffers the
    graph's kernels point at: the next call must capture again and still
    equal the oracle.  Changing the queue layout (same slot total, other
    split between queues) must not leave stale task words behind."""
    wl, eI, eU = wl3s
    import torch
    sel = np.arange(0, wl.n_pairs, 3)
    dwl = device_workload(wl.A, wl.B, wl.pa[sel], wl.pb[sel])
    # the same output tensors every time, so that only the scratch changes
    out = (torch.empty(len(sel), dtype=torch.int64, device="cuda"),
           torch.empty(len(sel), dtype=torch.int64, device="cuda"))
    c = graph_context(heavy_verts=1, min_queue_cells=1, n_queues=2, queue_cap=4096)
    try:
        gI, gU = run_graph(c, dwl, out=out)
        assert_exact(gI, gU, eI[sel], eU[sel], "first captured call")
        c.reserve(wl.A.n, wl.B.n, 40 * len(sel))  # reallocates the pair scratch
        gI, gU = run_graph(c, dwl, out=out)
        assert_exact(gI, gU, eI[sel], eU[sel], "after reserve")
        gI, gU = run_graph(c, dwl, out=out)
        assert_exact(gI, gU, eI[sel], eU[sel], "replay after reserve")
        c.set_params(heavy_verts=1, min_queue_cells=1, n_queues=4, queue_cap=2048)
        gI, gU = run_graph(c, dwl, out=out)
        assert_exact(gI, gU, eI[sel], eU[sel], "after a queue layout change")
        c.set_params(heavy_verts=1, min_queue_cells=1, n_queues=2, queue_cap=4096)
        gI, gU = run_graph(c, dwl, out=out)
        assert_exact(gI, gU, eI[sel], eU[sel], "after the layout changed back")
    finally:
        c.close()


@pytest.mark.parametrize("mode", MODES)
def test_shuffled_and_repeated_pairs(ctx, wl1, mode):
    wl, eI, eU = wl1
    rng = np.random.default_rng(3)
    perm = rng.permutation(np.concatenate([np.arange(wl.n_pairs)] * 3))
    gI, gU = run(ctx, device_workload(wl.A, wl.B, wl.pa[perm], wl.pb[perm]), mode)
    assert_exact(gI, gU, eI[perm], eU[perm], f"shuffled mode {mode}")


def test_graph_replays_match_eager(wl3s):
    """The batched sequence is captured once and replayed; every replay, with
    eager device work in between, gives the same counts."""
    import torch
    wl, eI, eU = wl3s
    c = sccg.Context(0, stream=torch.cuda.Stream())
    dwl = device_workload(wl.A, wl.B, wl.pa, wl.pb)
    I = torch.empty(wl.n_pairs, dtype=torch.int64, device="cuda")
    U = torch.empty(wl.n_pairs, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    for rep in range(4):
        I.fill_(-1)
        U.fill_(-1)
        torch.cuda.synchronize()
        with torch.cuda.stream(c.stream):
            c.area_pairs(*dwl, out_inter=I, out_union=U, mode=sccg.SCCG_BATCHED)
        c.sync()
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        assert_exact(I.cpu().numpy(), U.cpu().numpy(), eI, eU, f"replay {rep}")
        del junk
    c.close()


@pytest.mark.parametrize("mode", MODES)
def test_degenerate_rings(ctx, mode):
    sq = band_ring([0, 5], [0], [5])
    dup = np.concatenate([sq, sq[:1], sq[:1]])          # repeated closing vertex twice
    col = np.array([[0, 0], [2, 0], [5, 0], [5, 3], [5, 5], [0, 5]], np.int32)  # collinear points
    far = sq + np.array([1000, 0], np.int32)             # disjoint: empty pair box
    touch = sq + np.array([5, 0], np.int32)              # shares an edge only
    corner = sq + np.array([5, 5], np.int32)             # shares a corner only
    A = concat([sq, dup, col, sq, sq, sq])
    B = concat([dup, col, sq, far, touch, corner])
    idx = np.arange(6, dtype=np.int32)
    gI, gU = run(ctx, device_workload(A, B, idx, idx), mode)
    assert gI.tolist() == [25, 25, 25, 0, 0, 0]
    assert gU.tolist() == [25, 25, 25, 50, 50, 50]


def _redundant(ring, rng, n_extra):
    """The same polygon with n_extra redundant vertices: edge midpoints
    (collinear points on vertical or horizontal runs) and repeated vertices."""
    r = [tuple(v) for v in ring]
    for _ in range(n_extra):
        k = int(rng.integers(0, len(r)))
        a, b = r[k], r[(k + 1) % len(r)]
        if rng.random() < 0.5 and abs(a[0] - b[0]) + abs(a[1] - b[1]) >= 2:
            r.insert(k + 1, ((a[0] + b[0]) // 2, (a[1] + b[1]) // 2))
        else:
            r.insert(k + 1, a)
    return np.array(r, np.int32)


@pytest.mark.parametrize("mode", MODES)
def test_redundant_vertices(ctx, mode):
    """Rings with collinear and repeated vertices (every vertex is then not a
    corner), sized so that the extra vertices fall at 64-vertex chunk
    boundaries of the sweep's registers (63, 64, 65, 127, 128, 129 vertices
    and more): counts equal the oracle's and those of the clean rings."""
    wl = sccg_gen.pairs(3, 3000)
    rng = np.random.default_rng(17)
    ra, rb, pa_clean, pb_clean = [], [], [], []
    for i in range(wl.n_pairs):
        a, b = wl.A.ring(wl.pa[i]), wl.B.ring(wl.pb[i])
        if len(a) > 200 or len(b) > 200:
            continue
        ta = int(rng.choice([len(a) + 1, 63, 64, 65, 127, 128, 129, len(a) + 40]))
        tb = int(rng.choice([len(b) + 1, 63, 64, 65, 127, 128, 129, len(b) + 40]))
        ra.append(_redundant(a, rng, max(1, ta - len(a))))
        rb.append(_redundant(b, rng, max(1, tb - len(b))))
        pa_clean.append(wl.pa[i])
        pb_clean.append(wl.pb[i])
    A, B = concat(ra), concat(rb)
    idx = np.arange(len(ra), dtype=np.int32)
    eI, eU = oracle.area_pairs(A, B, idx, idx, form=oracle.ROWS)
    cI, cU = oracle.area_pairs(wl.A, wl.B, np.array(pa_clean, np.int32), np.array(pb_clean, np.int32),
                               form=oracle.ROWS)
    assert np.array_equal(eI, cI) and np.array_equal(eU, cU)
    if mode == sccg.SCCG_PLAIN:
        idx = idx[:300]
        eI, eU = eI[:300], eU[:300]
    gI, gU = run(ctx, device_workload(A, B, idx, idx), mode)
    assert_exact(gI, gU, eI, eU, f"redundant vertices mode {mode}")


def _boundary_pairs(seed=23, n=400):
    """Band-polygon pairs sitting on BATCHED mode's class boundaries: union
    boxes of 31-33 and 63-65 pixels a side (the union tile, its halves, the
    medium sweep), rings padded to 64, 65, 128, 129, 256 and 257 vertices,
    and some pairs of 255 + 256 and 256 + 256 vertices (heavy_verts 512).
    Returns the rings and the closed-form counts."""
    rng = np.random.default_rng(seed)
    targets = {31, 32, 33, 63, 64, 65}
    sizes = [0, 64, 65, 128, 129, 256, 257]
    ra, rb, expect = [], [], []
    while len(ra) < n:
        def stair():
            nb = int(rng.integers(1, 5))
            w = int(rng.integers(8, 60))
            return staircase(nb, int(rng.integers(8, 70)), int(rng.integers(0, w)), w)
        (ya, aa, ba), (yb, ab, bb) = stair(), stair()
        dx, dy = (int(v) for v in rng.integers(-12, 13, 2))
        yb, ab, bb = [y + dy for y in yb], [x + dx for x in ab], [x + dx for x in bb]
        ux = max(max(ba), max(bb)) - min(min(aa), min(ab))
        uy = max(ya[-1], yb[-1]) - min(ya[0], yb[0])
        if ux not in targets and uy not in targets and rng.random() < 0.9:
            continue
        ring_a, rects_a = band_ring(ya, aa, ba), band_rects(ya, aa, ba)
        ring_b, rects_b = band_ring(yb, ab, bb), band_rects(yb, ab, bb)
        if rng.random() < 0.1:
            na, nq = 256, int(rng.choice([255, 256]))
        else:
            na, nq = int(rng.choice(sizes)), int(rng.choice(sizes))
        if na > len(ring_a):
            ring_a = _redundant(ring_a, rng, na - len(ring_a))
        if nq > len(ring_b):
            ring_b = _redundant(ring_b, rng, nq - len(ring_b))
        sx, sy = (1 if rng.random() < 0.5 else -1), (1 if rng.random() < 0.5 else -1)
        sw = bool(rng.random() < 0.5)
        tx, ty = (int(v) for v in rng.integers(-50000, 50000, 2))
        ring_a, rects_a = transform(ring_a, rects_a, sx, sy, sw, tx, ty, 1)
        ring_b, rects_b = transform(ring_b, rects_b, sx, sy, sw, tx, ty, 1)
        ra.append(np.asarray(ring_a, np.int32))
        rb.append(np.asarray(ring_b, np.int32))
        i = rects_inter(rects_a, rects_b)
        expect.append((i, rects_area(rects_a) + rects_area(rects_b) - i))
    return ra, rb, expect


@pytest.mark.parametrize("case", ["plain", "batched", "batched_heavy64", "batched_pair_box", "batched_pair_box_only"])
def test_class_boundaries(case):
    """Counts at every class boundary of BATCHED mode equal the closed form
    (and the oracle), in both modes, with heavy_verts moved to 64, and with
    the union sweep counting pair boxes (alone: without the union tile)."""
    ra, rb, expect = _boundary_pairs()
    A, B = concat(ra), concat(rb)
    idx = np.arange(len(ra), dtype=np.int32)
    eI = np.array([e[0] for e in expect], np.int64)
    eU = np.array([e[1] for e in expect], np.int64)
    oI, oU = oracle.area_pairs(A, B, idx, idx, form=oracle.ROWS)
    assert np.array_equal(oI, eI) and np.array_equal(oU, eU)
    kw = {"batched_heavy64": dict(heavy_verts=64), "batched_pair_box": dict(sweep_pair_box=2),
          "batched_pair_box_only": dict(sweep_pair_box=2, flags=sccg.SCCG_F_NO_UNION_TILE)}.get(case, {})
    c = sccg.Context(0, **kw)
    try:
        mode = sccg.SCCG_PLAIN if case == "plain" else sccg.SCCG_BATCHED
        gI, gU = run(c, device_workload(A, B, idx, idx), mode)
    finally:
        c.close()
    assert_exact(gI, gU, eI, eU, f"class boundaries ({case})")


def _comb(width, height, base, tooth, gap):
    """A comb: `base` full rows, then teeth `tooth` px wide every
    tooth + gap px up to `height`: many vertical edges in every 64-row band."""
    m = np.zeros((height, width), np.uint8)
    m[:base, :] = 1
    for x in range(0, width, tooth + gap):
        m[base:, x:x + tooth] = 1
    ring = sccg_gen.trace_mask(m)
    assert ring is not None
    return ring


@pytest.mark.parametrize("mode", MODES)
def test_dense_band_rows(ctx, mode):
    """Rings with more vertical edges in one 64-row band than a band list
    holds (the per-tile path takes over), rows of several leaf tiles, and
    tiles known to lie inside one polygon; counts equal the oracle's."""
    comb = _comb(520, 150, 8, 2, 2)          # about 260 vertical edges per band
    sparse = _comb(520, 150, 8, 2, 30)       # a few dozen per band
    rect = band_ring([20, 130], [40], [480])
    big = band_ring([-10, 200], [-10], [600])
    A = concat([comb, comb, comb, sparse, sparse, comb])
    B = concat([comb + np.array([1, 3], np.int32), rect, big, sparse + np.array([5, -2], np.int32), rect, sparse])
    idx = np.arange(6, dtype=np.int32)
    eI, eU = oracle.area_pairs(A, B, idx, idx, form=oracle.ROWS)
    gI, gU = run(ctx, device_workload(A, B, idx, idx), mode)
    assert_exact(gI, gU, eI, eU, f"dense band rows mode {mode}")


@pytest.mark.parametrize("bad", [dict(sweep_pair_box=3), dict(sweep_pair_box=-1), dict(min_classify_cells=66),
                                 dict(queue_chunk=65), dict(waves_per_wg=9), dict(wg_size=96)])
def test_parameter_ranges(ctx, bad):
    """A tuning value outside its documented range is refused with
    SCCG_E_ARG, at creation and by set_params (which keeps the old values)."""
    with pytest.raises(sccg.SccgError) as e:
        sccg.Context(0, **bad)
    assert e.value.code == sccg.SCCG_E_ARG
    before = ctx.get_params()
    with pytest.raises(sccg.SccgError) as e:
        ctx.set_params(**bad)
    assert e.value.code == sccg.SCCG_E_ARG
    assert ctx.get_params() == before


@pytest.mark.parametrize("mode", MODES)
def test_empty_call_and_argument_errors(ctx, wl1, mode):
    import torch
    wl, _, _ = wl1
    dA, dB, tpa, tpb = device_workload(wl.A, wl.B, wl.pa, wl.pb)
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    I, U = ctx.area_pairs(dA, dB, e, e, mode=mode)  # n = 0: nothing queued
    assert I.numel() == 0
    lib = sccg.load_library()
    ca = dA.c()
    rc = lib.sccg_area_pairs(ctx.h, None, None, 1, None, None, None, None, mode)
    assert rc == sccg.SCCG_E_ARG
    rc = lib.sccg_area_pairs(ctx.h, __import__("ctypes").byref(ca), __import__("ctypes").byref(ca), -1,
                             None, None, None, None, mode)
    assert rc == sccg.SCCG_E_ARG
    rc = lib.sccg_area_pairs(ctx.h, __import__("ctypes").byref(ca), __import__("ctypes").byref(ca), 1,
                             None, None, None, None, 7)
    assert rc == sccg.SCCG_E_ARG
    assert ctx.sync_code() == sccg.SCCG_OK


@pytest.mark.parametrize("mode", MODES)
def test_range_errors_latch_and_zero(ctx, mode):
    sq = band_ring([0, 5], [0], [5])
    big = band_ring([0, 40000], [0], [40000])           # pair box side 40000 > 32767
    huge = sq + np.array([1 << 30, 0], np.int32)          # x beyond 2^30
    A = concat([sq, big, huge])
    B = concat([sq, big, sq])
    # pair 0 fine; pair 1 side too large; pair 2 coordinate out of range; pair 3 index out of range
    pa = np.array([0, 1, 2, 5], np.int32)
    pb = np.array([0, 1, 2, 0], np.int32)
    dwl = device_workload(A, B, pa, pb)
    # BATCHED also with the union sweep counting pair boxes (where the side
    # and coordinate checks then run)
    ctxs = [ctx] + ([sccg.Context(0, sweep_pair_box=2)] if mode == sccg.SCCG_BATCHED else [])
    for c in ctxs:
        I, U = c.area_pairs(*dwl, mode=mode)
        assert c.sync_code() == sccg.SCCG_E_RANGE
        assert c.sync_code() == sccg.SCCG_OK  # latched error is cleared by the sync that reports it
        gI, gU = I.cpu().numpy(), U.cpu().numpy()
        assert gI.tolist() == [25, 0, 0, 0]
        assert gU.tolist()[0] == 25 and gU.tolist()[1] == 0 and gU.tolist()[3] == 0
        assert gU.tolist()[2] == 25  # the rejected polygon counts as empty
    for c in ctxs[1:]:
        c.close()


@pytest.mark.parametrize("mode", MODES)
def test_wide_rings_exact_areas(ctx, mode):
    """Rings whose extent reaches 2^14 or more on an axis take the 64-bit
    area path; each is paired with a small ring so that the pair box stays in
    range.  Counts are closed forms of band rectangles."""
    sq = lambda x, y, s: ([y, y + s], [x], [x + s])
    cases = [
        (([0, 10], [0], [20000]), sq(100, -5, 30)),                # 20000 x 10 band
        (staircase(150, 30000, 200, 1000), sq(15100, 15050, 50)),  # 600 vertices, 30800 x 30000
        (staircase(300, 30000, 100, 2000), sq(15100, 15050, 50)),  # 1200 vertices (heavy pair)
        (([-(1 << 29), 1 << 29], [-(1 << 29)], [1 << 29]), sq(7, -3, 10)),  # twice its area needs 62 bits
        (staircase(150, 30000, 200, 1000), sq(29000, 100, 40)),    # wide ring, no common pixel
    ]
    rings_a, rings_b, expect = [], [], []
    for pa_b, pb_b in cases:
        rings_a.append(band_ring(*pa_b))
        rings_b.append(band_ring(*pb_b))
        ra, rb = band_rects(*pa_b), band_rects(*pb_b)
        i = rects_inter(ra, rb)
        expect.append((i, rects_area(ra) + rects_area(rb) - i))
    A, B = concat(rings_a), concat(rings_b)
    idx = np.arange(len(cases), dtype=np.int32)
    for c in with_pair_box_sweep(ctx, mode):
        I, U = c.area_pairs(*device_workload(A, B, idx, idx), mode=mode)
        assert c.sync_code() == sccg.SCCG_OK
        got = list(zip(I.cpu().numpy().tolist(), U.cpu().numpy().tolist()))
        assert got == expect, f"params {c.get_params()}"


@pytest.mark.parametrize("mode", MODES)
def test_coordinates_at_the_limit(ctx, mode):
    """Rectangles reaching |coordinate| = 2^30 paired with small ones at the
    opposite extreme: a coordinate minus a box side reaches 2^31 in the leaf,
    band-row and classification paths, a union box is 2^31 wide, and one ring
    has twice its area equal to 2^63.  q lies inside p: I = |q|, U = |p|."""
    cases = limit_cases()
    A, B = concat([rect_ring(p) for p, _ in cases]), concat([rect_ring(q) for _, q in cases])
    area = lambda r: (r[2] - r[0]) * (r[3] - r[1])
    idx = np.arange(len(cases), dtype=np.int32)
    for c in with_pair_box_sweep(ctx, mode):
        I, U = c.area_pairs(*device_workload(A, B, idx, idx), mode=mode)
        assert c.sync_code() == sccg.SCCG_OK
        got = list(zip(I.cpu().numpy().tolist(), U.cpu().numpy().tolist()))
        assert got == [(area(q), area(p)) for p, q in cases], f"params {c.get_params()}"


@pytest.mark.parametrize("mode", MODES)
def test_full_range_pair_box_is_rejected(mode):
    """Two rings spanning [-2^30, 2^30] make a pair box 2^31 wide: beyond the
    32767 limit, so the call reports SCCG_E_RANGE."""
    M = 1 << 30
    A = concat([rect_ring((-M, 0, M, 10))])
    B = concat([rect_ring((-M, 5, M, 20))])
    idx = np.zeros(1, np.int32)
    c = sccg.Context(0)
    try:
        c.area_pairs(*device_workload(A, B, idx, idx), mode=mode)
        assert c.sync_code() == sccg.SCCG_E_RANGE
    finally:
        c.close()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("flags", [0, sccg.SCCG_F_NO_UNION_TILE])
def test_comb_band_rows(mode, flags):
    """Combs whose 64-row bands meet 300 and 640 vertical edges: band lists
    that overflow their share of the staging list, are staged again one row at
    a time, and (640 edges) fall back to scattering from the rings; with and
    without cell classification.  Counts are closed forms."""
    cases = comb_pairs(150, 300) + comb_pairs(320, 200)
    A, B = concat([k[0] for k in cases]), concat([k[1] for k in cases])
    idx = np.arange(len(cases), dtype=np.int32)
    for mcc, spb in ((1, 1), (26, 1), (65, 1), (26, 2)):
        c = sccg.Context(0, flags=flags, min_classify_cells=mcc, sweep_pair_box=spb)
        try:
            I, U = c.area_pairs(*device_workload(A, B, idx, idx), mode=mode)
            assert c.sync_code() == sccg.SCCG_OK
            got = list(zip(I.cpu().numpy().tolist(), U.cpu().numpy().tolist()))
        finally:
            c.close()
        assert got == [(k[2], k[3]) for k in cases], f"min_classify_cells {mcc}, sweep_pair_box {spb}"


def _stair_bands(n_bands, x0, y0, width, step=1, h=1):
    """Bands of a staircase whose ring has 4 * n_bands vertices (band_ring
    keeps every corner): band k is [x0 + step*k, x0 + step*k + width) x
    [y0 + h*k, y0 + h*k + h)."""
    y = [y0 + h * k for k in range(n_bands + 1)]
    a = [x0 + step * k for k in range(n_bands)]
    return y, a, [v + width for v in a]


@pytest.mark.parametrize("mode", MODES)
def test_tile_and_chunk_boundaries(ctx, mode):
    """Union boxes of width and height 63..65 around the one-tile limit and
    the 32-row mask switch, and rings of 16, 17, 32, 33 bands (64, 68, 128,
    132 vertices) around the register chunks: counts equal closed forms."""
    rng = np.random.default_rng(31)
    cases = []
    for uw in (31, 32, 33, 63, 64, 65):
        for uh in (32, 33, 64, 65):
            # p: [0, uw - 5) x [0, uh - 3); q: [5, uw) x [3, uh): union exactly uw x uh
            cases.append((([0, uh - 3], [0], [uw - 5]), ([3, uh], [5], [uw])))
    for nb in (16, 17, 32, 33):
        for dx in (0, 7, 40):
            cases.append((_stair_bands(nb, 0, 0, 20, 1, 1), _stair_bands(nb, dx, 2, 15, 1, 1)))
    for _ in range(20):
        nb_p, nb_q = int(rng.integers(1, 40)), int(rng.integers(1, 40))
        cases.append((_stair_bands(nb_p, 0, 0, int(rng.integers(3, 40)), int(rng.integers(0, 2)), 1),
                      _stair_bands(nb_q, int(rng.integers(-10, 30)), int(rng.integers(-10, 30)),
                                   int(rng.integers(3, 40)), int(rng.integers(0, 2)), int(rng.integers(1, 3)))))
    rings_a, rings_b, expect = [], [], []
    for pb_, qb_ in cases:
        rings_a.append(band_ring(*pb_))
        rings_b.append(band_ring(*qb_))
        ra, rb = band_rects(*pb_), band_rects(*qb_)
        i = rects_inter(ra, rb)
        expect.append((i, rects_area(ra) + rects_area(rb) - i))
    A, B = concat(rings_a), concat(rings_b)
    assert {4 * 16, 4 * 17, 4 * 32, 4 * 33} <= set(np.diff(A.off).tolist())
    idx = np.arange(len(cases), dtype=np.int32)
    for flags, spb in ((0, 1), (sccg.SCCG_F_NO_UNION_TILE, 1), (0, 2), (sccg.SCCG_F_NO_UNION_TILE, 2)):
        c = sccg.Context(0, flags=flags, sweep_pair_box=spb) if mode == sccg.SCCG_BATCHED else ctx
        I, U = c.area_pairs(*device_workload(A, B, idx, idx), mode=mode)
        assert c.sync_code() == sccg.SCCG_OK
        got = list(zip(I.cpu().numpy().tolist(), U.cpu().numpy().tolist()))
        if c is not ctx:
            c.close()
        assert got == expect, f"flags {flags}, sweep_pair_box {spb}"


def test_validate_polys(ctx):
    sq = band_ring([0, 5], [0], [5])
    diag = np.array([[0, 0], [5, 0], [5, 5], [1, 4]], np.int32)
    tri = np.array([[0, 0], [5, 0], [5, 5]], np.int32)
    P = concat([sq, sq, diag, sq, tri])
    dP = sccg.DevicePolys.from_host(P.off, P.xy)
    out = ctx.validate_polys(dP)
    ctx.sync()
    assert int(out.item()) == 2
    Q = concat([sq, sq])
    out = ctx.validate_polys(sccg.DevicePolys.from_host(Q.off, Q.xy))
    ctx.sync()
    assert int(out.item()) == -1


@pytest.mark.parametrize("include_zero", [False, True])
def test_jaccard_sets(ctx, wl3s, include_zero):
    import torch
    wl, eI, eU = wl3s
    rng = np.random.default_rng(2)
    cuts = np.sort(rng.integers(0, wl.n_pairs, 30))
    so = np.concatenate([[0], cuts, cuts[-1:], [wl.n_pairs]]).astype(np.int64)  # includes an empty set
    tI = torch.from_numpy(eI).cuda()
    tU = torch.from_numpy(eU).cuda()
    tso = torch.from_numpy(so).cuda()
    flags = sccg.SCCG_J_INCLUDE_ZERO if include_zero else sccg.SCCG_J_NONZERO_ONLY
    si, su, nn, j, jp = ctx.jaccard_sets(tso, tI, tU, flags=flags)
    ctx.sync()
    osi, osu, onn, oj, ojp = oracle.jaccard_sets(so, eI, eU, include_zero=include_zero)
    assert np.array_equal(si.cpu().numpy(), osi)
    assert np.array_equal(su.cpu().numpy(), osu)
    assert np.array_equal(nn.cpu().numpy(), onn)
    assert np.array_equal(j.cpu().numpy(), oj)       # bit-identical binary64
    assert np.array_equal(jp.cpu().numpy(), ojp)


@pytest.mark.parametrize("layout", ["one_set", "tiny_sets", "offset_start"])
def test_jaccard_sets_layouts(ctx, wl3s, layout):
    """Set sums against the oracle when one set spans every chunk of the
    pair range, when a chunk holds hundreds of sets, and when the first set
    starts past pair 0."""
    import torch
    wl, eI, eU = wl3s
    n = wl.n_pairs
    if layout == "one_set":
        so = np.array([0, n], np.int64)
    elif layout == "tiny_sets":
        so = np.concatenate([np.arange(0, n, 7), [n]]).astype(np.int64)
    else:
        so = np.array([12345, 12345, 20000, 40001, n - 3], np.int64)
    tI, tU = torch.from_numpy(eI).cuda(), torch.from_numpy(eU).cuda()
    si, su, nn, j, jp = ctx.jaccard_sets(torch.from_numpy(so).cuda(), tI, tU)
    ctx.sync()
    osi, osu, onn, oj, ojp = oracle.jaccard_sets(so, eI, eU)
    assert np.array_equal(si.cpu().numpy(), osi) and np.array_equal(su.cpu().numpy(), osu)
    assert np.array_equal(nn.cpu().numpy(), onn)
    assert np.array_equal(j.cpu().numpy(), oj) and np.array_equal(jp.cpu().numpy(), ojp)


@pytest.mark.parametrize("spb", [1, 2])
def test_batched_stats(wl3s, spb):
    """The kernel instances that keep work counters give the oracle's counts
    too, and the counters add up (each pair is small, large or empty)."""
    wl, eI, eU = wl3s
    c = sccg.Context(0, min_classify_cells=1, sweep_pair_box=spb)
    c.set_stats(True)
    gI, gU = run(c, device_workload(wl.A, wl.B, wl.pa, wl.pb), sccg.SCCG_BATCHED)
    s = c.get_stats()
    c.close()
    assert_exact(gI, gU, eI, eU, f"counters on, sweep_pair_box {spb}")
    assert s["small_pairs"] + s["large_pairs"] + s["empty_pairs"] == wl.n_pairs
    assert s["leaf_pixel_tests"] > 0 and s["leaf_boxes"] >= s["small_pairs"]
    assert s["large_pairs"] > 0 and s["split_boxes"] >= s["large_pairs"]
    assert s["leaf_edge_updates"] > 0 and s["classify_edge_visits"] > 0
    assert s["union_tile_vertices"] > 0 and s["ring_scan_vertices"] > 0


def test_wave_stamps(wl3s):
    """Every wave of the three batched kernels stamps a start and a later end;
    the kernels run in stream order."""
    import torch
    wl, _, _ = wl3s
    c = sccg.Context(0)
    assert len(c.wave_times(0)) == 0  # no call with stamps yet
    c.set_stats(False, stamps=True)
    run(c, device_workload(wl.A, wl.B, wl.pa, wl.pb), sccg.SCCG_BATCHED)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    spans = []
    for k in range(3):
        wt = c.wave_times(k)
        assert len(wt) >= cus, f"kernel {k}: {len(wt)} waves"
        assert (wt[:, 0] > 0).all() and (wt[:, 1] >= wt[:, 0]).all(), f"kernel {k}"
        spans.append((int(wt[:, 0].min()), int(wt[:, 1].max())))
    # the union sweep ends before the medium sweep starts, and so on
    assert spans[0][1] <= spans[1][0] and spans[1][1] <= spans[2][0], spans
    with pytest.raises(sccg.SccgError):
        c.wave_times(3)
    c.close()


def test_kernel_timing(wl3s):
    wl, _, _ = wl3s
    c = sccg.Context(0)
    c.set_timing(True)
    dwl = device_workload(wl.A, wl.B, wl.pa, wl.pb)
    for mode in MODES:
        for _ in range(2):
            run(c, dwl, mode)
        ms, n = c.get_timing()
        assert n == 2 and ms > 0
    c.close()


@pytest.fixture(scope="module")
def sets4():
    wl = sccg_gen.sets(n_tiles=4, tile_side=2048, cell=64)
    I, U = oracle.area_pairs(wl.A, wl.B, wl.pa, wl.pb, form=oracle.ROWS)
    return wl, I, U


@pytest.mark.parametrize("mode", MODES)
def test_set_workload_tiles(ctx, sets4, mode):
    """Workload 4 on four tiles: pair counts of the grid-join candidates and the
    per-tile J and J' bit-identical to the oracle."""
    import torch
    wl, eI, eU = sets4
    dwl = device_workload(wl.A, wl.B, wl.pa, wl.pb)
    I, U = ctx.area_pairs(*dwl, mode=mode)
    so = torch.from_numpy(wl.set_off).cuda()
    si, su, nn, j, jp = ctx.jaccard_sets(so, I, U)
    ctx.sync()
    assert_exact(I.cpu().numpy(), U.cpu().numpy(), eI, eU, f"set workload mode {mode}")
    osi, osu, onn, oj, ojp = oracle.jaccard_sets(wl.set_off, eI, eU)
    assert np.array_equal(si.cpu().numpy(), osi) and np.array_equal(su.cpu().numpy(), osu)
    assert np.array_equal(nn.cpu().numpy(), onn)
    assert np.array_equal(j.cpu().numpy(), oj) and np.array_equal(jp.cpu().numpy(), ojp)


def _dev_i64(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.int64)).to("cuda")


@pytest.mark.parametrize("cell", [64, 7, 1000])
def test_join_sets_equals_oracle(ctx, sets4, cell):
    """Filter stage on the device: the same pairs, in the same order, as the
    oracle's all-pairs test (and the generator's host grid join)."""
    wl, _, _ = sets4
    dA, dB, _, _ = device_workload(wl.A, wl.B, wl.pa, wl.pb)
    pa, pb, so = ctx.join_sets(dA, dB, _dev_i64(wl.a_set_off), _dev_i64(wl.b_set_off), cell=cell)
    ctx.sync()
    ea, eb, eso = oracle.join_sets(wl.A, wl.B, wl.a_set_off, wl.b_set_off)
    assert np.array_equal(pa.cpu().numpy(), ea) and np.array_equal(pb.cpu().numpy(), eb)
    assert np.array_equal(so.cpu().numpy(), eso)


def test_join_edge_cases_and_capacity(ctx):
    sq = band_ring([0, 5], [0], [5])
    empty = np.zeros((0, 2), np.int32)
    # set 0: touching, overlapping, empty, far-away B; set 1: no A; set 2: no B; set 3: empty
    ra = [sq, sq + np.array([20, 0], np.int32), empty, sq + np.array([100, 100], np.int32)]
    rb = [sq + np.array([5, 0], np.int32), sq + np.array([4, 4], np.int32), empty, sq + np.array([-500, 0], np.int32),
          band_ring([-3, 30], [-3], [40]), sq + np.array([100, 100], np.int32)]
    A, B = concat(ra), concat(rb)
    a_off = np.array([0, 3, 3, 4, 4], np.int64)
    b_off = np.array([0, 5, 6, 6, 6], np.int64)
    ea, eb, eso = oracle.join_sets(A, B, a_off, b_off)
    assert len(ea) > 0
    dA, dB, _, _ = device_workload(A, B, np.zeros(1, np.int32), np.zeros(1, np.int32))
    for cell in (1, 3, 64):
        pa, pb, so = ctx.join_sets(dA, dB, _dev_i64(a_off), _dev_i64(b_off), cell=cell)
        ctx.sync()
        assert list(zip(pa.cpu().tolist(), pb.cpu().tolist())) == list(zip(ea.tolist(), eb.tolist()))
        assert np.array_equal(so.cpu().numpy(), eso)
    # a buffer that is too small: the total comes back and nothing is written
    import ctypes
    import torch
    out_a = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    out_b = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    so = torch.empty(5, dtype=torch.int64, device="cuda")
    total = ctypes.c_int64(0)
    cA, cB = dA.c(), dB.c()
    rc = ctx.lib.sccg_join_sets(ctx.h, ctypes.byref(cA), ctypes.byref(cB), 4, _dev_i64(a_off).data_ptr(),
                                _dev_i64(b_off).data_ptr(), 64, 1, out_a.data_ptr(), out_b.data_ptr(),
                                so.data_ptr(), ctypes.byref(total))
    ctx.sync()
    assert rc == sccg.SCCG_OK and total.value == len(ea) > 1
    assert out_a.item() == -7 and out_b.item() == -7
    assert np.array_equal(so.cpu().numpy(), eso)


@pytest.mark.parametrize("mode", MODES)
def test_join_then_pairs_then_sets_on_device(ctx, sets4, mode):
    """Filter, pair counts and set reduction all on the device: per-tile
    sums and Jaccard equal the oracle's."""
    wl, eI, eU = sets4
    dA, dB, _, _ = device_workload(wl.A, wl.B, wl.pa, wl.pb)
    pa, pb, so = ctx.join_sets(dA, dB, _dev_i64(wl.a_set_off), _dev_i64(wl.b_set_off))
    I, U = ctx.area_pairs(dA, dB, pa.contiguous(), pb.contiguous(), mode=mode)
    si, su, nn, j, jp = ctx.jaccard_sets(so, I, U)
    ctx.sync()
    osi, osu, onn, oj, ojp = oracle.jaccard_sets(wl.set_off, eI, eU)
    assert np.array_equal(si.cpu().numpy(), osi) and np.array_equal(su.cpu().numpy(), osu)
    assert np.array_equal(j.cpu().numpy(), oj) and np.array_equal(jp.cpu().numpy(), ojp)


def _relate_cases():
    sq = band_ring([0, 5], [0], [5])
    small = band_ring([1, 3], [1], [3])
    empty = np.zeros((0, 2), np.int32)
    L = band_ring([0, 2, 5], [0, 0], [6, 2])
    pairs = [(sq, sq + np.array([5, 0], np.int32)), (sq, sq + np.array([5, 5], np.int32)),
             (sq, sq + np.array([6, 0], np.int32)), (sq, sq + np.array([4, 4], np.int32)), (sq, small), (small, sq),
             (sq, sq[::-1].copy()), (sq, empty), (L, band_ring([2, 5], [2], [6]))]
    return concat([a for a, _ in pairs]), concat([b for _, b in pairs])


@pytest.mark.parametrize("which", ["closed_forms", "tiny_shifted", "workload1", "set_tiles"])
def test_relate_pairs_equals_oracle(ctx, tiny, wl1, sets4, which):
    """Section 3.4's operators on the device (counts from BATCHED mode, then
    sccg_relate_pairs) equal the oracle's, bit for bit."""
    if which == "closed_forms":
        A, B = _relate_cases()
        pa = pb = np.arange(A.n, dtype=np.int32)
    elif which == "tiny_shifted":
        A, B, pa, pb = tiny[0], tiny[1], tiny[2][:5000], tiny[3][:5000]
    elif which == "workload1":
        A, B, pa, pb = wl1[0].A, wl1[0].B, wl1[0].pa, wl1[0].pb
    else:
        wl = sets4[0]
        A, B, pa, pb = wl.A, wl.B, wl.pa[:4000], wl.pb[:4000]
    dA, dB, dpa, dpb = device_workload(A, B, pa, pb)
    I, U = ctx.area_pairs(dA, dB, dpa, dpb, mode=sccg.SCCG_BATCHED)
    rel = ctx.relate_pairs(dA, dB, dpa, dpb, I)
    ctx.sync()
    expect = oracle.relate_pairs(A, B, pa, pb)
    got = rel.cpu().numpy().astype(np.uint32)
    bad = np.nonzero(got != expect)[0]
    assert len(bad) == 0, [(int(k), int(got[k]), int(expect[k])) for k in bad[:5]]
    if which == "closed_forms":
        assert got.tolist() == [16, 16, 0, 1, 3, 5, 15, 0, 16]

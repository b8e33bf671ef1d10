"""PixelBox on the host CPU (sccg_host_area_pairs, the CPU path of the
serving migration): its counts equal the oracle's exactly.  Runs without a
GPU: the entry point is plain host code in the device library."""

import os

import numpy as np
import pytest

import oracle
import paper_1208_0277_amd as sccg
import sccg_gen
from sccg_gen import concat
from tests.shapes import (band_rects, band_ring, comb_pairs, limit_cases, random_bands, rect_ring, rects_area,
                          rects_inter, staircase, transform)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(sccg.LIB_PATH):
        pytest.skip("device library not built")
    return sccg.load_library()


def _run(wl_A, wl_B, pa, pb, threads=4):
    return sccg.host_area_pairs(wl_A.off, wl_A.xy, wl_B.off, wl_B.xy, pa, pb, threads=threads)


def test_workload1_and_tiny(lib, cfg1):
    I, U = _run(cfg1.A, cfg1.B, cfg1.pa, cfg1.pb)
    eI, eU = oracle.area_pairs(cfg1.A, cfg1.B, cfg1.pa, cfg1.pb)
    assert np.array_equal(I, eI) and np.array_equal(U, eU)


def test_heavy_tailed_sample_with_blobs(lib):
    wl = sccg_gen.pairs(3, 3000)
    sel = np.concatenate([np.nonzero(wl.blob)[0][:15], np.arange(0, 3000, 5)])
    I, U = _run(wl.A, wl.B, wl.pa[sel], wl.pb[sel])
    eI, eU = oracle.area_pairs(wl.A, wl.B, wl.pa[sel], wl.pb[sel], form=oracle.ROWS)
    assert np.array_equal(I, eI) and np.array_equal(U, eU)


def test_band_polygons_closed_form(lib):
    rng = np.random.default_rng(77)
    ra, rb, expect = [], [], []
    for _ in range(500):
        a, ar = random_bands(rng, int(rng.integers(1, 10)), span=int(rng.integers(8, 300)),
                            hmax=int(rng.integers(1, 80)))
        b, br = random_bands(rng, int(rng.integers(1, 10)), x0=int(rng.integers(-30, 30)),
                             y0=int(rng.integers(-30, 80)), span=int(rng.integers(8, 300)),
                             hmax=int(rng.integers(1, 80)))
        sx, sy, sw = (1 if rng.random() < 0.5 else -1), (1 if rng.random() < 0.5 else -1), bool(rng.random() < .5)
        a, ar = transform(a, ar, sx, sy, sw)
        b, br = transform(b, br, sx, sy, sw)
        ra.append(a)
        rb.append(b)
        i = rects_inter(ar, br)
        expect.append((i, rects_area(ar) + rects_area(br) - i))
    A, B = concat(ra), concat(rb)
    idx = np.arange(len(ra), dtype=np.int32)
    I, U = _run(A, B, idx, idx, threads=1)
    assert [tuple(t) for t in zip(I.tolist(), U.tolist())] == expect


def test_range_error_and_empty(lib, cfg1):
    with pytest.raises(sccg.SccgError):
        _run(cfg1.A, cfg1.B, np.array([cfg1.A.n], np.int32), np.array([0], np.int32))
    I, U = _run(cfg1.A, cfg1.B, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert len(I) == 0 and len(U) == 0


def test_rejections_report_range_after_writing(lib):
    """A ring beyond 2^30 covers nothing and a pair box wider than 32767
    gives (0, 0); both make the call fail with SCCG_E_RANGE."""
    sq = lambda x, y, w, h: np.array([[x, y], [x + w, y], [x + w, y + h], [x, y + h]], np.int32)
    off = np.array([0, 4, 8], np.int64)
    a_xy = np.concatenate([sq((1 << 30) + 5, 0, 10, 10), sq(0, 0, 40000, 3)]).reshape(-1)
    b_xy = np.concatenate([sq((1 << 30) + 6, 1, 4, 4), sq(0, 0, 40000, 3)]).reshape(-1)
    for k in range(2):
        idx = np.array([k], np.int32)
        with pytest.raises(sccg.SccgError) as e:
            sccg.host_area_pairs(off, a_xy, off, b_xy, idx, idx)
        assert e.value.code == sccg.SCCG_E_RANGE


def test_wide_rings_closed_form(lib):
    sq = lambda x, y, s: ([y, y + s], [x], [x + s])
    cases = [(([0, 10], [0], [20000]), sq(100, -5, 30)),
             (staircase(300, 30000, 100, 2000), sq(15100, 15050, 50)),
             (([-(1 << 29), 1 << 29], [-(1 << 29)], [1 << 29]), sq(7, -3, 10))]
    A = concat([band_ring(*p) for p, _ in cases])
    B = concat([band_ring(*q) for _, q in cases])
    expect = []
    for p, q in cases:
        i = rects_inter(band_rects(*p), band_rects(*q))
        expect.append((i, rects_area(band_rects(*p)) + rects_area(band_rects(*q)) - i))
    idx = np.arange(len(cases), dtype=np.int32)
    I, U = _run(A, B, idx, idx)
    assert list(zip(I.tolist(), U.tolist())) == expect


def test_leaf_limit_boxes_closed_form(lib):
    """Pair boxes of 1, 63, 64 and 65 pixels a side around the 64-wide leaf
    limit, with staircases whose edges toggle runs of rows that start and end
    at the box's first and last rows: counts equal closed forms."""
    cases = []
    for w in (1, 63, 64, 65, 130):
        for h in (1, 63, 64, 65, 130):
            # p: [0, w) x [0, h), q covers p's box with a notch cut at its
            # left side, so the pair box is exactly p's box
            cases.append((([0, h], [0], [w]), ([-2, h // 3, h + 2], [-1, w // 2], [w + 1, w + 1])))
            cases.append((staircase(max(1, h // 4), h, 1, max(2, w - h // 4)), ([0, h], [0], [w])))
    A = concat([band_ring(*p) for p, _ in cases])
    B = concat([band_ring(*q) for _, q in cases])
    expect = []
    for p, q in cases:
        i = rects_inter(band_rects(*p), band_rects(*q))
        expect.append((i, rects_area(band_rects(*p)) + rects_area(band_rects(*q)) - i))
    idx = np.arange(len(cases), dtype=np.int32)
    for threads in (1, 3):
        I, U = _run(A, B, idx, idx, threads=threads)
        assert list(zip(I.tolist(), U.tolist())) == expect


def test_comb_closed_forms_match_oracle():
    cases = comb_pairs(12, 90)
    A, B = concat([c[0] for c in cases]), concat([c[1] for c in cases])
    idx = np.arange(len(cases), dtype=np.int32)
    eI, eU = oracle.area_pairs(A, B, idx, idx)
    assert list(zip(eI.tolist(), eU.tolist())) == [(c[2], c[3]) for c in cases]


def test_combs_closed_form(lib):
    """Combs whose 64-row bands meet 300 and 640 vertical edges each."""
    cases = comb_pairs(150, 300) + comb_pairs(320, 200)
    A, B = concat([c[0] for c in cases]), concat([c[1] for c in cases])
    idx = np.arange(len(cases), dtype=np.int32)
    I, U = _run(A, B, idx, idx)
    assert list(zip(I.tolist(), U.tolist())) == [(c[2], c[3]) for c in cases]


def test_coordinates_at_the_limit(lib):
    cases = limit_cases()
    A, B = concat([rect_ring(p) for p, _ in cases]), concat([rect_ring(q) for _, q in cases])
    area = lambda r: (r[2] - r[0]) * (r[3] - r[1])
    idx = np.arange(len(cases), dtype=np.int32)
    I, U = _run(A, B, idx, idx)
    assert list(zip(I.tolist(), U.tolist())) == [(area(q), area(p)) for p, q in cases]

"""Pins of the CPU oracle against facts it does not compute itself.

Each test fixes the oracle's output to something independent of it: closed
forms from rectangle overlaps, raster-mask popcounts (exhaustive tiny grids
and the generator's own masks), the shoelace formula, invariants of the
definition, and exact rational arithmetic for J.
"""

from fractions import Fraction

import numpy as np
import pytest

import oracle
import sccg_gen
from sccg_gen import concat
from tests.shapes import (band_ring, band_rects, random_bands, rects_area, rects_inter, transform)


def _pairs_from(rings_a, rings_b):
    A, B = concat(rings_a), concat(rings_b)
    idx = np.arange(len(rings_a), dtype=np.int32)
    return A, B, idx, idx


def test_pixel_inside_square():
    ring = np.array([[0, 0], [3, 0], [3, 2], [0, 2]], np.int32)
    inside = [(x, y) for y in range(-1, 4) for x in range(-1, 5) if oracle.pixel_inside(ring, x, y)]
    assert inside == [(x, y) for y in range(2) for x in range(3)]


def test_rectangles_closed_form():
    rng = np.random.default_rng(1)
    ra, rb, expect = [], [], []
    for _ in range(400):
        x0, y0 = (int(v) for v in rng.integers(-50, 50, 2))
        w, h = (int(v) for v in rng.integers(1, 30, 2))
        u0, v0 = (int(v) for v in rng.integers(-50, 50, 2))
        w2, h2 = (int(v) for v in rng.integers(1, 30, 2))
        r = (x0, y0, x0 + w, y0 + h)
        s = (u0, v0, u0 + w2, v0 + h2)
        ra.append(band_ring([y0, y0 + h], [x0], [x0 + w]))
        rb.append(band_ring([v0, v0 + h2], [u0], [u0 + w2])[::-1])  # clockwise
        i = rects_inter([r], [s])
        expect.append((i, w * h + w2 * h2 - i))
    A, B, pa, pb = _pairs_from(ra, rb)
    for form in (oracle.PURE, oracle.ROWS):
        I, U = oracle.area_pairs(A, B, pa, pb, form=form)
        assert [tuple(t) for t in zip(I.tolist(), U.tolist())] == expect


@pytest.mark.parametrize("nb", [2, 3, 7, 12])
def test_band_polygons_closed_form(nb):
    rng = np.random.default_rng(100 + nb)
    ra, rb, expect, areas = [], [], [], []
    for t in range(300):
        ring_a, rects_a = random_bands(rng, nb, x0=0, y0=0)
        ring_b, rects_b = random_bands(rng, int(rng.integers(1, nb + 1)), x0=int(rng.integers(-10, 10)),
                                       y0=int(rng.integers(-10, 20)))
        # random reflections / transposes keep the rectangle decomposition exact
        sx, sy = (1 if rng.random() < 0.5 else -1), (1 if rng.random() < 0.5 else -1)
        sw = bool(rng.random() < 0.5)
        ring_a, rects_a = transform(ring_a, rects_a, sx, sy, sw)
        ring_b, rects_b = transform(ring_b, rects_b, sx, sy, sw)
        ra.append(ring_a)
        rb.append(ring_b)
        i = rects_inter(rects_a, rects_b)
        expect.append((i, rects_area(rects_a) + rects_area(rects_b) - i))
        areas.append(rects_area(rects_a))
    A, B, pa, pb = _pairs_from(ra, rb)
    for form in (oracle.PURE, oracle.ROWS):
        I, U = oracle.area_pairs(A, B, pa, pb, form=form)
        assert [tuple(t) for t in zip(I.tolist(), U.tolist())] == expect
    assert oracle.poly_areas(A).tolist() == areas


def test_l_shapes_closed_form():
    # L = [0,6)x[0,2) + [0,2)x[2,5): 12 + 6 = 18 pixels
    L = band_ring([0, 2, 5], [0, 0], [6, 2])
    Lr = band_rects([0, 2, 5], [0, 0], [6, 2])
    R = band_ring([1, 4], [1], [4])  # [1,4)x[1,4)
    # overlap: [1,4)x[1,2) = 3 and [1,2)x[2,4) = 2  -> 5
    A, B, pa, pb = _pairs_from([L, L], [R, L])
    I, U = oracle.area_pairs(A, B, pa, pb)
    assert I.tolist() == [5, 18]
    assert U.tolist() == [18 + 9 - 5, 18]
    assert rects_inter(Lr, [(1, 1, 4, 4)]) == 5


def _valid_4x4_masks():
    def ok(m):
        cells = {(x, y) for y in range(4) for x in range(4) if m >> (y * 4 + x) & 1}
        start = next(iter(cells))
        seen, st = {start}, [start]
        while st:
            x, y = st.pop()
            for c in ((x + 1, y), (x - 1, y), (x, y + 1), (x, y - 1)):
                if c in cells and c not in seen:
                    seen.add(c)
                    st.append(c)
        if len(seen) != len(cells):
            return False
        bg = {(x, y) for x in range(-1, 5) for y in range(-1, 5)} - cells
        seen, st = {(-1, -1)}, [(-1, -1)]
        while st:
            x, y = st.pop()
            for c in ((x + 1, y), (x - 1, y), (x, y + 1), (x, y - 1)):
                if c in bg and c not in seen:
                    seen.add(c)
                    st.append(c)
        return len(seen) == len(bg)
    return [m for m in range(1, 1 << 16) if ok(m)]


def _bits(m):
    return np.array([[(m >> (y * 4 + x)) & 1 for x in range(4)] for y in range(4)], np.uint8)


@pytest.fixture(scope="module")
def tiny_corpus():
    masks = _valid_4x4_masks()
    rings = [sccg_gen.trace_mask(_bits(m)) for m in masks]
    assert all(r is not None for r in rings)
    return masks, rings


def test_tiny_grid_exhaustive_single(tiny_corpus):
    """Every hole-free 4-connected mask on a 4x4 grid: I(A,A) = U(A,A) =
    popcount(mask) = |shoelace|."""
    masks, rings = tiny_corpus
    assert len(masks) == 9349
    A = concat(rings)
    idx = np.arange(len(rings), dtype=np.int32)
    I, U = oracle.area_pairs(A, A, idx, idx)
    pop = np.array([bin(m).count("1") for m in masks], np.int64)
    assert np.array_equal(I, pop) and np.array_equal(U, pop)
    assert np.array_equal(oracle.poly_areas(A), pop)


def test_tiny_grid_pairs_with_shifts(tiny_corpus):
    """Random pairs of tiny-grid masks with shifts in [-4,4]^2: I and U equal
    popcount(a & b) and popcount(a | b) of the shifted masks."""
    masks, rings = tiny_corpus
    rng = np.random.default_rng(7)
    n = 60000
    ia = rng.integers(0, len(masks), n)
    ib = rng.integers(0, len(masks), n)
    sh = rng.integers(-4, 5, (n, 2))
    rb = [rings[j] + sh[k].astype(np.int32) for k, j in enumerate(ib)]
    ra = [rings[j] for j in ia]
    A, B, pa, pb = _pairs_from(ra, rb)
    I, U = oracle.area_pairs(A, B, pa, pb)
    # truth from 12x12 canvases
    big = np.zeros((len(masks), 12, 12), np.uint8)
    for k, m in enumerate(masks):
        big[k, 4:8, 4:8] = _bits(m)
    eI = np.empty(n, np.int64)
    eU = np.empty(n, np.int64)
    for k in range(n):
        a = big[ia[k]]
        b = np.roll(np.roll(big[ib[k]], sh[k, 1], axis=0), sh[k, 0], axis=1)
        eI[k] = int(np.sum(a & b))
        eU[k] = int(np.sum(a | b))
    assert np.array_equal(I, eI)
    assert np.array_equal(U, eU)


def _mask_truth(wl, i):
    a, ax, ay = wl.mask(0, i)
    b, bx, by = wl.mask(1, i)
    x0, y0 = min(ax, bx), min(ay, by)
    x1 = max(ax + a.shape[1], bx + b.shape[1])
    y1 = max(ay + a.shape[0], by + b.shape[0])
    ca = np.zeros((y1 - y0, x1 - x0), np.uint8)
    cb = np.zeros_like(ca)
    ca[ay - y0:ay - y0 + a.shape[0], ax - x0:ax - x0 + a.shape[1]] = a
    cb[by - y0:by - y0 + b.shape[0], bx - x0:bx - x0 + b.shape[1]] = b
    return int(np.sum(ca & cb)), int(np.sum(ca | cb)), int(a.sum()), int(b.sum())


def test_generator_masks_config1(cfg1):
    """Workload 1 in full: oracle counts equal popcounts of the generator's
    raster masks (the pixels the rings were traced from)."""
    I, U = oracle.area_pairs(cfg1.A, cfg1.B, cfg1.pa, cfg1.pb)
    areas_a = oracle.poly_areas(cfg1.A)
    for i in range(cfg1.n_pairs):
        ti, tu, na, nb = _mask_truth(cfg1, i)
        assert (I[i], U[i], areas_a[i]) == (ti, tu, na), i


def test_generator_masks_config3_sample():
    wl = sccg_gen.pairs(3, 3000)
    sel = np.concatenate([np.nonzero(wl.blob)[0][:10], np.arange(0, 3000, 37)])
    pa, pb = wl.pa[sel], wl.pb[sel]
    I, U = oracle.area_pairs(wl.A, wl.B, pa, pb, form=oracle.ROWS)
    for k, i in enumerate(sel):
        ti, tu, _, _ = _mask_truth(wl, int(i))
        assert (I[k], U[k]) == (ti, tu), i


def test_invariants_config1(cfg1):
    A, B, pa, pb = cfg1.A, cfg1.B, cfg1.pa, cfg1.pb
    I, U = oracle.area_pairs(A, B, pa, pb)
    aa, ab = oracle.poly_areas(A), oracle.poly_areas(B)
    assert np.array_equal(I + U, aa[pa] + ab[pb])             # |p|+|q| = I + U
    I2, U2 = oracle.area_pairs(B, A, pb, pa)
    assert np.array_equal(I, I2) and np.array_equal(U, U2)     # symmetry
    Is, Us = oracle.area_pairs(A, A, pa, pa)
    assert np.array_equal(Is, aa) and np.array_equal(Us, aa)   # J(A,A) = 1
    assert np.all(I <= np.minimum(aa[pa], ab[pb])) and np.all(U >= np.maximum(aa[pa], ab[pb]))
    # translation, including into negative coordinates
    shift = np.array([-70001, -123457], np.int32)
    At = sccg_gen.Polys(A.off, A.xy + shift)
    Bt = sccg_gen.Polys(B.off, B.xy + shift)
    It, Ut = oracle.area_pairs(At, Bt, pa, pb)
    assert np.array_equal(I, It) and np.array_equal(U, Ut)
    # disjoint: B moved past A (every shape is under 50 px wide)
    Bf = sccg_gen.Polys(B.off, B.xy + np.array([100, 0], np.int32))
    Id, Ud = oracle.area_pairs(A, Bf, pa, pb)
    assert np.all(Id == 0) and np.array_equal(Ud, aa[pa] + ab[pb])
    # rows form = pure form
    Ir, Ur = oracle.area_pairs(A, B, pa, pb, form=oracle.ROWS)
    assert np.array_equal(I, Ir) and np.array_equal(U, Ur)


@pytest.mark.parametrize("k", [2, 3, 5])
def test_scale_k_squared(cfg1, k):
    """Scaling all coordinates by k (Section 5.2's scale factors) multiplies
    every pixel count by k^2."""
    sel = np.arange(0, cfg1.n_pairs, 5)
    pa, pb = cfg1.pa[sel], cfg1.pb[sel]
    I, U = oracle.area_pairs(cfg1.A, cfg1.B, pa, pb, form=oracle.ROWS)
    As = sccg_gen.Polys(cfg1.A.off, cfg1.A.xy * k)
    Bs = sccg_gen.Polys(cfg1.B.off, cfg1.B.xy * k)
    Ik, Uk = oracle.area_pairs(As, Bs, pa, pb, form=oracle.ROWS)
    assert np.array_equal(Ik, k * k * I) and np.array_equal(Uk, k * k * U)


def test_containment_and_degenerate():
    inner = band_ring([2, 4, 6], [2, 1], [5, 4])
    outer = band_ring([0, 10], [0], [10])
    tiny = band_ring([3, 4], [3], [4])
    dup = np.concatenate([inner, inner[:1]])  # repeated closing vertex
    A, B, pa, pb = _pairs_from([inner, tiny, dup, outer], [outer, outer, inner, inner])
    I, U = oracle.area_pairs(A, B, pa, pb)
    assert I.tolist() == [12, 1, 12, 12]
    assert U.tolist() == [100, 100, 12, 100]


def test_empty_rings():
    """A ring without vertices has no edges, so no pixel centre sees a
    crossing: it covers nothing, and the other ring is counted alone."""
    R = band_ring([0, 3], [0], [5])  # [0,5)x[0,3): 15 pixels
    empty = np.zeros((0, 2), np.int32)
    A, B, pa, pb = _pairs_from([empty, R, empty], [R, empty, empty])
    for form in (oracle.PURE, oracle.ROWS):
        I, U = oracle.area_pairs(A, B, pa, pb, form=form)
        assert I.tolist() == [0, 0, 0] and U.tolist() == [15, 15, 0]
    assert oracle.poly_areas(A).tolist() == [0, 15, 0]


def test_jaccard_exact_rational():
    rng = np.random.default_rng(3)
    n = 5000
    I = rng.integers(0, 10 ** 6, n).astype(np.int64)
    I[rng.random(n) < 0.2] = 0
    U = I + rng.integers(1, 10 ** 6, n).astype(np.int64)
    so = np.array([0, 10, 10, 2500, n], np.int64)
    for inc in (False, True):
        si, su, nn, j, jp = oracle.jaccard_sets(so, I, U, include_zero=inc)
        for s in range(len(so) - 1):
            ks = [k for k in range(so[s], so[s + 1]) if inc or I[k] > 0]
            ti = sum(int(I[k]) for k in ks)
            tu = sum(int(U[k]) for k in ks)
            assert (si[s], su[s], nn[s]) == (ti, tu, len(ks))
            # one correctly rounded division of the exact sums
            assert j[s] == (float(Fraction(ti, tu)) if tu else 0.0)
    # J' of ratios 1/2 and 1/4 is exactly 3/8; identical pairs give exactly 1
    si, su, nn, j, jp = oracle.jaccard_sets(np.array([0, 2, 5]), np.array([1, 1, 7, 7, 7]),
                                            np.array([2, 4, 7, 7, 7]))
    assert jp.tolist() == [0.375, 1.0] and j.tolist() == [2 / 6, 1.0]


def test_jprime_exact_sum():
    """J' = (sum of the binary64 ratios, rounded once from its exact value) / n,
    checked with exact rationals."""
    rng = np.random.default_rng(11)
    for trial in range(20):
        n = int(rng.integers(1, 3000))
        U = rng.integers(1, 10 ** 9, n).astype(np.int64)
        I = (U * rng.random(n)).astype(np.int64) + 1
        I = np.minimum(I, U)
        _, _, nn, _, jp = oracle.jaccard_sets(np.array([0, n]), I, U)
        exact = sum(Fraction(float(I[k]) / float(U[k])) for k in range(n))
        assert nn[0] == n
        assert jp[0] == float(exact) / n


def test_set_workload_join_is_exact():
    """Workload 4's candidate pairs are exactly the (A, B) pairs of one tile
    whose MBRs share a pixel, each once (brute force over small tiles; a B
    shape near a tile's edge may reach into the next tile, whose A shapes
    belong to another set)."""
    wl = sccg_gen.sets(n_tiles=2, tile_side=768, cell=64)

    def mbrs(P):
        m = np.zeros((P.n, 4), np.int64)
        for k in range(P.n):
            r = P.ring(k)
            m[k] = (r[:, 0].min(), r[:, 1].min(), r[:, 0].max(), r[:, 1].max())
        return m
    ma, mb = mbrs(wl.A), mbrs(wl.B)
    got = set(zip(wl.pa.tolist(), wl.pb.tolist()))
    assert len(got) == wl.n_pairs  # no duplicates
    a_ids = np.arange(len(ma))
    by_b = {}
    for (a, b) in got:
        by_b.setdefault(b, set()).add(a)
    for t in range(len(wl.a_set_off) - 1):
        a_lo, a_hi = int(wl.a_set_off[t]), int(wl.a_set_off[t + 1])
        ids = a_ids[a_lo:a_hi]
        for b in range(int(wl.b_set_off[t]), int(wl.b_set_off[t + 1])):
            x0 = np.maximum(ma[a_lo:a_hi, 0], mb[b, 0])
            y0 = np.maximum(ma[a_lo:a_hi, 1], mb[b, 1])
            x1 = np.minimum(ma[a_lo:a_hi, 2], mb[b, 2])
            y1 = np.minimum(ma[a_lo:a_hi, 3], mb[b, 3])
            hit = set(ids[(x0 < x1) & (y0 < y1)].tolist())
            assert hit == by_b.get(b, set()), b
    assert wl.stats["polys_a"] > 0 and wl.n_pairs > 0


def test_join_closed_forms():
    """MBRs that only touch along a side or at a corner share no pixel; one
    pixel of overlap is enough; a ring without vertices meets nothing."""
    sq = band_ring([0, 5], [0], [5])
    A = concat([sq])
    cases = [(sq + np.array([5, 0], np.int32), 0), (sq + np.array([5, 5], np.int32), 0),
             (sq + np.array([4, 4], np.int32), 1), (sq + np.array([-4, 0], np.int32), 1),
             (np.zeros((0, 2), np.int32), 0), (band_ring([1, 2], [1], [2]), 1)]
    B = concat([r for r, _ in cases])
    pa, pb, so = oracle.join_sets(A, B, np.array([0, 1], np.int64), np.array([0, len(cases)], np.int64))
    assert pb.tolist() == [k for k, (_, hit) in enumerate(cases) if hit] and set(pa.tolist()) <= {0}
    assert so.tolist() == [0, len(pb)]


def test_join_brute_force_and_sets():
    """Random rectangles in three sets against a brute-force overlap test;
    pairs never cross sets; order is set, then b, then a."""
    rng = np.random.default_rng(21)
    ra, rb, a_off, b_off = [], [], [0], [0]
    for s in range(3):
        na, nb = int(rng.integers(0, 40)), int(rng.integers(0, 40))
        for _ in range(na):
            x, y, w, h = (int(v) for v in rng.integers([0, 0, 1, 1], [100, 100, 20, 20]))
            ra.append(band_ring([y, y + h], [x], [x + w]))
        for _ in range(nb):
            x, y, w, h = (int(v) for v in rng.integers([0, 0, 1, 1], [100, 100, 20, 20]))
            rb.append(band_ring([y, y + h], [x], [x + w]))
        a_off.append(a_off[-1] + na)
        b_off.append(b_off[-1] + nb)
    A, B = concat(ra), concat(rb)
    pa, pb, so = oracle.join_sets(A, B, np.array(a_off), np.array(b_off))
    expect = []
    for s in range(3):
        for b in range(b_off[s], b_off[s + 1]):
            rbx = rb[b]
            for a in range(a_off[s], a_off[s + 1]):
                rax = ra[a]
                if (max(rax[:, 0].min(), rbx[:, 0].min()) < min(rax[:, 0].max(), rbx[:, 0].max()) and
                        max(rax[:, 1].min(), rbx[:, 1].min()) < min(rax[:, 1].max(), rbx[:, 1].max())):
                    expect.append((a, b))
    assert list(zip(pa.tolist(), pb.tolist())) == expect
    assert so[-1] == len(expect)


def test_join_agrees_with_grid_join():
    """The oracle's all-pairs test and the generator's uniform-grid join
    (reference-point dedup) are independent and give the same pair list."""
    wl = sccg_gen.sets(n_tiles=3, tile_side=1536, cell=64)
    pa, pb, so = oracle.join_sets(wl.A, wl.B, wl.a_set_off, wl.b_set_off)
    assert np.array_equal(pa, wl.pa) and np.array_equal(pb, wl.pb) and np.array_equal(so, wl.set_off)


def test_relate_closed_forms():
    """Section 3.4's operators from counts: shared side or corner touches;
    a gap, or any common pixel, does not; containment both ways; equality;
    an empty ring relates to nothing."""
    sq = band_ring([0, 5], [0], [5])
    small = band_ring([1, 3], [1], [3])
    empty = np.zeros((0, 2), np.int32)
    L = band_ring([0, 2, 5], [0, 0], [6, 2])       # L-shape; its notch touches the square below
    cases = [
        (sq, sq + np.array([5, 0], np.int32), oracle.REL_TOUCHES),     # shared side
        (sq, sq + np.array([5, 5], np.int32), oracle.REL_TOUCHES),     # shared corner
        (sq, sq + np.array([6, 0], np.int32), 0),                      # gap of one pixel
        (sq, sq + np.array([4, 4], np.int32), oracle.REL_INTERSECTS),  # one common pixel
        (sq, small, oracle.REL_INTERSECTS | oracle.REL_CONTAINS),
        (small, sq, oracle.REL_INTERSECTS | oracle.REL_WITHIN),
        (sq, sq[::-1].copy(), 15),                                     # equal (other orientation)
        (sq, empty, 0),
        (L, band_ring([2, 5], [2], [6]), oracle.REL_TOUCHES),           # fills the notch: touch along two sides
    ]
    A = concat([a for a, _, _ in cases])
    B = concat([b for _, b, _ in cases])
    idx = np.arange(len(cases), dtype=np.int32)
    assert oracle.relate_pairs(A, B, idx, idx).tolist() == [r for _, _, r in cases]


def test_relate_brute_force_on_tiny_masks(tiny_corpus):
    """Random tiny-grid pairs with shifts: contains/within/equal/intersects
    against mask set relations, touches against pixel adjacency (two
    disjoint pixel sets touch iff some pixels share a side or a corner)."""
    masks, rings = tiny_corpus
    rng = np.random.default_rng(31)
    n = 3000
    ia = rng.integers(0, len(masks), n)
    ib = rng.integers(0, len(masks), n)
    sh = rng.integers(-5, 6, (n, 2))
    A = concat([rings[j] for j in ia])
    B = concat([rings[j] + sh[k].astype(np.int32) for k, j in enumerate(ib)])
    idx = np.arange(n, dtype=np.int32)
    rel = oracle.relate_pairs(A, B, idx, idx)
    for k in range(n):
        a = {(x, y) for y in range(4) for x in range(4) if masks[ia[k]] >> (y * 4 + x) & 1}
        b = {(x + sh[k, 0], y + sh[k, 1]) for y in range(4) for x in range(4) if masks[ib[k]] >> (y * 4 + x) & 1}
        i = a & b
        exp = 0
        if i:
            exp |= oracle.REL_INTERSECTS
            exp |= oracle.REL_CONTAINS if i == b else 0
            exp |= oracle.REL_WITHIN if i == a else 0
            exp |= oracle.REL_EQUALS if a == b else 0
        elif any((x + dx, y + dy) in b for (x, y) in a for dx in (-1, 0, 1) for dy in (-1, 0, 1)):
            exp |= oracle.REL_TOUCHES
        assert rel[k] == exp, (k, rel[k], exp)

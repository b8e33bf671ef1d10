"""Closed-form test shapes: rectilinear polygons built as stacks of disjoint
horizontal bands, so that every pixel count has an exact value from rectangle
overlaps alone (no ray casting, no shoelace)."""

from __future__ import annotations

import numpy as np


def band_ring(y, a, b):
    """Ring of the polygon whose band k is the rectangle [a[k], b[k]) x [y[k], y[k+1]).

    Consecutive bands must overlap in x so that the union is one simple
    polygon.  The ring runs up the right side and back down the left side
    (counter-clockwise); repeated or collinear points are kept on purpose.
    """
    n = len(a)
    assert len(y) == n + 1 and len(b) == n
    pts = [(b[0], y[0])]
    for k in range(n):
        pts.append((b[k], y[k + 1]))
        if k + 1 < n:
            pts.append((b[k + 1], y[k + 1]))
    pts.append((a[n - 1], y[n]))
    for k in range(n - 1, -1, -1):
        pts.append((a[k], y[k]))
        if k > 0:
            pts.append((a[k - 1], y[k]))
    return np.array(pts, np.int32)


def staircase(n_bands, height, step, width):
    """Bands (y, a, b) of a staircase: n_bands bands over [0, height), band k
    spanning [step*k, step*k + width); step < width keeps it one polygon."""
    y = [round(k * height / n_bands) for k in range(n_bands + 1)]
    a = [step * k for k in range(n_bands)]
    return y, a, [x + width for x in a]


def band_rects(y, a, b):
    return [(a[k], y[k], b[k], y[k + 1]) for k in range(len(a))]


def rect_overlap(r, s):
    ox = min(r[2], s[2]) - max(r[0], s[0])
    oy = min(r[3], s[3]) - max(r[1], s[1])
    return max(ox, 0) * max(oy, 0)


def rects_area(rs):
    return sum((r[2] - r[0]) * (r[3] - r[1]) for r in rs)


def rects_inter(rs, ss):
    """|union(rs) & union(ss)| for two lists of pairwise-disjoint rectangles."""
    return sum(rect_overlap(r, s) for r in rs for s in ss)


def random_bands(rng, nb, x0=0, y0=0, span=40, hmax=6):
    """Random band polygon with nb bands: returns (ring, rects)."""
    ys = [y0]
    for _ in range(nb):
        ys.append(ys[-1] + int(rng.integers(1, hmax + 1)))
    a, b = [], []
    lo = x0 + int(rng.integers(0, span // 2))
    hi = lo + int(rng.integers(1, span // 2 + 1))
    for k in range(nb):
        if k > 0:
            # new band overlapping the previous one by at least one pixel
            pa, pb = a[-1], b[-1]
            lo = int(rng.integers(x0 - 2, pb))
            hi = int(rng.integers(max(lo, pa) + 1, x0 + span + 3))
            if hi <= max(lo, pa):
                hi = max(lo, pa) + 1
        a.append(lo)
        b.append(hi)
    return band_ring(ys, a, b), band_rects(ys, a, b)


def transform(ring, rects, sx=1, sy=1, swap=False, dx=0, dy=0, k=1):
    """Apply a reflection/transpose, an integer scale k and a translation to
    both the ring and its rectangle decomposition."""
    r = np.asarray(ring, np.int64).copy()
    out_rects = []
    for (x0, y0, x1, y1) in rects:
        xs = sorted([sx * x0, sx * x1])
        ys = sorted([sy * y0, sy * y1])
        q = (xs[0], ys[0], xs[1], ys[1])
        if swap:
            q = (q[1], q[0], q[3], q[2])
        out_rects.append((k * q[0] + dx, k * q[1] + dy, k * q[2] + dx, k * q[3] + dy))
    r[:, 0] *= sx
    r[:, 1] *= sy
    if swap:
        r = r[:, ::-1]
    r = r * k
    r[:, 0] += dx
    r[:, 1] += dy
    return r.astype(np.int32), out_rects


def comb_ring(n, height, base=10, x0=0):
    """Ring (4n vertices) of a comb: base [x0, x0 + 2n - 1) x [0, base) with
    n teeth [x0 + 2k, x0 + 2k + 1) x [base, height), one pixel wide and one
    pixel apart, so every 64-row band above the base meets 2n vertical edges."""
    pts = [(x0, 0), (x0 + 2 * n - 1, 0)]
    for k in range(n - 1, -1, -1):
        pts += [(x0 + 2 * k + 1, height), (x0 + 2 * k, height)]
        if k > 0:
            pts += [(x0 + 2 * k, base), (x0 + 2 * k - 1, base)]
    return np.array(pts, dtype=np.int32)


def comb_area(n, height, base=10):
    return (2 * n - 1) * base + n * (height - base)


def limit_cases():
    """Pairs of rectangles (x0, y0, x1, y1) reaching |coordinate| = 2^30, the
    largest accepted, where a coordinate minus a box side reaches 2^31.  In
    every pair q lies inside p, so I = |q| and U = |p|.  The pair boxes cover
    one leaf tile, a split into a few tiles, and a split that classifies
    cells; the last two pairs' p has twice its area equal to 2^63 (and the
    last one's pair box fits one leaf tile at the top corner of the range)."""
    M = 1 << 30
    return [
        ((0, -M, 10, M), (0, -M, 10, -M + 5)),
        ((-M, 0, M, 10), (-M, 0, -M + 10, 10)),
        ((-M, 0, M, 10), (0, 0, 10, 10)),
        ((0, -M, 100, M), (0, -M, 100, -M + 100)),
        ((-M, 0, M, 100), (-M, 0, -M + 100, 100)),
        ((0, -M, 600, M), (0, -M, 600, -M + 600)),
        ((-M, -M, M, M), (M - 70, M - 70, M, M)),
        ((-M, -M, M, M), (M - 40, M - 30, M, M)),
    ]


def rect_ring(r):
    x0, y0, x1, y1 = r
    return band_ring([y0, y1], [x0], [x1])


def comb_pairs(n, h):
    """(p ring, q ring, I, U) of a comb against its box, the box against the
    comb, the comb against itself shifted one pixel right (teeth interleave,
    only the bases overlap) and the comb against itself."""
    comb, shifted = comb_ring(n, h), comb_ring(n, h, x0=1)
    box = rect_ring((0, 0, 2 * n - 1, h))
    ca, ba, ia = comb_area(n, h), (2 * n - 1) * h, (2 * n - 2) * 10
    return [(comb, box, ca, ba), (box, comb, ca, ba), (comb, shifted, ia, 2 * ca - ia), (comb, comb, ca, ca)]

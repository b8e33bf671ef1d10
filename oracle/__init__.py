"""Test infrastructure: ctypes binding of the plain CPU oracle.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the device library
and its binding) never calls it.  See ``sccg_oracle.c`` for what each function
computes and the passage of the paper it follows.
"""

from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsccg_oracle.so")
_lib = None

PURE = 0
ROWS = 1


class _Polys(ctypes.Structure):
    _fields_ = [("n_polys", ctypes.c_int64), ("offsets", ctypes.c_void_p), ("xy", ctypes.c_void_p)]


def _load():
    global _lib
    if _lib is None:
        _lib = load_library(LIB_PATH)
    return _lib


def load_library(path: str):
    """Load an oracle library build with its signatures set (the pin-strength
    tests load deliberately broken builds this way)."""
    if not os.path.exists(path):
        raise RuntimeError(f"oracle library not built: {path} (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    lib.sccg_oracle_pixel_inside.restype = ctypes.c_int
    lib.sccg_oracle_pixel_inside.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
    lib.sccg_oracle_poly_area.restype = ctypes.c_int64
    lib.sccg_oracle_poly_area.argtypes = [ctypes.POINTER(_Polys), ctypes.c_int64]
    lib.sccg_oracle_area_pairs.restype = None
    lib.sccg_oracle_area_pairs.argtypes = [ctypes.POINTER(_Polys), ctypes.POINTER(_Polys), ctypes.c_int64,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_int, ctypes.c_int]
    lib.sccg_oracle_jaccard_sets.restype = None
    lib.sccg_oracle_jaccard_sets.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]
    lib.sccg_oracle_relate_pairs.restype = None
    lib.sccg_oracle_relate_pairs.argtypes = [ctypes.POINTER(_Polys), ctypes.POINTER(_Polys), ctypes.c_int64,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.sccg_oracle_join_sets.restype = ctypes.c_int64
    lib.sccg_oracle_join_sets.argtypes = [ctypes.POINTER(_Polys), ctypes.POINTER(_Polys), ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]
    return lib


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _polys(P):
    off = _c(P.off, np.int64)
    xy = _c(P.xy, np.int32)
    s = _Polys(len(off) - 1, off.ctypes.data, xy.ctypes.data)
    return s, (off, xy)


def pixel_inside(ring, x: int, y: int) -> int:
    r = _c(ring, np.int32)
    return int(_load().sccg_oracle_pixel_inside(r.ctypes.data, len(r), x, y))


def poly_areas(P) -> np.ndarray:
    lib = _load()
    s, keep = _polys(P)
    return np.array([lib.sccg_oracle_poly_area(ctypes.byref(s), k) for k in range(s.n_polys)], np.int64)


def area_pairs(A, B, pa, pb, form: int = PURE, threads: int | None = None):
    """Exact (I, U) int64 per pair; form PURE or ROWS."""
    lib = _load()
    sa, ka = _polys(A)
    sb, kb = _polys(B)
    pa = _c(pa, np.int32)
    pb = _c(pb, np.int32)
    n = len(pa)
    I = np.zeros(n, np.int64)
    U = np.zeros(n, np.int64)
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    lib.sccg_oracle_area_pairs(ctypes.byref(sa), ctypes.byref(sb), n, pa.ctypes.data, pb.ctypes.data,
                               I.ctypes.data, U.ctypes.data, form, threads)
    return I, U


def jaccard_sets(set_off, I, U, include_zero: bool = False):
    """Per set: (sum_i, sum_u, n_contrib, J, J').

    J = sum I / sum U (Section 2.1) with one binary64 division.  J' (Equation
    1) = mean of I/U over the contributing pairs: each ratio is one binary64
    division, their sum is rounded once from the exact value (math.fsum), then
    divided by the count.  Fixing the rounding this way makes J' independent
    of summation order; the paper does not fix one.
    """
    lib = _load()
    so = _c(set_off, np.int64)
    I = _c(I, np.int64)
    U = _c(U, np.int64)
    ns = len(so) - 1
    si = np.zeros(ns, np.int64)
    su = np.zeros(ns, np.int64)
    nn = np.zeros(ns, np.int64)
    j = np.zeros(ns, np.float64)
    jp = np.zeros(ns, np.float64)
    lib.sccg_oracle_jaccard_sets(ns, so.ctypes.data, I.ctypes.data, U.ctypes.data, int(include_zero),
                                 si.ctypes.data, su.ctypes.data, nn.ctypes.data, j.ctypes.data)
    for s in range(ns):
        i_s = I[so[s]:so[s + 1]]
        u_s = U[so[s]:so[s + 1]]
        keep = np.ones(len(i_s), bool) if include_zero else (i_s > 0)
        i_k, u_k = i_s[keep], u_s[keep]
        pos = u_k > 0
        ratios = np.zeros(len(i_k), np.float64)
        ratios[pos] = i_k[pos].astype(np.float64) / u_k[pos].astype(np.float64)
        n = len(i_k)
        jp[s] = math.fsum(ratios.tolist()) / n if n else 0.0
    return si, su, nn, j, jp


#: relation bits of relate_pairs (Section 3.4)
REL_INTERSECTS, REL_CONTAINS, REL_WITHIN, REL_EQUALS, REL_TOUCHES = 1, 2, 4, 8, 16


def relate_pairs(A, B, pa, pb):
    """Per pair the relation bits: intersects, A contains B, A within B,
    equal (from the pixel counts and areas), touches (no common pixel, but
    boundaries that share a point, by comparing every pair of edges)."""
    lib = _load()
    sa, ka = _polys(A)
    sb, kb = _polys(B)
    pa = _c(pa, np.int32)
    pb = _c(pb, np.int32)
    out = np.zeros(len(pa), np.uint32)
    lib.sccg_oracle_relate_pairs(ctypes.byref(sa), ctypes.byref(sb), len(pa), pa.ctypes.data, pb.ctypes.data,
                                 out.ctypes.data)
    return out


def join_sets(A, B, a_set_off, b_set_off):
    """Candidate pairs with intersecting MBRs, per set (Section 4.1's filter
    stage), by testing every pair of each set: (pa, pb, set_off), ordered by
    set, then b, then a."""
    lib = _load()
    sa, ka = _polys(A)
    sb, kb = _polys(B)
    ao = _c(a_set_off, np.int64)
    bo = _c(b_set_off, np.int64)
    ns = len(ao) - 1
    so = np.zeros(ns + 1, np.int64)
    total = lib.sccg_oracle_join_sets(ctypes.byref(sa), ctypes.byref(sb), ns, ao.ctypes.data, bo.ctypes.data, 0,
                                      None, None, so.ctypes.data)
    pa = np.zeros(total, np.int32)
    pb = np.zeros(total, np.int32)
    lib.sccg_oracle_join_sets(ctypes.byref(sa), ctypes.byref(sb), ns, ao.ctypes.data, bo.ctypes.data, total,
                              pa.ctypes.data, pb.ctypes.data, so.ctypes.data)
    return pa, pb, so

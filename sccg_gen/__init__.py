"""Seeded synthetic workloads (input generator only).

Builds rectilinear integer-vertex polygons the way segmentation of a raster
image yields them (paper Section 2.1, Figure 3): unions of integer ellipses are
rasterised, reduced to their largest 4-connected component, hole-filled and
traced along pixel sides.  Pairs (A_i, B_i) follow the workload recipes in
this package's docstrings; B_i is A_i shifted by up to 3 px and dilated or
eroded by one pixel.

This module computes nothing of the PixelBox method: no crossing tests, no
areas, no box classification.  Both the oracle tests and the device tests take
their inputs from here.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsccg_gen.so")
_lib = None

#: the seed of workload k is BASE_SEED + k
BASE_SEED = 20120277

#: pairs per workload: 1 = 1k pairs of <=32 px shapes on a 4096^2 tile,
#: 2 = 200k pairs of 10-60 px shapes, 3 = 2M pairs with a heavy-tailed size
#: mix (lognormal side, median 24 px, clipped to 8-400 px, 1% merged blobs).
DEFAULT_PAIRS = {1: 1000, 2: 200_000, 3: 2_000_000}


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"generator library not built: {_LIB_PATH} (run __graft_entry__.build())")
    lib = ctypes.CDLL(_LIB_PATH)
    lib.sccg_gen_pairs.restype = ctypes.c_void_p
    lib.sccg_gen_pairs.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int]
    lib.sccg_gen_free.argtypes = [ctypes.c_void_p]
    lib.sccg_gen_counts.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.sccg_gen_copy.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 7
    lib.sccg_gen_blob_flags.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.sccg_gen_mask.restype = ctypes.c_int
    lib.sccg_gen_mask.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_int64]
    lib.sccg_gen_sets_create.restype = ctypes.c_void_p
    lib.sccg_gen_sets_create.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int]
    lib.sccg_gen_sets_free.argtypes = [ctypes.c_void_p]
    lib.sccg_gen_sets_counts.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.sccg_gen_sets_copy.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 7
    lib.sccg_gen_sets_poly_off.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.sccg_gen_trace_mask.restype = ctypes.c_int64
    lib.sccg_gen_trace_mask.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_int64]
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


@dataclass
class Polys:
    """CSR rings: polygon k has vertices xy[off[k]:off[k+1]] (int32 pairs)."""
    off: np.ndarray  # int64 [n+1]
    xy: np.ndarray   # int32 [V, 2]

    @property
    def n(self) -> int:
        return len(self.off) - 1

    def ring(self, k: int) -> np.ndarray:
        return self.xy[self.off[k]:self.off[k + 1]]


@dataclass
class PairWorkload:
    config: int
    seed: int
    A: Polys
    B: Polys
    pa: np.ndarray      # int32 [n_pairs]
    pb: np.ndarray      # int32 [n_pairs]
    set_off: np.ndarray  # int64 [n_sets+1]
    blob: np.ndarray    # uint8 [n_pairs]
    stats: dict
    _handle: int = 0

    @property
    def n_pairs(self) -> int:
        return len(self.pa)

    def mask(self, which: int, i: int):
        """Raster mask of polygon i of A (which=0) or B (which=1):
        returns (bits[h, w] uint8, ox, oy) with pixel (ox+x, oy+y) = bits[y, x]."""
        lib = _load()
        info = np.zeros(4, np.int64)
        if lib.sccg_gen_mask(self._handle, which, i, _ptr(info), None, 0) != 0:
            raise IndexError(i)
        w, h, ox, oy = (int(v) for v in info)
        bits = np.zeros((h, w), np.uint8)
        lib.sccg_gen_mask(self._handle, which, i, _ptr(info), _ptr(bits), bits.size)
        return bits, ox, oy

    def close(self):
        if self._handle:
            _load().sccg_gen_free(self._handle)
            self._handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pairs(config: int, n_pairs: int | None = None, seed: int | None = None,
          threads: int | None = None) -> PairWorkload:
    """Generate the pair workload `config` (1, 2 or 3)."""
    lib = _load()
    if n_pairs is None:
        n_pairs = DEFAULT_PAIRS[config]
    if seed is None:
        seed = BASE_SEED + config
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    h = lib.sccg_gen_pairs(config, seed, n_pairs, threads)
    if not h:
        raise ValueError("generator rejected the arguments")
    c = np.zeros(10, np.int64)
    lib.sccg_gen_counts(h, _ptr(c))
    nA, vA, nB, vB, npairs, nsets = (int(v) for v in c[:6])
    offA = np.zeros(nA + 1, np.int64)
    xyA = np.zeros((vA, 2), np.int32)
    offB = np.zeros(nB + 1, np.int64)
    xyB = np.zeros((vB, 2), np.int32)
    pa = np.zeros(npairs, np.int32)
    pb = np.zeros(npairs, np.int32)
    so = np.zeros(nsets + 1, np.int64)
    lib.sccg_gen_copy(h, _ptr(offA), _ptr(xyA), _ptr(offB), _ptr(xyB), _ptr(pa), _ptr(pb), _ptr(so))
    blob = np.zeros(npairs, np.uint8)
    lib.sccg_gen_blob_flags(h, _ptr(blob))
    stats = dict(tiles_used=int(c[6]), shapes_outside_vertex_range=int(c[7]), attempts=int(c[8]),
                 n_blobs=int(c[9]))
    return PairWorkload(config, seed, Polys(offA, xyA), Polys(offB, xyB), pa, pb, so, blob, stats, h)


@dataclass
class SetWorkload:
    """Set-level workload: per tile, a result set A and a result set B of
    polygons; candidate pairs from a uniform-grid MBR join, grouped by tile
    (pairs set_off[t]:set_off[t+1] belong to tile t)."""
    seed: int
    A: Polys
    B: Polys
    pa: np.ndarray
    pb: np.ndarray
    set_off: np.ndarray
    stats: dict
    a_set_off: np.ndarray = None  # int64 [n_tiles+1]: A polygons of tile t
    b_set_off: np.ndarray = None  # int64 [n_tiles+1]: B polygons of tile t

    @property
    def n_pairs(self) -> int:
        return len(self.pa)


def sets(n_tiles: int = 64, tile_side: int = 8192, cell: int = 64, seed: int | None = None,
         threads: int | None = None) -> SetWorkload:
    """Workload 4: n_tiles tiles of tile_side^2 px.  In each tile set A is
    filled pixel-disjoint with workload-2 shapes (10-60 px, 16-120 vertices),
    each dropped onto a per-column skyline near a cursor that walks the tile,
    until the tile is full; set B holds a shifted, dilated or eroded copy of
    85% of A's shapes plus 15% * |A| fresh shapes at uniform positions."""
    lib = _load()
    if seed is None:
        seed = BASE_SEED + 4
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    h = lib.sccg_gen_sets_create(seed, n_tiles, tile_side, cell, threads)
    if not h:
        raise ValueError("generator rejected the arguments")
    try:
        c = np.zeros(6, np.int64)
        lib.sccg_gen_sets_counts(h, _ptr(c))
        nA, vA, nB, vB, npairs, nt = (int(v) for v in c)
        offA = np.zeros(nA + 1, np.int64)
        xyA = np.zeros((vA, 2), np.int32)
        offB = np.zeros(nB + 1, np.int64)
        xyB = np.zeros((vB, 2), np.int32)
        pa = np.zeros(npairs, np.int32)
        pb = np.zeros(npairs, np.int32)
        so = np.zeros(nt + 1, np.int64)
        lib.sccg_gen_sets_copy(h, _ptr(offA), _ptr(xyA), _ptr(offB), _ptr(xyB), _ptr(pa), _ptr(pb), _ptr(so))
        aso = np.zeros(nt + 1, np.int64)
        bso = np.zeros(nt + 1, np.int64)
        lib.sccg_gen_sets_poly_off(h, _ptr(aso), _ptr(bso))
    finally:
        lib.sccg_gen_sets_free(h)
    stats = dict(tiles=nt, polys_a=nA, polys_b=nB, pairs=npairs, tile_side=tile_side, cell=cell)
    return SetWorkload(seed, Polys(offA, xyA), Polys(offB, xyB), pa, pb, so, stats, aso, bso)


def trace_mask(bits: np.ndarray) -> np.ndarray | None:
    """Largest 4-component of a small mask (bits[y, x], y up), holes filled,
    traced into a counter-clockwise rectilinear ring; None if empty."""
    lib = _load()
    b = np.ascontiguousarray(bits, dtype=np.uint8)
    h, w = b.shape
    cap = 4 * (w + 1) * (h + 1)
    xy = np.zeros((cap, 2), np.int32)
    nv = lib.sccg_gen_trace_mask(_ptr(b), w, h, _ptr(xy), cap)
    if nv < 0:
        return None
    return xy[:nv].copy()


def concat(rings: list[np.ndarray]) -> Polys:
    """Pack a list of rings into CSR."""
    off = np.zeros(len(rings) + 1, np.int64)
    for k, r in enumerate(rings):
        off[k + 1] = off[k] + len(r)
    xy = np.concatenate([np.asarray(r, np.int32).reshape(-1, 2) for r in rings]) if rings else \
        np.zeros((0, 2), np.int32)
    return Polys(off, np.ascontiguousarray(xy, dtype=np.int32))

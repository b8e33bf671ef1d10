"""Strength of the oracle's pins: plant one plausible mistake at a time in a
copy of the oracle's C source (a shifted ray, a closed span, a dropped
absolute value, a wrong box, a swapped operand ...), build it, and check that
the pins of tests/test_oracle.py reject every such build while accepting the
real one.  Everything runs on the CPU; the real oracle is never modified."""

import math
import os

import numpy as np
import pytest

import oracle
import sccg_gen
from oracle import build as oracle_build
from tests import test_oracle as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "sccg_oracle.c")

# (name, text in the source, replacement); each text occurs exactly once
MUTANTS = [
    ("ray starts at the pixel edge", "if (xi > x && lo <= y && y < hi) inside ^= 1;",
     "if (xi >= x && lo <= y && y < hi) inside ^= 1;"),
    ("closed edge span", "if (xi > x && lo <= y && y < hi) inside ^= 1;",
     "if (xi > x && lo <= y && y <= hi) inside ^= 1;"),
    ("open lower span end", "if (xi > x && lo <= y && y < hi) inside ^= 1;",
     "if (xi > x && lo < y && y < hi) inside ^= 1;"),
    ("x and y swapped in the ray test", "if (xi > x && lo <= y && y < hi) inside ^= 1;",
     "if (yi > x && lo <= y && y < hi) inside ^= 1;"),
    ("horizontal edges taken for vertical", "if (xi != xj) continue; /* not vertical",
     "if (xi == xj) continue; /* not vertical"),
    ("no absolute value of the shoelace sum", "  if (s < 0) s = -s;\n", "\n"),
    ("shoelace operand swapped", "- (__int128)xy[2 * j] * xy[2 * i + 1];", "- (__int128)xy[2 * j + 1] * xy[2 * i];"),
    ("shoelace without its closing edge", "int64_t j = (i + 1 == nv) ? 0 : i + 1;\n    s +=",
     "int64_t j = (i + 1 == nv) ? i : i + 1;\n    s +="),
    ("shoelace not halved", "return (int64_t)(s / 2);", "return (int64_t)(s);"),
    ("union counted as symmetric difference", "*I += a & b;\n      *U += a | b;\n    }\n}",
     "*I += a & b;\n      *U += a ^ b;\n    }\n}"),
    ("intersection counted as union", "*I += a & b;\n      *U += a | b;\n    }\n}",
     "*I += a | b;\n      *U += a | b;\n    }\n}"),
    ("box of the pair is the MBR intersection",
     "int64_t x0 = px0 < qx0 ? px0 : qx0, y0 = py0 < qy0 ? py0 : qy0;\n"
     "  int64_t x1 = px1 > qx1 ? px1 : qx1, y1 = py1 > qy1 ? py1 : qy1;\n  for (int64_t y = y0; y < y1; ++y)\n    for",
     "int64_t x0 = px0 > qx0 ? px0 : qx0, y0 = py0 > qy0 ? py0 : qy0;\n"
     "  int64_t x1 = px1 < qx1 ? px1 : qx1, y1 = py1 < qy1 ? py1 : qy1;\n  for (int64_t y = y0; y < y1; ++y)\n    for"),
    ("MBR misses its last column", "if (x > *x1) *x1 = x;", "if (x > *x1) *x1 = x - 1;"),
    ("row form: ray starts at the pixel edge", "a ^= (bufp[e] > x);", "a ^= (bufp[e] >= x);"),
    ("row form: closed edge span", "if (lo <= y && y < hi) xs[k++] = xi;", "if (lo <= y && y <= hi) xs[k++] = xi;"),
    ("row form: q tested against p's edges", "b ^= (bufq[e] > x);", "b ^= (bufp[e] > x);"),
    ("row form: columns start at p's MBR", "for (int64_t x = x0; x < x1; ++x) {\n      int a = 0, b = 0;",
     "for (int64_t x = px0; x < x1; ++x) {\n      int a = 0, b = 0;"),
    ("empty ring counted into the intersection", "*U += sccg_oracle_pixel_inside(r, nr, x, y);",
     "*I += sccg_oracle_pixel_inside(r, nr, x, y);"),
    ("zero-intersection pairs kept in the set sums", "if (!include_zero && inter[k] == 0) continue;",
     "if (!include_zero && inter[k] < 0) continue;"),
    ("J by integer division", "(double)si / (double)su", "(double)(si / su)"),
]


@pytest.fixture(scope="module")
def fixtures():
    masks = pins._valid_4x4_masks()
    rings = [sccg_gen.trace_mask(pins._bits(m)) for m in masks]
    return (masks, rings), sccg_gen.pairs(1)


def battery(fixtures):
    """The pins, cheapest first; returns the name of the first that fails,
    or None if all hold."""
    tiny, cfg1 = fixtures
    checks = [
        ("pixel_inside_square", lambda: pins.test_pixel_inside_square()),
        ("rectangles", lambda: pins.test_rectangles_closed_form()),
        ("l_shapes", lambda: pins.test_l_shapes_closed_form()),
        ("containment", lambda: pins.test_containment_and_degenerate()),
        ("empty_rings", lambda: pins.test_empty_rings()),
        ("band_polygons", lambda: pins.test_band_polygons_closed_form(3)),
        ("band_polygons_7", lambda: pins.test_band_polygons_closed_form(7)),
        ("tiny_grid", lambda: pins.test_tiny_grid_exhaustive_single(tiny)),
        ("invariants", lambda: pins.test_invariants_config1(cfg1)),
        ("k_squared", lambda: pins.test_scale_k_squared(cfg1, 3)),
        ("generator_masks", lambda: pins.test_generator_masks_config1(cfg1)),
        ("jaccard_rational", lambda: pins.test_jaccard_exact_rational()),
        ("jprime_sum", lambda: pins.test_jprime_exact_sum()),
    ]
    for name, f in checks:
        try:
            f()
        except AssertionError:
            return name
    return None


def _with_library(lib, fn):
    saved = oracle._lib
    oracle._lib = lib
    try:
        return fn()
    finally:
        oracle._lib = saved


def test_real_oracle_passes_every_pin(fixtures, tmp_path):
    out = str(tmp_path / "libreal.so")
    oracle_build.build(src=SRC, out=out)
    assert _with_library(oracle.load_library(out), lambda: battery(fixtures)) is None


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(fixtures, tmp_path, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site of '{name}' is not unique in the oracle source"
    src = tmp_path / "mutant.c"
    src.write_text(text.replace(old, new))
    out = str(tmp_path / "libmutant.so")
    oracle_build.build(src=str(src), out=out)
    caught = _with_library(oracle.load_library(out), lambda: battery(fixtures))
    assert caught is not None, f"no pin rejects the mistake '{name}'"


def test_naive_summation_of_jprime_is_caught(monkeypatch):
    """J' summed left to right in binary64 instead of rounded once from the
    exact sum: the exact-rational pin rejects it."""
    monkeypatch.setattr(math, "fsum", lambda xs: sum(xs))
    with pytest.raises(AssertionError):
        pins.test_jprime_exact_sum()

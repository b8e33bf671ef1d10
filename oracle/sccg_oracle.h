/* Test infrastructure: the plain CPU oracle for the PixelBox pair areas.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use
 * this library.  It shares no code with the device library: it computes the
 * definition of the result directly, pixel by pixel, as Section 3.1 of the
 * paper states it (a pixel is in a polygon iff a ray cast from it crosses the
 * boundary an odd number of times; intersection = pixels in both, union =
 * pixels in either), never by sampling boxes.
 *
 * Host pointers only.  Polygon k of a set is the ring
 * xy[2*off[k] .. 2*off[k+1]-1] (x0,y0,x1,y1,...), implicitly closed, either
 * orientation.
 */
#ifndef SCCG_ORACLE_H
#define SCCG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int64_t n_polys;
  const int64_t* offsets; /* [n_polys+1] */
  const int32_t* xy;      /* [2*offsets[n_polys]] */
} sccg_oracle_polys;

/* Even-odd crossing test of pixel (x,y) (centre (x+1/2, y+1/2)) against one
 * ring of nv vertices: 1 if inside. */
int sccg_oracle_pixel_inside(const int32_t* xy, int64_t nv, int64_t x, int64_t y);

/* |shoelace| / 2 of polygon k (Section 3.2's area formula, cyclic index,
 * absolute value per polygon). */
int64_t sccg_oracle_poly_area(const sccg_oracle_polys* P, int64_t k);

/* Per pair, exact pixel counts of intersection and union over every pixel of
 * the bounding box of MBR(p) and MBR(q).  form 0 = pure (every edge tested
 * per pixel); form 1 = row-bucketed (per row, only the vertical edges whose
 * y-span holds that row).  n_threads <= 0 means 1. */
void sccg_oracle_area_pairs(const sccg_oracle_polys* A, const sccg_oracle_polys* B, int64_t n_pairs,
                            const int32_t* pair_a, const int32_t* pair_b, int64_t* out_inter,
                            int64_t* out_union, int form, int n_threads);

/* Per set s over pairs [set_off[s], set_off[s+1]): sums of I and U, the number
 * of contributing pairs and J = sum I / sum U (one binary64 division).  With
 * include_zero = 0 only pairs with I > 0 contribute (the paper's ratio > 0
 * filter).  J' (the mean of the ratios) is formed by the Python wrapper with
 * an exactly rounded sum. */
void sccg_oracle_jaccard_sets(int64_t n_sets, const int64_t* set_off, const int64_t* inter,
                              const int64_t* uni, int include_zero, int64_t* out_sum_i,
                              int64_t* out_sum_u, int64_t* out_n, double* out_j);

/* The filter stage of Section 4.1: candidate pairs with intersecting MBRs.
 * For each set s, every (a, b) with a in [a_off[s], a_off[s+1]) and b in
 * [b_off[s], b_off[s+1]) whose MBRs (the pixel extents [min x, max x) x
 * [min y, max y) of their vertices) share at least one pixel, ordered by set,
 * then b, then a.  Writes the first min(total, cap) pairs and the per-set
 * offsets (out_set_off[n_sets+1], counting every pair); returns the total. */
int64_t sccg_oracle_join_sets(const sccg_oracle_polys* A, const sccg_oracle_polys* B, int64_t n_sets,
                              const int64_t* a_off, const int64_t* b_off, int64_t cap, int32_t* out_pa,
                              int32_t* out_pb, int64_t* out_set_off);

/* Section 3.4's other operators, from the pixel counts: per pair a bit set
 *   1 intersects (I > 0),  2 A contains B (I == |B| > 0),  4 A within B
 *   (I == |A| > 0),  8 equal (I == |A| == |B| > 0),  16 touches (I == 0 and
 *   the two boundaries, as closed point sets, share a point).
 * The boundary test compares every edge of one ring with every edge of the
 * other (axis-parallel closed segments).  I comes from the pure pixel count. */
void sccg_oracle_relate_pairs(const sccg_oracle_polys* A, const sccg_oracle_polys* B, int64_t n_pairs,
                              const int32_t* pair_a, const int32_t* pair_b, uint32_t* out_rel);

#ifdef __cplusplus
}
#endif
#endif

/* Test infrastructure: the plain CPU oracle for the PixelBox pair areas.
 * Only tests, the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * What it computes, and where the paper defines it:
 *  - Pixelization (Section 3.1): a pixel is the unit square [x,x+1)x[y,y+1);
 *    the intersection area of p and q is the number of pixels inside both,
 *    the union area the number inside either.  Pixels whose centre lies
 *    inside a rectilinear integer polygon lie wholly inside it, because its
 *    boundary runs along pixel sides (Figure 3 and the accuracy discussion of
 *    Section 3.4).
 *  - Ray casting (Section 3.1): a pixel is inside iff a ray from it crosses
 *    the boundary an odd number of times.  Here the ray runs from the pixel
 *    centre towards +x.  At a half-integer height it never meets a vertex
 *    and never runs along a horizontal edge, so a crossing is exactly a
 *    vertical edge with X > x whose y-span [min, max) holds y.
 *  - Polygon area (Section 3.2): the shoelace sum, cyclic, absolute value
 *    taken per polygon.
 *  - The filter stage (Section 4.1): the candidate pairs of two polygon sets
 *    are those whose MBRs intersect; here MBR = pixel extent of the vertices,
 *    and two MBRs intersect when they share a pixel.  Every pair of a set is
 *    tested (no index).
 *  - Other operators (Section 3.4): containment when the intersection area
 *    equals the contained polygon's area; touching when the polygons share
 *    boundary points but no interior (here: no common pixel), tested by
 *    comparing every edge of one polygon with every edge of the other.
 *  - Jaccard (Section 2.1): J = total intersection / total union of a set of
 *    pairs.  J' (Equation 1, the mean of the per-pair ratios over the pairs
 *    with non-zero intersection) is formed in the Python wrapper.
 *
 * The union is counted directly (pixels in p or q), never as |p|+|q|-I, so
 * the identity I + U = |p| + |q| that the method relies on (Section 3.2)
 * stays a test, not an assumption.
 *
 * Parity pins (checked by the CPU tests): closed forms for rectangles and
 * L-shapes, pixel count of a polygon = its shoelace area, I + U = |p| + |q|,
 * symmetry, containment, disjointness, translation, k^2 scaling (the
 * coordinate scaling of Section 5.2), exhaustive 4x4 masks against mask
 * popcounts, generator masks against mask popcounts, and the rounding of J
 * against exact rational arithmetic.
 */
#include "sccg_oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

int sccg_oracle_pixel_inside(const int32_t* xy, int64_t nv, int64_t x, int64_t y) {
  int inside = 0;
  for (int64_t i = 0; i < nv; ++i) {
    int64_t j = (i + 1 == nv) ? 0 : i + 1;
    int64_t xi = xy[2 * i], yi = xy[2 * i + 1];
    int64_t xj = xy[2 * j], yj = xy[2 * j + 1];
    if (xi != xj) continue; /* not vertical: the ray never crosses it */
    int64_t lo = yi < yj ? yi : yj, hi = yi < yj ? yj : yi;
    if (xi > x && lo <= y && y < hi) inside ^= 1;
  }
  return inside;
}

int64_t sccg_oracle_poly_area(const sccg_oracle_polys* P, int64_t k) {
  const int32_t* xy = P->xy + 2 * P->offsets[k];
  int64_t nv = P->offsets[k + 1] - P->offsets[k];
  __int128 s = 0;
  for (int64_t i = 0; i < nv; ++i) {
    int64_t j = (i + 1 == nv) ? 0 : i + 1;
    s += (__int128)xy[2 * i] * xy[2 * j + 1] - (__int128)xy[2 * j] * xy[2 * i + 1];
  }
  if (s < 0) s = -s;
  return (int64_t)(s / 2);
}

static void ring_mbr(const int32_t* xy, int64_t nv, int64_t* x0, int64_t* y0, int64_t* x1, int64_t* y1) {
  /* pixel extent [x0,x1) x [y0,y1) of the ring's vertices */
  *x0 = *y0 = INT64_MAX;
  *x1 = *y1 = INT64_MIN;
  for (int64_t i = 0; i < nv; ++i) {
    int64_t x = xy[2 * i], y = xy[2 * i + 1];
    if (x < *x0) *x0 = x;
    if (x > *x1) *x1 = x;
    if (y < *y0) *y0 = y;
    if (y > *y1) *y1 = y;
  }
}

/* Pure form: every pixel of the box, every edge of both rings. */
static void pair_pure(const int32_t* p, int64_t np, const int32_t* q, int64_t nq, int64_t* I, int64_t* U) {
  int64_t px0, py0, px1, py1, qx0, qy0, qx1, qy1;
  *I = 0;
  *U = 0;
  if (np == 0 || nq == 0) {
    /* an empty ring covers no pixel; the other is counted on its own box */
    const int32_t* r = np ? p : q;
    int64_t nr = np ? np : nq;
    if (nr == 0) return;
    ring_mbr(r, nr, &px0, &py0, &px1, &py1);
    for (int64_t y = py0; y < py1; ++y)
      for (int64_t x = px0; x < px1; ++x) *U += sccg_oracle_pixel_inside(r, nr, x, y);
    return;
  }
  ring_mbr(p, np, &px0, &py0, &px1, &py1);
  ring_mbr(q, nq, &qx0, &qy0, &qx1, &qy1);
  int64_t x0 = px0 < qx0 ? px0 : qx0, y0 = py0 < qy0 ? py0 : qy0;
  int64_t x1 = px1 > qx1 ? px1 : qx1, y1 = py1 > qy1 ? py1 : qy1;
  for (int64_t y = y0; y < y1; ++y)
    for (int64_t x = x0; x < x1; ++x) {
      int a = sccg_oracle_pixel_inside(p, np, x, y);
      int b = sccg_oracle_pixel_inside(q, nq, x, y);
      *I += a & b;
      *U += a | b;
    }
}

/* Row-bucketed form: for each row, first collect the X of the vertical edges
 * whose y-span holds the row, then test each pixel of the row against only
 * those.  Same definition, fewer edge visits. */
static int64_t collect_row(const int32_t* r, int64_t nr, int64_t y, int64_t* xs) {
  int64_t k = 0;
  for (int64_t i = 0; i < nr; ++i) {
    int64_t j = (i + 1 == nr) ? 0 : i + 1;
    int64_t xi = r[2 * i], yi = r[2 * i + 1], xj = r[2 * j], yj = r[2 * j + 1];
    if (xi != xj) continue;
    int64_t lo = yi < yj ? yi : yj, hi = yi < yj ? yj : yi;
    if (lo <= y && y < hi) xs[k++] = xi;
  }
  return k;
}

static void pair_rows(const int32_t* p, int64_t np, const int32_t* q, int64_t nq, int64_t* I, int64_t* U,
                      int64_t* bufp, int64_t* bufq) {
  int64_t px0, py0, px1, py1, qx0, qy0, qx1, qy1;
  *I = 0;
  *U = 0;
  if (np == 0 || nq == 0) {
    pair_pure(p, np, q, nq, I, U);
    return;
  }
  ring_mbr(p, np, &px0, &py0, &px1, &py1);
  ring_mbr(q, nq, &qx0, &qy0, &qx1, &qy1);
  int64_t x0 = px0 < qx0 ? px0 : qx0, y0 = py0 < qy0 ? py0 : qy0;
  int64_t x1 = px1 > qx1 ? px1 : qx1, y1 = py1 > qy1 ? py1 : qy1;
  for (int64_t y = y0; y < y1; ++y) {
    int64_t kp = collect_row(p, np, y, bufp);
    int64_t kq = collect_row(q, nq, y, bufq);
    for (int64_t x = x0; x < x1; ++x) {
      int a = 0, b = 0;
      for (int64_t e = 0; e < kp; ++e) a ^= (bufp[e] > x);
      for (int64_t e = 0; e < kq; ++e) b ^= (bufq[e] > x);
      *I += a & b;
      *U += a | b;
    }
  }
}

typedef struct {
  const sccg_oracle_polys *A, *B;
  int64_t n_pairs;
  const int32_t *pa, *pb;
  int64_t *I, *U;
  int form;
  int64_t next; /* shared work counter */
} job_t;

static void* worker(void* arg) {
  job_t* J = (job_t*)arg;
  int64_t cap = 0;
  int64_t *bp = NULL, *bq = NULL;
  for (;;) {
    int64_t i0 = __atomic_fetch_add(&J->next, 16, __ATOMIC_RELAXED);
    if (i0 >= J->n_pairs) break;
    int64_t i1 = i0 + 16 < J->n_pairs ? i0 + 16 : J->n_pairs;
    for (int64_t i = i0; i < i1; ++i) {
      int64_t a = J->pa[i], b = J->pb[i];
      const int32_t* p = J->A->xy + 2 * J->A->offsets[a];
      int64_t np = J->A->offsets[a + 1] - J->A->offsets[a];
      const int32_t* q = J->B->xy + 2 * J->B->offsets[b];
      int64_t nq = J->B->offsets[b + 1] - J->B->offsets[b];
      if (J->form == 0) {
        pair_pure(p, np, q, nq, &J->I[i], &J->U[i]);
      } else {
        int64_t need = (np > nq ? np : nq) + 1;
        if (need > cap) {
          free(bp);
          free(bq);
          cap = need;
          bp = (int64_t*)malloc(sizeof(int64_t) * cap);
          bq = (int64_t*)malloc(sizeof(int64_t) * cap);
        }
        pair_rows(p, np, q, nq, &J->I[i], &J->U[i], bp, bq);
      }
    }
  }
  free(bp);
  free(bq);
  return NULL;
}

void sccg_oracle_area_pairs(const sccg_oracle_polys* A, const sccg_oracle_polys* B, int64_t n_pairs,
                            const int32_t* pair_a, const int32_t* pair_b, int64_t* out_inter,
                            int64_t* out_union, int form, int n_threads) {
  job_t J;
  J.A = A;
  J.B = B;
  J.n_pairs = n_pairs;
  J.pa = pair_a;
  J.pb = pair_b;
  J.I = out_inter;
  J.U = out_union;
  J.form = form;
  J.next = 0;
  if (n_threads <= 1) {
    worker(&J);
    return;
  }
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)n_threads);
  for (int t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, worker, &J);
  for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
  free(th);
}

void sccg_oracle_jaccard_sets(int64_t n_sets, const int64_t* set_off, const int64_t* inter,
                              const int64_t* uni, int include_zero, int64_t* out_sum_i,
                              int64_t* out_sum_u, int64_t* out_n, double* out_j) {
  for (int64_t s = 0; s < n_sets; ++s) {
    int64_t si = 0, su = 0, n = 0;
    for (int64_t k = set_off[s]; k < set_off[s + 1]; ++k) {
      if (!include_zero && inter[k] == 0) continue;
      si += inter[k];
      su += uni[k];
      n += 1;
    }
    out_sum_i[s] = si;
    out_sum_u[s] = su;
    out_n[s] = n;
    out_j[s] = (su > 0) ? (double)si / (double)su : 0.0;
  }
}

static void poly_mbr(const sccg_oracle_polys* P, int64_t k, int64_t* m) {
  const int64_t o = P->offsets[k], nv = P->offsets[k + 1] - o;
  if (nv <= 0) { /* no vertices: an MBR that holds no pixel */
    m[0] = m[1] = 1;
    m[2] = m[3] = 0;
    return;
  }
  ring_mbr(P->xy + 2 * o, nv, &m[0], &m[1], &m[2], &m[3]);
}

int64_t sccg_oracle_join_sets(const sccg_oracle_polys* A, const sccg_oracle_polys* B, int64_t n_sets,
                              const int64_t* a_off, const int64_t* b_off, int64_t cap, int32_t* out_pa,
                              int32_t* out_pb, int64_t* out_set_off) {
  int64_t total = 0;
  for (int64_t s = 0; s < n_sets; ++s) {
    if (out_set_off) out_set_off[s] = total;
    for (int64_t b = b_off[s]; b < b_off[s + 1]; ++b) {
      int64_t mb[4];
      poly_mbr(B, b, mb);
      for (int64_t a = a_off[s]; a < a_off[s + 1]; ++a) {
        int64_t ma[4];
        poly_mbr(A, a, ma);
        const int64_t x0 = ma[0] > mb[0] ? ma[0] : mb[0], x1 = ma[2] < mb[2] ? ma[2] : mb[2];
        const int64_t y0 = ma[1] > mb[1] ? ma[1] : mb[1], y1 = ma[3] < mb[3] ? ma[3] : mb[3];
        if (x0 < x1 && y0 < y1) {
          if (total < cap) {
            out_pa[total] = (int32_t)a;
            out_pb[total] = (int32_t)b;
          }
          ++total;
        }
      }
    }
  }
  if (out_set_off) out_set_off[n_sets] = total;
  return total;
}

/* Do the closed axis-parallel segments (a0-a1) and (b0-b1) share a point?
 * Each segment equals its own bounding box. */
static int segments_meet(const int32_t* a0, const int32_t* a1, const int32_t* b0, const int32_t* b1) {
  const int64_t ax0 = a0[0] < a1[0] ? a0[0] : a1[0], ax1 = a0[0] < a1[0] ? a1[0] : a0[0];
  const int64_t ay0 = a0[1] < a1[1] ? a0[1] : a1[1], ay1 = a0[1] < a1[1] ? a1[1] : a0[1];
  const int64_t bx0 = b0[0] < b1[0] ? b0[0] : b1[0], bx1 = b0[0] < b1[0] ? b1[0] : b0[0];
  const int64_t by0 = b0[1] < b1[1] ? b0[1] : b1[1], by1 = b0[1] < b1[1] ? b1[1] : b0[1];
  return (ax0 > bx0 ? ax0 : bx0) <= (ax1 < bx1 ? ax1 : bx1) && (ay0 > by0 ? ay0 : by0) <= (ay1 < by1 ? ay1 : by1);
}

void sccg_oracle_relate_pairs(const sccg_oracle_polys* A, const sccg_oracle_polys* B, int64_t n_pairs,
                              const int32_t* pair_a, const int32_t* pair_b, uint32_t* out_rel) {
  for (int64_t k = 0; k < n_pairs; ++k) {
    const int64_t a = pair_a[k], b = pair_b[k];
    const int32_t* p = A->xy + 2 * A->offsets[a];
    const int64_t np = A->offsets[a + 1] - A->offsets[a];
    const int32_t* q = B->xy + 2 * B->offsets[b];
    const int64_t nq = B->offsets[b + 1] - B->offsets[b];
    int64_t I = 0, U = 0;
    pair_pure(p, np, q, nq, &I, &U);
    const int64_t ap = sccg_oracle_poly_area(A, a), aq = sccg_oracle_poly_area(B, b);
    uint32_t r = 0;
    if (I > 0) r |= 1u;
    if (I > 0 && I == aq) r |= 2u;
    if (I > 0 && I == ap) r |= 4u;
    if (I > 0 && I == ap && I == aq) r |= 8u;
    if (I == 0 && np > 0 && nq > 0) {
      int meet = 0;
      for (int64_t i = 0; i < np && !meet; ++i) {
        const int64_t i1 = (i + 1 == np) ? 0 : i + 1;
        for (int64_t j = 0; j < nq && !meet; ++j) {
          const int64_t j1 = (j + 1 == nq) ? 0 : j + 1;
          meet = segments_meet(p + 2 * i, p + 2 * i1, q + 2 * j, q + 2 * j1);
        }
      }
      if (meet) r |= 16u;
    }
    out_rel[k] = r;
  }
}

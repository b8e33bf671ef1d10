// Section 3.4's other operators from the same machinery: containment and
// equality from the intersection count and the polygon areas, and touching
// (no common pixel, boundaries that share a point) from the edges.  One
// wave per pair; only pairs with no common pixel whose closed MBRs meet go
// on to the edge test, in which each lane holds one edge of p and the wave
// walks q's edges, stopping at the first pair of edges that meet.
#include <limits.h>

#include "sccg_device.h"

namespace sccg {

namespace {

// Do the closed axis-parallel segments v0-v1 and w0-w1 share a point?  Each
// equals its own bounding box.
__device__ __forceinline__ bool segments_meet(int2 v0, int2 v1, int2 w0, int2 w1) {
  return max(min(v0.x, v1.x), min(w0.x, w1.x)) <= min(max(v0.x, v1.x), max(w0.x, w1.x)) &&
         max(min(v0.y, v1.y), min(w0.y, w1.y)) <= min(max(v0.y, v1.y), max(w0.y, w1.y));
}

}  // namespace

__global__ void __launch_bounds__(256) k_relate(Polys A, Polys B, const Meta* metaA, const Meta* metaB,
                                                const int64_t* areaA, const int64_t* areaB, int64_t n_pairs,
                                                const int32_t* pa, const int32_t* pb, const int64_t* inter,
                                                uint32_t* out, uint32_t* err) {
  const int lane = lane_id();
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t k = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; k < n_pairs; k += waves) {
    const int64_t a = pa[k], b = pb[k];
    if (a < 0 || a >= A.n || b < 0 || b >= B.n) {
      if (lane == 0) {
        out[k] = 0;
        latch_error(err, kErrIndex);
      }
      continue;
    }
    const int64_t I = inter[k], ap = areaA[a], aq = areaB[b];
    uint32_t r = 0;
    if (I > 0) {
      r |= SCCG_REL_INTERSECTS;
      if (I == aq) r |= SCCG_REL_CONTAINS;
      if (I == ap) r |= SCCG_REL_WITHIN;
      if (I == ap && I == aq) r |= SCCG_REL_EQUALS;
    } else {
      // MBR extents are [x0, x1) in pixels: the vertices span [x0, x1] x [y0, y1]
      const Meta mp = load_meta(metaA, a), mq = load_meta(metaB, b);
      const bool near = mp.x0 < mp.x1 && mq.x0 < mq.x1 && max(mp.x0, mq.x0) <= min(mp.x1, mq.x1) &&
                        max(mp.y0, mq.y0) <= min(mp.y1, mq.y1);
      if (near) {
        const int64_t op = A.off[a], np = A.off[a + 1] - op;
        const int64_t oq = B.off[b], nq = B.off[b + 1] - oq;
        bool meet = false;
        for (int64_t base = 0; base < np && !meet; base += kWave) {
          const int64_t i = base + lane;
          int2 v0 = make_int2(0, 0), v1 = make_int2(0, 0);
          const bool mine = i < np;
          if (mine) {
            v0 = A.xy[op + i];
            v1 = A.xy[op + (i + 1 == np ? 0 : i + 1)];
          }
          bool hit = false;
          int2 w0 = B.xy[oq];
          for (int64_t j = 0; j < nq; ++j) {
            const int2 w1 = B.xy[oq + (j + 1 == nq ? 0 : j + 1)];
            hit = hit || (mine && segments_meet(v0, v1, w0, w1));
            w0 = w1;
            if ((j & 15) == 15 && ballot(hit)) break;
          }
          meet = ballot(hit) != 0ull;
        }
        if (meet) r |= SCCG_REL_TOUCHES;
      }
    }
    if (lane == 0) out[k] = r;
  }
}

hipError_t launch_relate(const Polys& A, const Polys& B, const Meta* metaA, const Meta* metaB, const int64_t* areaA,
                         const int64_t* areaB, int64_t n_pairs, const int32_t* pa, const int32_t* pb,
                         const int64_t* inter, uint32_t* out, uint32_t* err, hipStream_t s) {
  if (n_pairs <= 0) return hipSuccess;
  const int64_t blocks = min((n_pairs + 3) / 4, (int64_t)65536);
  hipLaunchKernelGGL(k_relate, dim3((unsigned)blocks), dim3(256), 0, s, A, B, metaA, metaB, areaA, areaB, n_pairs, pa,
                     pb, inter, out, err);
  return hipGetLastError();
}

}  // namespace sccg

// PLAIN mode: Algorithm 1 of the paper as printed, on gfx950.
//
// One polygon pair per workgroup (grid-stride over pairs, Algorithm 1's
// outer loop).  The pair box is pushed on a shared stack of sampling boxes
// with a "continue" flag; each popped box is either pixelized (BOXSIZE < T:
// every thread tests its pixels against every edge of both polygons with the
// crossing rule) or split into one sub-box per thread (SUBSAMPBOX), each
// thread classifies its sub-box against both polygons (BOXPOSITION, Lemma 1),
// adds the size of sub-boxes inside both, and pushes its sub-box with the
// continue flag above the popped entry, which is marked dead instead of being
// overwritten (Section 3.3).  Shared-memory vertex staging with a static cap,
// a split (structure-of-arrays) stack and an unrolled edge loop are the
// implementation optimizations of Section 3.3.
//
// Differences from the printed listing, none of which changes a count:
//   - the per-thread partial sums are reduced on the device (wave shuffles)
//     instead of being copied to the host;
//   - a second barrier after reading the popped entry, so that no thread can
//     still be reading it when thread 0 marks it dead (the listing relies on a
//     warp being the whole block);
//   - the polygon areas come from the per-polygon prepass.
#include <limits.h>

#include "sccg_device.h"

namespace sccg {

enum : int { kOut = 0, kIn = 1, kHover = 2 };

// Stack depth bound: ceil-splitting a side of 32767 by g until it reaches 1.
__host__ __device__ inline int plain_levels(int g) {
  int levels = 0;
  for (int s = kMaxSide; s > 1; s = (s + g - 1) / g) ++levels;
  return levels + 1;
}

__host__ __device__ inline int plain_stack_cap(int wg, int gx, int gy) {
  return plain_levels(gx < gy ? gx : gy) * (wg + 1) + 2;
}

int plain_lds_bytes(int wg_size, int lds_vertex_cap) {
  // gx*gy == wg_size with min side >= 4 in every accepted configuration; size
  // the stack for the worst (min side 4)
  const int cap = plain_stack_cap(wg_size, 4, 4);
  return lds_vertex_cap * 8 + cap * 9 + 64 + 16 * 8;
}

// Even-odd crossing count of the +x ray from the centre of pixel (px, py):
// a vertical edge at X > px whose y-span [lo, hi) holds py.  Horizontal edges
// never satisfy the span test.
__device__ __forceinline__ int pixel_in_poly(const int2* R, int n, int px, int py) {
  int par = 0;
  int2 v = R[0];
#pragma unroll 4
  for (int i = 1; i < n; ++i) {
    const int2 w = R[i];
    par ^= ((v.y <= py) != (w.y <= py)) & (v.x > px);
    v = w;
  }
  const int2 w = R[0];
  par ^= ((v.y <= py) != (w.y <= py)) & (v.x > px);
  return par;
}

// Lemma 1 with the open-interior reading: a box hovers iff some edge meets
// its open interior (an edge crossing its sides or a vertex inside it);
// otherwise all its pixels share the position of its first pixel.
__device__ __forceinline__ int box_position(const int2* R, int n, int x0, int y0, int x1, int y1) {
  bool hover = false;
  int par = 0;
  auto edge = [&](int2 v, int2 w) {
    if (v.x == w.x) {
      const int X = v.x, lo = min(v.y, w.y), hi = max(v.y, w.y);
      hover |= (x0 < X) & (X < x1) & (lo < y1) & (hi > y0);
      par ^= (X > x0) & (lo <= y0) & (y0 < hi);
    } else {
      const int Y = v.y, lo = min(v.x, w.x), hi = max(v.x, w.x);
      hover |= (y0 < Y) & (Y < y1) & (lo < x1) & (hi > x0);
    }
  };
  int2 v = R[0];
#pragma unroll 4
  for (int i = 1; i < n; ++i) {
    const int2 w = R[i];
    edge(v, w);
    v = w;
  }
  edge(v, R[0]);
  return hover ? kHover : (par ? kIn : kOut);
}

template <int WG>
__global__ void __launch_bounds__(WG) k_plain(PlainArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int cap_v = a.lds_vertex_cap;
  const int scap = plain_stack_cap(WG, a.gx, a.gy);
  int2* verts = reinterpret_cast<int2*>(smem);
  int16_t* sx0 = reinterpret_cast<int16_t*>(smem + (size_t)cap_v * 8);
  int16_t* sy0 = sx0 + scap;
  int16_t* sx1 = sy0 + scap;
  int16_t* sy1 = sx1 + scap;
  uint8_t* sc = reinterpret_cast<uint8_t*>(sy1 + scap);
  unsigned long long* wred = reinterpret_cast<unsigned long long*>(
      smem + (((size_t)cap_v * 8 + (size_t)scap * 9 + 15) & ~(size_t)15));

  const int tid = threadIdx.x;
  const int T = a.box_threshold;
  const int gx = a.gx, gy = a.gy;
  const int si = tid % gx, sj = tid / gx;  // this thread's sub-box in the split grid

  for (int64_t i = blockIdx.x; i < a.n_pairs; i += gridDim.x) {
    const int64_t ia = a.pa[i], ib = a.pb[i];
    if (ia < 0 || ia >= a.A.n || ib < 0 || ib >= a.B.n) {
      if (tid == 0) {
        latch_error(a.err, kErrIndex);
        a.inter[i] = 0;
        a.uni[i] = 0;
      }
      continue;
    }
    const Meta mp = load_meta(a.metaA, ia), mq = load_meta(a.metaB, ib);
    const int64_t ap = a.areaA[ia], aq = a.areaB[ib];
    const Meta bx = pair_box(mp, mq);
    if (bx.x0 >= bx.x1 || bx.y0 >= bx.y1) {
      if (tid == 0) {
        a.inter[i] = 0;
        a.uni[i] = ap + aq;
      }
      continue;
    }
    if (side_u(bx.x0, bx.x1) > (uint32_t)kMaxSide || side_u(bx.y0, bx.y1) > (uint32_t)kMaxSide) {
      if (tid == 0) {
        latch_error(a.err, kErrSide);
        a.inter[i] = 0;
        a.uni[i] = 0;
      }
      continue;
    }
    const int64_t op = a.A.off[ia], oq = a.B.off[ib];
    const int np = (int)(a.A.off[ia + 1] - op), nq = (int)(a.B.off[ib + 1] - oq);
    const int2* P;
    const int2* Q;
    if (np + nq <= cap_v) {
      for (int k = tid; k < np; k += WG) verts[k] = a.A.xy[op + k];
      for (int k = tid; k < nq; k += WG) verts[np + k] = a.B.xy[oq + k];
      P = verts;
      Q = verts + np;
    } else {
      P = a.A.xy + op;
      Q = a.B.xy + oq;
    }
    // the stack holds boxes relative to the pair box origin
    const int ox = bx.x0, oy = bx.y0;
    if (tid == 0) {
      sx0[0] = 0;
      sy0[0] = 0;
      sx1[0] = (int16_t)(bx.x1 - ox);
      sy1[0] = (int16_t)(bx.y1 - oy);
      sc[0] = 1;
    }
    unsigned long long acc = 0, tests = 0, nleaf = 0, nsplit = 0, edge_tests = 0, box_tests = 0;
    int top = 1;
    bool overflow = false;
    while (top > 0) {
      top -= 1;
      __syncthreads();
      const int bx0 = sx0[top], by0 = sy0[top], bx1 = sx1[top], by1 = sy1[top];
      const int c = sc[top];
      __syncthreads();
      if (c == 0) continue;
      const int w = bx1 - bx0, h = by1 - by0;
      const int size = w * h;
      if (size < T) {
        // PIXELINPOLY over the box's pixels, WG at a time
        const int stepy = WG / w, stepx = WG % w;
        int jx = tid % w, jy = tid / w;
        for (int j = tid; j < size; j += WG) {
          const int px = ox + bx0 + jx, py = oy + by0 + jy;
          const int in_p = pixel_in_poly(P, np, px, py);
          const int in_q = pixel_in_poly(Q, nq, px, py);
          acc += (unsigned)(in_p & in_q);
          jx += stepx;
          jy += stepy;
          if (jx >= w) {
            jx -= w;
            jy += 1;
          }
        }
        tests += 2ull * (unsigned)size;
        edge_tests += (unsigned long long)size * (unsigned)(np + nq);
        nleaf += 1;
      } else {
        // SUBSAMPBOX: cut lines at x0 + floor(k*w/gx), y0 + floor(k*h/gy)
        const int cx0 = bx0 + (si * w) / gx, cx1 = bx0 + ((si + 1) * w) / gx;
        const int cy0 = by0 + (sj * h) / gy, cy1 = by0 + ((sj + 1) * h) / gy;
        int cnext = 0;
        if (cx0 < cx1 && cy0 < cy1) {
          const int p1 = box_position(P, np, ox + cx0, oy + cy0, ox + cx1, oy + cy1);
          const int p2 = box_position(Q, nq, ox + cx0, oy + cy0, ox + cx1, oy + cy1);
          // BOXCONTINUE / BOXCONTRIBUTE
          cnext = (p1 != kOut) & (p2 != kOut) & !((p1 == kIn) & (p2 == kIn));
          const int t = (p1 == kIn) & (p2 == kIn);
          acc += (unsigned long long)((1 - cnext) * t) * (unsigned)((cx1 - cx0) * (cy1 - cy0));
          box_tests += (unsigned)(np + nq);
        }
        if (top + 1 + WG > scap) {
          overflow = true;  // cannot happen for sides <= 32767; kept as a guard
          break;
        }
        sx0[top + 1 + tid] = (int16_t)cx0;
        sy0[top + 1 + tid] = (int16_t)cy0;
        sx1[top + 1 + tid] = (int16_t)cx1;
        sy1[top + 1 + tid] = (int16_t)cy1;
        sc[top + 1 + tid] = (uint8_t)cnext;
        if (tid == 0) sc[top] = 0;
        top += 1 + WG;
        nsplit += 1;
      }
    }
    // on-device reduction of the per-thread partial intersections
    unsigned long long s = wave_sum_u64(acc);
    if (WG > kWave) {
      if ((tid & (kWave - 1)) == 0) wred[tid / kWave] = s;
      __syncthreads();
      if (tid == 0)
        for (int k = 1; k < WG / kWave; ++k) s += wred[k];
    }
    if (a.stats) {
      const unsigned long long bt = wave_sum_u64(box_tests);
      if ((tid & (kWave - 1)) == 0) atomicAdd(&a.stats[9], bt);
    }
    if (tid == 0) {
      if (overflow) latch_error(a.err, kErrWatchdog);
      a.inter[i] = (int64_t)s;
      a.uni[i] = ap + aq - (int64_t)s;
      if (a.stats) {
        atomicAdd(&a.stats[0], tests);
        atomicAdd(&a.stats[1], nleaf);
        atomicAdd(&a.stats[2], nsplit);
        atomicAdd(&a.stats[8], edge_tests);
      }
    }
    __syncthreads();
  }
}

int plain_occupancy(int wg_size, int lds_vertex_cap) {
  int n = 0;
  const size_t lds = (size_t)plain_lds_bytes(wg_size, lds_vertex_cap);
  hipError_t e = hipErrorInvalidValue;
  switch (wg_size) {
    case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_plain<64>, 64, lds); break;
    case 128: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_plain<128>, 128, lds); break;
    case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_plain<256>, 256, lds); break;
  }
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_plain(const PlainArgs& a, int wg_size, int grid, hipStream_t s) {
  if (a.n_pairs <= 0) return hipSuccess;
  const size_t lds = (size_t)plain_lds_bytes(wg_size, a.lds_vertex_cap);
  switch (wg_size) {
    case 64: hipLaunchKernelGGL(k_plain<64>, dim3(grid), dim3(64), lds, s, a); break;
    case 128: hipLaunchKernelGGL(k_plain<128>, dim3(grid), dim3(128), lds, s, a); break;
    case 256: hipLaunchKernelGGL(k_plain<256>, dim3(grid), dim3(256), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sccg

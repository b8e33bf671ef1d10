// PLAIN mode: the PixelBox method of Section 3.3 in its direct GPU form, one
// polygon pair per workgroup, one sampling sub-box or one pixel per thread.
//
// A workgroup takes pairs in a grid-stride loop.  For its pair it keeps, in
// LDS, a stack of the boxes still to be decided ("live" boxes), starting with
// the pair box MBR(p) ∩ MBR(q):
//   - a live box of fewer than T pixels is pixelized (Section 3.1): its pixels
//     are dealt out to the threads row by row, and each pixel centre is tested
//     against both rings with the even-odd crossing rule;
//   - a larger live box is cut into a gx x gy grid of sub-boxes, one per
//     thread.  Each thread places its sub-box against both polygons by Lemma 1
//     (inside, outside or hovering), counts its pixels at once if it lies
//     inside both, drops it if it lies outside either, and otherwise keeps it.
//     The kept sub-boxes are compacted onto the stack with a workgroup-wide
//     count of the keep flags, so the stack only ever holds live boxes.
// The pixels counted by all threads are summed on the device; the union comes
// from the polygon areas of the per-polygon prepass, |p ∪ q| = |p| + |q| −
// |p ∩ q| (Section 3.2).  Both rings are staged in LDS when they fit
// lds_vertex_cap (Section 3.3's use of shared memory), else read from global
// memory.
#include <limits.h>

#include "sccg_device.h"

namespace sccg {

namespace {

enum Place : int { kOutside = 0, kInside = 1, kHovering = 2 };

// Depth bound of the stack: the longest side (at most kMaxSide) shrinks to
// ceil(side / g) per split, g = the smaller grid side.
__host__ __device__ inline int plain_depth(int g) {
  int d = 1;
  for (int side = kMaxSide; side > 1; side = (side + g - 1) / g) ++d;
  return d;
}

// A split keeps at most wg sub-boxes, and only the newest split's sub-boxes
// are split further, so every level of the depth bound holds at most wg boxes.
__host__ __device__ inline int plain_stack_boxes(int wg, int g_min) { return plain_depth(g_min) * wg + 1; }

// Crossing parity of the pixel centre (px + 1/2, py + 1/2) against ring R
// (Section 3.1): the number of vertical edges at X > px whose span
// [min y, max y) holds py, taken mod 2.  Every edge is the pair
// (previous vertex, vertex), the first one closing the ring.
__device__ __forceinline__ unsigned crossing_parity(const int2* R, int n, int px, int py) {
  unsigned odd = 0;
  if (n <= 0) return 0;  // a ring without edges covers nothing
  int2 prev = R[n - 1];
#pragma unroll 4
  for (int i = 0; i < n; ++i) {
    const int2 cur = R[i];
    const bool spans = (prev.y <= py) != (cur.y <= py);  // false for a horizontal edge
    odd ^= (unsigned)(spans && cur.x > px);
    prev = cur;
  }
  return odd;
}

// Lemma 1 (open-interior reading): the box [x0, x1) x [y0, y1) hovers R when
// an edge of R meets the box's open interior; otherwise the box lies wholly
// inside or wholly outside, and the crossing parity of its first pixel says
// which (a box's geometric centre can fall on a grid line, a pixel centre
// never does).
__device__ __forceinline__ Place place_box(const int2* R, int n, int x0, int y0, int x1, int y1) {
  bool meets = false;
  unsigned odd = 0;
  if (n <= 0) return kOutside;
  int2 prev = R[n - 1];
#pragma unroll 4
  for (int i = 0; i < n; ++i) {
    const int2 cur = R[i];
    if (prev.x == cur.x) {
      const int lo = min(prev.y, cur.y), hi = max(prev.y, cur.y);
      meets |= x0 < cur.x && cur.x < x1 && lo < y1 && y0 < hi;
      odd ^= (unsigned)(cur.x > x0 && lo <= y0 && y0 < hi);
    } else {
      const int lo = min(prev.x, cur.x), hi = max(prev.x, cur.x);
      meets |= y0 < cur.y && cur.y < y1 && lo < x1 && x0 < hi;
    }
    prev = cur;
  }
  return meets ? kHovering : (odd ? kInside : kOutside);
}

// Live boxes, relative to the pair-box origin (sides <= 32767 fit int16).
struct BoxStack {
  int16_t* x0;
  int16_t* y0;
  int16_t* x1;
  int16_t* y1;
};

}  // namespace

int plain_lds_bytes(int wg_size, int lds_vertex_cap) {
  // every accepted grid has both sides >= 4: size the stack for that worst case
  const int boxes = plain_stack_boxes(wg_size, 4);
  return lds_vertex_cap * 8 + boxes * 8 + 16 * 8 + 16;
}

template <int WG>
__global__ void __launch_bounds__(WG) k_plain(PlainArgs a) {
  constexpr int kWaves = WG / kWave;
  extern __shared__ __align__(16) unsigned char smem[];
  const int cap_v = a.lds_vertex_cap;
  const int gx = a.gx, gy = a.gy;
  const int boxes = plain_stack_boxes(WG, min(gx, gy));
  int2* staged = reinterpret_cast<int2*>(smem);
  BoxStack st;
  st.x0 = reinterpret_cast<int16_t*>(smem + (size_t)cap_v * 8);
  st.y0 = st.x0 + boxes;
  st.x1 = st.y0 + boxes;
  st.y1 = st.x1 + boxes;
  // per-wave keep counts (compaction) and partial sums (final reduction)
  unsigned long long* wave_word =
      reinterpret_cast<unsigned long long*>(smem + (((size_t)cap_v * 8 + (size_t)boxes * 8 + 15) & ~(size_t)15));

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  const int T = a.box_threshold;
  const int gi = tid % gx, gj = tid / gx;  // this thread's cell of a split grid

  for (int64_t k = blockIdx.x; k < a.n_pairs; k += gridDim.x) {
    const int64_t ia = a.pa[k], ib = a.pb[k];
    if (ia < 0 || ia >= a.A.n || ib < 0 || ib >= a.B.n) {
      if (tid == 0) {
        latch_error(a.err, kErrIndex);
        a.inter[k] = 0;
        a.uni[k] = 0;
      }
      continue;
    }
    const Meta box = pair_box(load_meta(a.metaA, ia), load_meta(a.metaB, ib));
    const int64_t area_sum = a.areaA[ia] + a.areaB[ib];
    if (box.x0 >= box.x1 || box.y0 >= box.y1) {  // the MBRs do not overlap
      if (tid == 0) {
        a.inter[k] = 0;
        a.uni[k] = area_sum;
      }
      continue;
    }
    if (side_u(box.x0, box.x1) > (uint32_t)kMaxSide || side_u(box.y0, box.y1) > (uint32_t)kMaxSide) {
      if (tid == 0) {
        latch_error(a.err, kErrSide);
        a.inter[k] = 0;
        a.uni[k] = 0;
      }
      continue;
    }
    const int64_t op = a.A.off[ia], oq = a.B.off[ib];
    const int np = (int)(a.A.off[ia + 1] - op), nq = (int)(a.B.off[ib + 1] - oq);
    const int2* P = a.A.xy + op;
    const int2* Q = a.B.xy + oq;
    if (np + nq <= cap_v) {
      for (int v = tid; v < np; v += WG) staged[v] = P[v];
      for (int v = tid; v < nq; v += WG) staged[np + v] = Q[v];
      P = staged;
      Q = staged + np;
    }
    const int ox = box.x0, oy = box.y0;
    if (tid == 0) {
      st.x0[0] = 0;
      st.y0[0] = 0;
      st.x1[0] = (int16_t)(box.x1 - ox);
      st.y1[0] = (int16_t)(box.y1 - oy);
    }
    unsigned long long inside = 0;  // pixels of p ∩ q this thread counted
    unsigned long long n_pix = 0, n_leaf = 0, n_split = 0, n_pix_edges = 0, n_box_edges = 0;
    int live = 1;  // boxes on the stack (the same in every thread)
    bool too_deep = false;
    while (live > 0) {
      __syncthreads();  // the last pushes (and the staged rings) are visible
      const int bx0 = st.x0[live - 1], by0 = st.y0[live - 1], bx1 = st.x1[live - 1], by1 = st.y1[live - 1];
      __syncthreads();  // every thread has the box before its slot is reused
      live -= 1;
      const int w = bx1 - bx0, h = by1 - by0;
      const int pixels = w * h;
      if (pixels < T) {
        // pixelize: thread t takes pixels t, t + WG, ... in row-major order
        const int dy = WG / w, dx = WG % w;
        int px = tid % w, py = tid / w;
        for (int t = tid; t < pixels; t += WG) {
          const int X = ox + bx0 + px, Y = oy + by0 + py;
          inside += crossing_parity(P, np, X, Y) & crossing_parity(Q, nq, X, Y);
          px += dx;
          py += dy;
          if (px >= w) {
            px -= w;
            py += 1;
          }
        }
        n_pix += 2ull * (unsigned)pixels;
        n_pix_edges += (unsigned long long)pixels * (unsigned)(np + nq);
        n_leaf += 1;
        continue;
      }
      // split: cell (gi, gj) spans [bx0 + floor(gi w / gx), bx0 + floor((gi + 1) w / gx)), likewise in y
      const int cx0 = bx0 + gi * w / gx, cx1 = bx0 + (gi + 1) * w / gx;
      const int cy0 = by0 + gj * h / gy, cy1 = by0 + (gj + 1) * h / gy;
      bool keep = false;
      if (cx0 < cx1 && cy0 < cy1) {
        const Place in_p = place_box(P, np, ox + cx0, oy + cy0, ox + cx1, oy + cy1);
        const Place in_q = place_box(Q, nq, ox + cx0, oy + cy0, ox + cx1, oy + cy1);
        if (in_p == kInside && in_q == kInside)
          inside += (unsigned long long)((cx1 - cx0) * (cy1 - cy0));
        else
          keep = in_p != kOutside && in_q != kOutside;
        n_box_edges += (unsigned)(np + nq);
      }
      // compaction of the kept cells onto the stack, in thread order
      const uint64_t kept = ballot(keep);
      if (lane == 0) wave_word[wave] = (unsigned long long)__popcll(kept);
      __syncthreads();
      int below = 0, total = 0;
#pragma unroll
      for (int v = 0; v < kWaves; ++v) {
        const int c = (int)wave_word[v];
        below += v < wave ? c : 0;
        total += c;
      }
      if (live + total > boxes) {  // cannot happen for sides <= 32767; a guard
        too_deep = true;
        break;
      }
      if (keep) {
        const int slot = live + below + lanes_below(kept);
        st.x0[slot] = (int16_t)cx0;
        st.y0[slot] = (int16_t)cy0;
        st.x1[slot] = (int16_t)cx1;
        st.y1[slot] = (int16_t)cy1;
      }
      live += total;
      n_split += 1;
    }
    // sum the threads' pixels: DPP within each wave, then across waves
    __syncthreads();
    unsigned long long sum = wave_sum_u64(inside);
    if (kWaves > 1) {
      if (lane == 0) wave_word[wave] = sum;
      __syncthreads();
      sum = 0;
#pragma unroll
      for (int v = 0; v < kWaves; ++v) sum += wave_word[v];
    }
    if (a.stats) {
      const unsigned long long be = wave_sum_u64(n_box_edges);
      if (lane == 0) atomicAdd(&a.stats[9], be);
    }
    if (tid == 0) {
      if (too_deep) latch_error(a.err, kErrWatchdog);
      a.inter[k] = (int64_t)sum;
      a.uni[k] = area_sum - (int64_t)sum;
      if (a.stats) {
        atomicAdd(&a.stats[0], n_pix);
        atomicAdd(&a.stats[1], n_leaf);
        atomicAdd(&a.stats[2], n_split);
        atomicAdd(&a.stats[8], n_pix_edges);
      }
    }
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

// BATCHED mode: every pair of a call in one persistent launch.
//
// The method is PixelBox (Section 3): a pair box is split into sampling
// boxes, each box is classified against both polygons with Lemma 1 (open-
// interior reading: a box hovers iff an edge meets its open interior,
// otherwise its first pixel decides), boxes inside both polygons count at
// once, boxes outside either are dropped, the rest are split again, and boxes
// that fit one leaf tile are pixelized with the even-odd crossing rule.
//
// How it is laid out on gfx950 (wave64, 256 CUs in 8 XCDs):
//   - A pair box that fits one 64x64 leaf tile (the small pairs, most of any
//     pathology workload) is pixelized at once: it is below the pixelization
//     threshold T = 64*64, the n^2 end of Section 3.4's range for n = 64.
//     When even the union of the two MBRs fits one tile, that tile is used
//     and I and U are both counted there, so the ring areas are not needed
//     (SCCG_F_NO_UNION_TILE turns this off).
//   - Larger boxes are split into at most 8x8 cells whose side is 64*8^l, so
//     that every split lands on leaf tiles after l more levels.  One wave
//     classifies all cells of a box in one pass over the edges: each lane
//     takes one edge and sets the bits of the cells it hovers and of the
//     cells whose first pixel it crosses, in two 64-bit masks, which are then
//     OR- and XOR-reduced across the wave.  Cost O(edges) per split instead of
//     O(cells x edges).  A split into fewer than min_classify_cells leaf
//     tiles is not classified: its tiles are pixelized directly.
//   - Rings are read 64 vertices at a time with the next chunk in flight
//     (RingStream); a vertex's successor comes from the next lane.
//   - Leaf tiles use bit-sliced crossing tests: a lane holds one column of
//     the tile as a row mask.  Each vertical edge of the tile's band XORs its
//     row mask into the LDS slot of the rightmost column it toggles (one
//     atomic per edge), and a prefix XOR over the lanes turns the slots into
//     every column's crossing parities.  A polygon known to contain a tile
//     is not tested again (its mask is all ones).  When a split leaves
//     several leaf tiles, each ring is read once into per-row lists of its
//     band edges in LDS, and every tile scatters from its row's list.
//   - The pair's MBRs and shoelace areas are reduced by the wave that takes
//     the pair, from the same coalesced ring loads it needs anyway; only the
//     pairs with many vertices ("heavy", claimed first: a largest-first
//     order) get them from a prepass, run by a quarter of the medium
//     sweep's waves beside the others' computation, so that any wave can
//     take one of their boxes.
//   - One persistent grid.  Waves claim, in this order: boxes from their
//     queue, heavy pairs, chunks of the other pairs, boxes from any queue.
//     Claims go through per-stream counters (one stream per XCD) on cache
//     lines of their own.  A heavy pair's split publishes its continuing
//     boxes to a device queue when there are enough of them, so that idle
//     waves share the pair.  Queue slots are single 64-bit words written and
//     taken with atomics, so no cache flushes are needed; a consumer that
//     overshoots the tail marks the slot skipped and the producer keeps that
//     box, so every box is processed exactly once and nobody waits on work
//     that may never come.  The one remaining wait (a slot reserved but not
//     yet written) is on a producer that writes right after reserving; it is
//     bounded anyway and latches SCCG_E_DEVICE if the bound is hit.
#include <limits.h>
#include <stddef.h>

#include <algorithm>

#include <type_traits>

#include "sccg_device.h"

namespace sccg {

constexpr int kLeafSlots = 2 * kWave;  // per-wave leaf slots: one per column of p and of q
constexpr int kLocalCap = 256;          // per-wave stack of boxes to process inline
constexpr uint32_t kSpinLimit = 1u << 22;
// per-wave LDS of the persistent kernel: the slots of one band row of each
// ring (a single tile's leaf slots are the first of them), the inline box
// stack
constexpr int kRowSlotsPerWave = 2 * kMaxGrid * kWave;
constexpr int kLdsPerWave = kRowSlotsPerWave * 8 + kLocalCap * 8;
constexpr unsigned long long kSkip = 1ull;  // slot abandoned by an overshooting consumer
constexpr int kSetupPerThread = 16;         // most pairs per thread of the setup pass

int batch_lds_bytes_per_wave() { return kLdsPerWave; }

// ---------------------------------------------------------------- task words
// [63] valid | [56:55] level | [54] p inside | [53] q inside | [52:44] ty |
// [43:35] tx | [30:0] heavy-list index.  tx, ty: cell origin in 64-px units
// from the pair-box origin; level l: cell side 64 * 8^l (0 = leaf tile).
__device__ __forceinline__ uint64_t task_word(int64_t hidx, int level, int tx, int ty, bool kp, bool kq) {
  return (1ull << 63) | ((uint64_t)level << 55) | ((uint64_t)kp << 54) | ((uint64_t)kq << 53) |
         ((uint64_t)ty << 44) | ((uint64_t)tx << 35) | (uint64_t)hidx;
}
struct Task {
  int64_t hidx;
  int level, tx, ty;
  bool kp, kq;
};
__device__ __forceinline__ Task task_decode(uint64_t w) {
  Task t;
  t.hidx = (int64_t)(w & 0x7fffffffull);
  t.tx = (int)((w >> 35) & 0x1ff);
  t.ty = (int)((w >> 44) & 0x1ff);
  t.kq = (w >> 53) & 1;
  t.kp = (w >> 54) & 1;
  t.level = (int)((w >> 55) & 3);
  return t;
}

// ------------------------------------------------------------- bit helpers
// cell (i, j) of an 8x8 grid is bit 8*j + i
__device__ __forceinline__ uint64_t rows_bits(int j0, int j1) {
  return (~0ull >> (8 * (7 - j1))) & (~0ull << (8 * j0));
}
__device__ __forceinline__ uint64_t spread(uint32_t colbyte) { return (uint64_t)colbyte * 0x0101010101010101ull; }
__device__ __forceinline__ uint32_t cols_bits(int i0, int i1) { return (0xFFu >> (7 - i1)) & (0xFFu << i0) & 0xFFu; }
// rows [lo, hi) of a 64-row tile, 0 <= lo < hi <= 64
__device__ __forceinline__ uint64_t row_range(int lo, int hi) {
  return (~0ull << lo) & (~0ull >> (64 - hi));
}
// x limited to [lo, hi]: a coordinate clamped to a box's sides before the
// box origin is subtracted, since |x| <= 2^30 on both sides of a difference
// could leave int32
__device__ __forceinline__ int clamp_to(int x, int lo, int hi) { return min(max(x, lo), hi); }

// ----------------------------------------------------------------- context
struct Ctx {
  const BatchArgs* a;
  bool stats;       // work counters on (a compile-time false in the sweeps' plain instances)
  int lane;
  uint64_t* slots;  // per-wave leaf slots (kLeafSlots; in the persistent kernel, two band rows' worth)
  uint64_t* local;  // per-wave inline stack, kLocalCap entries
  int lsp;          // inline stack depth (wave-uniform)
  int home;         // preferred queue
  int xcd;          // first claim stream (the workgroup's XCD under round-robin dispatch)
};

// Work counters (only with sccg_set_stats): one atomic per event from lane 0.
// The first stream at or after `from` (cyclically, kStreams of them) not in
// the exhausted mask `empty` (wave-uniform; at least one must be left).
__device__ __forceinline__ int next_stream(uint32_t empty, int from) {
  const uint32_t avail = ~empty & ((1u << kStreams) - 1u);
  const uint32_t rot = ((avail >> from) | (avail << (kStreams - from))) & ((1u << kStreams) - 1u);
  return uniform((from + __ffs((int)rot) - 1) % kStreams);
}

// Stamp of the device's constant-rate counter (100 MHz), read by the wave.
__device__ __forceinline__ unsigned long long wave_stamp(const BatchArgs& a) {
  return a.wave_t ? (unsigned long long)__builtin_amdgcn_s_memrealtime() : 0ull;
}
// A wave's (start, end) stamps of kernel `kernel` (see BatchArgs::wave_t).
__device__ __forceinline__ void wave_stamps(const BatchArgs& a, int kernel, unsigned long long t0, int lane) {
  if (!a.wave_t || lane != 0) return;
  const unsigned w = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (w >= (unsigned)a.wave_cap) return;
  unsigned long long* p = a.wave_t + 2 * ((size_t)kernel * (size_t)a.wave_cap + w);
  p[0] = t0;
  p[1] = (unsigned long long)__builtin_amdgcn_s_memrealtime();
}

__device__ __forceinline__ void stat_add(const Ctx& c, int k, unsigned long long v) {
  if (c.stats && c.lane == 0 && v) atomicAdd(&c.a->st->stats[k], v);
}

// What a wave needs to work on one pair.
struct PairInfo {
  int64_t pair;     // index into the pair arrays
  int64_t hidx;     // heavy-list index, or -1 when the pair is not shared
  int64_t op, np, oq, nq;
  Meta box;
  int64_t area_sum;  // |p| + |q|
};

// PairInfo fields are wave-uniform: keep them in scalar registers.
__device__ __forceinline__ void make_uniform(PairInfo& pi) {
  pi.pair = uniform64(pi.pair);
  pi.hidx = uniform64(pi.hidx);
  pi.op = uniform64(pi.op);
  pi.np = uniform64(pi.np);
  pi.oq = uniform64(pi.oq);
  pi.nq = uniform64(pi.nq);
  pi.box.x0 = uniform(pi.box.x0);
  pi.box.y0 = uniform(pi.box.y0);
  pi.box.x1 = uniform(pi.box.x1);
  pi.box.y1 = uniform(pi.box.y1);
  pi.area_sum = uniform64(pi.area_sum);
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------- ring scans
// A lane's view of the first two 64-vertex chunks of a ring: vertex k and its
// successor for k = lane and k = lane + 64.  Loaded once (coalesced), used for
// the extent, the area and the leaf edges.
struct RingRegs {
  int2 v0, w0, v1, w1;
};

// The first two chunks of a ring when they are already in registers
// (vertex lane in v0, vertex lane + 64 in v1, (0, 0) past the end).
struct Held {
  bool have;
  int2 v0, v1;
};

// The value of the next lane (DPP wave shift left by one; lane 63 reads 0).
__device__ __forceinline__ int2 next_lane(int2 v) {
  return make_int2(__builtin_amdgcn_update_dpp(0, v.x, 0x130, 0xf, 0xf, false),
                   __builtin_amdgcn_update_dpp(0, v.y, 0x130, 0xf, 0xf, false));
}

__device__ __forceinline__ int2 lane_value(int2 v, int l) {
  return make_int2(__builtin_amdgcn_readlane(v.x, l), __builtin_amdgcn_readlane(v.y, l));
}

// A ring read 64 vertices at a time with loads running ahead: lane L holds
// vertex base + L in `cur` and vertex base + 64 + L in `nxt`; ahead(), called
// at the top of each iteration, starts the load of the chunk after `nxt`, so
// that it arrives while the current chunk is processed.  A vertex's
// successor is the next lane's vertex; lane 63's is lane 0 of `nxt`, and the
// last vertex's is the first.  `nv` (>= 1) must be wave-uniform.  Lanes past the end load the
// last vertex again (the index is clamped, so the loads need no branch) and
// must be masked with valid(): the successor shift reads across lanes, so
// no lane may be switched off around it, and a per-lane branch in the loop
// body lets the compiler split the wave.
struct RingStream {
  const int2* p;
  int nv, base, lane;
  int2 first, cur, nxt, nn;

  __device__ __forceinline__ int2 at(int k) const { return p[min(k, nv - 1)]; }
  __device__ __forceinline__ RingStream(const int2* xy, int64_t o, int nv_, int lane_, int base0 = 0,
                                        const int2* first_ = nullptr)
      : p(xy + o), nv(uniform(nv_)), base(uniform(base0)), lane(lane_) {
    cur = at(base + lane);
    nxt = at(base + kWave + lane);
    first = first_ ? *first_ : lane_value(cur, 0);
  }
  __device__ __forceinline__ void ahead() { nn = at(base + 2 * kWave + lane); }
  __device__ __forceinline__ bool valid() const { return base + lane < nv; }
  // successor of this lane's vertex (every lane takes part)
  __device__ __forceinline__ int2 succ() const {
    const int2 s = next_lane(cur);
    const int2 n0 = lane_value(nxt, 0);
    const bool wrap = base + lane + 1 == nv, last = lane == kWave - 1;
    return make_int2(wrap ? first.x : (last ? n0.x : s.x), wrap ? first.y : (last ? n0.y : s.y));
  }
  __device__ __forceinline__ bool next() {
    base = uniform(base + kWave);
    if (base >= nv) return false;
    cur = nxt;
    nxt = nn;
    return true;
  }
};

// Load the first two 64-vertex chunks of a ring with one coalesced load each;
// each vertex's successor comes from the neighbouring lane, lane 63's from
// the next chunk, and the last vertex's is vertex 0.
__device__ __forceinline__ void load_ring2(const int2* xy, int64_t o, int nv, int lane, RingRegs& r,
                                           int2& first, const Held& pre) {
  const int k0 = lane, k1 = lane + kWave;
  r.v0 = pre.have ? pre.v0 : (k0 < nv ? xy[o + k0] : make_int2(0, 0));
  r.v1 = pre.have ? pre.v1 : (k1 < nv ? xy[o + k1] : make_int2(0, 0));
  first = lane_value(r.v0, 0);
  const int2 a64 = nv > kWave ? lane_value(r.v1, 0) : first;
  const int2 a128 = nv > 2 * kWave ? xy[o + 2 * kWave] : first;
  int2 s0 = next_lane(r.v0), s1 = next_lane(r.v1);
  if (lane == kWave - 1) {
    s0 = a64;
    s1 = a128;
  }
  if (k0 + 1 == nv) s0 = first;
  if (k1 + 1 == nv) s1 = first;
  r.w0 = s0;
  r.w1 = s1;
}

// Extent and |shoelace|/2 of one ring (Section 3.2's area formula), reduced
// across the wave.  Lanes past the end of the ring stand at the first vertex:
// they leave the extent alone and add a zero shoelace term.  The terms use
// coordinates relative to the first vertex in wrapping 32-bit arithmetic with
// 24-bit multiplies, which is exact when the extent is below 2^14 on both
// axes (twice the area is then below 2^29); a wider ring has its area summed
// again in 64 bits.  Empty rings and rings with |coordinate| > 2^30 come back
// empty.
__device__ __forceinline__ void ring_extent(const int2* xy, int64_t o, int64_t nv64, int lane, RingRegs& r, Meta& m,
                                            int64_t& area, const Held& pre = Held{false, {0, 0}, {0, 0}}) {
  const int nv = uniform((int)nv64);
  int2 first;
  load_ring2(xy, o, nv, lane, r, first, pre);
  int x0, y0, x1, y1;
  uint32_t twice;
  {
    const bool ok = lane < nv;
    const int vx = ok ? r.v0.x : first.x, vy = ok ? r.v0.y : first.y;
    x0 = x1 = vx;
    y0 = y1 = vy;
    const int dx = vx - first.x, dy = vy - first.y;
    twice = (uint32_t)__mul24(dx, r.w0.y - first.y) - (uint32_t)__mul24(r.w0.x - first.x, dy);
  }
  if (nv > kWave) {
    const bool ok = lane + kWave < nv;
    const int vx = ok ? r.v1.x : first.x, vy = ok ? r.v1.y : first.y;
    x0 = min(x0, vx);
    y0 = min(y0, vy);
    x1 = max(x1, vx);
    y1 = max(y1, vy);
    const int dx = vx - first.x, dy = vy - first.y;
    twice += (uint32_t)__mul24(dx, r.w1.y - first.y) - (uint32_t)__mul24(r.w1.x - first.x, dy);
  }
  if (nv > 2 * kWave) {
    RingStream rs(xy, o, nv, lane, 2 * kWave, &first);
#pragma unroll 1
    do {
      rs.ahead();
      const int2 w = rs.succ();
      const bool ok = rs.valid();
      const int vx = ok ? rs.cur.x : first.x, vy = ok ? rs.cur.y : first.y;
      x0 = min(x0, vx);
      y0 = min(y0, vy);
      x1 = max(x1, vx);
      y1 = max(y1, vy);
      const int dx = vx - first.x, dy = vy - first.y;
      twice += (uint32_t)__mul24(dx, w.y - first.y) - (uint32_t)__mul24(w.x - first.x, dy);
    } while (rs.next());
  }
  m.x0 = wave_min_i32(x0);
  m.y0 = wave_min_i32(y0);
  m.x1 = wave_max_i32(x1);
  m.y1 = wave_max_i32(y1);
  const int32_t t = (int32_t)wave_sum_u32(twice);
  if (side_u(m.x0, m.x1) < 16384u && side_u(m.y0, m.y1) < 16384u) {
    area = (int64_t)(t < 0 ? -(int64_t)t : (int64_t)t) / 2;
  } else {
    uint64_t tw = 0;
    RingStream rs(xy, o, nv, lane);
#pragma unroll 1
    do {
      rs.ahead();
      const int2 w = rs.succ();
      if (rs.valid()) tw += (uint64_t)((int64_t)rs.cur.x * w.y) - (uint64_t)((int64_t)w.x * rs.cur.y);
    } while (rs.next());
    // twice the area is at most 2^63 in size, so the magnitude of the wrapped
    // sum is exact in unsigned form
    const uint64_t t64 = wave_sum_u64(tw);
    area = (int64_t)(((int64_t)t64 < 0 ? 0 - t64 : t64) / 2);
  }
  if (nv <= 0 || m.x0 < -kMaxCoord || m.y0 < -kMaxCoord || m.x1 > kMaxCoord || m.y1 > kMaxCoord) {
    m = Meta{INT_MAX, INT_MAX, INT_MIN, INT_MIN};  // covers nothing
    area = 0;
  }
}

// The same extent and area for the prepass of listed (long) rings: each
// lane loads its vertices and their successors directly, kScanBatch chunks
// of 64 per round trip, so that a long ring costs few memory latencies (four:
// the prepass shares its kernel with the medium sweep, whose computation
// hides them).
constexpr int kScanBatch = 4;
__device__ __forceinline__ void ring_scan(const int2* xy, int64_t o, int64_t nv64, int lane, Meta& m, int64_t& area) {
  const int nv = uniform((int)nv64);
  m = Meta{INT_MAX, INT_MAX, INT_MIN, INT_MIN};  // covers nothing
  area = 0;
  if (nv <= 0) return;
  const int2* R = xy + o;
  const int2 f = R[0];
  int x0 = f.x, y0 = f.y, x1 = f.x, y1 = f.y;
  uint32_t twice = 0;  // relative to the first vertex, wrapping (exact for extents below 2^14)
#pragma unroll 1
  for (int base = 0; base < nv; base += kScanBatch * kWave) {
    int2 v[kScanBatch], w[kScanBatch];
#pragma unroll
    for (int c = 0; c < kScanBatch; ++c) {
      v[c] = w[c] = f;
      if (base + c * kWave < nv) {
        const int k = base + c * kWave + lane;
        v[c] = R[min(k, nv - 1)];
        w[c] = R[k + 1 < nv ? k + 1 : 0];
      }
    }
#pragma unroll
    for (int c = 0; c < kScanBatch; ++c) {
      if (base + c * kWave + lane < nv) {
        x0 = min(x0, v[c].x);
        y0 = min(y0, v[c].y);
        x1 = max(x1, v[c].x);
        y1 = max(y1, v[c].y);
        twice += (uint32_t)__mul24(v[c].x - f.x, w[c].y - f.y) - (uint32_t)__mul24(w[c].x - f.x, v[c].y - f.y);
      }
    }
  }
  m.x0 = wave_min_i32(x0);
  m.y0 = wave_min_i32(y0);
  m.x1 = wave_max_i32(x1);
  m.y1 = wave_max_i32(y1);
  if (side_u(m.x0, m.x1) < 16384u && side_u(m.y0, m.y1) < 16384u) {
    const int32_t t = (int32_t)wave_sum_u32(twice);
    area = (int64_t)(t < 0 ? -(int64_t)t : (int64_t)t) / 2;
  } else {
    // twice the area is at most 2^63 in size, so the magnitude of the
    // wrapped 64-bit sum is exact in unsigned form
    uint64_t tw = 0;
#pragma unroll 1
    for (int base = 0; base < nv; base += kScanBatch * kWave) {
      int2 v[kScanBatch], w[kScanBatch];
#pragma unroll
      for (int c = 0; c < kScanBatch; ++c) {
        v[c] = w[c] = f;
        if (base + c * kWave < nv) {
          const int k = base + c * kWave + lane;
          v[c] = R[min(k, nv - 1)];
          w[c] = R[k + 1 < nv ? k + 1 : 0];
        }
      }
#pragma unroll
      for (int c = 0; c < kScanBatch; ++c)
        if (base + c * kWave + lane < nv)
          tw += (uint64_t)((int64_t)v[c].x * w[c].y) - (uint64_t)((int64_t)w[c].x * v[c].y);
    }
    const uint64_t t64 = wave_sum_u64(tw);
    area = (int64_t)(((int64_t)t64 < 0 ? 0 - t64 : t64) / 2);
  }
  if (m.x0 < -kMaxCoord || m.y0 < -kMaxCoord || m.x1 > kMaxCoord || m.y1 > kMaxCoord) {
    m = Meta{INT_MAX, INT_MAX, INT_MIN, INT_MIN};
    area = 0;
  }
}

__device__ __forceinline__ bool coords_bad(const Meta& m, int64_t nv) {
  return nv > 0 && m.x0 == INT_MAX;
}

// The ablations of Section 5.2 (SCCG_F_PIXEL_ONLY, SCCG_F_NO_SEP) count the
// union directly, over the bounding box of both MBRs, instead of deriving it
// from the areas.  Counts of one box then travel packed: intersection in
// the low 32 bits, direct union in the high 32 (a processed box has at most
// 32767^2 < 2^32 pixels).
__device__ __forceinline__ bool direct_union(const BatchArgs& a) {
  return (a.flags & (SCCG_F_PIXEL_ONLY | SCCG_F_NO_SEP)) != 0u;
}

// Wave total of a lane's intersection count n and, when `direct`, of its
// union count nu, packed.
__device__ __forceinline__ uint64_t pack_counts(uint32_t n, uint32_t nu, bool direct) {
  if (!direct) return wave_sum_u32(n);
  // a lane holds at most 64 pixels of each, so both wave sums stay below
  // 2^13 and travel in the two halves of one 32-bit sum
  const uint32_t t = wave_sum_u32(n | (nu << 16));
  return (uint64_t)(t & 0xffffu) | ((uint64_t)(t >> 16) << 32);
}

// ------------------------------------------------------------------ leaves
// Scatter-and-scan leaves.  The columns of a leaf tile live in lanes in
// reverse order: in a W-column group (W = 64, or 32 when p and q share the
// wave as two halves), lane L holds column W - 1 - L.  A vertical edge at X
// whose span meets the tile's rows toggles those rows in every column left of
// X.  It XORs its row mask into one LDS slot: the slot of the rightmost column
// it toggles, W - min(X - x0, W).  Any number of edges may share a slot.  An
// inclusive prefix XOR over the lanes then leaves in every column the XOR of
// the edges right of it: bit r of lane L is the crossing parity of the centre
// of pixel (x0 + W - 1 - L, y0 + r) (Section 3.1).  Cost per tile: one atomic
// per edge of the band, no per-edge work in the other lanes.

// Inclusive prefix XOR over lanes (rows of 16 by shifts, then the row
// broadcasts); with kHalves the scan restarts at lane 32.
template <bool kHalves>
__device__ __forceinline__ uint32_t wave_prefix_xor(uint32_t x) {
  x ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
  if (!kHalves) x ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x;
}
template <bool kHalves>
__device__ __forceinline__ uint64_t wave_prefix_xor(uint64_t x) {
  return ((uint64_t)wave_prefix_xor<kHalves>((uint32_t)(x >> 32)) << 32) | wave_prefix_xor<kHalves>((uint32_t)x);
}

// The slot and row mask of edge (v, w) for the tile at (tx0, ty0) of height
// th in a W-column group: kept iff vertical, right of the tile's left side,
// with a span meeting the rows.
__device__ __forceinline__ bool leaf_edge(int2 v, int2 w, int tx0, int ty0, int th, int W, int& slot,
                                          uint64_t& rr) {
  if (v.x != w.x) return false;
  const int lo = clamp_to(min(v.y, w.y), ty0, ty0 + th) - ty0;
  const int hi = clamp_to(max(v.y, w.y), ty0, ty0 + th) - ty0;
  const int dx = min(v.x, tx0 + W) - tx0;
  if (!(lo < hi && dx > 0)) return false;
  slot = W - dx;
  rr = row_range(lo, hi);
  return true;
}

template <typename M>
__device__ __forceinline__ void slot_xor(M* slots, int k, uint64_t rr) {
  __hip_atomic_fetch_xor(slots + k, (M)rr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Scatter the leaf edges of one ring into slots[base ..).  The first two
// 64-vertex chunks come from registers when `r` is given, the rest (or all)
// from global memory.  With `full` given, edges right of the whole group
// (they toggle every column) are XORed into *full (per lane) instead of
// slot 0, so that they do not all hit one LDS address.
template <typename M>
__device__ __forceinline__ void scatter_ring(Ctx& c, const int2* xy, int64_t o, int64_t nv, const RingRegs* r,
                                             int tx0, int ty0, int th, int W, M* slots, int base,
                                             uint64_t* full = nullptr) {
  const int lane = c.lane;
  const int n = uniform((int)nv);
  uint32_t kept = 0;
  auto one = [&](int2 v, int2 w, bool ok) {
    int slot = 0;
    uint64_t rr = 0;
    const bool keep = ok && leaf_edge(v, w, tx0, ty0, th, W, slot, rr);
    if (keep) {
      if (full && slot == 0)
        *full ^= rr;
      else
        slot_xor(slots, base + slot, rr);
    }
    if (c.stats) kept += (uint32_t)__popcll(ballot(keep));
  };
  int b0 = 0;
  int2 first;
  if (r) {
    // the first two chunks are in registers
    one(r->v0, r->w0, lane < n);
    if (n > kWave) one(r->v1, r->w1, kWave + lane < n);
    b0 = 2 * kWave;
    first = lane_value(r->v0, 0);
  }
  if (b0 < n) {
    RingStream rs(xy, o, n, lane, b0, r ? &first : nullptr);
#pragma unroll 1
    do {
      rs.ahead();
      const int2 w = rs.succ();
      one(rs.cur, w, rs.valid());
    } while (rs.next());
  }
  if (c.stats) {
    stat_add(c, 8, (unsigned long long)kept);
    stat_add(c, 10, (unsigned long long)nv);
  }
}

// Zero for clearing leaf slots, made where it is stored: a zero the compiler
// hoists into a long-lived register pair gets spilled to scratch under this
// kernel's register pressure.
template <typename M>
__device__ __forceinline__ M fresh_zero() {
  uint32_t lo, hi;
  asm volatile("v_mov_b32 %0, 0" : "=v"(lo));
  if (sizeof(M) == 4) return (M)lo;
  asm volatile("v_mov_b32 %0, 0" : "=v"(hi));
  return (M)(((uint64_t)hi << 32) | lo);
}

// Intersection count of a small pair (box <= 64 x 64 = one leaf tile).
// Narrow boxes (w <= 32) run p in lanes 0-31 and q in lanes 32-63 with one
// scan; short boxes (h <= 32) use 32-bit row masks.
template <bool kRows64>
__device__ __forceinline__ int64_t leaf_small(Ctx& c, const PairInfo& pi, const RingRegs& rp, const RingRegs& rq,
                                              int tw, int th, bool direct) {
  using M = typename std::conditional<kRows64, uint64_t, uint32_t>::type;
  const BatchArgs& a = *c.a;
  const int lane = c.lane;
  const int tx0 = pi.box.x0, ty0 = pi.box.y0;
  M* slots = reinterpret_cast<M*>(c.slots);
  uint32_t n = 0, nu = 0;
  if (tw <= 32) {
    slots[lane] = fresh_zero<M>();
    wave_sync_lds();
    scatter_ring(c, a.A.xy, pi.op, pi.np, &rp, tx0, ty0, th, 32, slots, 0);
    scatter_ring(c, a.B.xy, pi.oq, pi.nq, &rq, tx0, ty0, th, 32, slots, 32);
    wave_sync_lds();
    const M m = wave_prefix_xor<true>(slots[lane]);
    // lanes 0-31 hold p's columns, lanes 32-63 q's: bring q's beside p's
    M mq;
    if (kRows64) {
      const uint64_t m64 = (uint64_t)m;
      const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)m64, 32, kWave);
      const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(m64 >> 32), 32, kWave);
      mq = (M)(((uint64_t)hi << 32) | lo);
    } else {
      mq = (M)(uint32_t)__shfl_xor((int)(uint32_t)m, 32, kWave);
    }
    if (lane < 32 && 31 - lane < tw) {
      n = (uint32_t)__popcll((uint64_t)(m & mq));
      nu = (uint32_t)__popcll((uint64_t)(m | mq));
    }
  } else {
    slots[lane] = fresh_zero<M>();
    slots[kWave + lane] = fresh_zero<M>();
    wave_sync_lds();
    scatter_ring(c, a.A.xy, pi.op, pi.np, &rp, tx0, ty0, th, kWave, slots, 0);
    scatter_ring(c, a.B.xy, pi.oq, pi.nq, &rq, tx0, ty0, th, kWave, slots, kWave);
    wave_sync_lds();
    const M mp = wave_prefix_xor<false>(slots[lane]);
    const M mq = wave_prefix_xor<false>(slots[kWave + lane]);
    if (kWave - 1 - lane < tw) {
      n = (uint32_t)__popcll((uint64_t)(mp & mq));
      nu = (uint32_t)__popcll((uint64_t)(mp | mq));
    }
  }
  wave_sync_lds();
  if (c.stats) {
    stat_add(c, 1, 1ull);
    stat_add(c, 0, 2ull * (unsigned long long)tw * th);
  }
  return (int64_t)pack_counts(n, nu, direct);
}

// Pixels of the tile [tx0, tx0+tw) x [ty0, ty0+th) inside both polygons; a
// polygon known to contain the tile is not scattered (all rows set).
__device__ __forceinline__ uint64_t leaf_count(Ctx& c, const PairInfo& pi, int tx0, int ty0, int tw, int th, bool kp,
                                               bool kq) {
  const BatchArgs& a = *c.a;
  const int lane = c.lane;
  uint64_t* slots = c.slots;
  slots[lane] = fresh_zero<uint64_t>();
  slots[kWave + lane] = fresh_zero<uint64_t>();
  wave_sync_lds();
  uint64_t fp = 0, fq = 0;
  if (!kp) scatter_ring(c, a.A.xy, pi.op, pi.np, (const RingRegs*)nullptr, tx0, ty0, th, kWave, slots, 0, &fp);
  if (!kq) scatter_ring(c, a.B.xy, pi.oq, pi.nq, (const RingRegs*)nullptr, tx0, ty0, th, kWave, slots, kWave, &fq);
  wave_sync_lds();
  const uint64_t full = row_range(0, th);
  const uint64_t mp = kp ? full : wave_prefix_xor<false>(slots[lane]) ^ wave_xor64(fp);
  const uint64_t mq = kq ? full : wave_prefix_xor<false>(slots[kWave + lane]) ^ wave_xor64(fq);
  wave_sync_lds();
  const bool in_tile = kWave - 1 - lane < tw;
  const uint32_t n = in_tile ? (uint32_t)__popcll(mp & mq) : 0u;
  const uint32_t nu = in_tile ? (uint32_t)__popcll(mp | mq) : 0u;
  if (c.stats) {
    stat_add(c, 1, 1ull);
    stat_add(c, 0, (unsigned long long)tw * th * ((kp ? 0 : 1) + (kq ? 0 : 1)));
  }
  return pack_counts(n, nu, direct_union(a));
}

// Row-wide leaves.  When a split leaves several leaf tiles, each band row of
// it (up to kMaxGrid tiles) is pixelized at once: one slot array per ring
// holds every column of the row, position Wpad - 1 - (column - bx0) for
// Wpad = 64 x (tiles per row), so that a vertical edge at X toggles the
// positions from Wpad - min(X - bx0, Wpad) up, with one atomic whatever its
// distance.  Each ring is streamed once per band row (from L2: its pair's
// rings were read moments before).  Inside each tile's block of 64 positions
// a prefix XOR over the lanes gives the tile's columns their crossing
// parities for the edges that end inside it; the blocks of the tiles to its
// right add the XOR of all their slots, carried from block to block.
constexpr int kRowSlots = kMaxGrid * kWave;  // slots of one ring's band row

// Scatter the vertical edges of one ring that meet rows [ry0, ry0 + th) into
// a row's slots (wpad positions from bx0).
__device__ __forceinline__ void scatter_row(Ctx& c, const int2* xy, int64_t o, int64_t nv, int bx0, int wpad, int ry0,
                                            int th, uint64_t* slots) {
  const int n = uniform((int)nv);
  if (n <= 0) return;
  uint32_t kept = 0;
  RingStream rs(xy, o, n, c.lane);
#pragma unroll 1
  do {
    rs.ahead();
    const int2 w = rs.succ();
    int slot = 0;
    uint64_t rr = 0;
    const bool keep = rs.valid() && leaf_edge(rs.cur, w, bx0, ry0, th, wpad, slot, rr);
    if (keep) slot_xor(slots, slot, rr);
    if (c.stats) kept += (uint32_t)__popcll(ballot(keep));
  } while (rs.next());
  if (c.stats) {
    stat_add(c, 8, (unsigned long long)kept);
    stat_add(c, 10, (unsigned long long)n);
  }
}

// The leaf tiles `cont` (bit 8j + i = tile (i, j) of side 64 from (bx0, by0))
// of a split.  kin_p / kin_q: tiles known to lie inside p / q.  A lone tile
// is scattered straight from the rings; otherwise a band row at a time.
__device__ __forceinline__ void leaf_rows(Ctx& c, const PairInfo& pi, int bx0, int by0, int bx1, int by1, int gy,
                                          uint64_t cont, uint64_t kin_p, uint64_t kin_q, uint64_t& acc) {
  const BatchArgs& a = *c.a;
  if (__popcll(cont) == 1) {
    const int t = __ffsll((long long)cont) - 1, i = t & 7, j = t >> 3;
    const int tx0 = bx0 + kTile * i, ty0 = by0 + kTile * j;
    acc += leaf_count(c, pi, tx0, ty0, min(kTile, bx1 - tx0), min(kTile, by1 - ty0), (kin_p >> t) & 1ull,
                      (kin_q >> t) & 1ull);
    return;
  }
  const int lane = c.lane;
  const bool direct = direct_union(a);
  const int gx = uniform((bx1 - bx0 + kTile - 1) / kTile);
  const int wpad = gx * kTile;
  uint64_t* sp = c.slots;
  uint64_t* sq = c.slots + kRowSlots;
  uint32_t ni = 0, nu = 0;  // this lane's pixels counted, over every tile
  unsigned long long n_leaf = 0, n_tests = 0;
#pragma unroll 1
  for (int j = 0; j < gy; ++j) {
    const uint32_t row = (uint32_t)(cont >> (8 * j)) & 0xffu;
    if (!row) continue;
    const uint32_t kp_row = (uint32_t)(kin_p >> (8 * j)) & row, kq_row = (uint32_t)(kin_q >> (8 * j)) & row;
    const bool need_p = kp_row != row, need_q = kq_row != row;
    const int ry0 = by0 + kTile * j, th = min(kTile, by1 - ry0);
    const uint64_t full = row_range(0, th);
#pragma unroll 1
    for (int b = 0; b < gx; ++b) {
      sp[b * kWave + lane] = fresh_zero<uint64_t>();
      sq[b * kWave + lane] = fresh_zero<uint64_t>();
    }
    wave_sync_lds();
    if (need_p) scatter_row(c, a.A.xy, pi.op, pi.np, bx0, wpad, ry0, th, sp);
    if (need_q) scatter_row(c, a.B.xy, pi.oq, pi.nq, bx0, wpad, ry0, th, sq);
    wave_sync_lds();
    // tiles right to left: block b = gx - 1 - i holds tile i
    uint64_t carry_p = 0, carry_q = 0;
#pragma unroll 1
    for (int i = gx - 1; i >= 0; --i) {
      const int b = gx - 1 - i;
      const uint64_t xp = wave_prefix_xor<false>(sp[b * kWave + lane]);
      const uint64_t xq = wave_prefix_xor<false>(sq[b * kWave + lane]);
      if ((row >> i) & 1u) {
        const int tw = min(kTile, bx1 - (bx0 + kTile * i));
        const uint64_t mp = ((kp_row >> i) & 1u) ? full : (xp ^ carry_p);
        const uint64_t mq = ((kq_row >> i) & 1u) ? full : (xq ^ carry_q);
        if (kWave - 1 - lane < tw) {
          ni += (uint32_t)__popcll(mp & mq);
          nu += (uint32_t)__popcll(mp | mq);
        }
        n_leaf += 1;
        n_tests += (unsigned long long)tw * th * ((((kp_row >> i) & 1u) ? 0 : 1) + (((kq_row >> i) & 1u) ? 0 : 1));
      }
      carry_p ^= (uint64_t)readlane64((int64_t)xp, kWave - 1);
      carry_q ^= (uint64_t)readlane64((int64_t)xq, kWave - 1);
    }
    wave_sync_lds();
  }
  const uint64_t si = wave_sum_u32(ni);
  acc += direct ? (si | ((uint64_t)wave_sum_u32(nu) << 32)) : si;
  if (c.stats) {
    stat_add(c, 1, n_leaf);
    stat_add(c, 0, n_tests);
  }
}

// One pass over the ring: hover mask H and first-pixel parity mask P of the
// gx x gy cells of side 2^ls covering [bx0,bx1) x [by0,by1).
__device__ __forceinline__ void classify(Ctx& c, const int2* xy, int64_t o, int64_t nv, int bx0, int by0, int bx1, int by1, int ls,
                         int gx, int gy, uint64_t& H, uint64_t& P) {
  const int S = 1 << ls;
  uint64_t h = 0, p = 0;
  if (uniform((int)nv) <= 0) {
    H = 0;
    P = 0;
    return;
  }
  RingStream rs(xy, o, uniform((int)nv), c.lane);
#pragma unroll 1
  do {
    rs.ahead();
    const int2 v = rs.cur, w = rs.succ();
    if (!rs.valid()) {
      // past the end of the ring
    } else if (v.x == w.x) {
      // coordinates past the box's far sides are clamped to them (the tests
      // below do not change), so that no difference leaves int32
      const int X = min(v.x, bx1), lo = min(min(v.y, w.y), by1), hi = min(max(v.y, w.y), by1);
      const int dx = X - bx0;
      if (dx > 0 && hi > by0) {
        // hover: X strictly inside a column, span meeting the open rows
        if (X < bx1 && (dx & (S - 1)) != 0 && lo < by1) {
          const int i = dx >> ls;
          const int j0 = lo > by0 ? (lo - by0) >> ls : 0;
          const int j1 = min(gy - 1, ((hi - by0 + S - 1) >> ls) - 1);
          if (j0 <= j1) h |= rows_bits(j0, j1) & spread(1u << i);
        }
        // crossing of the first pixel (c_i, r_j) of cells with c_i < X, lo <= r_j < hi
        const int ic = min(gx - 1, ((dx + S - 1) >> ls) - 1);
        const int ja = lo > by0 ? ((lo - by0 + S - 1) >> ls) : 0;
        const int jb = min(gy - 1, ((hi - by0 + S - 1) >> ls) - 1);
        if (ja <= jb) p ^= rows_bits(ja, jb) & spread(0xFFu >> (7 - ic));
      }
    } else {
      const int Y = min(v.y, by1), lo = min(min(v.x, w.x), bx1), hi = min(max(v.x, w.x), bx1);
      const int dy = Y - by0;
      if (dy > 0 && Y < by1 && (dy & (S - 1)) != 0 && lo < bx1 && hi > bx0) {
        const int j = dy >> ls;
        const int i0 = lo > bx0 ? (lo - bx0) >> ls : 0;
        const int i1 = min(gx - 1, ((hi - bx0 + S - 1) >> ls) - 1);
        if (i0 <= i1) h |= rows_bits(j, j) & spread(cols_bits(i0, i1));
      }
    }
  } while (rs.next());
  H = wave_or64(h);
  P = wave_xor64(p);
  stat_add(c, 9, (unsigned long long)nv);
}

// Add a shared pair's partial counts: `n` packed as by pack_counts.  The
// union starts at |p| + |q| and loses every intersection pixel, or (direct
// union) starts at 0 and gains every union pixel.
__device__ __forceinline__ void add_counts(const BatchArgs& a, int64_t pair, uint64_t n) {
  if (n == 0) return;
  const unsigned long long i = n & 0xffffffffull;
  const unsigned long long u = direct_union(a) ? (n >> 32) : (0 - i);
  if (i) atomicAdd(reinterpret_cast<unsigned long long*>(a.inter + pair), i);
  if (u) atomicAdd(reinterpret_cast<unsigned long long*>(a.uni + pair), u);
}

// ------------------------------------------------------------------- queue
// Queue q is a head counter, a tail counter and queue_cap slots.  A producer
// reserves slots with one atomic add on the tail and fills each with a
// compare-and-swap from 0; a consumer takes a ticket with one atomic add on
// the head.  A ticket below the tail is a reserved slot: the consumer waits
// for its word.  A ticket at or past the tail tries to mark its slot skipped;
// if it wins, the producer that later reserves the slot finds it taken and
// keeps the box; if it loses, the word is there and the consumer takes it.
__device__ __forceinline__ bool queue_claim_one(Ctx& c, int q, uint64_t* out) {
  const BatchArgs& a = *c.a;
  uint64_t word = 0;
  if (c.lane == 0) {
    unsigned long long* head = &a.st->q_head[q].v;
    unsigned long long* tail = &a.st->q_tail[q].v;
    const unsigned long long cap = (unsigned long long)a.queue_cap;
    const unsigned long long h0 = __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned long long t = __hip_atomic_load(tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (h0 < cap && h0 < t) {
      const unsigned long long h = atomicAdd(head, 1ull);
      if (h < cap) {
        unsigned long long* slot = a.queue + (size_t)q * a.queue_cap + h;
        t = __hip_atomic_load(tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (h < t) {
          uint32_t spins = 0;
          while ((word = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == 0) {
            if (++spins > kSpinLimit) {
              latch_error(a.err, kErrWatchdog);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
        } else {
          const unsigned long long prev = atomicCAS(slot, 0ull, kSkip);
          word = (prev == 0ull) ? 0ull : prev;
        }
        if (word == kSkip) word = 0;
      }
    }
  }
  const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)word, 0, kWave);
  const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(word >> 32), 0, kWave);
  *out = ((uint64_t)hi << 32) | lo;
  return *out != 0;
}

// Claim from the home queue only, or from every queue (home first).
__device__ __forceinline__ bool queue_claim(Ctx& c, bool all, uint64_t* out) {
  const int nq = all ? c.a->n_queues : 1;
  for (int r = 0; r < nq; ++r)
    if (queue_claim_one(c, (c.home + r) % c.a->n_queues, out)) return true;
  return false;
}

// Children of one split: lane j (< n) holds word j.  Publish them to the
// queue when the pair is shared and there are enough, else (and for what a
// full queue or a skip-marked slot refuses) keep them on the wave's stack.
__device__ __forceinline__ void emit_children(Ctx& c, const PairInfo& pi, uint64_t word, bool has, int n) {
  const BatchArgs& a = *c.a;
  const uint64_t b = ballot(has);
  const int rank = lanes_below(b);
  bool keep = has;
  if (pi.hidx >= 0 && !(a.flags & SCCG_F_NO_SPLIT_QUEUE) && n >= a.min_cells_to_queue) {
    unsigned long long t = 0;
    if (c.lane == 0) t = atomicAdd(&a.st->q_tail[c.home].v, (unsigned long long)n);
    t = (unsigned long long)uniform64((int64_t)__shfl((long long)t, 0, kWave));
    if (has && t + rank < (unsigned long long)a.queue_cap) {
      unsigned long long* slot = a.queue + (size_t)c.home * a.queue_cap + t + rank;
      const unsigned long long prev = atomicCAS(slot, 0ull, (unsigned long long)word);
      keep = prev != 0ull;  // skip-marked: the box stays here
    }
    if (c.stats) {
      const int kept = __popcll(ballot(keep));
      stat_add(c, 3, (unsigned long long)(n - kept));
      stat_add(c, 4, (unsigned long long)kept);
    }
  }
  const uint64_t bk = ballot(keep);
  const int nk = __popcll(bk);
  if (nk > 0) {
    if (keep) c.local[c.lsp + lanes_below(bk)] = word;
    c.lsp += nk;
    wave_sync_lds();
  }
}

// Pixels of the cells `m` of a gx x gy grid of side S whose last column and
// row are lw and lh wide.
__device__ __forceinline__ uint64_t cells_area(uint64_t m, int gx, int gy, int S, int lw, int lh) {
  uint64_t add = 0;
  for (int j = 0; j < gy; ++j) {
    const uint32_t row = (uint32_t)(m >> (8 * j)) & 0xFFu;
    if (!row) continue;
    const uint64_t hgt = (j == gy - 1) ? (uint64_t)lh : (uint64_t)S;
    const uint32_t last = (row >> (gx - 1)) & 1u;
    add += hgt * ((uint64_t)(__popc(row) - last) * S + (uint64_t)last * lw);
  }
  return add;
}

// Split box [bx0,bx1) x [by0,by1) of a pair (already known to be a
// continuing box) into cells of level `cl` (side 64*8^cl).  Cells inside
// both polygons add their size to `acc`; continuing cells become tasks.
__device__ __forceinline__ void split_box(Ctx& c, const PairInfo& pi, int bx0, int by0, int bx1, int by1, int cl, bool kp, bool kq,
                          uint64_t& acc) {
  const BatchArgs& a = *c.a;
  const int ls = 6 + 3 * cl;
  const int S = 1 << ls;
  const int gx = (bx1 - bx0 + S - 1) >> ls, gy = (by1 - by0 + S - 1) >> ls;
  const uint64_t valid = rows_bits(0, gy - 1) & spread(cols_bits(0, gx - 1));
  uint64_t Hp = 0, Pp = valid, Hq = 0, Pq = valid;
  if (a.flags & SCCG_F_PIXEL_ONLY) {
    Hp = Hq = valid;  // PixelOnly: no sampling boxes, every cell is pixelized
  } else if (cl == 0 && gx * gy < a.min_classify_cells) {
    // a split into a few leaf tiles: classifying them costs two ring passes
    // and rarely decides a tile, so every tile is pixelized (a polygon known
    // to contain the box still counts as inside)
    if (!kp) Hp = valid;
    if (!kq) Hq = valid;
  } else {
    if (!kp) classify(c, a.A.xy, pi.op, pi.np, bx0, by0, bx1, by1, ls, gx, gy, Hp, Pp);
    if (!kq) classify(c, a.B.xy, pi.oq, pi.nq, bx0, by0, bx1, by1, ls, gx, gy, Hq, Pq);
  }
  const uint64_t in_p = ~Hp & Pp & valid, out_p = ~Hp & ~Pp & valid;
  const uint64_t in_q = ~Hq & Pq & valid, out_q = ~Hq & ~Pq & valid;
  const uint64_t both = in_p & in_q;
  uint64_t cont = valid & ~out_p & ~out_q & ~both;
  uint64_t uni_add = 0;  // cells that stop inside p or q (direct union only)
  if (direct_union(a)) {
    // a cell stops only when decided for the intersection (inside both, or
    // outside one) and for the union (inside one, or outside both)
    const uint64_t dec_i = both | out_p | out_q, dec_u = in_p | in_q | (out_p & out_q);
    cont = valid & ~(dec_i & dec_u);
    uni_add = (in_p | in_q) & valid & ~cont;
  }
  const int lw = (bx1 - bx0) - (gx - 1) * S, lh = (by1 - by0) - (gy - 1) * S;
  // cells inside both polygons contribute their size at once
  if (both) acc += cells_area(both, gx, gy, S, lw, lh);
  if (uni_add) acc += cells_area(uni_add, gx, gy, S, lw, lh) << 32;
  stat_add(c, 2, 1ull);
  const int n = __popcll(cont);
  // leaf tiles that this wave keeps: process them now, a band row at a time
  const bool publish = pi.hidx >= 0 && !(a.flags & SCCG_F_NO_SPLIT_QUEUE) && n >= a.min_cells_to_queue;
  if (cl == 0 && n && !publish) {
    const uint64_t kn = (a.flags & SCCG_F_NO_KNOWN_INSIDE) ? 0ull : ~0ull;
    leaf_rows(c, pi, bx0, by0, bx1, by1, gy, cont, in_p & kn, in_q & kn, acc);
    return;
  }
  // one lane per continuing cell
  bool has = false;
  uint64_t word = 0;
  if ((cont >> c.lane) & 1ull) {
    const int i = c.lane & 7, j = c.lane >> 3;
    const int tx = ((bx0 - pi.box.x0) >> 6) + (i << (3 * cl));
    const int ty = ((by0 - pi.box.y0) >> 6) + (j << (3 * cl));
    has = true;
    word = task_word(pi.hidx < 0 ? 0 : pi.hidx, cl, tx, ty, (in_p >> c.lane) & 1ull, (in_q >> c.lane) & 1ull);
  }
  if (n) emit_children(c, pi, word, has, n);
}

// Process one box task of pair `pi`: a leaf tile or a further split.
__device__ __forceinline__ void run_box(Ctx& c, const PairInfo& pi, uint64_t w, uint64_t& acc) {
  const BatchArgs& a = *c.a;
  const Task t = task_decode(w);
  const int side = kTile << (3 * t.level);
  const int x0 = pi.box.x0 + t.tx * kTile, y0 = pi.box.y0 + t.ty * kTile;
  const int x1 = min(x0 + side, pi.box.x1), y1 = min(y0 + side, pi.box.y1);
  const bool kp = t.kp && !(a.flags & SCCG_F_NO_KNOWN_INSIDE);
  const bool kq = t.kq && !(a.flags & SCCG_F_NO_KNOWN_INSIDE);
  if (t.level == 0)
    acc += leaf_count(c, pi, x0, y0, x1 - x0, y1 - y0, kp, kq);
  else
    split_box(c, pi, x0, y0, x1, y1, t.level - 1, kp, kq, acc);
}

__device__ __forceinline__ void drain_local(Ctx& c, const PairInfo& pi, uint64_t& acc) {
  while (c.lsp > 0) {
    c.lsp -= 1;
    wave_sync_lds();
    const uint64_t w = c.local[c.lsp];
    wave_sync_lds();
    run_box(c, pi, uniform64((int64_t)w), acc);
  }
}

// The large path for one pair: `task` (a root box, a queued box or a leaf
// tile) goes on the wave's box stack and the stack is drained.  Every large
// box of the kernel goes through this one site.  Returns the intersection
// counted.
__device__ __forceinline__ uint64_t run_large(Ctx& c, const PairInfo& pi, uint64_t task) {
  c.local[c.lsp] = task;
  c.lsp += 1;
  wave_sync_lds();
  uint64_t acc = 0;
  drain_local(c, pi, acc);
  return acc;
}

// The task word of a whole pair box: a cell of the first level whose side
// covers the box, at the pair-box origin.
__device__ __forceinline__ uint64_t root_task(const PairInfo& pi) {
  const int side = max(pi.box.x1 - pi.box.x0, pi.box.y1 - pi.box.y0);
  int cl = 0;
  while ((kTile << (3 * cl)) < side) ++cl;
  return task_word(pi.hidx < 0 ? 0 : pi.hidx, cl, 0, 0, false, false);
}

// A listed pair (its box from the prepass or the sweep).  Its index also
// names it in the task words of its boxes.
__device__ __forceinline__ PairInfo heavy_info(const BatchArgs& a, int64_t pair) {
  PairInfo pi;
  pi.hidx = pair;
  pi.pair = pair;
  const int64_t ia = a.pa[pair], ib = a.pb[pair];
  pi.op = a.A.off[ia];
  pi.np = a.A.off[ia + 1] - pi.op;
  pi.oq = a.B.off[ib];
  pi.nq = a.B.off[ib + 1] - pi.oq;
  pi.box = load_meta(a.hbox, pair);
  pi.area_sum = 0;
  make_uniform(pi);
  return pi;
}

// The list bucket of a pair with n vertices (largest first; one bucket when
// the order is switched off).
__device__ __forceinline__ int lpt_bucket(const BatchArgs& a, int64_t n) {
  if (a.flags & SCCG_F_NO_LPT) return 0;
  const int64_t h = a.heavy_verts;
  return n >= 4 * h ? 3 : n >= 2 * h ? 2 : n >= h ? 1 : 0;
}

// Occupancy target of the persistent kernel (waves per SIMD); 0 leaves the
// register budget to the compiler.  A build-time tuning knob.
#ifndef SCCG_RUN_WAVES_PER_EU
#define SCCG_RUN_WAVES_PER_EU 4
#endif
#if SCCG_RUN_WAVES_PER_EU > 0
#define SCCG_RUN_ATTR __attribute__((amdgpu_waves_per_eu(SCCG_RUN_WAVES_PER_EU)))
#else
#define SCCG_RUN_ATTR
#endif

// -------------------------------------------------------------------- sweep
// First pass of a batched call: every pair the setup pass did not list as
// heavy, one pair at a time per wave, a chunk of consecutive pairs per claim.
// A pair whose two rings have at most kSweepRing vertices each is loaded
// into registers, both rings as one stream of positions (p's vertices, then
// q's); when the union of its MBRs fits one leaf tile it is counted there
// at once (below Section 3.4's pixelization threshold, I and U directly).
// Every other pair gets its MBRs and areas from its rings and is appended,
// with its pair box, to the persistent kernel's list.
constexpr int kSweepRing = 2 * kWave;                 // longest ring of the union sweep
constexpr int kMediumRing = 4 * kWave;                // longest ring of the medium sweep
constexpr int kSweepWaves = 4;                        // waves per workgroup of the sweep
constexpr int kSweepRowTiles = 4;                     // widest box (in leaf tiles) the sweep pixelizes
// Occupancy target of the sweep (waves per SIMD), a build-time tuning knob;
// the sweep that also counts pair boxes holds more wave-uniform values and
// runs fewer waves, each with the largest scalar register file.
#ifndef SCCG_SWEEP_WAVES_PER_EU
#define SCCG_SWEEP_WAVES_PER_EU 8
#endif
#ifndef SCCG_SWEEP_PB_WAVES_PER_EU
#define SCCG_SWEEP_PB_WAVES_PER_EU 6
#endif

// the lanes named by a wave-uniform mask (the mask is the lane condition)
__device__ __forceinline__ bool lane_in(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// lanes [0, n) of a chunk, for any n
__device__ __forceinline__ uint64_t lanes_lt(int n) {
  return n <= 0 ? 0ull : (n >= kWave ? ~0ull : (1ull << n) - 1ull);
}

// Lane L < 32 gets lane L + 32's value (v_permlane32_swap).
__device__ __forceinline__ uint32_t upper_half(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_permlane32_swap((int)v, (int)v, false, false)[1];
}
__device__ __forceinline__ uint64_t upper_half(uint64_t v) {
  return ((uint64_t)upper_half((uint32_t)(v >> 32)) << 32) | upper_half((uint32_t)v);
}

// The value of the next lane (DPP wave shift left by one; lane 63 reads 0).
__device__ __forceinline__ int next_lane_x(int x) { return __builtin_amdgcn_update_dpp(0, x, 0x130, 0xf, 0xf, false); }

// A sweep pair in registers: each ring in up to N 64-vertex chunks, lane L
// of chunk c holding vertex 64 c + L (lanes past the end hold the ring's last
// vertex again: neutral for extents).
constexpr int kUnionChunks = kSweepRing / kWave;    // chunks per ring in the union sweep
constexpr int kMediumChunks = kMediumRing / kWave;  // chunks per ring in the medium sweep
template <int N>
struct PairRegs {
  int2 p[N], q[N];
};
// pairs of the union sweep whose rings are in flight beyond the pair in
// hand (deeper lookahead measured no faster: the sweep is bound by
// instruction issue, not by load latency)
constexpr int kSweepAhead = 1;
#ifndef SCCG_RUN_STEAL
#define SCCG_RUN_STEAL 0
#endif
// whether the persistent kernel's waves also claim listed pairs from other
// XCDs' streams
constexpr bool kRunSteal = SCCG_RUN_STEAL != 0;
#ifndef SCCG_SWEEP_STEAL
#define SCCG_SWEEP_STEAL 0
#endif
// whether the sweeps' waves also claim from other XCDs' streams
constexpr bool kSweepSteal = SCCG_SWEEP_STEAL != 0;


// lanes [0, k) for 0 <= k <= 63, and lanes [0, m) for 1 <= m <= 64
__device__ __forceinline__ uint64_t lanes_below_k(int k) { return (1ull << k) - 1ull; }
__device__ __forceinline__ uint64_t lanes_upto_m(int m) { return ~0ull >> (kWave - m); }

// The corners of a ring held in registers: the vertices whose two edges are
// not both vertical or both horizontal (bit L of word c: vertex 64 c + L).
// A vertex's edge to its successor is vertical iff both have the same x;
// the successor is the next lane, the next chunk's first lane, and after
// the last vertex the first.
template <int N>
__device__ __forceinline__ void ring_corners(const int2 (&d)[N], int nr, uint64_t (&cm)[N]) {
#pragma unroll
  for (int c = 0; c < N; ++c) cm[c] = 0;
  if (nr <= 0) return;
  const int nc = (nr + kWave - 1) / kWave;
  const int le = (nr - 1) & (kWave - 1);  // lane of the last vertex, in the last chunk
  const int xl_lane = nc == 1 ? d[0].x : nc == 2 ? d[1 < N ? 1 : N - 1].x : nc == 3 ? d[2 < N ? 2 : N - 1].x
                                                                              : d[N - 1].x;
  const uint64_t last = __builtin_amdgcn_readlane(xl_lane, le) == __builtin_amdgcn_readlane(d[0].x, 0) ? 1ull : 0ull;
  uint64_t carry = last;  // the edge before vertex 0 is the ring's last
#pragma unroll
  for (int c = 0; c < N; ++c) {
    if (c < nc) {
      int xs;
      if (c + 1 < N && c + 1 < nc)
        xs = __builtin_amdgcn_update_dpp(__builtin_amdgcn_readlane(d[c + 1 < N ? c + 1 : c].x, 0), d[c].x,
                                         0x130, 0xf, 0xf, false);
      else
        xs = next_lane_x(d[c].x);
      uint64_t b = ballot(d[c].x == xs);
      if (c == nc - 1) b = (b & lanes_below_k(le)) | (last << le);
      cm[c] = (b ^ ((b << 1) | carry)) & (c == nc - 1 ? lanes_upto_m(nr - c * kWave) : ~0ull);
      carry = b >> 63;
    }
  }
}

// Scatter of one ring of a union tile (see union_counts): every corner XORs
// the rows at or above it into the slot of the rightmost column left of it.
// `base`: the ring's first slot.  kClip: vertices may lie outside the tile
// (see union_counts).  Returns the vertices scattered.
template <typename M, int W, int R, int N, bool kClip = false>
__device__ __forceinline__ uint32_t ring_scatter(M* slots, const int2 (&d)[N], int nr, int x0, int y0,
                                                 int lane, int base) {
  if (nr <= 0) return 0;
  uint64_t cm[N];
  ring_corners(d, nr, cm);
  uint32_t kept = 0;
#pragma unroll
  for (int c = 0; c < N; ++c) {
    if (c * kWave < nr) {
      const int dx = kClip ? min(d[c].x, x0 + W) - x0 : d[c].x - x0;
      const int ty = kClip ? max(min(d[c].y, y0 + R) - y0, 0) : d[c].y - y0;
      const uint64_t keep = cm[c] & ballot(dx > 0) & ballot(ty < R);
      M* sp = slots + (base + W - dx);
      if (lane_in(keep)) slot_xor(sp, 0, (M)(~(M)0 << ty));
      kept += (uint32_t)__popcll(keep);
    }
  }
  return kept;
}

// Counts of a pair whose MBR union [x0, x0 + W) x [y0, y0 + R) fits one leaf
// tile, from its rings in registers, packed as I | U << 16.
//
// Pixel (x, y) is inside a ring iff an odd number of its vertical edges lie
// right of x with a span holding row y (Section 3.1).  A vertical edge from
// (X, ya) to (X, yb) holds row y iff exactly one of ya, yb is <= y, so its
// term is the XOR of one term per end: "rows >= y_end, in the columns left of
// X".  Summed over a ring, a vertex contributes its term once for each
// vertical edge it bounds: once at a corner, twice (no effect) between two
// vertical edges, never between two horizontal ones.  So every vertex whose
// two edges are not both vertical or both horizontal XORs the mask of rows
// >= y_v into the slot of the rightmost column left of x_v, and the prefix
// XOR over the columns (lanes, in reverse order as in the other leaves)
// gives every column's crossing parities.  Every vertex lies in the tile:
// rows and columns past the union box come out outside, and nothing needs
// clipping.  kHalves: W = 32, p's columns in lanes 0-31 and q's in lanes
// 32-63, one scan; else W = 64 and one scan per ring.  M: 32- or 64-bit rows.
//
// kClip: the tile [x0, x0 + W) x [y0, y0 + R) is a pair box, and vertices
// may lie outside it.  A corner left of it toggles none of its columns and
// one right of it all of them (its x is taken as x0 + W); a corner below it
// sets all of its rows and one above it none.  Every pixel's parities in the
// tile stay exact, and a pixel of the tile outside the pair box is outside
// MBR(p) or MBR(q), so the intersection count is exact; the union count is
// not (the caller takes U from the areas).
template <bool kHalves, typename M, int N, bool kClip = false>
__device__ __forceinline__ uint32_t union_counts(Ctx& c, const PairRegs<N>& r, int np, int nq, int x0, int y0) {
  constexpr int W = kHalves ? 32 : kWave;
  constexpr int R = (int)sizeof(M) * 8;
  const int lane = c.lane;
  M* slots = reinterpret_cast<M*>(c.slots);
  slots[lane] = (M)0;
  if (!kHalves) slots[kWave + lane] = (M)0;
  wave_sync_lds();
  uint32_t kept = ring_scatter<M, W, R, N, kClip>(slots, r.p, np, x0, y0, lane, 0);
  kept += ring_scatter<M, W, R, N, kClip>(slots, r.q, nq, x0, y0, lane, W);
  wave_sync_lds();
  uint32_t t;
  if (kHalves) {
    const M m = wave_prefix_xor<true>(slots[lane]);
    const M o = upper_half(m);
    const uint32_t ni = lane < 32 ? (uint32_t)__popcll((uint64_t)(m & o)) : 0u;
    const uint32_t nu = lane < 32 ? (uint32_t)__popcll((uint64_t)(m | o)) : 0u;
    t = wave_sum_u32(ni | (nu << 16));
  } else {
    const M mp = wave_prefix_xor<false>(slots[lane]);
    const M mq = wave_prefix_xor<false>(slots[kWave + lane]);
    t = wave_sum_u32((uint32_t)__popcll((uint64_t)(mp & mq)) | ((uint32_t)__popcll((uint64_t)(mp | mq)) << 16));
  }
  wave_sync_lds();
  stat_add(c, 14, (unsigned long long)kept);
  return t;
}

// Scan and count of a union tile's 64-bit slots (see union_counts), packed as
// I | U << 16.  kHalves: W = 32, p's columns in slots 0-31 and q's in 32-63;
// else p's in 0-63 and q's in 64-127.  kRows64: rows 32-63 are in use
// (else those bits are all zero: rows past the union box come out outside).
template <bool kHalves, bool kRows64>
__device__ __forceinline__ uint32_t union_tile_count(const uint64_t* slots, int lane) {
  using M = typename std::conditional<kRows64, uint64_t, uint32_t>::type;
  auto slot = [&](int k) -> M {
    if (kRows64) return (M)slots[k];
    return (M)reinterpret_cast<const uint32_t*>(slots)[2 * k];  // low word: rows 0-31
  };
  uint32_t ni, nu;
  if (kHalves) {
    const M m = wave_prefix_xor<true>(slot(lane));
    const M o = upper_half(m);
    ni = lane < 32 ? (uint32_t)__popcll((uint64_t)(m & o)) : 0u;
    nu = lane < 32 ? (uint32_t)__popcll((uint64_t)(m | o)) : 0u;
  } else {
    const M mp = wave_prefix_xor<false>(slot(lane));
    const M mq = wave_prefix_xor<false>(slot(kWave + lane));
    ni = (uint32_t)__popcll((uint64_t)(mp & mq));
    nu = (uint32_t)__popcll((uint64_t)(mp | mq));
  }
  return wave_sum_u32(ni | (nu << 16));
}

// One ring of at most 64 vertices (lane L: vertex L; lanes past the end hold
// the last vertex again) scattered into a union tile's 64-bit slots from
// `base` on (see union_counts).  Each lane finds whether its vertex is a
// corner from its two neighbours' x (the last vertex's successor is the
// first, the first's predecessor the last), so that the lane masks combine
// in few scalar steps.  Returns the vertices scattered.
__device__ __forceinline__ uint32_t scatter_small_ring(uint64_t* slots, int2 v, int nr, int x0, int y0, int W, int base,
                                                       int lane) {
  if (nr <= 0) return 0;
  const int le = nr - 1;
  const int x_first = __builtin_amdgcn_readfirstlane(v.x), x_last = __builtin_amdgcn_readlane(v.x, le);
  // the neighbours' x, read by every lane before the selections
  const int xn = next_lane_x(v.x), xb = __builtin_amdgcn_update_dpp(0, v.x, 0x138, 0xf, 0xf, false);  // wave_shr:1
  const int xs = lane == le ? x_first : xn;
  const int xp = lane == 0 ? x_last : xb;
  const int dx = v.x - x0, ty = v.y - y0;
  const bool keep = (lane <= le) & ((v.x == xs) != (v.x == xp)) & (dx > 0) & (ty < kWave);
  if (keep) slot_xor(slots + (base + W - dx), 0, ~0ull << ty);
  return (uint32_t)__popcll(ballot(keep));
}

// A pair whose rings have at most 64 vertices each, one chunk per ring in
// registers: when the union of its MBRs fits one leaf tile (and every
// coordinate is in range), its counts packed as I | U << 16 in t, and true.
// The counts of such a pair on its union box [x0, x1) x [y0, y1), which fits
// one leaf tile, packed as I | U << 16 in t.
__device__ __forceinline__ void union_small_box(Ctx& c, int2 vp, int np, int2 vq, int nq, int x0, int y0, int x1,
                                                int y1, uint32_t& t) {
  const int lane = c.lane;
  const int uw = x1 - x0, uh = y1 - y0;
  const int W = uw <= 32 ? 32 : kWave;
  uint64_t* slots = c.slots;
  slots[lane] = fresh_zero<uint64_t>();
  slots[kWave + lane] = fresh_zero<uint64_t>();
  wave_sync_lds();
  uint32_t kept = scatter_small_ring(slots, vp, np, x0, y0, W, 0, lane);
  kept += scatter_small_ring(slots, vq, nq, x0, y0, W, W, lane);
  wave_sync_lds();
  if (W == 32)
    t = uh <= 32 ? union_tile_count<true, false>(slots, lane) : union_tile_count<true, true>(slots, lane);
  else
    t = uh <= 32 ? union_tile_count<false, false>(slots, lane) : union_tile_count<false, true>(slots, lane);
  wave_sync_lds();
  if (c.stats) {
    const int n = np + nq;
    stat_add(c, 14, (unsigned long long)kept);
    stat_add(c, 5, 1ull);
    stat_add(c, 11, (unsigned long long)uw * uh);
    stat_add(c, 13, (unsigned long long)n);
    stat_add(c, 1, 1ull);
    stat_add(c, 0, 2ull * (unsigned long long)uw * uh);
    stat_add(c, 10, (unsigned long long)n);
  }
}

__device__ __forceinline__ bool union_small(Ctx& c, int2 vp, int np, int2 vq, int nq, uint32_t& t) {
  const int2 a = np > 0 ? vp : vq, b = nq > 0 ? vq : vp;  // an empty ring takes the other's vertices
  const int x0 = wave_min_i32(min(a.x, b.x)), y0 = wave_min_i32(min(a.y, b.y));
  const int x1 = wave_max_i32(max(a.x, b.x)), y1 = wave_max_i32(max(a.y, b.y));
  if (!(x0 >= -kMaxCoord && y0 >= -kMaxCoord && x1 <= kMaxCoord && y1 <= kMaxCoord &&
        side_u(x0, x1) <= (uint32_t)kTile && side_u(y0, y1) <= (uint32_t)kTile))
    return false;
  union_small_box(c, vp, np, vq, nq, x0, y0, x1, y1, t);
  return true;
}

// The counts of such a pair on its union box [x0, x1) x [y0, y1), which fits
// one leaf tile, packed as I | U << 16 in t.
template <int N>
__device__ __forceinline__ void union_pair_box(Ctx& c, const PairRegs<N>& r, int np, int nq, int x0, int y0, int x1,
                                               int y1, uint32_t& t) {
  const int uw = x1 - x0, uh = y1 - y0;
  if (uw <= 32)
    t = uh <= 32 ? union_counts<true, uint32_t, N>(c, r, np, nq, x0, y0)
                 : union_counts<true, uint64_t, N>(c, r, np, nq, x0, y0);
  else
    t = uh <= 32 ? union_counts<false, uint32_t, N>(c, r, np, nq, x0, y0)
                 : union_counts<false, uint64_t, N>(c, r, np, nq, x0, y0);
  if (c.stats) {
    const int n = np + nq;
    stat_add(c, 5, 1ull);
    stat_add(c, 11, (unsigned long long)uw * uh);
    stat_add(c, 13, (unsigned long long)n);
    stat_add(c, 1, 1ull);
    stat_add(c, 0, 2ull * (unsigned long long)uw * uh);
    stat_add(c, 10, (unsigned long long)n);
  }
}

// A pair held in registers: when the union of its MBRs fits one leaf tile
// (and every coordinate is in range), its counts packed as I | U << 16 in t,
// and true.
template <int N>
__device__ __forceinline__ bool union_pair(Ctx& c, const PairRegs<N>& r, int np, int nq, uint32_t& t) {
  const int2 f = np > 0 ? r.p[0] : r.q[0];  // lanes of an empty ring take this vertex
  int mnx = f.x, mny = f.y, mxx = f.x, mxy = f.y;
  auto add = [&](int2 v) {
    mnx = min(mnx, v.x);
    mny = min(mny, v.y);
    mxx = max(mxx, v.x);
    mxy = max(mxy, v.y);
  };
#pragma unroll
  for (int c = 0; c < N; ++c) {
    if (c > 0 && c * kWave < np) add(r.p[c]);
    if (c * kWave < nq) add(r.q[c]);
  }
  const int x0 = wave_min_i32(mnx), y0 = wave_min_i32(mny);
  const int x1 = wave_max_i32(mxx), y1 = wave_max_i32(mxy);
  if (!(x0 >= -kMaxCoord && y0 >= -kMaxCoord && x1 <= kMaxCoord && y1 <= kMaxCoord &&
        side_u(x0, x1) <= (uint32_t)kTile && side_u(y0, y1) <= (uint32_t)kTile))
    return false;
  union_pair_box<N>(c, r, np, nq, x0, y0, x1, y1, t);
  return true;
}

// Extent of a ring held in registers (one or more chunks, lanes past the end
// holding the last vertex again): pixels [x0, x1) x [y0, y1) of its vertices.
// An empty ring, or one with a coordinate beyond 2^30 (returns true), comes
// back as the empty extent {INT_MAX, INT_MAX, INT_MIN, INT_MIN}.
template <int N>
__device__ __forceinline__ bool ring_extent_regs(const int2 (&d)[N], int nr, Meta& m) {
  m = Meta{INT_MAX, INT_MAX, INT_MIN, INT_MIN};
  if (nr <= 0) return false;
  const int nc = (nr + kWave - 1) / kWave;
  int mnx = d[0].x, mny = d[0].y, mxx = mnx, mxy = mny;
#pragma unroll
  for (int c = 1; c < N; ++c) {
    if (c < nc) {
      mnx = min(mnx, d[c].x);
      mny = min(mny, d[c].y);
      mxx = max(mxx, d[c].x);
      mxy = max(mxy, d[c].y);
    }
  }
  const Meta e{wave_min_i32(mnx), wave_min_i32(mny), wave_max_i32(mxx), wave_max_i32(mxy)};
  if (e.x0 < -kMaxCoord || e.y0 < -kMaxCoord || e.x1 > kMaxCoord || e.y1 > kMaxCoord) return true;
  m = e;
  return false;
}

// |shoelace|/2 of a non-empty ring held in registers whose extent e is in
// range (Section 3.2's area formula).  Twice the signed area is summed modulo
// 2^32 for a ring at most 32767 pixels on a side, else modulo 2^64, and its
// magnitude taken, which is exact while it stays within 2^31 (2^63).
template <int N>
__device__ __forceinline__ int64_t ring_area_regs(const int2 (&d)[N], int nr, int lane, const Meta& e) {
  const int nc = (nr + kWave - 1) / kWave;
  // A simple ring at most 32767 pixels wide and tall has |twice its area|
  // below 2^31: summed from coordinates relative to its first vertex (the
  // sum does not depend on the origin) it is exact modulo 2^32 in 32-bit
  // lanes.
  const bool narrow = side_u(e.x0, e.x1) <= (uint32_t)kMaxSide && side_u(e.y0, e.y1) <= (uint32_t)kMaxSide;
  // each vertex's successor: the next lane, the next chunk's first lane, and
  // the first vertex after the last
  const int le = (nr - 1) & (kWave - 1);
  const int2 f = lane_value(d[0], 0);
  uint64_t tw = 0;
  uint32_t tn = 0;
#pragma unroll
  for (int c = 0; c < N; ++c) {
    if (c < nc) {
      const bool last_chunk = c == nc - 1;
      const int2 nx = last_chunk ? f : lane_value(d[c + 1 < N ? c + 1 : c], 0);
      int sx = __builtin_amdgcn_update_dpp(nx.x, d[c].x, 0x130, 0xf, 0xf, false);
      int sy = __builtin_amdgcn_update_dpp(nx.y, d[c].y, 0x130, 0xf, 0xf, false);
      if (last_chunk && lane == le) {
        sx = f.x;
        sy = f.y;
      }
      if (!last_chunk || lane <= le) {
        if (narrow) {
          const uint32_t ux = (uint32_t)d[c].x - (uint32_t)f.x, uy = (uint32_t)d[c].y - (uint32_t)f.y;
          const uint32_t vx = (uint32_t)sx - (uint32_t)f.x, vy = (uint32_t)sy - (uint32_t)f.y;
          tn += ux * vy - vx * uy;
        } else {
          tw += (uint64_t)((int64_t)d[c].x * sy) - (uint64_t)((int64_t)sx * d[c].y);
        }
      }
    }
  }
  if (narrow) {
    const int32_t t = (int32_t)wave_sum_u32(tn);
    return (t < 0 ? -(int64_t)t : (int64_t)t) / 2;
  }
  const uint64_t t = wave_sum_u64(tw);
  return (int64_t)(((int64_t)t < 0 ? 0 - t : t) / 2);
}

// Extent and area of a ring held in registers (see ring_extent_regs and
// ring_area_regs); an empty or rejected ring has area 0, and a rejected one
// sets `bad`.
template <int N>
__device__ __forceinline__ void ring_meta_regs(const int2 (&d)[N], int nr, int lane, Meta& m, int64_t& area,
                                               bool& bad) {
  bad = ring_extent_regs(d, nr, m);
  area = nr > 0 && !bad ? ring_area_regs(d, nr, lane, m) : 0;
}

// Count of a pair box [bx0, bx1) x [by0, by1) at most kSweepRowTiles leaf
// tiles wide, from the rings in registers: the vertex form of the crossing
// test (see union_counts) with the box clipping it.  A corner left of the
// box toggles none of its columns and one right of it all of them; a corner
// below a band row of the box sets all of the band's rows and one above it
// none.  Each band row is laid out as in leaf_rows: the columns of both
// rings in one slot array each, tiles scanned right to left with the XOR of
// the tiles to their right carried.  kQ: q's first slot (p's is slot 0); a
// box gx tiles wide uses slots [0, gx kWave) and [kQ, kQ + gx kWave).
template <int N, int kQ = kSweepRowTiles * kWave>
__device__ __forceinline__ uint64_t sweep_rows(Ctx& c, const PairRegs<N>& r, int np, int nq, const Meta& box) {
  const int lane = c.lane;
  const int bw = box.x1 - box.x0, bh = box.y1 - box.y0;
  const int gx = (bw + kTile - 1) / kTile, gy = (bh + kTile - 1) / kTile;
  const int wpad = gx * kTile;
  // per vertex: its slot position when it is a corner right of the box's
  // left side, else -1
  int posp[N], posq[N];
  {
    uint64_t cm[N];
    ring_corners(r.p, np, cm);
#pragma unroll
    for (int ch = 0; ch < N; ++ch) {
      const int dx = min(r.p[ch].x, box.x0 + wpad) - box.x0;
      posp[ch] = lane_in(cm[ch]) && dx > 0 ? wpad - dx : -1;
    }
    ring_corners(r.q, nq, cm);
#pragma unroll
    for (int ch = 0; ch < N; ++ch) {
      const int dx = min(r.q[ch].x, box.x0 + wpad) - box.x0;
      posq[ch] = lane_in(cm[ch]) && dx > 0 ? kQ + wpad - dx : -1;
    }
  }
  uint64_t* slots = c.slots;
  uint32_t ni = 0;
#pragma unroll 1
  for (int j = 0; j < gy; ++j) {
    const int ry0 = box.y0 + kTile * j, th = min(kTile, box.y1 - ry0);
    const uint64_t full = row_range(0, th);
#pragma unroll 1
    for (int b = 0; b < gx; ++b) {
      slots[b * kWave + lane] = fresh_zero<uint64_t>();
      slots[kQ + b * kWave + lane] = fresh_zero<uint64_t>();
    }
    wave_sync_lds();
#pragma unroll
    for (int ch = 0; ch < N; ++ch) {
      if (ch * kWave < np) {
        const int ty = min(r.p[ch].y, ry0 + kTile) - ry0;
        if (posp[ch] >= 0 && ty < kTile) slot_xor(slots, posp[ch], ty <= 0 ? ~0ull : ~0ull << ty);
      }
      if (ch * kWave < nq) {
        const int ty = min(r.q[ch].y, ry0 + kTile) - ry0;
        if (posq[ch] >= 0 && ty < kTile) slot_xor(slots, posq[ch], ty <= 0 ? ~0ull : ~0ull << ty);
      }
    }
    wave_sync_lds();
    uint64_t carry_p = 0, carry_q = 0;
#pragma unroll 1
    for (int i = gx - 1; i >= 0; --i) {
      const int b = gx - 1 - i;
      const uint64_t xp = wave_prefix_xor<false>(slots[b * kWave + lane]);
      const uint64_t xq = wave_prefix_xor<false>(slots[kQ + b * kWave + lane]);
      const int tw = min(kTile, bw - kTile * i);
      if (kWave - 1 - lane < tw) ni += (uint32_t)__popcll((xp ^ carry_p) & (xq ^ carry_q) & full);
      carry_p ^= (uint64_t)readlane64((int64_t)xp, kWave - 1);
      carry_q ^= (uint64_t)readlane64((int64_t)xq, kWave - 1);
    }
    wave_sync_lds();
  }
  if (c.stats) {
    stat_add(c, 1, (unsigned long long)gx * gy);
    stat_add(c, 0, 2ull * (unsigned long long)bw * bh);
    stat_add(c, 10, (unsigned long long)(np + nq) * gy);
  }
  return wave_sum_u32(ni);
}

// A sweep pair held in registers that the union tile does not take: MBRs and
// areas, then the pair box (the union box when the union is counted
// directly).  Returns the pair's class: done (an empty box, or a box side
// out of range: I and U are final), or small / large (the pair is to be
// listed for the persistent kernel with `box`, I = 0 and U = |p| + |q|, or 0
// when the union is counted directly, as the values its boxes add to).
template <int N>
__device__ __forceinline__ uint8_t sweep_meta(Ctx& c, const PairRegs<N>& r, int np, int nq, int64_t& I, int64_t& U,
                                              Meta& box) {
  const BatchArgs& a = *c.a;
  Meta mp, mq;
  int64_t ap, aq;
  bool bp, bq;
  ring_meta_regs(r.p, np, c.lane, mp, ap, bp);
  ring_meta_regs(r.q, nq, c.lane, mq, aq, bq);
  if (c.lane == 0 && (bp || bq)) latch_error(a.err, kErrCoord);
  const bool direct = direct_union(a);
  box = direct ? union_box(mp, mq) : pair_box(mp, mq);
  I = 0;
  U = direct ? 0 : ap + aq;
  if (box.x0 >= box.x1 || box.y0 >= box.y1) {
    stat_add(c, 12, (unsigned long long)(np + nq));
    stat_add(c, 7, 1ull);  // empty pair box: nothing in common
    return kClsDone;
  }
  const uint32_t bw = side_u(box.x0, box.x1), bh = side_u(box.y0, box.y1);
  if (bw > (uint32_t)kMaxSide || bh > (uint32_t)kMaxSide) {
    if (c.lane == 0) latch_error(a.err, kErrSide);
    stat_add(c, 12, (unsigned long long)(np + nq));
    stat_add(c, 7, 1ull);
    U = 0;
    return kClsDone;
  }
  const bool small = bw <= (uint32_t)kTile && bh <= (uint32_t)kTile;
  stat_add(c, 12, (unsigned long long)(np + nq));
  stat_add(c, small ? 5 : 6, 1ull);
  stat_add(c, 11, (unsigned long long)bw * bh);
  return small ? kClsSmall : kClsLarge;
}

// A sweep pair as the setup pass recorded it (wave-uniform), taken from the
// chunk's records held one per lane.
struct SweepRec {
  int64_t op, oq;
  int np, nq, cls;
};
struct ChunkRecs {
  int op_lo, op_hi, oq_lo, oq_hi, np, nq, cls;
};
__device__ __forceinline__ SweepRec sweep_rec(const ChunkRecs& cr, int j) {
  SweepRec s;
  s.op = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(cr.op_hi, j) << 32) |
                   (uint32_t)__builtin_amdgcn_readlane(cr.op_lo, j));
  s.oq = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(cr.oq_hi, j) << 32) |
                   (uint32_t)__builtin_amdgcn_readlane(cr.oq_lo, j));
  s.np = __builtin_amdgcn_readlane(cr.np, j);
  s.nq = __builtin_amdgcn_readlane(cr.nq, j);
  s.cls = __builtin_amdgcn_readlane(cr.cls, j);
  return s;
}
// the records of pairs i0 + lane (lane < cnt) of a chunk, one coalesced load
__device__ __forceinline__ ChunkRecs chunk_recs(const BatchArgs& a, int64_t i0, int cnt, int lane) {
  ChunkRecs cr{0, 0, 0, 0, 0, 0, kClsDone};
  if (lane < cnt) {
    const int4 h = *reinterpret_cast<const int4*>(a.rec + i0 + lane);
    const int4 t = *(reinterpret_cast<const int4*>(a.rec + i0 + lane) + 1);
    cr = ChunkRecs{h.x, h.y, h.z, h.w, t.x, t.y, t.z};
  }
  return cr;
}

// the record of pair idx in every lane with `valid` set
__device__ __forceinline__ ChunkRecs gather_recs(const BatchArgs& a, int idx, bool valid) {
  ChunkRecs cr{0, 0, 0, 0, 0, 0, kClsDone};
  if (valid) {
    const int4 h = *reinterpret_cast<const int4*>(a.rec + idx);
    const int4 t = *(reinterpret_cast<const int4*>(a.rec + idx) + 1);
    cr = ChunkRecs{h.x, h.y, h.z, h.w, t.x, t.y, t.z};
  }
  return cr;
}

// Append pairs i0 + j (bit j of `m`) to a list with one reservation.
__device__ __forceinline__ void list_append(Counter& count, int32_t* list, uint64_t m, int64_t i0, int lane) {
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd(&count.v, (unsigned long long)__popcll(m));
  base = (unsigned long long)uniform64((int64_t)__shfl((long long)base, 0, kWave));
  if (lane_in(m)) list[base + (unsigned long long)lanes_below(m)] = (int32_t)(i0 + lane);
}

// Claim a chunk of `chunk` consecutive entries from per-stream counters (one
// stream per XCD, exhausted streams marked in `empty`): its first entry, or
// -1 when every stream is exhausted.
__device__ __forceinline__ int64_t claim_chunk(Counter* next, int64_t n, int chunk, int xcd, int lane,
                                               uint32_t& empty) {
  const unsigned long long n_chunks = ((unsigned long long)n + chunk - 1) / chunk;
  if (n_chunks == 0) empty = 0xffu;
  while (empty != 0xffu) {
    const int st = next_stream(empty, xcd);
    unsigned long long k = 0;
    if (lane == 0) k = atomicAdd(&next[st].v, 1ull);
    k = (unsigned long long)uniform64((int64_t)__shfl((long long)k, 0, kWave));
    const unsigned long long g = k * kStreams + st;
    if (g >= n_chunks) {
      empty = uniform_u(empty | (1u << st));
      continue;
    }
    return uniform64((int64_t)g * chunk);
  }
  return -1;
}

// The rings of a sweep pair (lane L: vertices L and 64 + L, clamped to the
// last), or for any other record a read of `dummy`: the same loads in every
// case, so that the compiler can count the loads in flight and wait only
// for those of the pair in hand, not for the ones just issued ahead of it.
__device__ __forceinline__ void sweep_load(const BatchArgs& a, const SweepRec& s, const int2* dummy, int lane,
                                           PairRegs<kUnionChunks>& r) {
  const bool mine = s.cls == kClsSweep;
  const int2* P = mine && s.np > 0 ? a.A.xy + s.op : dummy;
  const int2* Q = mine && s.nq > 0 ? a.B.xy + s.oq : dummy;
  const int lp = mine ? max(s.np - 1, 0) : 0, lq = mine ? max(s.nq - 1, 0) : 0;
#pragma unroll
  for (int c = 0; c < kUnionChunks; ++c) {
    r.p[c] = P[min(c * kWave + lane, lp)];
    r.q[c] = Q[min(c * kWave + lane, lq)];
  }
}

// I of a pair whose pair box fits one leaf tile, counted on that box (see
// union_counts with clipping): its columns in one half of the wave when it
// is at most 32 wide, 32-bit rows when it is at most 32 tall.
template <int N>
__device__ __forceinline__ uint32_t pair_box_count(Ctx& c, const PairRegs<N>& r, int np, int nq, const Meta& box) {
  const int bw = box.x1 - box.x0, bh = box.y1 - box.y0;
  uint32_t t;
  if (bw <= 32)
    t = bh <= 32 ? union_counts<true, uint32_t, N, true>(c, r, np, nq, box.x0, box.y0)
                 : union_counts<true, uint64_t, N, true>(c, r, np, nq, box.x0, box.y0);
  else
    t = bh <= 32 ? union_counts<false, uint32_t, N, true>(c, r, np, nq, box.x0, box.y0)
                 : union_counts<false, uint64_t, N, true>(c, r, np, nq, box.x0, box.y0);
  if (c.stats) {
    stat_add(c, 1, 1ull);
    stat_add(c, 0, 2ull * (unsigned long long)bw * bh);
    stat_add(c, 10, (unsigned long long)(np + nq));
  }
  return t & 0xffffu;
}

// Pair j of the chunk (a sweep pair): counted on its union tile, leaving
// I | U << 16 in lane j of `packed` and bit j in `wmask` (written out with
// the chunk); a pair left out (union box larger than a leaf tile) goes to
// the medium list with the chunk.
__device__ __forceinline__ void sweep_one(Ctx& c, const SweepRec& s, const PairRegs<kUnionChunks>& r, int j,
                                          bool union_ok, uint32_t& packed, uint64_t& wmask) {
  if (s.cls != kClsSweep) return;  // another class, or a bad index
  const int lane = c.lane;
  uint32_t t = 0;
  bool done = s.np + s.nq == 0;  // two empty rings: nothing in either
  if (done) stat_add(c, 7, 1ull);
  if (!done && union_ok)
    done = s.np <= kWave && s.nq <= kWave ? union_small(c, r.p[0], s.np, r.q[0], s.nq, t)
                                          : union_pair<kUnionChunks>(c, r, s.np, s.nq, t);
  if (done) {
    if (lane == j) packed = t;
    wmask |= 1ull << j;
  }
}

// Extent and area of a ring held wave-uniform; area < 0 until it is needed.
struct RingInfo {
  Meta m;
  int64_t area;
  bool bad;
};

// Pair j of the chunk (a sweep pair, index i0 + j) when the union sweep also
// counts pair boxes.  Both rings' extents come first, q's carried over from
// the previous pair of the wave when it is the same ring (a join's output
// grouped by one side repeats it).  When their union fits one leaf tile the
// pair is counted there, as in sweep_one; else, the union not being counted
// directly, the pair box MBR(p) ∩ MBR(q) decides as in the medium sweep: an
// empty box (nothing in common) or one that fits a leaf tile gives I and
// U = |p| + |q| - I (Section 3.2), written out at once with bit j in
// `dmask`; a box side out of range latches the error and gives I = U = 0; a
// larger box goes, with nothing counted, to the medium list with the chunk.
__device__ __forceinline__ void sweep_one_pb(Ctx& c, const SweepRec& s, const PairRegs<kUnionChunks>& r, int64_t i0,
                                             int j, bool union_ok, uint32_t& packed, uint64_t& wmask, uint64_t& dmask,
                                             int64_t& q_off, int& q_n, RingInfo& qi) {
  if (s.cls != kClsSweep) return;  // another class, or a bad index
  const BatchArgs& a = *c.a;
  const int lane = c.lane;
  if (s.np + s.nq == 0) {  // two empty rings: nothing in either
    stat_add(c, 7, 1ull);
    if (lane == j) packed = 0;
    wmask |= 1ull << j;
    return;
  }
  RingInfo pi;
  pi.bad = ring_extent_regs(r.p, s.np, pi.m);
  pi.area = -1;
  if (s.oq != q_off || s.nq != q_n) {
    qi.bad = ring_extent_regs(r.q, s.nq, qi.m);
    qi.area = -1;
    q_off = s.oq;
    q_n = s.nq;
  }
  const bool ok = !pi.bad && !qi.bad;
  const Meta u = union_box(pi.m, qi.m);  // an empty ring's extent drops out
  if (union_ok && ok && side_u(u.x0, u.x1) <= (uint32_t)kTile && side_u(u.y0, u.y1) <= (uint32_t)kTile) {
    uint32_t t;
    if (s.np <= kWave && s.nq <= kWave)
      union_small_box(c, r.p[0], s.np, r.q[0], s.nq, u.x0, u.y0, u.x1, u.y1, t);
    else
      union_pair_box<kUnionChunks>(c, r, s.np, s.nq, u.x0, u.y0, u.x1, u.y1, t);
    if (lane == j) packed = t;
    wmask |= 1ull << j;
    return;
  }
  if (direct_union(a)) return;
  const Meta box = pair_box(pi.m, qi.m);  // empty when a ring is empty or rejected
  const bool empty = box.x0 >= box.x1 || box.y0 >= box.y1;
  const uint32_t bw = side_u(box.x0, box.x1), bh = side_u(box.y0, box.y1);
  const bool wide = !empty && (bw > (uint32_t)kMaxSide || bh > (uint32_t)kMaxSide);
  const bool small = !empty && !wide && bw <= (uint32_t)kTile && bh <= (uint32_t)kTile;
  if (!empty && !wide && !small) return;
  if (lane == 0 && !ok) latch_error(a.err, kErrCoord);
  if (lane == 0 && wide) latch_error(a.err, kErrSide);
  stat_add(c, 12, (unsigned long long)(s.np + s.nq));
  stat_add(c, small ? 5 : 7, 1ull);
  if (small) stat_add(c, 11, (unsigned long long)bw * bh);
  int64_t I = 0, U = 0;
  if (!wide) {
    if (pi.area < 0) pi.area = s.np > 0 && !pi.bad ? ring_area_regs(r.p, s.np, lane, pi.m) : 0;
    if (qi.area < 0) qi.area = s.nq > 0 && !qi.bad ? ring_area_regs(r.q, s.nq, lane, qi.m) : 0;
    U = pi.area + qi.area;
    if (small) {
      I = (int64_t)pair_box_count(c, r, s.np, s.nq, box);
      U -= I;
    }
  }
  if (lane == 0) {
    a.inter[i0 + j] = I;
    a.uni[i0 + j] = U;
  }
  dmask |= 1ull << j;
}

// The prepass of a pair the setup pass listed (entry k of its buckets laid
// end to end, largest first, nb[b] entries in bucket b): one wave reduces
// the MBRs and areas of both rings and records the pair box and the pair's
// class; the outputs start at I = 0, U = |p| + |q| (boxes add to I and
// subtract from U atomically).
__device__ __forceinline__ void prepass_one(const BatchArgs& a, int64_t k, const int64_t (&nb)[kLptBuckets], int lane,
                                            bool stats) {
  int64_t kk = k;
  int bk = kLptBuckets - 1;
#pragma unroll
  for (int b = kLptBuckets - 1; b > 0; --b) {
    if (bk == b && kk >= nb[b]) {
      kk -= nb[b];
      bk = b - 1;
    }
  }
  const int64_t i = a.l_list[(int64_t)bk * a.n_pairs + kk];
  const int64_t ia = a.pa[i], ib = a.pb[i];
  const int64_t op = a.A.off[ia], oq = a.B.off[ib];
  Meta mp, mq;
  int64_t ap, aq;
  ring_scan(a.A.xy, op, a.A.off[ia + 1] - op, lane, mp, ap);
  ring_scan(a.B.xy, oq, a.B.off[ib + 1] - oq, lane, mq, aq);
  if (lane != 0) return;
  if (stats) atomicAdd(&a.st->stats[12], (unsigned long long)(a.A.off[ia + 1] - op + a.B.off[ib + 1] - oq));
  if (coords_bad(mp, a.A.off[ia + 1] - op) || coords_bad(mq, a.B.off[ib + 1] - oq)) latch_error(a.err, kErrCoord);
  const Meta b = direct_union(a) ? union_box(mp, mq) : pair_box(mp, mq);
  *reinterpret_cast<int4*>(a.hbox + i) = make_int4(b.x0, b.y0, b.x1, b.y1);
  const int64_t w = (int64_t)b.x1 - b.x0, h = (int64_t)b.y1 - b.y0;
  uint8_t cls = kClsDone;
  a.inter[i] = 0;
  a.uni[i] = direct_union(a) ? 0 : ap + aq;
  if (b.x0 >= b.x1 || b.y0 >= b.y1) {
    cls = kClsDone;
  } else if (w > kMaxSide || h > kMaxSide) {
    latch_error(a.err, kErrSide);
    a.uni[i] = 0;
  } else {
    cls = (w <= kTile && h <= kTile) ? kClsSmall : kClsLarge;
    if (stats) {
      atomicAdd(&a.st->stats[cls == kClsSmall ? 5 : 6], 1ull);
      atomicAdd(&a.st->stats[11], (unsigned long long)(w * h));
    }
  }
  a.cls[i] = cls;
}

// kPairBox: pairs whose union box exceeds a leaf tile are counted on their
// pair box when it fits one (the same counts as the medium sweep's, without
// loading the rings again); a separate instance keeps the extra registers
// off the plain sweep, which most mixes run.  kStats: the work counters are
// kept (an instance of its own, so that the others carry no test for them).
template <bool kPairBox, bool kStats>
__global__ void __launch_bounds__(kSweepWaves* kWave)
    __attribute__((amdgpu_waves_per_eu(kPairBox ? SCCG_SWEEP_PB_WAVES_PER_EU : SCCG_SWEEP_WAVES_PER_EU)))
k_batch_sweep(BatchArgs args) {
  __shared__ __align__(16) uint64_t sweep_slots[kSweepWaves * kLeafSlots];
  Ctx c;
  c.a = &args;
  c.stats = kStats;
  c.lane = lane_id();
  c.slots = sweep_slots + (threadIdx.x / kWave) * kLeafSlots;
  c.local = nullptr;
  c.lsp = 0;
  c.home = 0;
  c.xcd = (int)(blockIdx.x % (unsigned)kStreams);
  const BatchArgs& a = args;
  const int lane = c.lane;
  const bool union_ok = direct_union(a) || !(a.flags & SCCG_F_NO_UNION_TILE);
  const unsigned long long t_start = wave_stamp(a);
  // the prepass (run beside the medium sweep) takes the pairs the setup pass
  // listed: their counts, taken here, before the medium sweep lists more
  if (blockIdx.x == 0 && threadIdx.x < kLptBuckets) a.st->p_count[threadIdx.x].v = a.st->l_count[threadIdx.x].v;
  // claim streams found exhausted (wave-uniform); a wave claims only from
  // its own XCD's stream (the streams hold equal interleaved shares), so
  // that running dry costs it one claim, not one per stream (a grid too
  // small to give every stream a workgroup claims from all of them)
  uint32_t s_empty = kSweepSteal || gridDim.x < (unsigned)kStreams ? 0u : (0xffu & ~(1u << c.xcd));
  // kPairBox: the last q ring whose extent (and area, once needed) is held
  int64_t q_off = -1;
  int q_n = -1;
  RingInfo qi{Meta{INT_MAX, INT_MAX, INT_MIN, INT_MIN}, 0, false};
  for (;;) {
    const int64_t i0 = claim_chunk(a.st->s_next, a.n_pairs, a.chunk, c.xcd, lane, s_empty);
    if (i0 < 0) break;
    const int cnt = uniform((int)min((int64_t)a.chunk, a.n_pairs - i0));
    const ChunkRecs cr = chunk_recs(a, i0, cnt, lane);
    // lane j: I | U << 16 of pair i0 + j when it is counted on its union tile
    uint32_t packed = 0;
    uint64_t wmask = 0, dmask = 0;
    // the pair in hand (s[0], r[0]) and the next kSweepAhead ones, whose ring
    // loads are in flight while the pair in hand is processed
    SweepRec s[kSweepAhead + 1];
    PairRegs<kUnionChunks> r[kSweepAhead + 1];
    const int2* dummy = reinterpret_cast<const int2*>(a.rec + i0);
#pragma unroll
    for (int k = 0; k <= kSweepAhead; ++k) {
      s[k] = k < cnt ? sweep_rec(cr, k) : SweepRec{0, 0, 0, 0, kClsDone};
      sweep_load(a, s[k], dummy, lane, r[k]);
    }
#pragma unroll 1
    for (int j = 0; j < cnt; ++j) {
      if (kPairBox)
        sweep_one_pb(c, s[0], r[0], i0, j, union_ok, packed, wmask, dmask, q_off, q_n, qi);
      else
        sweep_one(c, s[0], r[0], j, union_ok, packed, wmask);
#pragma unroll
      for (int k = 0; k < kSweepAhead; ++k) {
        s[k] = s[k + 1];
        r[k] = r[k + 1];
      }
      const int jn = j + kSweepAhead + 1;
      s[kSweepAhead] = jn < cnt ? sweep_rec(cr, jn) : SweepRec{0, 0, 0, 0, kClsDone};
      sweep_load(a, s[kSweepAhead], dummy, lane, r[kSweepAhead]);
    }
    // the chunk's union-tile counts go out in one coalesced store per array,
    // the sweep pairs it left out to the medium list with one reservation
    if (lane_in(wmask)) {
      a.inter[i0 + lane] = (int64_t)(packed & 0xffffu);
      a.uni[i0 + lane] = (int64_t)(packed >> 16);
    }
    const uint64_t left = ballot(lane < cnt && cr.cls == kClsSweep) & ~(wmask | dmask);
    if (left) list_append(a.st->m_count, a.m_list, left, i0, lane);
  }
  wave_stamps(a, 0, t_start, lane);
}

// ------------------------------------------------------------ medium sweep
// Second pass over the medium list: pairs with rings of at most kMediumRing
// vertices that the union sweep did not finish (a ring over kSweepRing
// vertices, a pair box larger than a leaf tile, or, with the union counted
// directly, a union box larger than one).  MBRs and areas come from the
// rings in registers; a pair box at most kSweepRowTiles tiles wide is
// pixelized at once (a box the persistent kernel would not classify), a
// larger one is listed with its box.  A claim takes 64 consecutive entries.
// The same kernel runs the prepass of the pairs the setup pass listed: its
// ring scans wait on memory while the medium pairs compute, so a quarter of
// the waves start with it and the rest with the medium list, each turning
// to the other list when its own runs dry.  (Six waves per SIMD, a few registers
// spilled: at the unconstrained register count only four fit.)
//
// Every chunk of both rings of a medium pair (clamped to each ring's last
// vertex), or for no pair reads of `dummy`.
__device__ __forceinline__ void medium_load(const BatchArgs& a, const SweepRec& s, const int2* dummy, int lane,
                                            PairRegs<kMediumChunks>& r) {
  const int2* P = s.np > 0 ? a.A.xy + s.op : dummy;
  const int2* Q = s.nq > 0 ? a.B.xy + s.oq : dummy;
  const int lp = max(s.np - 1, 0), lq = max(s.nq - 1, 0);
#pragma unroll
  for (int c = 0; c < kMediumChunks; ++c) {
    r.p[c] = P[min(c * kWave + lane, lp)];
    r.q[c] = Q[min(c * kWave + lane, lq)];
  }
}

__device__ __forceinline__ void medium_one(Ctx& c, const SweepRec& s, const PairRegs<kMediumChunks>& r, int64_t i) {
  const BatchArgs& a = *c.a;
  int64_t I = 0, U = 0;
  Meta box{0, 0, 0, 0};
  uint8_t cls = sweep_meta(c, r, s.np, s.nq, I, U, box);
  if (cls != kClsDone && !direct_union(a)) {
    const int gx = (box.x1 - box.x0 + kTile - 1) / kTile, gy = (box.y1 - box.y0 + kTile - 1) / kTile;
    if (gx * gy == 1) {
      I = (int64_t)pair_box_count(c, r, s.np, s.nq, box);
      U -= I;
      cls = kClsDone;
    } else if (gx <= kSweepRowTiles && gy <= kMaxGrid && gx * gy < a.min_classify_cells) {
      I = (int64_t)sweep_rows(c, r, s.np, s.nq, box);
      U -= I;
      cls = kClsDone;
    }
  }
  if (c.lane == 0) {
    a.inter[i] = I;
    a.uni[i] = U;
    if (cls != kClsDone) {
      const int bk = lpt_bucket(a, (int64_t)s.np + s.nq);
      const unsigned long long k = atomicAdd(&a.st->l_count[bk].v, 1ull);
      a.l_list[(int64_t)bk * a.n_pairs + (int64_t)k] = (int32_t)i;
      *reinterpret_cast<int4*>(a.hbox + i) = make_int4(box.x0, box.y0, box.x1, box.y1);
      a.cls[i] = cls;
    }
  }
}

template <bool kStats>
__global__ void __launch_bounds__(kSweepWaves* kWave) __attribute__((amdgpu_waves_per_eu(6))) k_batch_medium(BatchArgs args) {
  constexpr int kMediumSlots = 2 * kSweepRowTiles * kWave;
  __shared__ __align__(16) uint64_t medium_slots[kSweepWaves * kMediumSlots];
  Ctx c;
  c.a = &args;
  c.stats = kStats;
  c.lane = lane_id();
  c.slots = medium_slots + (threadIdx.x / kWave) * kMediumSlots;
  c.local = nullptr;
  c.lsp = 0;
  c.home = 0;
  c.xcd = (int)(blockIdx.x % (unsigned)kStreams);
  const BatchArgs& a = args;
  const int lane = c.lane;
  const unsigned long long t_start = wave_stamp(a);
  // the prepass entries (the setup pass's listed pairs, counted by the union
  // sweep), one per claim
  int64_t nb[kLptBuckets], n_pre = 0;
#pragma unroll
  for (int b = 0; b < kLptBuckets; ++b) {
    nb[b] = (int64_t)a.st->p_count[b].v;
    n_pre += nb[b];
  }
  const int64_t n_med = (int64_t)a.st->m_count.v;
  // entries per claim: 64, or fewer when the list gives the grid's waves
  // less than 8 claims each
  const int64_t per_wave = n_med / ((int64_t)gridDim.x * kSweepWaves * 8);
  const int chunk = (int)max((int64_t)1, min((int64_t)kWave, per_wave));
  const uint32_t own = kSweepSteal || gridDim.x < (unsigned)kStreams ? 0u : (0xffu & ~(1u << c.xcd));
  uint32_t m_empty = own, p_empty = own;
  // the first wave of each workgroup starts with the prepass, which waits on
  // memory, the others with the medium list, which computes; each turns to
  // the other list when its own runs dry (a quarter of the waves measured
  // faster than a half, an eighth or none)
  const bool pre_first = threadIdx.x / kWave == 0;
#pragma unroll 1
  for (int phase = 0; phase < 2; ++phase) {
    if ((phase == 0) == pre_first) {
#pragma unroll 1
      for (;;) {
        const int64_t k = claim_chunk(a.st->p_next, n_pre, 1, c.xcd, lane, p_empty);
        if (k < 0) break;
        prepass_one(a, k, nb, lane, kStats);
      }
      continue;
    }
#pragma unroll 1
    for (;;) {
      const int64_t e0 = claim_chunk(a.st->m_next, n_med, chunk, c.xcd, lane, m_empty);
      if (e0 < 0) break;
      const int cnt = uniform((int)min((int64_t)chunk, n_med - e0));
      // lane j: pair index and record of entry e0 + j
      const int idx = lane < cnt ? a.m_list[e0 + lane] : 0;
      const ChunkRecs cr = gather_recs(a, idx, lane < cnt);
      const int2* dummy = reinterpret_cast<const int2*>(a.rec + __builtin_amdgcn_readfirstlane(idx));
      // the pair in hand (sc, rc) and the next one (sn, rn), whose loads are in
      // flight while the pair in hand is processed: every chunk of both rings,
      // loaded the same way whatever the pair, so that the compiler waits only
      // for the pair in hand's loads
      PairRegs<kMediumChunks> rc, rn;
      SweepRec sc = sweep_rec(cr, 0);
      medium_load(a, sc, dummy, lane, rc);
#pragma unroll 1
      for (int j = 0; j < cnt; ++j) {
        const SweepRec sn = j + 1 < cnt ? sweep_rec(cr, j + 1) : SweepRec{0, 0, 0, 0, kClsDone};
        medium_load(a, sn, dummy, lane, rn);
        medium_one(c, sc, rc, (int64_t)__builtin_amdgcn_readlane(idx, j));
        sc = sn;
        rc = rn;
      }
    }
  }
  wave_stamps(a, 1, t_start, lane);
}

// ----------------------------------------------------------- persistent run
// Second pass: the listed pairs (heavy pairs from the setup pass, claimed
// first, then the sweep's pairs whose box is larger than a leaf tile), each
// with its box from the prepass or the sweep.  Waves claim, in this order:
// boxes from their queue, listed pairs, boxes from any queue.
template <bool kStats>
__global__ void __launch_bounds__(512) SCCG_RUN_ATTR k_batch_run(BatchArgs args) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wave = threadIdx.x / kWave;
  Ctx c;
  c.a = &args;
  c.stats = kStats;
  c.lane = lane_id();
  unsigned char* lds = smem + (size_t)wave * kLdsPerWave;
  c.slots = reinterpret_cast<uint64_t*>(lds);
  c.local = reinterpret_cast<uint64_t*>(lds + kRowSlotsPerWave * 8);
  c.lsp = 0;
  c.xcd = (int)(blockIdx.x % (unsigned)kStreams);
  c.home = c.xcd % args.n_queues;
  const BatchArgs& a = args;
  const unsigned long long t_start = wave_stamp(a);
  unsigned long long n_list[kLptBuckets], n_all = 0;
#pragma unroll
  for (int b = 0; b < kLptBuckets; ++b) {
    n_list[b] = a.st->l_count[b].v;
    n_all += n_list[b];
  }
  // Boxes reach a queue only from splits with at least min_cells_to_queue
  // continuing cells (at most 64): otherwise no wave ever needs to look at
  // the queues.
  const bool queues_used = n_all > 0 && !(a.flags & SCCG_F_NO_SPLIT_QUEUE) && a.min_cells_to_queue <= kWave;
  int bucket = kLptBuckets - 1;  // the bucket being claimed, largest first (wave-uniform)
  // streams of that bucket found exhausted (wave-uniform); as in the sweeps,
  // a wave claims only from its XCD's stream unless kRunSteal
  const uint32_t l_start = kRunSteal || gridDim.x < (unsigned)kStreams ? 0u : (0xffu & ~(1u << c.xcd));
  uint32_t l_empty = l_start;
  for (;;) {
    PairInfo pi;
    uint64_t task = 0;  // 0: a box that fits one leaf tile
    uint64_t w;
    bool have = false;
    if (queues_used && queue_claim(c, false, &w)) {
      pi = heavy_info(a, task_decode(w).hidx);
      task = w;
      have = true;
    }
    while (!have && bucket >= 0) {
      const unsigned long long nb = bucket == 3 ? n_list[3] : bucket == 2 ? n_list[2] : bucket == 1 ? n_list[1]
                                                                                                     : n_list[0];
      const int64_t e = claim_chunk(a.st->l_next[bucket], (int64_t)nb, 1, c.xcd, c.lane, l_empty);
      if (e < 0) {
        bucket = uniform(bucket - 1);
        l_empty = l_start;
        continue;
      }
      pi = heavy_info(a, (int64_t)a.l_list[(int64_t)bucket * a.n_pairs + e]);
      const uint8_t cls = a.cls[pi.pair];
      if (cls == kClsDone) continue;  // settled by the prepass
      have = true;
      if (cls == kClsLarge) task = root_task(pi);
    }
    // nothing of its own left: help with every queue, then stop
    if (!have) {
      if (!queues_used || !queue_claim(c, true, &w)) break;
      pi = heavy_info(a, task_decode(w).hidx);
      task = w;
    }
    uint64_t I;
    if (task == 0)
      I = leaf_count(c, pi, pi.box.x0, pi.box.y0, pi.box.x1 - pi.box.x0, pi.box.y1 - pi.box.y0, false, false);
    else
      I = run_large(c, pi, task);
    if (c.lane == 0) add_counts(a, pi.pair, I);
  }
  wave_stamps(a, 2, t_start, c.lane);
}

// ------------------------------------------------------------ setup / reset
// Clear the queue slots the previous call touched, then the counters.
__global__ void __launch_bounds__(256) k_batch_clear_slots(BatchArgs a) {
  for (int q = 0; q < a.n_queues; ++q) {
    unsigned long long used = max(a.st->q_tail[q].v, a.st->q_head[q].v);
    if (used > (unsigned long long)a.queue_cap) used = (unsigned long long)a.queue_cap;
    unsigned long long* base = a.queue + (size_t)q * a.queue_cap;
    for (unsigned long long j = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; j < used;
         j += (unsigned long long)gridDim.x * blockDim.x)
      base[j] = 0;
  }
}

__global__ void k_batch_clear_counters(BatchArgs a) {
  unsigned long long* p = reinterpret_cast<unsigned long long*>(a.st);
  const int n = (int)(sizeof(BatchState) / sizeof(unsigned long long));
  for (int k = threadIdx.x; k < n; k += blockDim.x) p[k] = 0;
}

// Per pair: index check, the pair's record and class: swept (rings of at
// most kSweepRing vertices), medium (at most kMediumRing), or listed by
// vertex count for the prepass and the persistent kernel (longer rings, or
// at least heavy_verts vertices in all).
__global__ void __launch_bounds__(256) k_batch_setup(BatchArgs a, int per) {
  // a block takes per x 256 consecutive pairs (coalesced rows of 256) and
  // reserves room for its listed pairs with one atomic per bucket: the
  // per-thread counts of the four buckets travel as 16-bit fields of one
  // 64-bit scan
  __shared__ unsigned long long scan[256];
  __shared__ unsigned long long base_s[kLptBuckets];
  const int tid = threadIdx.x;
  const int64_t b0 = (int64_t)blockIdx.x * 256 * per;
  __shared__ unsigned mscan[256];
  __shared__ unsigned long long mbase_s;
  uint32_t lmask = 0;      // bit t: pair t of this thread is listed
  uint32_t bmask = 0;      // bits 2t, 2t+1: its bucket
  uint32_t mmask = 0;      // bit t: pair t of this thread is a medium pair
  unsigned long long cnt = 0;
  for (int t = 0; t < per; ++t) {
    const int64_t i = b0 + (int64_t)t * 256 + tid;
    if (i >= a.n_pairs) break;
    const int64_t ia = a.pa[i], ib = a.pb[i];
    uint8_t cls = kClsSweep;
    PairRec r{0, 0, 0, 0, 0, 0};
    if (ia < 0 || ia >= a.A.n || ib < 0 || ib >= a.B.n) {
      latch_error(a.err, kErrIndex);
      a.inter[i] = 0;
      a.uni[i] = 0;
      cls = kClsDone;
    } else {
      r.op = a.A.off[ia];
      r.np = (int32_t)(a.A.off[ia + 1] - r.op);
      r.oq = a.B.off[ib];
      r.nq = (int32_t)(a.B.off[ib + 1] - r.oq);
      const int64_t n = (int64_t)r.np + r.nq;
      if (r.np > kMediumRing || r.nq > kMediumRing || n >= a.heavy_verts) {
        const int bk = lpt_bucket(a, n);
        lmask |= 1u << t;
        bmask |= (uint32_t)bk << (2 * t);
        cnt += 1ull << (16 * bk);
        cls = kClsHeavy;
      } else if (r.np > kSweepRing || r.nq > kSweepRing) {
        mmask |= 1u << t;
        cls = kClsMedium;
      }
    }
    r.cls = cls;
    a.cls[i] = cls;
    a.rec[i] = r;
  }
  // exclusive prefix of the per-thread counts over the block
  const unsigned mcnt = (unsigned)__popc(mmask);
  scan[tid] = cnt;
  mscan[tid] = mcnt;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {
    const unsigned long long v = tid >= d ? scan[tid - d] : 0ull;
    const unsigned mv = tid >= d ? mscan[tid - d] : 0u;
    __syncthreads();
    scan[tid] += v;
    mscan[tid] += mv;
    __syncthreads();
  }
  const unsigned long long total = scan[255];
  if (tid < kLptBuckets) {
    const unsigned long long nb = (total >> (16 * tid)) & 0xffffull;
    base_s[tid] = nb ? atomicAdd(&a.st->l_count[tid].v, nb) : 0ull;
  } else if (tid == kLptBuckets) {
    const unsigned long long nm = mscan[255];
    mbase_s = nm ? atomicAdd(&a.st->m_count.v, nm) : 0ull;
  }
  __syncthreads();
  unsigned long long mpos = mbase_s + (mscan[tid] - mcnt);
  for (uint32_t m = mmask; m; m &= m - 1)
    a.m_list[mpos++] = (int32_t)(b0 + (int64_t)(__ffs((int)m) - 1) * 256 + tid);
  const unsigned long long before = scan[tid] - cnt;
  unsigned long long pos[kLptBuckets];
#pragma unroll
  for (int b = 0; b < kLptBuckets; ++b) pos[b] = base_s[b] + ((before >> (16 * b)) & 0xffffull);
  for (uint32_t m = lmask; m; m &= m - 1) {
    const int t = __ffs((int)m) - 1;
    const int bk = (int)((bmask >> (2 * t)) & 3u);
    const int64_t k = (int64_t)(bk == 3 ? pos[3]++ : bk == 2 ? pos[2]++ : bk == 1 ? pos[1]++ : pos[0]++);
    a.l_list[(int64_t)bk * a.n_pairs + k] = (int32_t)(b0 + (int64_t)t * 256 + tid);
  }
}

__global__ void k_batch_stats_empty(BatchArgs a) {
  // pairs that ended in setup or in the heavy prepass (stats only)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.n_pairs && a.cls[i] == kClsDone) atomicAdd(&a.st->stats[7], 1ull);
}

hipError_t launch_batch_reset(const BatchArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_clear_slots, dim3(1024), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_batch_clear_counters, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_batch_setup(const BatchArgs& a, hipStream_t s) {
  if (a.n_pairs <= 0) return hipSuccess;
  // enough blocks to fill the chip (about 1024), at most kSetupPerThread pairs per thread
  const int per = (int)std::max<int64_t>(1, std::min<int64_t>(kSetupPerThread, a.n_pairs / (256 * 1024)));
  const int64_t per_block = 256 * (int64_t)per;
  const unsigned blocks = (unsigned)((a.n_pairs + per_block - 1) / per_block);
  hipLaunchKernelGGL(k_batch_setup, dim3(blocks), dim3(256), 0, s, a, per);
  return hipGetLastError();
}

int batch_occupancy(int waves_per_wg) {
  int n = 0;
  const size_t lds = (size_t)waves_per_wg * batch_lds_bytes_per_wave();
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_run<false>, waves_per_wg * kWave, lds) != hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

int batch_sweep_occupancy(bool pair_box) {
  int n = 0;
  const hipError_t e =
      pair_box ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_sweep<true, false>, kSweepWaves * kWave, 0)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_sweep<false, false>, kSweepWaves * kWave, 0);
  return e == hipSuccess && n > 0 ? n : 1;
}

int batch_medium_occupancy() {
  int n = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_medium<false>, kSweepWaves * kWave, 0);
  return e == hipSuccess && n > 0 ? n : 1;
}

int batch_sweep_waves_per_wg() { return kSweepWaves; }

hipError_t launch_batch_sweeps(const BatchArgs& a, int sweep_grid, int medium_grid, bool pair_box, hipStream_t s) {
  if (a.n_pairs <= 0) return hipSuccess;
  // the instances with counters run the same grids as those without (a
  // workgroup the device cannot hold yet waits its turn; no wave waits on
  // another)
  const dim3 b(kSweepWaves * kWave);
  if (pair_box && a.stats_on)
    hipLaunchKernelGGL((k_batch_sweep<true, true>), dim3(sweep_grid), b, 0, s, a);
  else if (pair_box)
    hipLaunchKernelGGL((k_batch_sweep<true, false>), dim3(sweep_grid), b, 0, s, a);
  else if (a.stats_on)
    hipLaunchKernelGGL((k_batch_sweep<false, true>), dim3(sweep_grid), b, 0, s, a);
  else
    hipLaunchKernelGGL((k_batch_sweep<false, false>), dim3(sweep_grid), b, 0, s, a);
  if (a.stats_on)
    hipLaunchKernelGGL(k_batch_medium<true>, dim3(medium_grid), b, 0, s, a);
  else
    hipLaunchKernelGGL(k_batch_medium<false>, dim3(medium_grid), b, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_batch_persistent(const BatchArgs& a, int grid, int waves_per_wg, hipStream_t s) {
  if (a.n_pairs <= 0) return hipSuccess;
  const size_t lds = (size_t)waves_per_wg * batch_lds_bytes_per_wave();
  if (a.stats_on)
    hipLaunchKernelGGL(k_batch_run<true>, dim3(grid), dim3(waves_per_wg * kWave), lds, s, a);
  else
    hipLaunchKernelGGL(k_batch_run<false>, dim3(grid), dim3(waves_per_wg * kWave), lds, s, a);
  if (a.stats_on)
    hipLaunchKernelGGL(k_batch_stats_empty, dim3((unsigned)((a.n_pairs + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace sccg

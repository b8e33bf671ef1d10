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
//   - Larger boxes are split into at most 8x8 cells whose side is 64*8^l, so
//     that every split lands on leaf tiles after l more levels.  One wave
//     classifies all cells of a box in one pass over the edges: each lane
//     takes one edge and sets the bits of the cells it hovers and of the
//     cells whose first pixel it crosses, in two 64-bit masks, which are then
//     OR- and XOR-reduced across the wave.  Cost O(edges) per split instead of
//     O(cells x edges).
//   - Leaf tiles use bit-sliced crossing tests: lane x holds column x of the
//     tile as a 64-bit row mask; each vertical edge of the tile's band at X
//     toggles, in every column left of X, the rows its span holds.  Only the
//     edges whose span meets the tile's rows and that lie right of its left
//     side are staged (band culling); a polygon known to contain a tile is
//     not tested again (its mask is all ones).
//   - One persistent grid.  Waves claim, in this order: queued boxes, large
//     pairs (largest bucket first, an LPT ordering), chunks of small pairs.
//     A split with many hovering cells publishes them to a device queue so
//     other waves share the work of large pairs; queue words are single
//     64-bit atomics, so no cache flushes are needed.  Every wave that
//     reserves queue slots fills them before anything else, so the only wait
//     (a consumer reading a slot just reserved) always ends; it is bounded
//     anyway and latches SCCG_E_DEVICE if the bound is hit.
#include <limits.h>

#include "sccg_device.h"

namespace sccg {

constexpr int kLeafCap = 128;   // staged band edges per flush (per wave)
constexpr int kLocalCap = 256;  // per-wave stack of boxes to process inline
constexpr uint32_t kSpinLimit = 1u << 22;

constexpr int kLdsPerWave = kLeafCap * 16 + kLocalCap * 8;
int batch_lds_bytes_per_wave() { return kLdsPerWave; }

// ---------------------------------------------------------------- task words
// [63] valid | [56:55] level | [54] p inside | [53] q inside | [52:44] ty |
// [43:35] tx | [30:0] pair index.  tx, ty: cell origin in 64-px units from
// the pair-box origin; level l: cell side 64 * 8^l (0 = leaf tile).
__device__ __forceinline__ uint64_t task_word(int64_t pair, int level, int tx, int ty, bool kp, bool kq) {
  return (1ull << 63) | ((uint64_t)level << 55) | ((uint64_t)kp << 54) | ((uint64_t)kq << 53) |
         ((uint64_t)ty << 44) | ((uint64_t)tx << 35) | (uint64_t)pair;
}
struct Task {
  int64_t pair;
  int level, tx, ty;
  bool kp, kq;
};
__device__ __forceinline__ Task task_decode(uint64_t w) {
  Task t;
  t.pair = (int64_t)(w & 0x7fffffffull);
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
  const uint64_t top = (hi >= 64) ? ~0ull : ((1ull << hi) - 1);
  return top & ~((1ull << lo) - 1);
}

// ----------------------------------------------------------------- context
struct Ctx {
  const BatchArgs* a;
  int lane;
  uint4* edges;       // per-wave staging, kLeafCap entries
  uint64_t* local;    // per-wave inline stack, kLocalCap entries
  int lsp;            // inline stack depth (wave-uniform)
  int home;           // preferred queue
  unsigned long long st_leaf_tests, st_leaf, st_split, st_queued, st_inline;
  unsigned long long st_edge_updates, st_class_edges, st_stage_edges;
};

struct PairInfo {
  int64_t op, np, oq, nq;  // ring offsets and vertex counts
  Meta box;                // pair box
};

__device__ __forceinline__ PairInfo pair_info(const BatchArgs& a, int64_t i) {
  PairInfo r;
  const int64_t ia = a.pa[i], ib = a.pb[i];
  const Meta mp = load_meta(a.metaA, ia), mq = load_meta(a.metaB, ib);
  r.box = pair_box(mp, mq);
  r.op = a.A.off[ia];
  r.np = a.A.off[ia + 1] - r.op;
  r.oq = a.B.off[ib];
  r.nq = a.B.off[ib + 1] - r.oq;
  return r;
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// XOR the staged edges into this lane's column mask: an edge at relative
// X = xr toggles, in every column x < xr, the rows it spans.
__device__ __forceinline__ void flush_edges(const uint4* e, int cnt, int lane, uint64_t& m) {
  wave_sync_lds();
  uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
  int k = 0;
  for (; k + 2 <= cnt; k += 2) {
    const uint4 a = e[k], b = e[k + 1];
    const uint32_t sa = (uint32_t)lane < a.x ? ~0u : 0u;
    const uint32_t sb = (uint32_t)lane < b.x ? ~0u : 0u;
    lo ^= a.y & sa;
    hi ^= a.z & sa;
    lo ^= b.y & sb;
    hi ^= b.z & sb;
  }
  if (k < cnt) {
    const uint4 a = e[k];
    const uint32_t sa = (uint32_t)lane < a.x ? ~0u : 0u;
    lo ^= a.y & sa;
    hi ^= a.z & sa;
  }
  m = ((uint64_t)hi << 32) | lo;
  wave_sync_lds();
}

// Column masks of polygon ring xy[o .. o+nv) over the leaf tile
// [tx0, tx0+64) x [ty0, ty0+th): bit r of lane x is the crossing parity of
// pixel (tx0 + x, ty0 + r).
__device__ uint64_t leaf_masks(Ctx& c, const int2* xy, int64_t o, int64_t nv, int tx0, int ty0, int th) {
  const int lane = c.lane;
  uint64_t m = 0;
  int cnt = 0;
  for (int64_t base = 0; base < nv; base += kWave) {
    const int64_t k = base + lane;
    bool keep = false;
    uint32_t xr = 0;
    uint64_t rr = 0;
    if (k < nv) {
      const int2 v = xy[o + k];
      const int2 w = xy[o + (k + 1 == nv ? 0 : k + 1)];
      if (v.x == w.x) {
        const int lo = max(min(v.y, w.y) - ty0, 0);
        const int hi = min(max(v.y, w.y) - ty0, th);
        const int dx = v.x - tx0;
        keep = (lo < hi) && (dx > 0);
        if (keep) {
          xr = (uint32_t)min(dx, kTile);
          rr = row_range(lo, hi);
        }
      }
    }
    const uint64_t b = ballot(keep);
    const int nk = __popcll(b);
    if (cnt + nk > kLeafCap) {
      flush_edges(c.edges, cnt, lane, m);
      cnt = 0;
    }
    if (keep) c.edges[cnt + lanes_below(b)] = make_uint4(xr, (uint32_t)rr, (uint32_t)(rr >> 32), 0u);
    cnt += nk;
    if (c.a->stats_on) c.st_edge_updates += nk;
  }
  if (cnt > 0) flush_edges(c.edges, cnt, lane, m);
  if (c.a->stats_on) c.st_stage_edges += (unsigned long long)nv;
  return m;
}

// Pixels of the tile [tx0, tx0+tw) x [ty0, ty0+th) inside both polygons.
__device__ uint32_t leaf_count(Ctx& c, const PairInfo& pi, int tx0, int ty0, int tw, int th, bool kp, bool kq) {
  const BatchArgs& a = *c.a;
  const uint64_t full = row_range(0, th);
  const uint64_t mp = kp ? full : leaf_masks(c, a.A.xy, pi.op, pi.np, tx0, ty0, th);
  const uint64_t mq = kq ? full : leaf_masks(c, a.B.xy, pi.oq, pi.nq, tx0, ty0, th);
  const uint32_t n = (c.lane < tw) ? (uint32_t)__popcll(mp & mq) : 0u;
  if (a.stats_on) {
    c.st_leaf += 1;
    c.st_leaf_tests += (unsigned long long)tw * th * ((kp ? 0 : 1) + (kq ? 0 : 1));
  }
  return wave_sum_u32(n);
}

// One pass over the ring: hover mask H and first-pixel parity mask P of the
// gx x gy cells of side 2^ls covering [bx0,bx1) x [by0,by1).
__device__ void classify(Ctx& c, const int2* xy, int64_t o, int64_t nv, int bx0, int by0, int bx1, int by1,
                         int ls, int gx, int gy, uint64_t& H, uint64_t& P) {
  const int S = 1 << ls;
  uint64_t h = 0, p = 0;
  for (int64_t base = 0; base < nv; base += kWave) {
    const int64_t k = base + c.lane;
    if (k >= nv) break;
    const int2 v = xy[o + k];
    const int2 w = xy[o + (k + 1 == nv ? 0 : k + 1)];
    if (v.x == w.x) {
      const int X = v.x, lo = min(v.y, w.y), hi = max(v.y, w.y);
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
      const int Y = v.y, lo = min(v.x, w.x), hi = max(v.x, w.x);
      const int dy = Y - by0;
      if (dy > 0 && Y < by1 && (dy & (S - 1)) != 0 && lo < bx1 && hi > bx0) {
        const int j = dy >> ls;
        const int i0 = lo > bx0 ? (lo - bx0) >> ls : 0;
        const int i1 = min(gx - 1, ((hi - bx0 + S - 1) >> ls) - 1);
        if (i0 <= i1) h |= rows_bits(j, j) & spread(cols_bits(i0, i1));
      }
    }
  }
  H = wave_or64(h);
  P = wave_xor64(p);
  if (c.a->stats_on) c.st_class_edges += (unsigned long long)nv;
}

__device__ __forceinline__ void add_counts(const BatchArgs& a, int64_t pair, uint64_t n) {
  if (n == 0) return;
  atomicAdd(reinterpret_cast<unsigned long long*>(a.inter + pair), (unsigned long long)n);
  atomicAdd(reinterpret_cast<unsigned long long*>(a.uni + pair), (unsigned long long)(0 - n));
}

// ------------------------------------------------------------------- queue
// Reserve up to k slots of queue q; returns the first slot and how many fit.
__device__ bool queue_claim(Ctx& c, uint64_t* out) {
  const BatchArgs& a = *c.a;
  uint64_t word = 0;
  int found = 0;
  if (c.lane == 0) {
    for (int r = 0; r < a.n_queues && !found; ++r) {
      const int q = (c.home + r) % a.n_queues;
      unsigned long long t =
          __hip_atomic_load(&a.st->q_tail[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (t > (unsigned long long)a.queue_cap) t = (unsigned long long)a.queue_cap;
      unsigned long long h =
          __hip_atomic_load(&a.st->q_head[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      while (h < t) {
        const unsigned long long prev = atomicCAS(&a.st->q_head[q], h, h + 1);
        if (prev == h) {
          unsigned long long* slot = a.queue + (size_t)q * a.queue_cap + h;
          uint32_t spins = 0;
          while ((word = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == 0) {
            if (++spins > kSpinLimit) break;
            __builtin_amdgcn_s_sleep(1);
          }
          if (word == 0) latch_error(a.err, kErrWatchdog);
          found = 1;
          break;
        }
        h = prev;
      }
    }
  }
  found = __shfl(found, 0, kWave);
  const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)word, 0, kWave);
  const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(word >> 32), 0, kWave);
  *out = ((uint64_t)hi << 32) | lo;
  return found && (*out != 0);
}

// Children of one split: lane j (< n) holds word j.  Publish them to the
// queue when there are enough, else (or for what does not fit) keep them on
// the wave's inline stack.
__device__ void emit_children(Ctx& c, uint64_t word, bool has, int n) {
  const BatchArgs& a = *c.a;
  const uint64_t b = ballot(has);
  const int rank = lanes_below(b);
  int queued = 0;
  if (!(a.flags & SCCG_F_NO_SPLIT_QUEUE) && n >= a.min_cells_to_queue) {
    unsigned long long t = 0;
    if (c.lane == 0) t = atomicAdd(&a.st->q_tail[c.home], (unsigned long long)n);
    t = (unsigned long long)uniform64((int64_t)__shfl((long long)t, 0, kWave));
    const long long room = (long long)a.queue_cap - (long long)t;
    queued = room <= 0 ? 0 : (room < n ? (int)room : n);
    if (has && rank < queued) {
      unsigned long long* slot = a.queue + (size_t)c.home * a.queue_cap + t + rank;
      __hip_atomic_store(slot, (unsigned long long)word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (a.stats_on) {
      c.st_queued += queued;
      c.st_inline += n - queued;
    }
  }
  const int rest = n - queued;
  if (rest > 0) {
    if (has && rank >= queued) c.local[c.lsp + rank - queued] = word;
    c.lsp += rest;
    wave_sync_lds();
  }
}

// Split box [bx0,bx1) x [by0,by1) of pair `pair` (already known to be a
// continuing box) into cells of level `cl` (side 64*8^cl) and handle them.
__device__ void split_box(Ctx& c, int64_t pair, const PairInfo& pi, int bx0, int by0, int bx1, int by1, int cl,
                          bool kp, bool kq) {
  const BatchArgs& a = *c.a;
  const int ls = 6 + 3 * cl;
  const int S = 1 << ls;
  const int gx = (bx1 - bx0 + S - 1) >> ls, gy = (by1 - by0 + S - 1) >> ls;
  const uint64_t valid = rows_bits(0, gy - 1) & spread(cols_bits(0, gx - 1));
  uint64_t Hp = 0, Pp = valid, Hq = 0, Pq = valid;
  if (!kp) classify(c, a.A.xy, pi.op, pi.np, bx0, by0, bx1, by1, ls, gx, gy, Hp, Pp);
  if (!kq) classify(c, a.B.xy, pi.oq, pi.nq, bx0, by0, bx1, by1, ls, gx, gy, Hq, Pq);
  const uint64_t in_p = ~Hp & Pp & valid, out_p = ~Hp & ~Pp & valid;
  const uint64_t in_q = ~Hq & Pq & valid, out_q = ~Hq & ~Pq & valid;
  const uint64_t both = in_p & in_q;
  const uint64_t cont = valid & ~out_p & ~out_q & ~both;
  // cells inside both polygons contribute their size at once
  uint64_t add = 0;
  if (both) {
    const int lw = (bx1 - bx0) - (gx - 1) * S, lh = (by1 - by0) - (gy - 1) * S;
    for (int j = 0; j < gy; ++j) {
      const uint32_t row = (uint32_t)(both >> (8 * j)) & 0xFFu;
      if (!row) continue;
      const uint64_t hgt = (j == gy - 1) ? (uint64_t)lh : (uint64_t)S;
      const uint32_t last = (row >> (gx - 1)) & 1u;
      add += hgt * ((uint64_t)(__popc(row) - last) * S + (uint64_t)last * lw);
    }
  }
  if (c.lane == 0) add_counts(a, pair, add);
  if (a.stats_on) c.st_split += 1;
  // one lane per continuing cell
  const int n = __popcll(cont);
  bool has = false;
  uint64_t word = 0;
  if (c.lane < 64 && ((cont >> c.lane) & 1ull)) {
    const int i = c.lane & 7, j = c.lane >> 3;
    const Meta& B = pi.box;
    const int tx = ((bx0 - B.x0) >> 6) + (i << (3 * cl));
    const int ty = ((by0 - B.y0) >> 6) + (j << (3 * cl));
    has = true;
    word = task_word(pair, cl, tx, ty, (in_p >> c.lane) & 1ull, (in_q >> c.lane) & 1ull);
  }
  if (n) emit_children(c, word, has, n);
}

__device__ void run_task(Ctx& c, uint64_t w) {
  const BatchArgs& a = *c.a;
  const Task t = task_decode(w);
  if (t.pair >= a.n_pairs) {
    latch_error(a.err, kErrWatchdog);
    return;
  }
  const PairInfo pi = pair_info(a, t.pair);
  const int side = kTile << (3 * t.level);
  const int x0 = pi.box.x0 + t.tx * kTile, y0 = pi.box.y0 + t.ty * kTile;
  const int x1 = min(x0 + side, pi.box.x1), y1 = min(y0 + side, pi.box.y1);
  const bool kp = t.kp && !(a.flags & SCCG_F_NO_KNOWN_INSIDE);
  const bool kq = t.kq && !(a.flags & SCCG_F_NO_KNOWN_INSIDE);
  if (t.level == 0) {
    const uint32_t n = leaf_count(c, pi, x0, y0, x1 - x0, y1 - y0, kp, kq);
    if (c.lane == 0) add_counts(a, t.pair, n);
  } else {
    split_box(c, t.pair, pi, x0, y0, x1, y1, t.level - 1, kp, kq);
  }
}

__device__ void drain_local(Ctx& c) {
  while (c.lsp > 0) {
    c.lsp -= 1;
    wave_sync_lds();
    const uint64_t w = c.local[c.lsp];
    wave_sync_lds();
    run_task(c, uniform64((int64_t)w));
  }
}

__device__ void run_large(Ctx& c, int64_t pair) {
  const BatchArgs& a = *c.a;
  const PairInfo pi = pair_info(a, pair);
  const int w = pi.box.x1 - pi.box.x0, h = pi.box.y1 - pi.box.y0;
  const int side = max(w, h);
  int cl = 0;
  while ((kTile << (3 * cl)) * kMaxGrid < side) ++cl;
  split_box(c, pair, pi, pi.box.x0, pi.box.y0, pi.box.x1, pi.box.y1, cl, false, false);
  drain_local(c);
}

__device__ void run_small(Ctx& c, int64_t pair) {
  const BatchArgs& a = *c.a;
  const PairInfo pi = pair_info(a, pair);
  const int w = pi.box.x1 - pi.box.x0, h = pi.box.y1 - pi.box.y0;
  const uint32_t n = leaf_count(c, pi, pi.box.x0, pi.box.y0, w, h, false, false);
  if (c.lane == 0) {
    const int64_t ap = a.areaA[a.pa[pair]], aq = a.areaB[a.pb[pair]];
    a.inter[pair] = (int64_t)n;
    a.uni[pair] = ap + aq - (int64_t)n;
  }
}

__global__ void __launch_bounds__(512) k_batch_run(BatchArgs args) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wave = threadIdx.x / kWave;
  Ctx c;
  c.a = &args;
  c.lane = lane_id();
  c.edges = reinterpret_cast<uint4*>(smem + (size_t)wave * kLdsPerWave);
  c.local = reinterpret_cast<uint64_t*>(smem + (size_t)wave * kLdsPerWave + kLeafCap * 16);
  c.lsp = 0;
  c.home = (int)(blockIdx.x % (unsigned)args.n_queues);
  c.st_leaf_tests = c.st_leaf = c.st_split = c.st_queued = c.st_inline = 0;
  c.st_edge_updates = c.st_class_edges = c.st_stage_edges = 0;
  const BatchArgs& a = args;
  const unsigned long long n_heavy = a.st->l_count[0];
  const unsigned long long n_large = n_heavy + a.st->l_count[1];
  for (;;) {
    uint64_t w;
    if (queue_claim(c, &w)) {
      run_task(c, uniform64((int64_t)w));
      drain_local(c);
      continue;
    }
    unsigned long long k = 0;
    if (c.lane == 0) k = atomicAdd(&a.st->l_next, 1ull);
    k = (unsigned long long)uniform64((int64_t)__shfl((long long)k, 0, kWave));
    if (k < n_large) {
      const int64_t idx = (k < n_heavy) ? (int64_t)k : (int64_t)(a.n_pairs - 1 - (int64_t)(k - n_heavy));
      run_large(c, (int64_t)a.l_list[idx]);
      continue;
    }
    unsigned long long s0 = 0;
    if (c.lane == 0) s0 = atomicAdd(&a.st->s_next, (unsigned long long)a.chunk);
    s0 = (unsigned long long)uniform64((int64_t)__shfl((long long)s0, 0, kWave));
    if (s0 < (unsigned long long)a.n_pairs) {
      const int64_t e = min((int64_t)s0 + a.chunk, a.n_pairs);
      for (int64_t i = (int64_t)s0; i < e; ++i)
        if (a.cls[i] == kClsSmall) run_small(c, i);
      continue;
    }
    break;
  }
  if (a.stats_on && c.lane == 0) {
    atomicAdd(&a.st->stats[0], c.st_leaf_tests);
    atomicAdd(&a.st->stats[1], c.st_leaf);
    atomicAdd(&a.st->stats[2], c.st_split);
    atomicAdd(&a.st->stats[3], c.st_queued);
    atomicAdd(&a.st->stats[4], c.st_inline);
    atomicAdd(&a.st->stats[8], c.st_edge_updates);
    atomicAdd(&a.st->stats[9], c.st_class_edges);
    atomicAdd(&a.st->stats[10], c.st_stage_edges);
  }
}

// ------------------------------------------------------------ setup / reset
// Clear the queue slots the previous call wrote, then the counters.
__global__ void __launch_bounds__(256) k_batch_clear_slots(BatchArgs a) {
  for (int q = 0; q < a.n_queues; ++q) {
    unsigned long long used = a.st->q_tail[q];
    if (used > (unsigned long long)a.queue_cap) used = (unsigned long long)a.queue_cap;
    unsigned long long* base = a.queue + (size_t)q * a.queue_cap;
    for (unsigned long long j = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; j < used;
         j += (unsigned long long)gridDim.x * blockDim.x)
      base[j] = 0;
  }
}

__global__ void k_batch_clear_counters(BatchArgs a) {
  const int t = threadIdx.x;
  unsigned long long* p = reinterpret_cast<unsigned long long*>(a.st);
  const int n = (int)(sizeof(BatchState) / sizeof(unsigned long long));
  for (int k = t; k < n; k += blockDim.x) p[k] = 0;
}

__global__ void __launch_bounds__(256) k_batch_setup(BatchArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool large = false, heavy = false;
  if (i < a.n_pairs) {
    const int64_t ia = a.pa[i], ib = a.pb[i];
    uint8_t cls = kClsDone;
    if (ia < 0 || ia >= a.A.n || ib < 0 || ib >= a.B.n) {
      latch_error(a.err, kErrIndex);
      a.inter[i] = 0;
      a.uni[i] = 0;
    } else {
      const Meta bx = pair_box(load_meta(a.metaA, ia), load_meta(a.metaB, ib));
      const int64_t ap = a.areaA[ia], aq = a.areaB[ib];
      if (bx.x0 >= bx.x1 || bx.y0 >= bx.y1) {
        a.inter[i] = 0;
        a.uni[i] = ap + aq;
      } else {
        const int w = bx.x1 - bx.x0, h = bx.y1 - bx.y0;
        if (w > kMaxSide || h > kMaxSide) {
          latch_error(a.err, kErrSide);
          a.inter[i] = 0;
          a.uni[i] = 0;
        } else if (w <= kTile && h <= kTile) {
          cls = kClsSmall;
        } else {
          cls = kClsLarge;
          large = true;
          heavy = !(a.flags & SCCG_F_NO_LPT) && (int64_t)w * h >= (int64_t)a.heavy_area;
          a.inter[i] = 0;
          a.uni[i] = ap + aq;
        }
      }
    }
    a.cls[i] = cls;
  }
  // heavy pairs fill the list from the front, the other large pairs from the back
  const uint64_t bh = ballot(large && heavy), bl = ballot(large && !heavy);
  unsigned long long baseh = 0, basel = 0;
  if (lane_id() == 0) {
    if (bh) baseh = atomicAdd(&a.st->l_count[0], (unsigned long long)__popcll(bh));
    if (bl) basel = atomicAdd(&a.st->l_count[1], (unsigned long long)__popcll(bl));
  }
  baseh = (unsigned long long)__shfl((long long)baseh, 0, kWave);
  basel = (unsigned long long)__shfl((long long)basel, 0, kWave);
  if (large && heavy) a.l_list[baseh + lanes_below(bh)] = (int32_t)i;
  if (large && !heavy) a.l_list[a.n_pairs - 1 - (int64_t)(basel + lanes_below(bl))] = (int32_t)i;
}

__global__ void k_batch_stats_classes(BatchArgs a) {
  // small / large / done-with-empty-box counts (stats only)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_pairs) return;
  const uint8_t c = a.cls[i];
  if (c == kClsSmall) atomicAdd(&a.st->stats[5], 1ull);
  else if (c == kClsLarge) atomicAdd(&a.st->stats[6], 1ull);
  else atomicAdd(&a.st->stats[7], 1ull);
}

hipError_t launch_batch_reset(const BatchArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_clear_slots, dim3(1024), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_batch_clear_counters, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_batch_setup(const BatchArgs& a, hipStream_t s) {
  if (a.n_pairs <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((a.n_pairs + 255) / 256);
  hipLaunchKernelGGL(k_batch_setup, dim3(blocks), dim3(256), 0, s, a);
  if (a.stats_on) hipLaunchKernelGGL(k_batch_stats_classes, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

int batch_occupancy(int waves_per_wg) {
  int n = 0;
  const size_t lds = (size_t)waves_per_wg * batch_lds_bytes_per_wave();
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_run, waves_per_wg * kWave, lds) != hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

hipError_t launch_batch_run(const BatchArgs& a, int grid, int waves_per_wg, hipStream_t s) {
  if (a.n_pairs <= 0) return hipSuccess;
  const size_t lds = (size_t)waves_per_wg * batch_lds_bytes_per_wave();
  hipLaunchKernelGGL(k_batch_run, dim3(grid), dim3(waves_per_wg * kWave), lds, s, a);
  return hipGetLastError();
}

}  // namespace sccg

// PixelBox on the host CPU (the PixelBox-CPU of Section 4.2), for the
// serving path's migration of small jobs when the device is congested.
//
// Per pair: extents and areas of both rings (Section 3.2), the pair box
// MBR(p) ∩ MBR(q), then sampling boxes (Section 3.3): a box is classified
// against each polygon by Lemma 1 (it hovers when an edge meets its open
// interior; otherwise the centre of its first pixel decides), boxes inside
// both add their size, boxes outside either are dropped, the rest are split
// in four until they are at most 64 pixels wide and below the pixelization
// threshold.  Such a box is not classified: each of its rows is tested at
// once, a 64-bit mask per row whose bit c is the crossing parity of pixel
// column x0 + c (Section 3.1).  The
// union is |p| + |q| - I.  The counts equal the device's exactly.
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

#include "host_pixelbox.h"

namespace {

struct Ring {
  const int32_t* xy;
  int64_t n;
  int32_t x0, y0, x1, y1;  // pixel extent [x0, x1) x [y0, y1); empty if x0 >= x1
  int64_t area;
};

constexpr int64_t kMaxCoord = int64_t(1) << 30;

Ring make_ring(const sccg_polys* P, int64_t k, bool* rejected) {
  Ring r;
  r.xy = P->xy + 2 * P->offsets[k];
  r.n = P->offsets[k + 1] - P->offsets[k];
  r.x0 = r.y0 = INT32_MAX;
  r.x1 = r.y1 = INT32_MIN;
  uint64_t twice = 0;  // wrapping sum: twice the area can reach 2^63 in size
  for (int64_t i = 0; i < r.n; ++i) {
    const int64_t j = i + 1 == r.n ? 0 : i + 1;
    const int32_t x = r.xy[2 * i], y = r.xy[2 * i + 1];
    r.x0 = std::min(r.x0, x);
    r.y0 = std::min(r.y0, y);
    r.x1 = std::max(r.x1, x);
    r.y1 = std::max(r.y1, y);
    twice += (uint64_t)((int64_t)x * r.xy[2 * j + 1] - (int64_t)r.xy[2 * j] * y);
  }
  const bool bad = r.n > 0 && (r.x0 < -kMaxCoord || r.y0 < -kMaxCoord || r.x1 > kMaxCoord || r.y1 > kMaxCoord);
  *rejected = bad;
  if (r.n == 0 || bad) {
    r.n = 0;  // an empty or rejected ring covers nothing
    r.x0 = r.y0 = INT32_MAX;
    r.x1 = r.y1 = INT32_MIN;
    r.area = 0;
  } else {
    r.area = (int64_t)(((int64_t)twice < 0 ? 0 - twice : twice) / 2);
  }
  return r;
}

enum Pos { kOut = 0, kIn = 1, kHover = 2 };

// Lemma 1 for box [x0, x1) x [y0, y1).
Pos position(const Ring& r, int32_t x0, int32_t y0, int32_t x1, int32_t y1) {
  int parity = 0;
  for (int64_t i = 0; i < r.n; ++i) {
    const int64_t j = i + 1 == r.n ? 0 : i + 1;
    const int32_t ax = r.xy[2 * i], ay = r.xy[2 * i + 1], bx = r.xy[2 * j], by = r.xy[2 * j + 1];
    if (ax == bx) {
      const int32_t lo = std::min(ay, by), hi = std::max(ay, by);
      if (x0 < ax && ax < x1 && lo < y1 && hi > y0) return kHover;
      if (ax > x0 && lo <= y0 && y0 < hi) parity ^= 1;
    } else {
      const int32_t lo = std::min(ax, bx), hi = std::max(ax, bx);
      if (y0 < ay && ay < y1 && lo < x1 && hi > x0) return kHover;
    }
  }
  return parity ? kIn : kOut;
}

// Row masks of a box at most 64 wide: bit c of rows[y - y0] is the parity of
// pixel (x0 + c, y).  Each vertical edge toggles the same mask on a run of
// rows, so its mask is XORed at the run's first row and just past its last,
// and a prefix XOR down the rows then gives every row's mask.
void row_masks(const Ring& r, int32_t x0, int32_t y0, int32_t w, int32_t h, uint64_t* rows) {
  std::fill(rows, rows + h + 1, 0ull);
  for (int64_t i = 0; i < r.n; ++i) {
    const int64_t j = i + 1 == r.n ? 0 : i + 1;
    const int32_t ax = r.xy[2 * i], ay = r.xy[2 * i + 1], bx = r.xy[2 * j], by = r.xy[2 * j + 1];
    if (ax != bx || ax <= x0) continue;
    const int32_t lo = std::max(std::min(ay, by), y0), hi = std::min(std::max(ay, by), y0 + h);
    if (lo >= hi) continue;
    // ax > x0; ax - x0 itself can reach 2^31
    const int32_t c = ax >= x0 + w ? w : ax - x0;
    const uint64_t m = c >= 64 ? ~0ull : ((1ull << c) - 1);
    rows[lo - y0] ^= m;
    rows[hi - y0] ^= m;
  }
  for (int32_t y = 1; y < h; ++y) rows[y] ^= rows[y - 1];
}

struct Box {
  int32_t x0, y0, x1, y1;
  bool kp, kq;  // known to lie inside p / q
};

int64_t pair_intersection(const Ring& p, const Ring& q, std::vector<Box>& stack) {
  const int32_t bx0 = std::max(p.x0, q.x0), by0 = std::max(p.y0, q.y0);
  const int32_t bx1 = std::min(p.x1, q.x1), by1 = std::min(p.y1, q.y1);
  if (bx0 >= bx1 || by0 >= by1) return 0;
  int64_t acc = 0;
  uint64_t rp[65], rq[65];
  stack.clear();
  stack.push_back(Box{bx0, by0, bx1, by1, false, false});
  while (!stack.empty()) {
    const Box b = stack.back();
    stack.pop_back();
    const int32_t w = b.x1 - b.x0, h = b.y1 - b.y0;
    const bool leaf = w <= 64 && h <= 64 && (int64_t)w * h < 4096;
    // a box that is pixelized anyway is not classified first: its row masks
    // give the same count
    const Pos sp = b.kp ? kIn : (leaf ? kHover : position(p, b.x0, b.y0, b.x1, b.y1));
    if (sp == kOut) continue;
    const Pos sq = b.kq ? kIn : (leaf ? kHover : position(q, b.x0, b.y0, b.x1, b.y1));
    if (sq == kOut) continue;
    if (sp == kIn && sq == kIn) {
      acc += (int64_t)w * h;
      continue;
    }
    if (leaf) {
      if (sp == kIn)
        std::fill(rp, rp + h, w >= 64 ? ~0ull : ((1ull << w) - 1));
      else
        row_masks(p, b.x0, b.y0, w, h, rp);
      if (sq == kIn)
        std::fill(rq, rq + h, w >= 64 ? ~0ull : ((1ull << w) - 1));
      else
        row_masks(q, b.x0, b.y0, w, h, rq);
      for (int32_t y = 0; y < h; ++y) acc += __builtin_popcountll(rp[y] & rq[y]);
      continue;
    }
    // split in four (halves of each side; a side of one pixel is not split)
    const int32_t mx = w > 1 ? b.x0 + w / 2 : b.x1, my = h > 1 ? b.y0 + h / 2 : b.y1;
    const bool kp = sp == kIn, kq = sq == kIn;
    stack.push_back(Box{b.x0, b.y0, mx, my, kp, kq});
    if (mx < b.x1) stack.push_back(Box{mx, b.y0, b.x1, my, kp, kq});
    if (my < b.y1) stack.push_back(Box{b.x0, my, mx, b.y1, kp, kq});
    if (mx < b.x1 && my < b.y1) stack.push_back(Box{mx, my, b.x1, b.y1, kp, kq});
  }
  return acc;
}

}  // namespace

namespace sccg {

// One participant's share of a HostWork: chunks of 64 pairs taken from the
// shared counter until none is left.  Returns the kHostErr* bits it saw.
uint32_t host_area_worker(HostWork& w) {
  std::vector<Box> stack;
  stack.reserve(256);
  uint32_t e = 0;
  for (;;) {
    const int64_t k0 = w.next.fetch_add(64);
    if (k0 >= w.n) break;
    const int64_t k1 = std::min(k0 + 64, w.n);
    for (int64_t k = k0; k < k1; ++k) {
      bool bad_p = false, bad_q = false;
      const Ring p = make_ring(w.A, w.pa[k], &bad_p), q = make_ring(w.B, w.pb[k], &bad_q);
      if (bad_p || bad_q) e |= kHostErrCoord;
      const int64_t bw = (int64_t)std::min(p.x1, q.x1) - std::max(p.x0, q.x0);
      const int64_t bh = (int64_t)std::min(p.y1, q.y1) - std::max(p.y0, q.y0);
      if (bw > 32767 || bh > 32767) {  // rejected like the device rejects it
        e |= kHostErrSide;
        w.out_i[k] = 0;
        w.out_u[k] = 0;
        continue;
      }
      const int64_t I = pair_intersection(p, q, stack);
      w.out_i[k] = I;
      w.out_u[k] = p.area + q.area - I;
    }
  }
  return e;
}

// Pairs [0, n) on `threads` host threads started for this call.
uint32_t host_area_pairs(const sccg_polys* A, const sccg_polys* B, int64_t n, const int32_t* pa, const int32_t* pb,
                         int64_t* out_i, int64_t* out_u, int threads) {
  HostWork w{A, B, pa, pb, out_i, out_u, n};
  threads = std::max(1, threads);
  if (threads == 1 || n < 256) return host_area_worker(w);
  std::atomic<uint32_t> err{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t) pool.emplace_back([&] { err.fetch_or(host_area_worker(w)); });
  for (auto& t : pool) t.join();
  return err.load();
}

}  // namespace sccg

extern "C" int sccg_host_area_pairs(const sccg_polys* A, const sccg_polys* B, int64_t n_pairs, const int32_t* pair_a,
                                    const int32_t* pair_b, int64_t* out_inter, int64_t* out_union, int n_threads) {
  if (!A || !B || n_pairs < 0 || !A->offsets || !B->offsets) return SCCG_E_ARG;
  if (n_pairs == 0) return SCCG_OK;
  if (!pair_a || !pair_b || !out_inter || !out_union) return SCCG_E_ARG;
  for (int64_t k = 0; k < n_pairs; ++k)
    if (pair_a[k] < 0 || pair_a[k] >= A->n_polys || pair_b[k] < 0 || pair_b[k] >= B->n_polys) return SCCG_E_RANGE;
  const uint32_t e = sccg::host_area_pairs(A, B, n_pairs, pair_a, pair_b, out_inter, out_union, n_threads);
  return e ? SCCG_E_RANGE : SCCG_OK;
}

// Seeded synthetic polygon workloads for the PixelBox pair-area path.
//
// This module only manufactures inputs: raster masks built from unions of
// integer ellipses, their outer boundaries traced into rectilinear integer
// rings, placement of the rings on tiles, and the pair/set index arrays.
// It holds none of the method's arithmetic (no crossing tests, no areas, no
// box classification) and is shared by the oracle tests and the device path
// only as a source of inputs.
//
// The polygons mimic the segmented nuclei of Section 2.1 and Figure 3 of the
// paper: integer vertices, axis-aligned edges, because they follow pixel
// boundaries of a raster image.  Each pair is drawn from its own
// counter-based stream (splitmix64 of seed and pair index), so a pair's shapes
// do not depend on the thread count or on any other pair.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

// ---------------------------------------------------------------- RNG ----
// splitmix64 (Steele, Lea, Flood 2014; the published finaliser constants).
struct Rng {
  uint64_t s;
  explicit Rng(uint64_t seed, uint64_t stream) {
    s = seed ^ (0x9E3779B97F4A7C15ull * (stream + 1));
    next();
  }
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  // uniform integer in [lo, hi]
  int64_t uni(int64_t lo, int64_t hi) {
    if (hi <= lo) return lo;
    return lo + (int64_t)(next() % (uint64_t)(hi - lo + 1));
  }
  double unit() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
  double normal() {  // Box-Muller
    double u1 = unit(), u2 = unit();
    if (u1 < 1e-300) u1 = 1e-300;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

// --------------------------------------------------------------- Mask ----
struct Mask {
  int w = 0, h = 0;
  std::vector<uint8_t> m;  // row-major, y up: m[y*w + x]
  void init(int W, int H) { w = W; h = H; m.assign((size_t)W * H, 0); }
  uint8_t at(int x, int y) const {
    if (x < 0 || y < 0 || x >= w || y >= h) return 0;
    return m[(size_t)y * w + x];
  }
};

// Pixel (x,y) lies in the ellipse with integer centre (cx,cy) and integer
// semi-axes (a,b) iff its centre (x+1/2, y+1/2) does:
//   (2x+1-2cx)^2 b^2 + (2y+1-2cy)^2 a^2 <= 4 a^2 b^2   (all int64).
void raster_ellipse(Mask& M, int64_t cx, int64_t cy, int64_t a, int64_t b) {
  int64_t x0 = std::max<int64_t>(0, cx - a), x1 = std::min<int64_t>(M.w, cx + a);
  int64_t y0 = std::max<int64_t>(0, cy - b), y1 = std::min<int64_t>(M.h, cy + b);
  const int64_t a2 = a * a, b2 = b * b, r = 4 * a2 * b2;
  for (int64_t y = y0; y < y1; ++y) {
    int64_t dy = 2 * y + 1 - 2 * cy;
    int64_t ty = dy * dy * a2;
    uint8_t* row = &M.m[(size_t)y * M.w];
    for (int64_t x = x0; x < x1; ++x) {
      int64_t dx = 2 * x + 1 - 2 * cx;
      if (dx * dx * b2 + ty <= r) row[x] = 1;
    }
  }
}

// Keep only the largest 4-connected foreground component (ties: the one found
// first in row-major scan order).  Returns its pixel count.
int64_t keep_largest_component(Mask& M) {
  const int W = M.w, H = M.h;
  std::vector<int32_t> lab((size_t)W * H, -1);
  std::vector<int32_t> stack;
  int32_t best = -1, nlab = 0;
  int64_t best_n = 0;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      size_t i = (size_t)y * W + x;
      if (!M.m[i] || lab[i] >= 0) continue;
      int32_t L = nlab++;
      int64_t cnt = 0;
      lab[i] = L;
      stack.clear();
      stack.push_back((int32_t)i);
      while (!stack.empty()) {
        int32_t j = stack.back();
        stack.pop_back();
        ++cnt;
        int jx = j % W, jy = j / W;
        const int nx[4] = {jx - 1, jx + 1, jx, jx};
        const int ny[4] = {jy, jy, jy - 1, jy + 1};
        for (int k = 0; k < 4; ++k) {
          if (nx[k] < 0 || ny[k] < 0 || nx[k] >= W || ny[k] >= H) continue;
          size_t q = (size_t)ny[k] * W + nx[k];
          if (M.m[q] && lab[q] < 0) {
            lab[q] = L;
            stack.push_back((int32_t)q);
          }
        }
      }
      if (cnt > best_n) { best_n = cnt; best = L; }
    }
  for (size_t i = 0; i < lab.size(); ++i) M.m[i] = (lab[i] == best && best >= 0) ? 1 : 0;
  return best_n;
}

// Fill holes: background pixels not 4-connected to the outside of the canvas
// become foreground.
void fill_holes(Mask& M) {
  const int W = M.w, H = M.h;
  std::vector<uint8_t> outside((size_t)W * H, 0);
  std::vector<int32_t> stack;
  auto seed = [&](int x, int y) {
    size_t i = (size_t)y * W + x;
    if (!M.m[i] && !outside[i]) { outside[i] = 1; stack.push_back((int32_t)i); }
  };
  for (int x = 0; x < W; ++x) { seed(x, 0); seed(x, H - 1); }
  for (int y = 0; y < H; ++y) { seed(0, y); seed(W - 1, y); }
  while (!stack.empty()) {
    int32_t j = stack.back();
    stack.pop_back();
    int jx = j % W, jy = j / W;
    if (jx > 0) seed(jx - 1, jy);
    if (jx + 1 < W) seed(jx + 1, jy);
    if (jy > 0) seed(jx, jy - 1);
    if (jy + 1 < H) seed(jx, jy + 1);
  }
  for (size_t i = 0; i < M.m.size(); ++i)
    if (!M.m[i] && !outside[i]) M.m[i] = 1;
}

// Crop to the foreground bounding box.  Returns false when empty.
bool crop(Mask& M, int& ox, int& oy) {
  int x0 = M.w, y0 = M.h, x1 = -1, y1 = -1;
  for (int y = 0; y < M.h; ++y)
    for (int x = 0; x < M.w; ++x)
      if (M.m[(size_t)y * M.w + x]) {
        x0 = std::min(x0, x); x1 = std::max(x1, x);
        y0 = std::min(y0, y); y1 = std::max(y1, y);
      }
  if (x1 < 0) return false;
  Mask C;
  C.init(x1 - x0 + 1, y1 - y0 + 1);
  for (int y = y0; y <= y1; ++y)
    std::memcpy(&C.m[(size_t)(y - y0) * C.w], &M.m[(size_t)y * M.w + x0], C.w);
  ox = x0; oy = y0;
  M = std::move(C);
  return true;
}

// Trace the outer boundary of a single hole-free 4-connected component along
// pixel sides, interior on the left (counter-clockwise, y up).  Vertices are
// emitted only where the direction changes, so collinear points are merged.
// Returns false if the boundary is not one simple loop.
bool trace(const Mask& M, std::vector<int32_t>& ring) {
  const int W = M.w, H = M.h, PW = W + 1;
  // out[p] = direction of the boundary edge leaving lattice point p
  //   0:+x 1:+y 2:-x 3:-y, -1 none; 4 = more than one (not simple)
  std::vector<int8_t> out((size_t)(W + 1) * (H + 1), -1);
  int64_t n_edges = 0;
  auto put = [&](int px, int py, int d) {
    int8_t& o = out[(size_t)py * PW + px];
    o = (o == -1) ? (int8_t)d : (int8_t)4;
    ++n_edges;
  };
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      if (!M.at(x, y)) continue;
      if (!M.at(x, y - 1)) put(x, y, 0);
      if (!M.at(x + 1, y)) put(x + 1, y, 1);
      if (!M.at(x, y + 1)) put(x + 1, y + 1, 2);
      if (!M.at(x - 1, y)) put(x, y + 1, 3);
    }
  if (n_edges == 0) return false;
  int sx = -1, sy = -1;
  for (int y = 0; y <= H && sx < 0; ++y)
    for (int x = 0; x <= W; ++x)
      if (out[(size_t)y * PW + x] >= 0) { sx = x; sy = y; break; }
  const int DX[4] = {1, 0, -1, 0}, DY[4] = {0, 1, 0, -1};
  ring.clear();
  int px = sx, py = sy, prev = -1;
  int64_t walked = 0;
  do {
    int d = out[(size_t)py * PW + px];
    if (d < 0 || d > 3) return false;
    if (d != prev) { ring.push_back(px); ring.push_back(py); }
    prev = d;
    px += DX[d]; py += DY[d];
    if (++walked > n_edges) return false;
  } while (px != sx || py != sy);
  if (walked != n_edges) return false;
  // the start point is a corner (entered moving -y, left moving +x) unless the
  // first and last runs are collinear, which cannot happen at the lowest-left
  // boundary point; keep the check anyway.
  if (out[(size_t)sy * PW + sx] == prev && ring.size() >= 4) ring.erase(ring.begin(), ring.begin() + 2);
  return ring.size() >= 8;
}

// 4-neighbour (cross) dilation or erosion by one pixel on a canvas padded by 1.
Mask morph(const Mask& A, bool dilate) {
  Mask R;
  R.init(A.w + 2, A.h + 2);
  for (int y = 0; y < R.h; ++y)
    for (int x = 0; x < R.w; ++x) {
      int ax = x - 1, ay = y - 1;
      uint8_t c = A.at(ax, ay), l = A.at(ax - 1, ay), r = A.at(ax + 1, ay), d = A.at(ax, ay - 1),
              u = A.at(ax, ay + 1);
      R.m[(size_t)y * R.w + x] = dilate ? (c | l | r | d | u) : (c & l & r & d & u);
    }
  return R;
}

// ------------------------------------------------------------- Shapes ----
struct Shape {
  Mask mask;               // cropped to its bounding box
  std::vector<int32_t> ring;  // local coordinates, relative to the mask origin
};

struct ShapeSpec {
  int canvas;          // square canvas side
  int kmin, kmax;      // number of ellipses
  int amin, amax;      // semi-axis range
  int vmin, vmax;      // accepted vertex-count range (0 = unchecked)
};

// Union of k random ellipses -> largest 4-component -> holes filled -> traced.
// Redrawn (same stream) until the vertex count is in range or attempts run out.
bool make_shape(Rng& g, const ShapeSpec& sp, Shape& out, int* attempts_used) {
  const int max_attempts = 64;
  for (int att = 1; att <= max_attempts; ++att) {
    Mask M;
    M.init(sp.canvas, sp.canvas);
    int k = (int)g.uni(sp.kmin, sp.kmax);
    for (int e = 0; e < k; ++e) {
      int a = (int)g.uni(sp.amin, sp.amax), b = (int)g.uni(sp.amin, sp.amax);
      a = std::max(1, std::min(a, sp.canvas / 2));
      b = std::max(1, std::min(b, sp.canvas / 2));
      int cx = (int)g.uni(a, sp.canvas - a), cy = (int)g.uni(b, sp.canvas - b);
      raster_ellipse(M, cx, cy, a, b);
    }
    if (keep_largest_component(M) == 0) continue;
    fill_holes(M);
    int ox, oy;
    if (!crop(M, ox, oy)) continue;
    std::vector<int32_t> ring;
    if (!trace(M, ring)) continue;
    int nv = (int)(ring.size() / 2);
    bool ok = (sp.vmin == 0 || nv >= sp.vmin) && (sp.vmax == 0 || nv <= sp.vmax);
    if (ok || att == max_attempts) {
      out.mask = std::move(M);
      out.ring = std::move(ring);
      if (attempts_used) *attempts_used = att;
      return ok;
    }
  }
  return false;
}

// B = A shifted by (dx,dy), then dilated or eroded by one pixel and retraced.
// Returns the offset of B's mask origin relative to A's mask origin.
bool derive_b(Rng& g, const Shape& A, Shape& B, int& bx, int& by) {
  int dx = (int)g.uni(-3, 3), dy = (int)g.uni(-3, 3);
  bool dilate = (g.next() & 1) != 0;
  for (int tries = 0; tries < 2; ++tries) {
    Mask M = morph(A.mask, dilate);
    if (keep_largest_component(M) > 0) {
      fill_holes(M);
      int ox, oy;
      if (crop(M, ox, oy) && trace(M, B.ring)) {
        B.mask = std::move(M);
        bx = dx + ox - 1;  // morph padded by 1
        by = dy + oy - 1;
        return true;
      }
    }
    dilate = true;  // erosion emptied the shape: dilate instead
  }
  return false;
}

// ------------------------------------------------------------ Dataset ----
struct Dataset {
  int config = 0;
  uint64_t seed = 0;
  std::vector<int32_t> wa, ha;  // A mask extents (placement)
  int64_t n_pairs = 0;
  std::vector<Shape> A, B;
  std::vector<int64_t> ax, ay, bx, by;  // global mask origins
  std::vector<uint8_t> blob;
  int64_t tiles_used = 0;
  int64_t rejected = 0;  // shapes accepted only after exhausting attempts
  int64_t attempts = 0;
  // set-level workloads
  int64_t n_sets = 0;
  std::vector<int32_t> pa, pb;
  std::vector<int64_t> set_off;
};

ShapeSpec spec_for(int config, Rng& g, bool& is_blob) {
  is_blob = false;
  ShapeSpec sp{};
  switch (config) {
    case 1: sp = {32, 1, 4, 4, 14, 8, 40}; break;
    case 2: case 4: case 5: sp = {64, 1, 4, 5, 30, 16, 120}; break;
    case 3: {
      if (g.unit() < 0.01) {
        is_blob = true;
        int s = (int)g.uni(150, 400);
        sp = {s, 10, 40, std::max(4, s / 10), std::max(5, s / 4), 8, 2000};
      } else {
        double side = 24.0 * std::exp(0.7 * g.normal());
        int s = (int)std::lround(std::min(400.0, std::max(8.0, side)));
        sp = {s, 1, 4, std::max(2, s / 4), std::max(2, s / 2), 0, 2000};
      }
      break;
    }
    default: sp = {32, 1, 4, 4, 14, 8, 40};
  }
  return sp;
}

// Shelf placement of MBRs (each padded for B's shift and dilation) on square
// tiles; tiles are laid out 16 to a row of tiles.
void place(Dataset& D, int64_t tile, int64_t pad) {
  int64_t t = 0, cx = 0, cy = 0, shelf_h = 0;
  const int64_t n = D.n_pairs;
  D.ax.resize(n); D.ay.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    int64_t w = D.wa[i] + 2 * pad, h = D.ha[i] + 2 * pad;
    if (cx + w > tile) { cx = 0; cy += shelf_h; shelf_h = 0; }
    if (cy + h > tile) { ++t; cx = 0; cy = 0; shelf_h = 0; }
    int64_t tx = (t % 16) * tile, ty = (t / 16) * tile;
    D.ax[i] = tx + cx + pad;
    D.ay[i] = ty + cy + pad;
    cx += w;
    shelf_h = std::max(shelf_h, h);
  }
  D.tiles_used = t + 1;
}

// Draw pair i (shapes in local mask coordinates, B's offset from A's origin).
void draw_pair(int config, uint64_t seed, int64_t i, Shape& A, Shape& B, int& bx, int& by, uint8_t& blob,
               int64_t& attempts, int64_t& rejected) {
  Rng g(seed, (uint64_t)i);
  for (;;) {
    bool is_blob = false;
    ShapeSpec sp = spec_for(config, g, is_blob);
    int used = 0;
    bool ok = make_shape(g, sp, A, &used);
    attempts += used;
    if (!ok) rejected++;
    if (A.ring.size() >= 8 && derive_b(g, A, B, bx, by)) {
      blob = is_blob;
      return;
    }
  }
}

void gen_pairs(Dataset& D, int config, uint64_t seed, int64_t n, int n_threads, bool keep_masks) {
  D.config = config;
  D.seed = seed;
  D.n_pairs = n;
  D.A.resize(n); D.B.resize(n);
  D.wa.resize(n); D.ha.resize(n);
  std::vector<int64_t> rbx(n), rby(n);
  D.blob.assign(n, 0);
  std::atomic<int64_t> next{0}, rej{0}, att{0};
  auto worker = [&]() {
    for (;;) {
      int64_t i0 = next.fetch_add(64);
      if (i0 >= n) break;
      int64_t a_loc = 0, r_loc = 0;
      for (int64_t i = i0; i < std::min(n, i0 + 64); ++i) {
        int bx = 0, by = 0;
        draw_pair(config, seed, i, D.A[i], D.B[i], bx, by, D.blob[i], a_loc, r_loc);
        rbx[i] = bx; rby[i] = by;
        D.wa[i] = D.A[i].mask.w; D.ha[i] = D.A[i].mask.h;
        if (!keep_masks) {
          D.A[i].mask = Mask();
          D.B[i].mask = Mask();
        }
      }
      att += a_loc;
      rej += r_loc;
    }
  };
  int nt = std::max(1, n_threads);
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) th.emplace_back(worker);
  for (auto& x : th) x.join();
  D.rejected = rej;
  D.attempts = att;
  int64_t tile = (config == 1) ? 4096 : 16384;
  place(D, tile, 6);
  D.bx.resize(n); D.by.resize(n);
  for (int64_t i = 0; i < n; ++i) { D.bx[i] = D.ax[i] + rbx[i]; D.by[i] = D.ay[i] + rby[i]; }
  D.pa.resize(n); D.pb.resize(n);
  for (int64_t i = 0; i < n; ++i) { D.pa[i] = (int32_t)i; D.pb[i] = (int32_t)i; }
  D.n_sets = 1;
  D.set_off = {0, n};
}


// ------------------------------------------------------- set-level tiles ----
// Workload 4: n_tiles square tiles; in each, set A is filled with
// workload-2 shapes until the tile is full, pixel-disjoint: a cursor walks
// the tile's columns left to right (wrapping), and each shape drops onto a
// per-column skyline (the row above the highest pixel placed in the column)
// until one of its columns touches, at the lowest such drop within half its
// width of the cursor, so that shapes nest into the profile of the row
// below; set B holds, for 85% of A's shapes (one draw per shape),
// a shifted and dilated or eroded copy, plus 15% * |A| fresh shapes at
// uniform positions in the tile.
// Candidate pairs come from a uniform-grid join of the MBRs (cell side
// `cell`): a pair is emitted when the MBRs share at least one pixel, once, in
// the cell that holds the lower-left pixel of their intersection.
struct TileSets {
  std::vector<Shape> A, B;
  std::vector<int64_t> ax, ay, bx, by;
  std::vector<int32_t> pa, pb;  // tile-local indices
};

void gen_tile(TileSets& T, uint64_t seed, int64_t tile, int64_t tile_side, int64_t ox, int64_t oy, int cell) {
  const uint64_t base = (uint64_t)tile << 32;
  // A: skyline drop (see above; each shape takes the lowest drop within
  // half its width of the cursor); a run of shapes that no longer fit below
  // the top of the tile ends the tile
  std::vector<int64_t> sky((size_t)tile_side, 0);
  std::vector<int64_t> lo, hi;
  int64_t cx = 0, misses = 0;
  for (int64_t k = 0; misses < 256; ++k) {
    Rng g(seed, base | (uint64_t)k);
    bool blob = false;
    ShapeSpec sp = spec_for(2, g, blob);
    Shape A;
    int used = 0;
    make_shape(g, sp, A, &used);
    if (A.ring.size() < 8) continue;
    const int64_t w = A.mask.w, h = A.mask.h;
    if (w > tile_side || h > tile_side) continue;
    if (cx + w > tile_side) cx = 0;
    // lowest and one past the highest pixel row of each column (a cropped,
    // connected shape has a pixel in every column)
    lo.assign((size_t)w, h);
    hi.assign((size_t)w, 0);
    for (int64_t y = 0; y < h; ++y)
      for (int64_t x = 0; x < w; ++x)
        if (A.mask.at((int)x, (int)y)) {
          lo[(size_t)x] = std::min(lo[(size_t)x], y);
          hi[(size_t)x] = std::max(hi[(size_t)x], y + 1);
        }
    // the lowest drop among positions around the cursor
    int64_t y0 = INT64_MAX, bx = cx;
    for (int64_t x0 = std::max<int64_t>(0, cx - w / 2); x0 <= std::min(cx + w / 2, tile_side - w); x0 += 2) {
      int64_t y = 0;
      for (int64_t x = 0; x < w && y < y0; ++x) y = std::max(y, sky[(size_t)(x0 + x)] - lo[(size_t)x]);
      if (y < y0) {
        y0 = y;
        bx = x0;
      }
    }
    cx = bx;
    if (y0 + h > tile_side) {
      ++misses;
      cx += w;
      continue;
    }
    misses = 0;
    for (int64_t x = 0; x < w; ++x) sky[(size_t)(cx + x)] = y0 + hi[(size_t)x];
    T.ax.push_back(ox + cx);
    T.ay.push_back(oy + y0);
    cx += w;
    // B derived from A with probability 0.85
    Rng gb(seed ^ 0x5bd1e995ull, base | (uint64_t)k);
    if (gb.unit() < 0.85) {
      Shape B;
      int bx = 0, by = 0;
      if (derive_b(gb, A, B, bx, by)) {
        T.bx.push_back(T.ax.back() + bx);
        T.by.push_back(T.ay.back() + by);
        B.mask = Mask();
        T.B.push_back(std::move(B));
      }
    }
    T.A.push_back(std::move(A));
    T.A.back().mask.m.shrink_to_fit();
  }
  // unmatched B shapes at uniform positions
  const int64_t n_fresh = (int64_t)std::llround(0.15 * (double)T.A.size());
  for (int64_t k = 0; k < n_fresh; ++k) {
    Rng g(seed ^ 0x9e3779b9ull, base | (uint64_t)k);
    bool blob = false;
    ShapeSpec sp = spec_for(2, g, blob);
    Shape B;
    int used = 0;
    make_shape(g, sp, B, &used);
    if (B.ring.size() < 8) continue;
    const int64_t px = g.uni(0, tile_side - B.mask.w), py = g.uni(0, tile_side - B.mask.h);
    T.bx.push_back(ox + px);
    T.by.push_back(oy + py);
    B.mask = Mask();
    T.B.push_back(std::move(B));
  }
  for (auto& a : T.A) a.mask = Mask();
  // MBRs (pixel extents) of both sets, tile-local cell grid
  auto mbr = [](const Shape& S, int64_t gx, int64_t gy, int64_t* m) {
    int64_t x0 = INT64_MAX, y0 = INT64_MAX, x1 = INT64_MIN, y1 = INT64_MIN;
    for (size_t k = 0; k < S.ring.size(); k += 2) {
      x0 = std::min<int64_t>(x0, S.ring[k] + gx);
      x1 = std::max<int64_t>(x1, S.ring[k] + gx);
      y0 = std::min<int64_t>(y0, S.ring[k + 1] + gy);
      y1 = std::max<int64_t>(y1, S.ring[k + 1] + gy);
    }
    m[0] = x0; m[1] = y0; m[2] = x1; m[3] = y1;
  };
  const int64_t ncell = (tile_side + cell - 1) / cell + 2;  // B shapes may reach a little past the tile
  std::vector<std::vector<int32_t>> grid((size_t)(ncell * ncell));
  std::vector<int64_t> ma(4 * T.A.size());
  auto cell_of = [&](int64_t v, int64_t o) { return std::min<int64_t>(ncell - 1, std::max<int64_t>(0, (v - o) / cell + 1)); };
  for (size_t k = 0; k < T.A.size(); ++k) {
    int64_t* m = &ma[4 * k];
    mbr(T.A[k], T.ax[k], T.ay[k], m);
    for (int64_t gy = cell_of(m[1], oy); gy <= cell_of(m[3] - 1, oy); ++gy)
      for (int64_t gx = cell_of(m[0], ox); gx <= cell_of(m[2] - 1, ox); ++gx)
        grid[(size_t)(gy * ncell + gx)].push_back((int32_t)k);
  }
  for (size_t k = 0; k < T.B.size(); ++k) {
    int64_t mb[4];
    mbr(T.B[k], T.bx[k], T.by[k], mb);
    std::vector<int32_t> found;
    for (int64_t gy = cell_of(mb[1], oy); gy <= cell_of(mb[3] - 1, oy); ++gy)
      for (int64_t gx = cell_of(mb[0], ox); gx <= cell_of(mb[2] - 1, ox); ++gx)
        for (int32_t a : grid[(size_t)(gy * ncell + gx)]) {
          const int64_t* m = &ma[4 * (size_t)a];
          const int64_t ix0 = std::max(m[0], mb[0]), iy0 = std::max(m[1], mb[1]);
          const int64_t ix1 = std::min(m[2], mb[2]), iy1 = std::min(m[3], mb[3]);
          if (ix0 >= ix1 || iy0 >= iy1) continue;
          // reference point: emit only in the cell of the intersection's lower-left pixel
          if (cell_of(ix0, ox) != gx || cell_of(iy0, oy) != gy) continue;
          found.push_back(a);
        }
    std::sort(found.begin(), found.end());
    for (int32_t a : found) {
      T.pa.push_back(a);
      T.pb.push_back((int32_t)k);
    }
  }
}

struct SetsDataset {
  int64_t n_tiles = 0;
  std::vector<TileSets> tiles;
};

void gen_sets(SetsDataset& D, uint64_t seed, int64_t n_tiles, int64_t tile_side, int cell, int n_threads) {
  D.n_tiles = n_tiles;
  D.tiles.resize((size_t)n_tiles);
  std::atomic<int64_t> next{0};
  auto worker = [&]() {
    for (;;) {
      const int64_t t = next.fetch_add(1);
      if (t >= n_tiles) break;
      gen_tile(D.tiles[(size_t)t], seed, t, tile_side, (t % 8) * tile_side, (t / 8) * tile_side, cell);
    }
  };
  std::vector<std::thread> th;
  for (int k = 0; k < std::max(1, n_threads); ++k) th.emplace_back(worker);
  for (auto& x : th) x.join();
}

}  // namespace

// ============================================================== C ABI ====
extern "C" {

typedef struct sccg_gen sccg_gen;
struct sccg_gen { Dataset d; };

// Generate a pair workload of the given config (1, 2 or 3).  Pair i is (A_i, B_i).
// Masks are not kept (a blob mask is up to 160 KB); sccg_gen_mask redraws the
// pair from its own stream when one is asked for.
sccg_gen* sccg_gen_pairs(int config, uint64_t seed, int64_t n_pairs, int n_threads) {
  if (n_pairs < 0) return nullptr;
  sccg_gen* h = new sccg_gen();
  gen_pairs(h->d, config, seed, n_pairs, n_threads, false);
  return h;
}

void sccg_gen_free(sccg_gen* h) { delete h; }

// counts[0..] = n_polys_A, n_verts_A, n_polys_B, n_verts_B, n_pairs, n_sets,
//               tiles_used, rejected, attempts, n_blobs
void sccg_gen_counts(const sccg_gen* h, int64_t* c) {
  const Dataset& D = h->d;
  int64_t va = 0, vb = 0, nb = 0;
  for (auto& s : D.A) va += (int64_t)s.ring.size() / 2;
  for (auto& s : D.B) vb += (int64_t)s.ring.size() / 2;
  for (auto b : D.blob) nb += b;
  c[0] = (int64_t)D.A.size(); c[1] = va; c[2] = (int64_t)D.B.size(); c[3] = vb;
  c[4] = (int64_t)D.pa.size(); c[5] = D.n_sets; c[6] = D.tiles_used; c[7] = D.rejected;
  c[8] = D.attempts; c[9] = nb;
}

static void emit(const std::vector<Shape>& S, const std::vector<int64_t>& ox, const std::vector<int64_t>& oy,
                 int64_t* off, int32_t* xy) {
  int64_t v = 0;
  off[0] = 0;
  for (size_t i = 0; i < S.size(); ++i) {
    const auto& r = S[i].ring;
    for (size_t k = 0; k < r.size(); k += 2) {
      xy[2 * v] = (int32_t)(r[k] + ox[i]);
      xy[2 * v + 1] = (int32_t)(r[k + 1] + oy[i]);
      ++v;
    }
    off[i + 1] = v;
  }
}

// Copy out CSR rings (global coordinates), pair index arrays and set offsets.
void sccg_gen_copy(const sccg_gen* h, int64_t* offA, int32_t* xyA, int64_t* offB, int32_t* xyB, int32_t* pa,
                   int32_t* pb, int64_t* set_off) {
  const Dataset& D = h->d;
  emit(D.A, D.ax, D.ay, offA, xyA);
  emit(D.B, D.bx, D.by, offB, xyB);
  std::memcpy(pa, D.pa.data(), D.pa.size() * 4);
  std::memcpy(pb, D.pb.data(), D.pb.size() * 4);
  std::memcpy(set_off, D.set_off.data(), D.set_off.size() * 8);
}

// Per-pair flags: 1 = large merged blob (config 3).
void sccg_gen_blob_flags(const sccg_gen* h, uint8_t* out) {
  std::memcpy(out, h->d.blob.data(), h->d.blob.size());
}

// Raster mask of polygon i of set `which` (0 = A, 1 = B): writes its size and
// global origin to info[0..3] = (w, h, ox, oy); copies w*h bytes (row-major,
// y up) into `bits` if non-null and cap >= w*h.
int sccg_gen_mask(const sccg_gen* h, int which, int64_t i, int64_t* info, uint8_t* bits, int64_t cap) {
  const Dataset& D = h->d;
  if (i < 0 || i >= D.n_pairs || D.config > 3) return -1;
  Shape A, B;
  int bx = 0, by = 0;
  uint8_t blob = 0;
  int64_t a = 0, r = 0;
  draw_pair(D.config, D.seed, i, A, B, bx, by, blob, a, r);
  const Mask& M = which ? B.mask : A.mask;
  info[0] = M.w; info[1] = M.h;
  info[2] = which ? D.bx[i] : D.ax[i];
  info[3] = which ? D.by[i] : D.ay[i];
  if (bits && cap >= (int64_t)M.w * M.h) std::memcpy(bits, M.m.data(), M.m.size());
  return 0;
}

// Trace a caller-supplied mask (w*h bytes, y up) after keeping its largest
// 4-connected component and filling holes.  Writes up to cap vertices
// (x,y interleaved, relative to the mask's (0,0)) and returns the vertex
// count, or -1 if the mask is empty.  Used to build exhaustive tiny-grid
// corpora.
int64_t sccg_gen_trace_mask(const uint8_t* bits, int w, int h, int32_t* xy, int64_t cap) {
  Mask M;
  M.init(w, h);
  std::memcpy(M.m.data(), bits, (size_t)w * h);
  if (keep_largest_component(M) == 0) return -1;
  fill_holes(M);
  std::vector<int32_t> ring;
  if (!trace(M, ring)) return -1;
  int64_t nv = (int64_t)ring.size() / 2;
  for (int64_t k = 0; k < std::min(nv, cap); ++k) { xy[2 * k] = ring[2 * k]; xy[2 * k + 1] = ring[2 * k + 1]; }
  return nv;
}

typedef struct sccg_gen_sets sccg_gen_sets;
struct sccg_gen_sets { SetsDataset d; };

// Set-level workload 4: n_tiles tiles of tile_side^2 pixels (8 tiles to a
// row of tiles), candidate pairs from a uniform grid of `cell`-pixel cells.
sccg_gen_sets* sccg_gen_sets_create(uint64_t seed, int64_t n_tiles, int64_t tile_side, int cell, int n_threads) {
  if (n_tiles < 0 || tile_side < 64 || cell < 1) return nullptr;
  sccg_gen_sets* h = new sccg_gen_sets();
  gen_sets(h->d, seed, n_tiles, tile_side, cell, n_threads);
  return h;
}

void sccg_gen_sets_free(sccg_gen_sets* h) { delete h; }

// c[0..3] = polygons in A, vertices in A, polygons in B, vertices in B; c[4] = pairs; c[5] = tiles
void sccg_gen_sets_counts(const sccg_gen_sets* h, int64_t* c) {
  int64_t na = 0, va = 0, nb = 0, vb = 0, np = 0;
  for (const auto& T : h->d.tiles) {
    na += (int64_t)T.A.size();
    nb += (int64_t)T.B.size();
    for (auto& s : T.A) va += (int64_t)s.ring.size() / 2;
    for (auto& s : T.B) vb += (int64_t)s.ring.size() / 2;
    np += (int64_t)T.pa.size();
  }
  c[0] = na; c[1] = va; c[2] = nb; c[3] = vb; c[4] = np; c[5] = h->d.n_tiles;
}

// CSR rings of both sets (tiles concatenated in order), global pair indices
// and the pair offsets of each tile (set_off[n_tiles+1]).
void sccg_gen_sets_copy(const sccg_gen_sets* h, int64_t* offA, int32_t* xyA, int64_t* offB, int32_t* xyB, int32_t* pa,
                        int32_t* pb, int64_t* set_off) {
  int64_t ia = 0, ib = 0, va = 0, vb = 0, np = 0;
  offA[0] = 0;
  offB[0] = 0;
  set_off[0] = 0;
  for (size_t t = 0; t < h->d.tiles.size(); ++t) {
    const TileSets& T = h->d.tiles[t];
    const int64_t a0 = ia, b0 = ib;
    for (size_t k = 0; k < T.A.size(); ++k) {
      const auto& r = T.A[k].ring;
      for (size_t j = 0; j < r.size(); j += 2) {
        xyA[2 * va] = (int32_t)(r[j] + T.ax[k]);
        xyA[2 * va + 1] = (int32_t)(r[j + 1] + T.ay[k]);
        ++va;
      }
      offA[++ia] = va;
    }
    for (size_t k = 0; k < T.B.size(); ++k) {
      const auto& r = T.B[k].ring;
      for (size_t j = 0; j < r.size(); j += 2) {
        xyB[2 * vb] = (int32_t)(r[j] + T.bx[k]);
        xyB[2 * vb + 1] = (int32_t)(r[j + 1] + T.by[k]);
        ++vb;
      }
      offB[++ib] = vb;
    }
    for (size_t k = 0; k < T.pa.size(); ++k) {
      pa[np] = (int32_t)(a0 + T.pa[k]);
      pb[np] = (int32_t)(b0 + T.pb[k]);
      ++np;
    }
    set_off[t + 1] = np;
  }
}

// Polygon ranges of each tile: A polygons [a_off[t], a_off[t+1]), B polygons
// [b_off[t], b_off[t+1]) (both [n_tiles+1]).
void sccg_gen_sets_poly_off(const sccg_gen_sets* h, int64_t* a_off, int64_t* b_off) {
  a_off[0] = 0;
  b_off[0] = 0;
  for (size_t t = 0; t < h->d.tiles.size(); ++t) {
    a_off[t + 1] = a_off[t] + (int64_t)h->d.tiles[t].A.size();
    b_off[t + 1] = b_off[t] + (int64_t)h->d.tiles[t].B.size();
  }
}

}  // extern "C"

// The filter stage of Section 4.1 on the device: candidate pairs of two
// polygon sets are the pairs whose MBRs intersect.  Per set, a uniform grid
// over the extent of the set's A polygons indexes them (a counting sort of
// (cell, polygon) entries); each B polygon visits the cells its MBR covers
// and keeps the A polygons whose MBR shares a pixel with its own, reporting
// a pair only from the cell that holds the lower-left pixel of the two MBRs'
// intersection, so that every pair is found once.  Each B polygon's pairs are
// written to a segment of their own (offsets from a scan of the counts) and
// sorted there by A index: the output is ordered by set, then B, then A.
#include <limits.h>

#include "sccg_device.h"

namespace sccg {

namespace {

// The set holding index k: the largest s with off[s] <= k, or -1 when k lies
// outside [off[0], off[n]).
__device__ __forceinline__ int64_t set_of(const int64_t* off, int64_t n, int64_t k) {
  if (n <= 0 || k < off[0] || k >= off[n]) return -1;
  int64_t lo = 0, hi = n;  // off[lo] <= k < off[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (off[mid] <= k)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ bool meta_empty(const Meta& m) { return m.x0 >= m.x1 || m.y0 >= m.y1; }

// cell index of pixel coordinate v in a grid starting at o (floor division,
// v >= o)
// cell index of v >= o; v - o can reach 2^31 with coordinates up to 2^30 in size
__device__ __forceinline__ int cell_of(int v, int o, int cell) {
  return (int)(((uint32_t)v - (uint32_t)o) / (uint32_t)cell);
}

}  // namespace

__global__ void k_join_init_sets(int64_t n_sets, int4* bbox) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n_sets) bbox[s] = make_int4(INT_MAX, INT_MAX, INT_MIN, INT_MIN);
}

// Extent of each set's A polygons.  Sets are contiguous ranges, so the
// lanes of a wave usually share one set: then the wave reduces first and one
// lane updates the set (a set holds many thousand polygons; per-polygon
// atomics on its four words would serialize).
__global__ void k_join_bbox(Polys A, const Meta* metaA, const int64_t* a_off, int64_t n_sets, int4* bbox) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t s = -1;
  Meta m{INT_MAX, INT_MAX, INT_MIN, INT_MIN};
  if (a < A.n) {
    s = set_of(a_off, n_sets, a);
    const Meta t = load_meta(metaA, a);
    if (s >= 0 && !meta_empty(t)) m = t;
  }
  const int64_t s0 = uniform64(s);
  if (ballot(s != s0) == 0ull) {
    if (s0 < 0) return;
    const int x0 = wave_min_i32(m.x0), y0 = wave_min_i32(m.y0);
    const int x1 = wave_max_i32(m.x1), y1 = wave_max_i32(m.y1);
    if (lane_id() == 0 && x0 < x1 && y0 < y1) {
      atomicMin(&bbox[s0].x, x0);
      atomicMin(&bbox[s0].y, y0);
      atomicMax(&bbox[s0].z, x1);
      atomicMax(&bbox[s0].w, y1);
    }
    return;
  }
  if (s < 0 || meta_empty(m)) return;
  atomicMin(&bbox[s].x, m.x0);
  atomicMin(&bbox[s].y, m.y0);
  atomicMax(&bbox[s].z, m.x1);
  atomicMax(&bbox[s].w, m.y1);
}

// Grid of each set: origin, columns, rows; cells[s] = columns x rows.
__global__ void k_join_grid(int64_t n_sets, const int4* bbox, int cell, int4* grid, int64_t* cells,
                            uint32_t* err) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sets) return;
  const int4 b = bbox[s];
  int gw = 0, gh = 0;
  if (b.x < b.z && b.y < b.w) {
    const int64_t w = ((int64_t)b.z - b.x + cell - 1) / cell, h = ((int64_t)b.w - b.y + cell - 1) / cell;
    if (w * h > (1 << 24)) {
      latch_error(err, kErrSide);  // the set's grid is too large for the cell size
    } else {
      gw = (int)w;
      gh = (int)h;
    }
  }
  grid[s] = make_int4(b.x, b.y, gw, gh);
  cells[s] = (int64_t)gw * gh;
}

// Cells of an MBR clamped to a grid: [cx0, cx1] x [cy0, cy1] (empty if cx0 > cx1).
__device__ __forceinline__ void cell_range(const Meta& m, const int4& g, int cell, int& cx0, int& cy0, int& cx1,
                                           int& cy1) {
  cx0 = max(0, cell_of(max(m.x0, g.x), g.x, cell));
  cy0 = max(0, cell_of(max(m.y0, g.y), g.y, cell));
  cx1 = min(g.z - 1, cell_of(max(m.x1 - 1, g.x), g.x, cell));
  cy1 = min(g.w - 1, cell_of(max(m.y1 - 1, g.y), g.y, cell));
  if (m.x1 <= g.x || m.y1 <= g.y) cx1 = -1;  // wholly left of or below the grid
}

// mode 0: count the A polygons of each cell; mode 1: fill the cell lists.
__global__ void k_join_cells(Polys A, const Meta* metaA, const int64_t* a_off, int64_t n_sets, const int4* grid,
                             const int64_t* cell_base, int cell, int mode, int32_t* count, const int64_t* start,
                             int32_t* list) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= A.n) return;
  const int64_t s = set_of(a_off, n_sets, a);
  if (s < 0) return;
  const Meta m = load_meta(metaA, a);
  const int4 g = grid[s];
  if (meta_empty(m) || g.z == 0) return;
  int cx0, cy0, cx1, cy1;
  cell_range(m, g, cell, cx0, cy0, cx1, cy1);
  for (int cy = cy0; cy <= cy1; ++cy)
    for (int cx = cx0; cx <= cx1; ++cx) {
      const int64_t c = cell_base[s] + (int64_t)cy * g.z + cx;
      const int32_t k = atomicAdd(count + c, 1);
      if (mode == 1) list[start[c] + k] = (int32_t)a;
    }
}

// Per B polygon: the A polygons of its set whose MBR shares a pixel with its
// own, each found in the cell of the intersection's lower-left pixel.  mode
// 0 counts them; mode 1 writes them (up to cap) and sorts the segment by A.
__global__ void k_join_pairs(Polys B, const Meta* metaA, const Meta* metaB, const int64_t* b_off, int64_t n_sets,
                             const int4* grid, const int64_t* cell_base, const int64_t* start, const int32_t* list,
                             int cell, int mode, int32_t* b_count, const int64_t* b_start, int64_t cap,
                             int32_t* out_pa, int32_t* out_pb) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B.n) return;
  const int64_t s = set_of(b_off, n_sets, b);
  int32_t n = 0;
  const int64_t base = mode == 1 ? b_start[b] : 0;
  if (s >= 0) {
    const Meta mb = load_meta(metaB, b);
    const int4 g = grid[s];
    if (!meta_empty(mb) && g.z > 0) {
      int cx0, cy0, cx1, cy1;
      cell_range(mb, g, cell, cx0, cy0, cx1, cy1);
      for (int cy = cy0; cy <= cy1; ++cy)
        for (int cx = cx0; cx <= cx1; ++cx) {
          const int64_t c = cell_base[s] + (int64_t)cy * g.z + cx;
          for (int64_t e = start[c]; e < start[c + 1]; ++e) {
            const int32_t a = list[e];
            const Meta ma = load_meta(metaA, a);
            const int ix0 = max(ma.x0, mb.x0), iy0 = max(ma.y0, mb.y0);
            const int ix1 = min(ma.x1, mb.x1), iy1 = min(ma.y1, mb.y1);
            if (ix0 >= ix1 || iy0 >= iy1) continue;
            if (cell_of(ix0, g.x, cell) != cx || cell_of(iy0, g.y, cell) != cy) continue;
            if (mode == 1 && base + n < cap) {
              out_pa[base + n] = a;
              out_pb[base + n] = (int32_t)b;
            }
            ++n;
          }
        }
    }
  }
  if (mode == 0) {
    b_count[b] = n;
    return;
  }
  // insertion sort of this B polygon's segment by A index
  const int64_t end = min(base + (int64_t)n, cap);
  for (int64_t i = base + 1; i < end; ++i) {
    const int32_t v = out_pa[i];
    int64_t j = i - 1;
    while (j >= base && out_pa[j] > v) {
      out_pa[j + 1] = out_pa[j];
      --j;
    }
    out_pa[j + 1] = v;
  }
}

__global__ void k_join_set_off(int64_t n_sets, int64_t n_b, const int64_t* b_off, const int64_t* b_start,
                               int64_t* out_set_off) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s <= n_sets) out_set_off[s] = b_start[min(max(b_off[s], (int64_t)0), n_b)];
}

// ------------------------------------------------------- exclusive scan
// out[i] = sum of in[0 .. i) for i <= n (out has n + 1 entries).  Blocks of
// 256 threads scan 1024 entries each; the block totals are scanned by one
// block; then each block adds its offset.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kScanBlock = kScanThreads * kScanPer;

template <typename T>
__device__ __forceinline__ int64_t block_exclusive(int64_t v, int64_t* sh) {
  // Hillis-Steele over the threads of the block; returns the exclusive prefix
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = 1; d < (int)blockDim.x; d <<= 1) {
    const int64_t add = t >= d ? sh[t - d] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  const int64_t incl = sh[t];
  __syncthreads();
  return incl - v;
}

template <typename T>
__global__ void __launch_bounds__(kScanThreads) k_scan_blocks(const T* in, int64_t n, int64_t* out, int64_t* sums) {
  __shared__ int64_t sh[kScanThreads];
  const int64_t i0 = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  int64_t v[kScanPer];
  int64_t tot = 0;
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = (i0 + k < n) ? (int64_t)in[i0 + k] : 0;
    tot += v[k];
  }
  int64_t run = block_exclusive<T>(tot, sh);
  for (int k = 0; k < kScanPer; ++k) {
    if (i0 + k < n) out[i0 + k] = run;
    run += v[k];
  }
  if (threadIdx.x == blockDim.x - 1) sums[blockIdx.x] = run;
}

// One block: exclusive scan of the nb block totals in place; sums[nb] = total.
__global__ void __launch_bounds__(1024) k_scan_sums(int64_t* sums, int64_t nb) {
  __shared__ int64_t sh[1024];
  const int64_t per = (nb + blockDim.x - 1) / blockDim.x;
  const int64_t i0 = (int64_t)threadIdx.x * per;
  int64_t tot = 0;
  for (int64_t k = i0; k < min(i0 + per, nb); ++k) tot += sums[k];
  int64_t run = block_exclusive<int64_t>(tot, sh);
  for (int64_t k = i0; k < min(i0 + per, nb); ++k) {
    const int64_t x = sums[k];
    sums[k] = run;
    run += x;
  }
  if (threadIdx.x == blockDim.x - 1) sums[nb] = run;
}

__global__ void k_scan_add(int64_t* out, int64_t n, const int64_t* sums) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += sums[i / kScanBlock];
  if (i == n) out[n] = sums[(n + kScanBlock - 1) / kScanBlock];
}

int64_t scan_scratch(int64_t n) { return (n + kScanBlock - 1) / kScanBlock + 1; }

template <typename T>
hipError_t scan_exclusive(const T* in, int64_t n, int64_t* out, int64_t* sums, hipStream_t s) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb > 0) hipLaunchKernelGGL(k_scan_blocks<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, out, sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, sums, nb);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, s, out, n, sums);
  return hipGetLastError();
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_join_grid(const Polys& A, const Meta* metaA, const int64_t* a_off, int64_t n_sets, int cell,
                            int4* bbox, int4* grid, int64_t* cells, int64_t* cell_base, int64_t* sums,
                            uint32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(k_join_init_sets, dim3(blocks_for(n_sets)), dim3(256), 0, s, n_sets, bbox);
  if (A.n > 0)
    hipLaunchKernelGGL(k_join_bbox, dim3(blocks_for(A.n)), dim3(256), 0, s, A, metaA, a_off, n_sets, bbox);
  hipLaunchKernelGGL(k_join_grid, dim3(blocks_for(n_sets)), dim3(256), 0, s, n_sets, bbox, cell, grid, cells, err);
  return scan_exclusive<int64_t>(cells, n_sets, cell_base, sums, s);
}

hipError_t launch_join_cells(const Polys& A, const Meta* metaA, const int64_t* a_off, int64_t n_sets,
                             const int4* grid, const int64_t* cell_base, int cell, int mode, int32_t* count,
                             const int64_t* start, int32_t* list, hipStream_t s) {
  if (A.n > 0)
    hipLaunchKernelGGL(k_join_cells, dim3(blocks_for(A.n)), dim3(256), 0, s, A, metaA, a_off, n_sets, grid,
                       cell_base, cell, mode, count, start, list);
  return hipGetLastError();
}

hipError_t launch_join_scan_counts(const int32_t* count, int64_t n, int64_t* start, int64_t* sums, hipStream_t s) {
  return scan_exclusive<int32_t>(count, n, start, sums, s);
}

hipError_t launch_join_pairs(const Polys& B, const Meta* metaA, const Meta* metaB, const int64_t* b_off,
                             int64_t n_sets, const int4* grid, const int64_t* cell_base, const int64_t* start,
                             const int32_t* list, int cell, int mode, int32_t* b_count, const int64_t* b_start,
                             int64_t cap, int32_t* out_pa, int32_t* out_pb, hipStream_t s) {
  if (B.n > 0)
    hipLaunchKernelGGL(k_join_pairs, dim3(blocks_for(B.n)), dim3(256), 0, s, B, metaA, metaB, b_off, n_sets, grid,
                       cell_base, start, list, cell, mode, b_count, b_start, cap, out_pa, out_pb);
  return hipGetLastError();
}

hipError_t launch_join_set_off(int64_t n_sets, int64_t n_b, const int64_t* b_off, const int64_t* b_start,
                               int64_t* out_set_off, hipStream_t s) {
  hipLaunchKernelGGL(k_join_set_off, dim3(blocks_for(n_sets + 1)), dim3(256), 0, s, n_sets, n_b, b_off, b_start,
                     out_set_off);
  return hipGetLastError();
}

}  // namespace sccg

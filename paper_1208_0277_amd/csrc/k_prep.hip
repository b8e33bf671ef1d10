// Per-polygon prepass, ring validation and the set-level Jaccard reduction.
#include <limits.h>

#include "fix192.h"
#include "sccg_device.h"

namespace sccg {

// One polygon's extent and doubled signed area, accumulated over one lane's
// share of a ring.  The shoelace sum (Section 3.2) is taken
// in wrapping 64-bit arithmetic: partial sums may overflow, the final value
// (twice the area, at most 2^63 in size) is exact modulo 2^64.
struct MetaAcc {
  int32_t x0 = INT_MAX, y0 = INT_MAX, x1 = INT_MIN, y1 = INT_MIN;
  uint64_t twice = 0;
  __device__ void add(int2 v, int2 w) {
    x0 = min(x0, v.x);
    y0 = min(y0, v.y);
    x1 = max(x1, v.x);
    y1 = max(y1, v.y);
    twice += (uint64_t)((int64_t)v.x * w.y) - (uint64_t)((int64_t)w.x * v.y);
  }
};

__device__ void write_meta(const MetaAcc& a, int64_t nv, int64_t k, Meta* meta, int64_t* area, uint32_t* err) {
  bool empty = nv <= 0;
  bool bad = !empty && (a.x0 < -kMaxCoord || a.y0 < -kMaxCoord || a.x1 > kMaxCoord || a.y1 > kMaxCoord);
  if (bad) latch_error(err, kErrCoord);
  if (empty || bad) {
    *reinterpret_cast<int4*>(meta + k) = make_int4(INT_MAX, INT_MAX, INT_MIN, INT_MIN);
    area[k] = 0;
    return;
  }
  *reinterpret_cast<int4*>(meta + k) = make_int4(a.x0, a.y0, a.x1, a.y1);
  // twice the area is at most 2^63 in size: its magnitude is exact unsigned
  const uint64_t t = (uint64_t)a.twice;
  area[k] = (int64_t)(((int64_t)t < 0 ? 0 - t : t) / 2);
}


// Eight lanes per polygon: lane j of a group walks vertices j, j + 8, ...
// (eight consecutive vertices, 64 bytes, per step of the group), then the
// group combines its partial extents and shoelace sums in three exchanges.
constexpr int kGroup = 8;

__device__ __forceinline__ int32_t group_min(int32_t v) {
  v = min(v, __shfl_xor(v, 1, kWave));
  v = min(v, __shfl_xor(v, 2, kWave));
  return min(v, __shfl_xor(v, 4, kWave));
}
__device__ __forceinline__ int32_t group_max(int32_t v) {
  v = max(v, __shfl_xor(v, 1, kWave));
  v = max(v, __shfl_xor(v, 2, kWave));
  return max(v, __shfl_xor(v, 4, kWave));
}
__device__ __forceinline__ uint64_t group_sum64(uint64_t v) {
  for (int d = 1; d < kGroup; d <<= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, d, kWave);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), d, kWave);
    v += ((uint64_t)hi << 32) | lo;
  }
  return v;
}

__global__ void __launch_bounds__(256) k_meta_group(Polys P, Meta* meta, int64_t* area, uint32_t* err) {
  const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kGroup;
  const int j = (int)(threadIdx.x % kGroup);
  const bool live = gid < P.n;
  int64_t o0 = 0, nv = 0;
  if (live) {
    o0 = P.off[gid];
    nv = P.off[gid + 1] - o0;
  }
  MetaAcc a;
  for (int64_t i = j; i < nv; i += kGroup) {
    const int2 v = P.xy[o0 + i];
    const int2 w = P.xy[o0 + (i + 1 == nv ? 0 : i + 1)];
    a.add(v, w);
  }
  MetaAcc r;
  r.x0 = group_min(a.x0);
  r.y0 = group_min(a.y0);
  r.x1 = group_max(a.x1);
  r.y1 = group_max(a.y1);
  r.twice = group_sum64(a.twice);
  if (live && j == 0) write_meta(r, nv, gid, meta, area, err);
}

hipError_t launch_poly_meta(const Polys& P, Meta* meta, int64_t* area, int32_t* big_list, int32_t* big_count,
                            uint32_t* err, hipStream_t s) {
  (void)big_list;
  (void)big_count;
  if (P.n <= 0) return hipSuccess;
  const int64_t blocks = (P.n * kGroup + 255) / 256;
  hipLaunchKernelGGL(k_meta_group, dim3((unsigned)blocks), dim3(256), 0, s, P, meta, area, err);
  return hipGetLastError();
}

// ---------------------------------------------------------------- validation
__global__ void k_validate_init(unsigned long long* first_bad) { *first_bad = ~0ull; }

__global__ void __launch_bounds__(256) k_validate(Polys P, unsigned long long* first_bad) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P.n) return;
  const int64_t o0 = P.off[k];
  const int64_t nv = P.off[k + 1] - o0;
  bool bad = nv < 4;
  for (int64_t i = 0; i < nv && !bad; ++i) {
    const int2 v = P.xy[o0 + i];
    const int2 w = P.xy[o0 + (i + 1 == nv ? 0 : i + 1)];
    if (v.x != w.x && v.y != w.y) bad = true;
  }
  if (bad) atomicMin(first_bad, (unsigned long long)k);
}

__global__ void k_validate_fin(unsigned long long* first_bad) {
  if (*first_bad == ~0ull) *reinterpret_cast<int64_t*>(first_bad) = -1;
}

hipError_t launch_validate(const Polys& P, int64_t* first_bad, hipStream_t s) {
  auto* fb = reinterpret_cast<unsigned long long*>(first_bad);
  hipLaunchKernelGGL(k_validate_init, dim3(1), dim3(1), 0, s, fb);
  if (P.n > 0)
    hipLaunchKernelGGL(k_validate, dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, s, P, fb);
  hipLaunchKernelGGL(k_validate_fin, dim3(1), dim3(1), 0, s, fb);
  return hipGetLastError();
}

// ------------------------------------------------------------------- Jaccard
// Per-set sums of Eq. 1 over the pairs of each set; J' by the exact ratio
// sum of fix192.h.  Workgroups claim chunks of kJacChunk consecutive pairs
// of the whole pair range, so that a large set is shared by many
// workgroups and many small sets by one.  For each set a chunk overlaps,
// the workgroup reduces its part and adds it to the set's accumulator:
// 64-bit atomics for the integer sums, and for the Fix192 ratio sum six
// 32-bit limbs, each added into a 64-bit counter (carry-save: a set gets at
// most 2^31 / kJacChunk + 1 additions, far from overflowing a counter).
// Integer and fixed-point addition do not depend on order, so the result is
// the same bits as any sequential sum.  A second pass normalizes the limbs
// and divides.
constexpr int kJacChunk = 4096;

__global__ void k_jaccard_clear(JacAcc* acc, int64_t n_sets, unsigned long long* next) {
  unsigned long long* w = reinterpret_cast<unsigned long long*>(acc);
  const int64_t n = n_sets * (int64_t)(sizeof(JacAcc) / 8);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    w[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *next = 0;
}

__global__ void __launch_bounds__(256) k_jaccard_chunks(int64_t n_sets, const int64_t* set_off,
                                                        const int64_t* inter, const int64_t* uni, uint32_t flags,
                                                        bool want_jp, JacAcc* acc, unsigned long long* next) {
  __shared__ uint64_t red[6][256];
  __shared__ int64_t chunk_s;
  const bool include_zero = (flags & SCCG_J_INCLUDE_ZERO) != 0;
  const int64_t base = set_off[0], end = set_off[n_sets];  // the pairs of all sets
  const int64_t n_chunks = (end - base + kJacChunk - 1) / kJacChunk;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) chunk_s = (int64_t)atomicAdd(next, 1ull);
    __syncthreads();
    const int64_t chunk = chunk_s;
    __syncthreads();
    if (chunk >= n_chunks) break;
    const int64_t c0 = base + chunk * kJacChunk, c1 = min(c0 + (int64_t)kJacChunk, end);
    // the set holding pair c0: the last s with set_off[s] <= c0
    int64_t lo = 0, hi = n_sets - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) / 2;
      if (set_off[mid] <= c0) lo = mid;
      else hi = mid - 1;
    }
    for (int64_t s = lo; s < n_sets; ++s) {
      const int64_t o0 = max(set_off[s], c0), o1 = min(set_off[s + 1], c1);
      uint64_t si = 0, su = 0, nn = 0;
      Fix192 fx;
      for (int64_t k = o0 + tid; k < o1; k += blockDim.x) {
        const int64_t I = inter[k], U = uni[k];
        if (!include_zero && I == 0) continue;
        si += (uint64_t)I;
        su += (uint64_t)U;
        nn += 1;
        if (want_jp && U > 0) fx.add_ratio((double)I / (double)U);
      }
      red[0][tid] = si;
      red[1][tid] = su;
      red[2][tid] = nn;
      red[3][tid] = fx.w[0];
      red[4][tid] = fx.w[1];
      red[5][tid] = fx.w[2];
      __syncthreads();
      for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (tid < h) {
          red[0][tid] += red[0][tid + h];
          red[1][tid] += red[1][tid + h];
          red[2][tid] += red[2][tid + h];
          Fix192 x, y;
          x.w[0] = red[3][tid]; x.w[1] = red[4][tid]; x.w[2] = red[5][tid];
          y.w[0] = red[3][tid + h]; y.w[1] = red[4][tid + h]; y.w[2] = red[5][tid + h];
          x.add(y);
          red[3][tid] = x.w[0]; red[4][tid] = x.w[1]; red[5][tid] = x.w[2];
        }
        __syncthreads();
      }
      if (tid == 0 && red[2][0] != 0) {
        JacAcc& A = acc[s];
        atomicAdd(&A.si, (unsigned long long)red[0][0]);
        atomicAdd(&A.su, (unsigned long long)red[1][0]);
        atomicAdd(&A.nn, (unsigned long long)red[2][0]);
        for (int k = 0; k < 3; ++k) {
          const uint64_t w = red[3 + k][0];
          if (w & 0xffffffffull) atomicAdd(&A.limb[2 * k], (unsigned long long)(w & 0xffffffffull));
          if (w >> 32) atomicAdd(&A.limb[2 * k + 1], (unsigned long long)(w >> 32));
        }
      }
      __syncthreads();
      if (set_off[s + 1] >= c1) break;
    }
  }
}

__global__ void k_jaccard_final(int64_t n_sets, const JacAcc* acc, bool want_jp, int64_t* sum_i, int64_t* sum_u,
                                int64_t* n_contrib, double* jout, double* jprime) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sets) return;
  const JacAcc A = acc[s];
  const int64_t tI = (int64_t)A.si, tU = (int64_t)A.su, tn = (int64_t)A.nn;
  sum_i[s] = tI;
  sum_u[s] = tU;
  n_contrib[s] = tn;
  jout[s] = tU > 0 ? (double)tI / (double)tU : 0.0;
  if (want_jp) {
    // limb k weighs 2^(32 k): add them up with carries into three words
    Fix192 f;
    for (int k = 0; k < 6; ++k) {
      Fix192 t;
      const uint64_t v = A.limb[k];
      const int sh = 32 * k, w = sh >> 6, off = sh & 63;
      t.w[w] = v << off;
      if (off && w + 1 < 3) t.w[w + 1] = v >> (64 - off);
      f.add(t);
    }
    jprime[s] = tn > 0 ? f.to_double() / (double)tn : 0.0;
  }
}

hipError_t launch_jaccard(int64_t n_sets, const int64_t* set_off, const int64_t* inter, const int64_t* uni,
                          uint32_t flags, int64_t* sum_i, int64_t* sum_u, int64_t* n_contrib, double* j,
                          double* jprime, JacAcc* acc, unsigned long long* next, int grid, hipStream_t s) {
  if (n_sets <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_jaccard_clear, dim3(256), dim3(256), 0, s, acc, n_sets, next);
  hipLaunchKernelGGL(k_jaccard_chunks, dim3(grid), dim3(256), 0, s, n_sets, set_off, inter, uni, flags,
                     jprime != nullptr, acc, next);
  hipLaunchKernelGGL(k_jaccard_final, dim3((unsigned)((n_sets + 255) / 256)), dim3(256), 0, s, n_sets, acc,
                     jprime != nullptr, sum_i, sum_u, n_contrib, j, jprime);
  return hipGetLastError();
}

}  // namespace sccg

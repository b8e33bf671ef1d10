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
// Per-set sums; J' by the exact ratio sum of fix192.h.
__global__ void __launch_bounds__(256) k_jaccard(int64_t n_sets, const int64_t* set_off, const int64_t* inter,
                                                 const int64_t* uni, uint32_t flags, int64_t* sum_i,
                                                 int64_t* sum_u, int64_t* n_contrib, double* jout,
                                                 double* jprime) {
  __shared__ uint64_t red[4][256];
  __shared__ uint64_t fx[3][256];
  const bool include_zero = (flags & SCCG_J_INCLUDE_ZERO) != 0;
  const bool want_jp = jprime != nullptr;
  for (int64_t s = blockIdx.x; s < n_sets; s += gridDim.x) {
    const int64_t o0 = set_off[s], o1 = set_off[s + 1];
    uint64_t si = 0, su = 0, nn = 0;
    Fix192 acc;
    for (int64_t k = o0 + threadIdx.x; k < o1; k += blockDim.x) {
      const int64_t I = inter[k], U = uni[k];
      if (!include_zero && I == 0) continue;
      si += (uint64_t)I;
      su += (uint64_t)U;
      nn += 1;
      if (want_jp && U > 0) acc.add_ratio((double)I / (double)U);
    }
    red[0][threadIdx.x] = si;
    red[1][threadIdx.x] = su;
    red[2][threadIdx.x] = nn;
    fx[0][threadIdx.x] = acc.w[0];
    fx[1][threadIdx.x] = acc.w[1];
    fx[2][threadIdx.x] = acc.w[2];
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) {
        red[0][threadIdx.x] += red[0][threadIdx.x + h];
        red[1][threadIdx.x] += red[1][threadIdx.x + h];
        red[2][threadIdx.x] += red[2][threadIdx.x + h];
        Fix192 a, b;
        a.w[0] = fx[0][threadIdx.x]; a.w[1] = fx[1][threadIdx.x]; a.w[2] = fx[2][threadIdx.x];
        b.w[0] = fx[0][threadIdx.x + h]; b.w[1] = fx[1][threadIdx.x + h]; b.w[2] = fx[2][threadIdx.x + h];
        a.add(b);
        fx[0][threadIdx.x] = a.w[0]; fx[1][threadIdx.x] = a.w[1]; fx[2][threadIdx.x] = a.w[2];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const int64_t tI = (int64_t)red[0][0], tU = (int64_t)red[1][0], tn = (int64_t)red[2][0];
      sum_i[s] = tI;
      sum_u[s] = tU;
      n_contrib[s] = tn;
      jout[s] = tU > 0 ? (double)tI / (double)tU : 0.0;
      if (want_jp) {
        Fix192 a;
        a.w[0] = fx[0][0]; a.w[1] = fx[1][0]; a.w[2] = fx[2][0];
        jprime[s] = tn > 0 ? a.to_double() / (double)tn : 0.0;
      }
    }
    __syncthreads();
  }
}

hipError_t launch_jaccard(int64_t n_sets, const int64_t* set_off, const int64_t* inter, const int64_t* uni,
                          uint32_t flags, int64_t* sum_i, int64_t* sum_u, int64_t* n_contrib, double* j,
                          double* jprime, hipStream_t s) {
  if (n_sets <= 0) return hipSuccess;
  const unsigned grid = (unsigned)(n_sets < 65536 ? n_sets : 65536);
  hipLaunchKernelGGL(k_jaccard, dim3(grid), dim3(256), 0, s, n_sets, set_off, inter, uni, flags, sum_i, sum_u,
                     n_contrib, j, jprime);
  return hipGetLastError();
}

}  // namespace sccg

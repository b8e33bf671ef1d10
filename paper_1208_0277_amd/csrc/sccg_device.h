// Device-side helpers: lane ids, ballots, wave reductions (wave64, gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sccg_common.h"

namespace sccg {

__device__ __forceinline__ int lane_id() {
  return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// number of set bits of `mask` in lanes below this one
__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uniform_u(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <typename Op>
__device__ __forceinline__ uint32_t wave_reduce32(uint32_t v, Op op) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = op(v, (uint32_t)__shfl_xor((int)v, m, kWave));
  return v;
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
  uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, kWave);
  uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, kWave);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int32_t wave_min_i32(int32_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = min(v, __shfl_xor(v, m, kWave));
  return v;
}
__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m, kWave));
  return v;
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += shfl_xor64(v, m);
  return v;
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
  return wave_reduce32(v, [](uint32_t a, uint32_t b) { return a + b; });
}
__device__ __forceinline__ uint64_t wave_or64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v |= shfl_xor64(v, m);
  return v;
}
__device__ __forceinline__ uint64_t wave_xor64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v ^= shfl_xor64(v, m);
  return v;
}

__device__ __forceinline__ void latch_error(uint32_t* err, uint32_t bit) {
  __hip_atomic_fetch_or(err, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Pair box = MBR(p) ∩ MBR(q) (pixels [x0,x1) x [y0,y1)); empty if x0 >= x1 or y0 >= y1.
__device__ __forceinline__ Meta pair_box(const Meta& p, const Meta& q) {
  Meta b;
  b.x0 = max(p.x0, q.x0);
  b.y0 = max(p.y0, q.y0);
  b.x1 = min(p.x1, q.x1);
  b.y1 = min(p.y1, q.y1);
  return b;
}

__device__ __forceinline__ Meta load_meta(const Meta* m, int64_t k) {
  const int4 v = *reinterpret_cast<const int4*>(m + k);
  return Meta{v.x, v.y, v.z, v.w};
}

}  // namespace sccg

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

// Wave reductions on the DPP network (no LDS traffic): pairs, quads, half
// rows, rows, then the row broadcasts; lane 63 ends with the result, which is
// returned to every lane (wave-uniform).  Lanes whose source is masked off
// read the identity, so the result is right for any exec mask as long as the
// inactive lanes are not needed.
#define SCCG_DPP_REDUCE(NAME, T, OP, ID)                                                 \
  __device__ __forceinline__ T NAME(T v) {                                               \
    const int id = (int)(ID);                                                            \
    int x = (int)v;                                                                      \
    x = (int)OP((T)x, (T)__builtin_amdgcn_update_dpp(id, x, 0xb1, 0xf, 0xf, false));     \
    x = (int)OP((T)x, (T)__builtin_amdgcn_update_dpp(id, x, 0x4e, 0xf, 0xf, false));     \
    x = (int)OP((T)x, (T)__builtin_amdgcn_update_dpp(id, x, 0x141, 0xf, 0xf, false));    \
    x = (int)OP((T)x, (T)__builtin_amdgcn_update_dpp(id, x, 0x140, 0xf, 0xf, false));    \
    x = (int)OP((T)x, (T)__builtin_amdgcn_update_dpp(id, x, 0x142, 0xa, 0xf, false));    \
    x = (int)OP((T)x, (T)__builtin_amdgcn_update_dpp(id, x, 0x143, 0xc, 0xf, false));    \
    return (T)__builtin_amdgcn_readlane(x, 63);                                          \
  }

__device__ __forceinline__ int32_t op_min_i32(int32_t a, int32_t b) { return a < b ? a : b; }
__device__ __forceinline__ int32_t op_max_i32(int32_t a, int32_t b) { return a > b ? a : b; }
__device__ __forceinline__ uint32_t op_add_u32(uint32_t a, uint32_t b) { return a + b; }
__device__ __forceinline__ uint32_t op_or_u32(uint32_t a, uint32_t b) { return a | b; }
__device__ __forceinline__ uint32_t op_xor_u32(uint32_t a, uint32_t b) { return a ^ b; }

typedef short sccg_short2 __attribute__((ext_vector_type(2)));
// lane-wise min / max of two packed int16 pairs (v_pk_min_i16 / v_pk_max_i16)
__device__ __forceinline__ uint32_t op_pkmin_i16(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(sccg_short2, a),
                                                                 __builtin_bit_cast(sccg_short2, b)));
}
__device__ __forceinline__ uint32_t op_pkmax_i16(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(sccg_short2, a),
                                                                 __builtin_bit_cast(sccg_short2, b)));
}

SCCG_DPP_REDUCE(wave_min_i32, int32_t, op_min_i32, 0x7fffffff)
SCCG_DPP_REDUCE(wave_max_i32, int32_t, op_max_i32, 0x80000000u)
SCCG_DPP_REDUCE(wave_sum_u32, uint32_t, op_add_u32, 0u)
SCCG_DPP_REDUCE(wave_or_u32, uint32_t, op_or_u32, 0u)
SCCG_DPP_REDUCE(wave_xor_u32, uint32_t, op_xor_u32, 0u)
SCCG_DPP_REDUCE(wave_pkmin_i16, uint32_t, op_pkmin_i16, 0x7fff7fffu)
SCCG_DPP_REDUCE(wave_pkmax_i16, uint32_t, op_pkmax_i16, 0x80008000u)

__device__ __forceinline__ uint64_t wave_or64(uint64_t v) {
  return ((uint64_t)wave_or_u32((uint32_t)(v >> 32)) << 32) | wave_or_u32((uint32_t)v);
}
__device__ __forceinline__ uint64_t wave_xor64(uint64_t v) {
  return ((uint64_t)wave_xor_u32((uint32_t)(v >> 32)) << 32) | wave_xor_u32((uint32_t)v);
}
// 64-bit sum from three 22-bit limbs (each limb sum stays below 2^28 for
// 64 lanes), carried back together exactly modulo 2^64
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  const uint64_t m = (1ull << 22) - 1;
  const uint64_t s0 = wave_sum_u32((uint32_t)(v & m));
  const uint64_t s1 = wave_sum_u32((uint32_t)((v >> 22) & m));
  const uint64_t s2 = wave_sum_u32((uint32_t)(v >> 44));
  return s0 + (s1 << 22) + (s2 << 44);
}

// hi - lo of a box side (lo <= hi): with coordinates up to 2^30 in size the
// difference can reach 2^31, which only the unsigned form holds
__device__ __forceinline__ uint32_t side_u(int32_t lo, int32_t hi) { return (uint32_t)hi - (uint32_t)lo; }

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

// Bounding box of MBR(p) ∪ MBR(q) (an empty MBR contributes nothing).
__device__ __forceinline__ Meta union_box(const Meta& p, const Meta& q) {
  Meta b;
  b.x0 = min(p.x0, q.x0);
  b.y0 = min(p.y0, q.y0);
  b.x1 = max(p.x1, q.x1);
  b.y1 = max(p.y1, q.y1);
  return b;
}

__device__ __forceinline__ Meta load_meta(const Meta* m, int64_t k) {
  const int4 v = *reinterpret_cast<const int4*>(m + k);
  return Meta{v.x, v.y, v.z, v.w};
}

}  // namespace sccg

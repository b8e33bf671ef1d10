// Exact sum of binary64 ratios in [0, 1] (the J' of Eq. 1 is the mean of
// the pair ratios): a 192-bit fixed-point integer in units of 2^-128.  A
// ratio I/U with I >= 1 and U < 2^63 is at least 2^-63, so its lowest
// mantissa bit is at least 2^-115 and the conversion is exact; the sum of up
// to 2^62 ratios stays below 2^191.  The sum does not depend on the order of
// the additions, so the device's tree reduction and a host loop over the
// same ratios give the same bits.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace sccg {

struct Fix192 {
  uint64_t w[3] = {0, 0, 0};  // little-endian limbs

  __host__ __device__ void add(const Fix192& o) {
    uint64_t c = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const uint64_t s = w[i] + o.w[i];
      const uint64_t c1 = s < w[i];
      const uint64_t s2 = s + c;
      const uint64_t c2 = s2 < s;
      w[i] = s2;
      c = c1 | c2;
    }
  }

  __host__ __device__ void add_ratio(double r) {
    if (!(r > 0.0)) return;
    const uint64_t bits = __builtin_bit_cast(uint64_t, r);
    const int e = (int)((bits >> 52) & 0x7ff);
    uint64_t m = bits & ((1ull << 52) - 1);
    if (e == 0) return;  // subnormal: impossible for a ratio >= 2^-63
    m |= 1ull << 52;
    // r = m * 2^(e - 1075); in 2^-128 units: m << (e - 1075 + 128)
    const int sh = e - 947;
    if (sh < 0) return;
    Fix192 t;
    const int limb = sh >> 6, off = sh & 63;
    if (limb < 3) t.w[limb] = m << off;
    if (off && limb + 1 < 3) t.w[limb + 1] = m >> (64 - off);
    add(t);
  }

  // Round to nearest binary64 (ties to even): the leading 64 bits with a
  // sticky bit for everything below are enough for one correct rounding.
  __host__ __device__ double to_double() const {
    int top = 2;
    while (top >= 0 && w[top] == 0) --top;
    if (top < 0) return 0.0;
    const int lz = __builtin_clzll(w[top]);
    const int msb = top * 64 + (63 - lz);  // bit index of the leading one
    const int lo_bit = msb - 63;           // bit index that lands in bit 0 of the lead
    if (lo_bit <= 0) return ldexp((double)w[0], -128);  // the whole value fits in 64 bits
    const int limb = lo_bit >> 6, off = lo_bit & 63;
    uint64_t lead = w[limb] >> off;
    if (off && limb + 1 < 3) lead |= w[limb + 1] << (64 - off);
    bool sticky = false;
    for (int i = 0; i < limb; ++i) sticky |= w[i] != 0;
    if (off) sticky |= (w[limb] & ((1ull << off) - 1)) != 0;
    lead |= sticky ? 1ull : 0ull;
    return ldexp((double)lead, lo_bit - 128);
  }
};

}  // namespace sccg

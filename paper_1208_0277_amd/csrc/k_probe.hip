// Diagnostics: the sustained VALU issue rate of the device, against which the
// persistent kernel's integer work is measured.
#include "sccg_common.h"

namespace sccg {

// Every lane runs eight independent chains of 32-bit integer adds and XORs,
// 32 operations per loop trip.  They are written as inline assembly so that
// the compiler can neither fold nor drop them; nothing is loaded.
__global__ void __launch_bounds__(256) k_valu_peak(int iters, unsigned long long* sink) {
  uint32_t a0 = threadIdx.x, a1 = a0 * 3u, a2 = a0 * 5u, a3 = a0 * 7u, a4 = a0 + 11u, a5 = a0 + 13u,
           a6 = a0 + 17u, a7 = a0 + 19u;
  const uint32_t k = blockIdx.x | 1u;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      asm volatile(
          "v_add_u32 %0, %0, %8\n\tv_add_u32 %1, %1, %8\n\tv_add_u32 %2, %2, %8\n\tv_add_u32 %3, %3, %8\n\t"
          "v_add_u32 %4, %4, %8\n\tv_add_u32 %5, %5, %8\n\tv_add_u32 %6, %6, %8\n\tv_add_u32 %7, %7, %8\n\t"
          "v_xor_b32 %0, %0, %8\n\tv_xor_b32 %1, %1, %8\n\tv_xor_b32 %2, %2, %8\n\tv_xor_b32 %3, %3, %8\n\t"
          "v_xor_b32 %4, %4, %8\n\tv_xor_b32 %5, %5, %8\n\tv_xor_b32 %6, %6, %8\n\tv_xor_b32 %7, %7, %8"
          : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
          : "v"(k));
    }
  }
  const uint32_t x = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
  if (x == 0xdeadbeefu) sink[0] = x;  // keeps the result observable; practically never stored
}

hipError_t launch_valu_peak(int grid, int iters, unsigned long long* sink, hipStream_t s) {
  hipLaunchKernelGGL(k_valu_peak, dim3(grid), dim3(256), 0, s, iters, sink);
  return hipGetLastError();
}

}  // namespace sccg

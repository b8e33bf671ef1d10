// PixelBox on the host CPU: the entry the serving path calls for jobs it
// moves off the device.
#pragma once

#include <stdint.h>

#include <atomic>

#include "sccg.h"

namespace sccg {

enum : uint32_t {
  kHostErrSide = 2u,   // a pair-box side above 32767: the pair gets (0, 0)
  kHostErrCoord = 4u,  // a ring with |coordinate| above 2^30: it covers nothing
};

// Counts of pairs (A[pa[k]], B[pb[k]]), k < n, on `threads` host threads;
// indices must already be checked.  Returns the kHostErr* bits seen.
uint32_t host_area_pairs(const sccg_polys* A, const sccg_polys* B, int64_t n, const int32_t* pa, const int32_t* pb,
                         int64_t* out_i, int64_t* out_u, int threads);

// The same work shared by any number of participants (threads of a pool):
// each calls host_area_worker, which takes chunks of 64 pairs from `next`
// until all n are done, and returns the kHostErr* bits it saw.
struct HostWork {
  const sccg_polys* A;
  const sccg_polys* B;
  const int32_t* pa;
  const int32_t* pb;
  int64_t* out_i;
  int64_t* out_u;
  int64_t n;
  std::atomic<int64_t> next{0};
};
uint32_t host_area_worker(HostWork& w);

}  // namespace sccg

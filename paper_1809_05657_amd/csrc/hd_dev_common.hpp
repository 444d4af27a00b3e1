// hd_dev_common.hpp — small device helpers shared by the data-path kernels:
// the float4 type, the 7 stencil weights, the XCD-aware workgroup order and
// the work-box lookup.
#pragma once
#include <hip/hip_runtime.h>

#include "hd_internal.hpp"

namespace hd {

typedef float f4 __attribute__((ext_vector_type(4)));

// Global-memory views of device buffers.  Loads through them compile to
// global (not flat) instructions, which count only against the vector-memory
// counter: a wait for an LDS operation (a cross-lane shuffle, an LDS read)
// then does not also wait for global loads still in flight.
typedef const float __attribute__((address_space(1))) gcf;
typedef const f4 __attribute__((address_space(1))) gcf4;
typedef float __attribute__((address_space(1))) gwf;
typedef f4 __attribute__((address_space(1))) gwf4;

struct Coef7 {
  float c[7];
};

// Flat tile index so that each XCD (workgroups are dealt round-robin over the
// 8 XCDs) walks a contiguous range of tiles: neighbouring tiles, which share
// halo rows, then hit the same L2.
__device__ inline int64_t xcd_remap(int64_t bid, int64_t ntiles) {
  const int64_t q = ntiles >> 3, r = ntiles & 7;
  const int64_t x = bid & 7, k = bid >> 3;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

__device__ inline int find_box(const WorkBox *__restrict__ wb, int nbox, int64_t t) {
  int lo = 0, hi = nbox - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wb[mid].tile0 <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

}  // namespace hd

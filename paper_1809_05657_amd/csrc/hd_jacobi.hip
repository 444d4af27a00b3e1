// hd_jacobi.hip — the per-call Jacobi / lower-triangular kernels over every
// logical device's work box in one launch (device code in hd_dev_jacobi.hpp).
// Two workgroup shapes: four waves walking a row of tiles, or one wave per
// workgroup with the tiles of an XCD walking down columns; the runtime picks
// one by timing both on real calls.
#include <hip/hip_runtime.h>

#include "hd_dev_jacobi.hpp"

namespace hd {

// Four waves per workgroup, one tile each (4 x 256 columns of the same rows).
template <int TH, bool TRI>
__global__ __launch_bounds__(256) void k_jacobi(const WorkBox *__restrict__ wb, int nbox,
                                                const ArrDev *__restrict__ A, int64_t ntiles) {
  const int64_t nwg = (ntiles + 3) >> 2;
  const int64_t t = xcd_remap(blockIdx.x, nwg) * 4 + (threadIdx.x >> 6);
  if (t >= ntiles) return;
  const WorkBox B = wb[find_box(wb, nbox, t)];
  dev_jacobi_tile<TH, TRI, true>(B, t - B.tile0, A);
}

// One wave per workgroup; the tiles of an XCD walk down columns of tiles.
template <int TH, bool TRI>
__global__ __launch_bounds__(64) void k_jacobi1(const WorkBox *__restrict__ wb, int nbox,
                                                const ArrDev *__restrict__ A, int64_t ntiles) {
  const int64_t t = xcd_remap(blockIdx.x, ntiles);
  const WorkBox B = wb[find_box(wb, nbox, t)];
  dev_jacobi_tile<TH, TRI, false>(B, t - B.tile0, A);
}

hipError_t launch_jacobi(bool tri, int th, int waves, const WorkBox *wb, int nbox, const ArrDev *A, int64_t ntiles,
                         hipStream_t s) {
  typedef void (*jk_t)(const WorkBox *, int, const ArrDev *, int64_t);
  if (waves == 4) {
    jk_t k = tri ? k_jacobi<8, true> : k_jacobi<8, false>;
    if (th == 4) k = tri ? k_jacobi<4, true> : k_jacobi<4, false>;
    if (th == 16) k = tri ? k_jacobi<16, true> : k_jacobi<16, false>;
    hipLaunchKernelGGL(k, dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, s, wb, nbox, A, ntiles);
  } else {
    jk_t k = tri ? k_jacobi1<8, true> : k_jacobi1<8, false>;
    if (th == 4) k = tri ? k_jacobi1<4, true> : k_jacobi1<4, false>;
    if (th == 16) k = tri ? k_jacobi1<16, true> : k_jacobi1<16, false>;
    hipLaunchKernelGGL(k, dim3((unsigned)ntiles), dim3(64), 0, s, wb, nbox, A, ntiles);
  }
  return hipGetLastError();
}

}  // namespace hd

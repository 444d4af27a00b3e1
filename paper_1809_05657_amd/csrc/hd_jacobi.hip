// hd_jacobi.hip — the per-call Jacobi / lower-triangular / 3 x 3
// convolution kernels over every logical device's work box in one launch
// (device code in hd_dev_jacobi.hpp).
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

// The 3 x 3 convolution on the same two workgroup shapes.
template <int TH>
__global__ __launch_bounds__(256) void k_conv(const WorkBox *__restrict__ wb, int nbox, const ArrDev *__restrict__ A,
                                              int64_t ntiles, Coef9 w) {
  const int64_t nwg = (ntiles + 3) >> 2;
  const int64_t t = xcd_remap(blockIdx.x, nwg) * 4 + (threadIdx.x >> 6);
  if (t >= ntiles) return;
  const WorkBox B = wb[find_box(wb, nbox, t)];
  dev_conv_tile<TH, true>(B, t - B.tile0, A, w);
}

template <int TH>
__global__ __launch_bounds__(64) void k_conv1(const WorkBox *__restrict__ wb, int nbox, const ArrDev *__restrict__ A,
                                              int64_t ntiles, Coef9 w) {
  const int64_t t = xcd_remap(blockIdx.x, ntiles);
  const WorkBox B = wb[find_box(wb, nbox, t)];
  dev_conv_tile<TH, false>(B, t - B.tile0, A, w);
}

hipError_t launch_conv(int th, int waves, const WorkBox *wb, int nbox, const ArrDev *A, int64_t ntiles,
                       const float *coef, hipStream_t s) {
  typedef void (*ck_t)(const WorkBox *, int, const ArrDev *, int64_t, Coef9);
  Coef9 w;
  for (int e = 0; e < 9; ++e) w.w[e] = coef ? coef[e] : 0.f;
  if (waves == 4) {
    ck_t k = th == 4 ? k_conv<4> : th == 16 ? k_conv<16> : k_conv<8>;
    hipLaunchKernelGGL(k, dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, s, wb, nbox, A, ntiles, w);
  } else {
    ck_t k = th == 4 ? k_conv1<4> : th == 16 ? k_conv1<16> : k_conv1<8>;
    hipLaunchKernelGGL(k, dim3((unsigned)ntiles), dim3(64), 0, s, wb, nbox, A, ntiles, w);
  }
  return hipGetLastError();
}

}  // namespace hd

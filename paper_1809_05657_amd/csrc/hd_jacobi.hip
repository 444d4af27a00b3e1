// hd_jacobi.hip — the per-call Jacobi / lower-triangular / 3 x 3
// convolution kernels over every logical device's work box in one launch
// (device code in hd_dev_jacobi.hpp).
// Workgroup shapes: four waves stacked down a tile (halo rows shared through
// LDS), one wave per tile (tiles of an XCD along rows or down columns), or
// tall one-wave strips; the runtime picks one by timing them on real calls.
#include <hip/hip_runtime.h>

#include "hd_dev_jacobi.hpp"

namespace hd {

// Four waves stacked down a tile of 4*TH rows x 256 columns, halo rows
// shared through LDS (OP: 0 Jacobi, 1 triangular, 2 convolution; VEC: all
// boxes float4-aligned).
template <int TH, int OP, bool VEC>
__global__ __launch_bounds__(256) void k_stack(const WorkBox *__restrict__ wb, int nbox,
                                               const ArrDev *__restrict__ A, int64_t ntiles, Coef9 w) {
  const int64_t t = xcd_remap(blockIdx.x, ntiles);
  const WorkBox B = wb[find_box(wb, nbox, t)];
  dev_stack_tile<4, TH, OP, VEC>(B, t - B.tile0, A, w);
}

// The same tiles with the boxes and buffers in the kernel arguments (float4
// rows, at most kArgBoxes boxes).
template <int TH, int OP>
__global__ __launch_bounds__(256) void k_stack_a(StackArgs a, int64_t ntiles, Coef9 w) {
  const int64_t t = xcd_remap(blockIdx.x, ntiles);
  int b = 0;
#pragma unroll
  for (int k = 1; k < kArgBoxes; ++k)
    if (k < a.nbox && a.tile0[k] <= t) b = k;
  WorkBox B;
  B.lo[1] = a.lo1[b];
  B.lo[2] = a.lo2[b];
  B.hi[1] = a.hi1[b];
  B.hi[2] = a.hi2[b];
  dev_stack_tile_p<4, TH, OP, true>(B, t - a.tile0[b], (gcf *)a.in[b], a.rsi[b], (gwf *)a.out[b], a.rso[b], a.N1, a.N2, w);
}

hipError_t launch_stack_args(int op, int th, const StackArgs &a, int64_t ntiles, const float *coef, hipStream_t s) {
  typedef void (*ak_t)(StackArgs, int64_t, Coef9);
  Coef9 w;
  for (int e = 0; e < 9; ++e) w.w[e] = coef ? coef[e] : 0.f;
  ak_t k;
  if (th == 4) k = op == 0 ? k_stack_a<4, 0> : op == 1 ? k_stack_a<4, 1> : k_stack_a<4, 2>;
  else if (th == 8) k = op == 0 ? k_stack_a<8, 0> : op == 1 ? k_stack_a<8, 1> : k_stack_a<8, 2>;
  else k = op == 0 ? k_stack_a<16, 0> : op == 1 ? k_stack_a<16, 1> : k_stack_a<16, 2>;
  if (ntiles > 0) hipLaunchKernelGGL(k, dim3((unsigned)ntiles), dim3(256), 0, s, a, ntiles, w);
  return hipGetLastError();
}

template <int TH, bool VEC>
static void *stack_kernel(int op) {
  return op == 0 ? (void *)k_stack<TH, 0, VEC> : op == 1 ? (void *)k_stack<TH, 1, VEC> : (void *)k_stack<TH, 2, VEC>;
}

static hipError_t launch_stack(int op, int th, bool vec, const WorkBox *wb, int nbox, const ArrDev *A, int64_t ntiles,
                               const Coef9 &w, hipStream_t s) {
  typedef void (*sk_t)(const WorkBox *, int, const ArrDev *, int64_t, Coef9);
  void *k;
  if (th == 4) k = vec ? stack_kernel<4, true>(op) : stack_kernel<4, false>(op);
  else if (th == 8) k = vec ? stack_kernel<8, true>(op) : stack_kernel<8, false>(op);
  else k = vec ? stack_kernel<16, true>(op) : stack_kernel<16, false>(op);
  hipLaunchKernelGGL((sk_t)k, dim3((unsigned)ntiles), dim3(256), 0, s, wb, nbox, A, ntiles, w);
  return hipGetLastError();
}

// One wave per workgroup; the tiles of an XCD walk along rows of tiles (HF)
// or down columns of tiles.
template <int TH, bool TRI, bool HF>
__global__ __launch_bounds__(64) void k_jacobi1(const WorkBox *__restrict__ wb, int nbox,
                                                const ArrDev *__restrict__ A, int64_t ntiles) {
  const int64_t t = xcd_remap(blockIdx.x, ntiles);
  const WorkBox B = wb[find_box(wb, nbox, t)];
  dev_jacobi_tile<TH, TRI, HF>(B, t - B.tile0, A);
}

// Tall strips (32 or 64 rows, one wave each) streaming through a register
// window of 8 rows; the strips of an XCD walk down columns.
template <int TS, int OP>
__global__ __launch_bounds__(64) void k_strip(const WorkBox *__restrict__ wb, int nbox, const ArrDev *__restrict__ A,
                                              int64_t ntiles, Coef9 w) {
  const int64_t t = xcd_remap(blockIdx.x, ntiles);
  const WorkBox B = wb[find_box(wb, nbox, t)];
  dev_strip<TS, 8, OP, false>(B, t - B.tile0, A, w);
}

static hipError_t launch_strip(int op, int th, const WorkBox *wb, int nbox, const ArrDev *A, int64_t ntiles,
                               const Coef9 &w, hipStream_t s) {
  typedef void (*sk_t)(const WorkBox *, int, const ArrDev *, int64_t, Coef9);
  sk_t k = th == 64 ? (op == 0 ? k_strip<64, 0> : op == 1 ? k_strip<64, 1> : k_strip<64, 2>)
                    : (op == 0 ? k_strip<32, 0> : op == 1 ? k_strip<32, 1> : k_strip<32, 2>);
  hipLaunchKernelGGL(k, dim3((unsigned)ntiles), dim3(64), 0, s, wb, nbox, A, ntiles, w);
  return hipGetLastError();
}

hipError_t launch_jacobi(bool tri, int th, int waves, int order, bool vec, const WorkBox *wb, int nbox,
                         const ArrDev *A, int64_t ntiles, hipStream_t s) {
  typedef void (*jk_t)(const WorkBox *, int, const ArrDev *, int64_t);
  if (th >= 32) return launch_strip(tri ? 1 : 0, th, wb, nbox, A, ntiles, Coef9{}, s);
  if (waves == 4) return launch_stack(tri ? 1 : 0, th, vec, wb, nbox, A, ntiles, Coef9{}, s);
  if (order) {
    jk_t k = tri ? k_jacobi1<8, true, true> : k_jacobi1<8, false, true>;
    if (th == 4) k = tri ? k_jacobi1<4, true, true> : k_jacobi1<4, false, true>;
    if (th == 16) k = tri ? k_jacobi1<16, true, true> : k_jacobi1<16, false, true>;
    hipLaunchKernelGGL(k, dim3((unsigned)ntiles), dim3(64), 0, s, wb, nbox, A, ntiles);
  } else {
    jk_t k = tri ? k_jacobi1<8, true, false> : k_jacobi1<8, false, false>;
    if (th == 4) k = tri ? k_jacobi1<4, true, false> : k_jacobi1<4, false, false>;
    if (th == 16) k = tri ? k_jacobi1<16, true, false> : k_jacobi1<16, false, false>;
    hipLaunchKernelGGL(k, dim3((unsigned)ntiles), dim3(64), 0, s, wb, nbox, A, ntiles);
  }
  return hipGetLastError();
}

// The 3 x 3 convolution on the same workgroup shapes.
template <int TH, bool HF>
__global__ __launch_bounds__(64) void k_conv1(const WorkBox *__restrict__ wb, int nbox, const ArrDev *__restrict__ A,
                                              int64_t ntiles, Coef9 w) {
  const int64_t t = xcd_remap(blockIdx.x, ntiles);
  const WorkBox B = wb[find_box(wb, nbox, t)];
  dev_conv_tile<TH, HF>(B, t - B.tile0, A, w);
}

hipError_t launch_conv(int th, int waves, int order, bool vec, const WorkBox *wb, int nbox, const ArrDev *A,
                       int64_t ntiles, const float *coef, hipStream_t s) {
  typedef void (*ck_t)(const WorkBox *, int, const ArrDev *, int64_t, Coef9);
  Coef9 w;
  for (int e = 0; e < 9; ++e) w.w[e] = coef ? coef[e] : 0.f;
  if (th >= 32) return launch_strip(2, th, wb, nbox, A, ntiles, w, s);
  if (waves == 4) return launch_stack(2, th, vec, wb, nbox, A, ntiles, w, s);
  if (order) {
    ck_t k = th == 4 ? k_conv1<4, true> : th == 16 ? k_conv1<16, true> : k_conv1<8, true>;
    hipLaunchKernelGGL(k, dim3((unsigned)ntiles), dim3(64), 0, s, wb, nbox, A, ntiles, w);
  } else {
    ck_t k = th == 4 ? k_conv1<4, false> : th == 16 ? k_conv1<16, false> : k_conv1<8, false>;
    hipLaunchKernelGGL(k, dim3((unsigned)ntiles), dim3(64), 0, s, wb, nbox, A, ntiles, w);
  }
  return hipGetLastError();
}

}  // namespace hd

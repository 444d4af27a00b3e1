// hd_meta.hip — per-phase kernels of the communication-set derivation
// (Sec. 2.2, Eq. 1-2) and the GDEF update (Eq. 3-4); the device code is in
// hd_dev_meta.hpp and shared with the persistent batched kernel.
#include <hip/hip_runtime.h>

#include "hd_dev_meta.hpp"

namespace hd {

constexpr int kRunWaves = 4;
constexpr int kGdefMaxB = 1024;

__global__ __launch_bounds__(256) void k_runs(PlanDev P, const ArrDev *__restrict__ A, Work W) {
  __shared__ Ivl s_iv[kRunWaves][kMaxCap];
  __shared__ Item s_run[kRunWaves][kMaxRunsRow];
  const int wv = threadIdx.x >> 6;
  for (int s = blockIdx.x * kRunWaves + wv; s < P.nsl1; s += gridDim.x * kRunWaves)
    dev_runs(P, A, W, s, s_iv[wv], s_run[wv]);
}

__global__ __launch_bounds__(256) void k_bandflags(Level L) { dev_bandflags(L, blockIdx.x * blockDim.x + threadIdx.x); }

__global__ __launch_bounds__(1024) void k_bandscan(Level L) { dev_bandscan(L); }

__global__ __launch_bounds__(256) void k_heads(Level L, int32_t *err) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < *L.nb) dev_heads(L, b, err);
}

__global__ __launch_bounds__(1024) void k_compact(PlanDev P, Level L, Work W, MsgRec *out, MsgHdr *hdr,
                                                  int64_t out_cap, int mode) {
  dev_compact(P, L, W, out, hdr, out_cap, mode);
}

// rows with at most 64 boundaries, register-only; larger rows are listed
__global__ __launch_bounds__(256) void k_gdef(PlanDev P, ArrDev *__restrict__ A, Work W) {
  const int wv = threadIdx.x >> 6;
  for (int t = blockIdx.x * 4 + wv; t < P.ngrow; t += gridDim.x * 4) {
    if (!dev_gdef_row_fast(P, A, W, t) && (threadIdx.x & 63) == 0) W.ovf_list[atomicAdd(W.ovf_cnt, 1)] = t;
  }
}

// the listed large rows, one wave each with LDS scratch; resets the list
__global__ __launch_bounds__(64) void k_gdef_large(PlanDev P, ArrDev *__restrict__ A, Work W) {
  __shared__ Ivl s_iv[kMaxCap];
  __shared__ int32_t s_b[kGdefMaxB], s_u[kGdefMaxB], s_own[kGdefMaxB];
  __shared__ uint64_t s_hold[kGdefMaxB];
  GdefLds S{s_iv, s_b, s_u, s_own, s_hold};
  const int cnt = *W.ovf_cnt;
  for (int q = blockIdx.x; q < cnt; q += gridDim.x) dev_gdef_row(P, A, W, W.ovf_list[q], S, kGdefMaxB);
}

__global__ void k_zero_ovf(int32_t *c) {
  if (threadIdx.x == 0) *c = 0;
}

// Every row starts as one interval [0, n2) owned and held by the host.
__global__ void k_init_rows(Ivl *ivl, int32_t *cnt, int64_t rows, int cap) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < rows; g += (int64_t)gridDim.x * blockDim.x) {
    ivl[g * cap] = Ivl{0, kHost, 1ull << kHost};
    cnt[g] = 1;
  }
}

// ------------------------------------------------------------- launchers
static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

hipError_t launch_runs(const PlanDev &P, const ArrDev *A, const Work &W, hipStream_t s) {
  if (P.nsl1 == 0) return hipSuccess;
  int grid = cdiv(P.nsl1, kRunWaves);
  if (grid > 8192) grid = 8192;
  hipLaunchKernelGGL(k_runs, dim3(grid), dim3(256), 0, s, P, A, W);
  return hipGetLastError();
}

hipError_t launch_level(const Level &L, int32_t *err, hipStream_t s) {
  if (L.nsl == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bandflags, dim3(cdiv(L.nsl, 256)), dim3(256), 0, s, L);
  hipLaunchKernelGGL(k_bandscan, dim3(1), dim3(1024), 0, s, L);
  hipLaunchKernelGGL(k_heads, dim3(cdiv(L.nsl, 256)), dim3(256), 0, s, L, err);
  return hipGetLastError();
}

hipError_t launch_compact(const PlanDev &P, const Level &L, const Work &W, MsgRec *out, MsgHdr *hdr,
                          int64_t cap, int mode, hipStream_t s) {
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, s, P, L, W, out, hdr, cap, mode);
  return hipGetLastError();
}

hipError_t launch_init_rows(Ivl *ivl, int32_t *cnt, int64_t rows, int cap, hipStream_t s) {
  int grid = cdiv(rows, 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_init_rows, dim3(grid), dim3(256), 0, s, ivl, cnt, rows, cap);
  return hipGetLastError();
}

hipError_t launch_gdef(const PlanDev &P, ArrDev *A, const Work &W, hipStream_t s) {
  if (P.ngrow == 0) return hipSuccess;
  int grid = cdiv(P.ngrow, 4);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_gdef, dim3(grid), dim3(256), 0, s, P, A, W);
  hipLaunchKernelGGL(k_gdef_large, dim3(256), dim3(64), 0, s, P, A, W);
  hipLaunchKernelGGL(k_zero_ovf, dim3(1), dim3(64), 0, s, W.ovf_cnt);
  return hipGetLastError();
}

}  // namespace hd

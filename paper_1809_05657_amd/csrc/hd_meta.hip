// hd_meta.hip — per-phase kernels of the communication-set derivation
// (Sec. 2.2, Eq. 1-2) and the GDEF update (Eq. 3-4); the device code is in
// hd_dev_meta.hpp and shared with the persistent batched kernel.
#include <hip/hip_runtime.h>

#include "hd_dev_meta.hpp"

namespace hd {

constexpr int kGdefMaxB = 1024;

// Runs of 4 consecutive use rows per workgroup plus the row before them
// (fifth wave, only to compare with): each row's band-start flag comes from
// comparing sorted run lists in LDS.  (No workgroup here waits for the
// others: a device-wide fence per workgroup costs more than a launch.)
constexpr int kRfWaves = 5;
template <int CAP>
__global__ __launch_bounds__(64 * kRfWaves) void k_runs_flags(PlanDev P, const ArrDev *__restrict__ A, Work W,
                                                              Level L, uint8_t *flag) {
  __shared__ Ivl s_iv[kRfWaves][CAP];
  __shared__ Run s_run[kRfWaves][kMaxRunsRow];
  __shared__ int s_nr[kRfWaves];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s0 = blockIdx.x * 4;
  const int s = wv < 4 ? s0 + wv : s0 - 1;
  bool work = s >= 0 && s < P.nsl1;
  if (wv == 4) work = work && L.grp[s0] == L.grp[s] && L.pos[s0] == L.pos[s] + 1;
  int nr = 0;
  if (work) {
    nr = dev_runs_find(P, A, W, s, s_iv[wv], s_run[wv]);
    if (wv < 4) dev_runs_store(P, W, s, s_run[wv], nr);
  }
  if (lane == 0) s_nr[wv] = nr;
  __syncthreads();
  if (wv < 4 && work) {
    const int pw = wv == 0 ? 4 : wv - 1;
    const bool st = runs_band_start(L, s, s_run[wv], nr, s_run[pw], s_nr[pw]);
    if (lane == 0) flag[s] = st ? 1 : 0;
  }
}

// Band masks from the flags, then the band scan (one workgroup).
__global__ __launch_bounds__(1024) void k_flags_scan(Level L, const uint8_t *flag) {
  const int nch = (L.nsl + 63) / 64;
  for (int c = threadIdx.x; c < nch; c += blockDim.x) dev_mask_from_flags(L, flag, c);
  __syncthreads();
  dev_bandscan(L);
}

__global__ __launch_bounds__(256) void k_bandflags(Level L) { dev_bandflags(L, blockIdx.x * blockDim.x + threadIdx.x); }

__global__ __launch_bounds__(1024) void k_bandscan(Level L) { dev_bandscan(L); }

// Heads of every band, one wave per band.
__global__ __launch_bounds__(256) void k_heads(Level L) {
  const int nb = *L.nb;
  for (int b = blockIdx.x * 4 + (threadIdx.x >> 6); b < nb; b += gridDim.x * 4) dev_heads(L, b);
}

__global__ __launch_bounds__(256) void k_compact(PlanDev P, Level L, Work W, MsgRec *out, MsgHdr *hdr,
                                                  int64_t out_cap, int mode) {
  dev_compact(P, L, W, out, hdr, out_cap, mode);
}

// Rows with at most 64 boundaries are updated register-only, one wave each;
// larger rows are listed for k_gdef_large.
__global__ __launch_bounds__(256) void k_gdef(PlanDev P, ArrDev *__restrict__ A, Work W) {
  const int wv = threadIdx.x >> 6;
  for (int t = blockIdx.x * 4 + wv; t < P.ngrow; t += gridDim.x * 4) {
    if (!dev_gdef_row_fast(P, A, W, t) && (threadIdx.x & 63) == 0) W.ovf_list[atomicAdd(W.ovf_cnt, 1)] = t;
  }
}

// The listed large rows, one wave each with LDS scratch (such rows are
// rare, so the grid is small); the last workgroup clears the list.
constexpr int kGdefLargeGrid = 32;
__global__ __launch_bounds__(64) void k_gdef_large(PlanDev P, ArrDev *__restrict__ A, Work W) {
  __shared__ Ivl s_iv[kMaxCap];
  __shared__ int32_t s_b[kGdefMaxB], s_u[kGdefMaxB], s_own[kGdefMaxB];
  __shared__ uint64_t s_hold[kGdefMaxB];
  GdefLds S{s_iv, s_b, s_u, s_own, s_hold};
  const int cnt = *W.ovf_cnt;
  for (int q = blockIdx.x; q < cnt; q += gridDim.x) dev_gdef_row(P, A, W, W.ovf_list[q], S, kGdefMaxB);
  if (last_workgroup(W.ovf_cnt + 1)) *W.ovf_cnt = 0;
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

hipError_t launch_compact(const PlanDev &P, const Level &L, const Work &W, MsgRec *out, MsgHdr *hdr,
                          int64_t cap, int mode, hipStream_t s);

// level 1: runs + band flags, band scan, heads, compaction
hipError_t launch_level1(const PlanDev &P, const ArrDev *A, const Work &W, const Level &L, uint8_t *flag,
                         MsgRec *out, MsgHdr *hdr, int64_t cap, int mode, int row_cap, hipStream_t s) {
  if (P.nsl1 == 0) return launch_compact(P, L, W, out, hdr, cap, mode, s);
  // LDS for the row's intervals sized to the row capacity (more workgroups
  // per CU at the default capacity)
  if (row_cap <= 64)
    hipLaunchKernelGGL(k_runs_flags<64>, dim3(cdiv(P.nsl1, 4)), dim3(64 * kRfWaves), 0, s, P, A, W, L, flag);
  else
    hipLaunchKernelGGL(k_runs_flags<kMaxCap>, dim3(cdiv(P.nsl1, 4)), dim3(64 * kRfWaves), 0, s, P, A, W, L, flag);
  hipLaunchKernelGGL(k_flags_scan, dim3(1), dim3(1024), 0, s, L, flag);
  int hg = cdiv(L.nsl, 4);
  if (hg > 2048) hg = 2048;
  hipLaunchKernelGGL(k_heads, dim3(hg), dim3(256), 0, s, L);
  return launch_compact(P, L, W, out, hdr, cap, mode, s);
}

// level 2 (stacking rectangles across planes): band flags, band scan, then
// heads + compaction
hipError_t launch_level2(const PlanDev &P, const Work &W, const Level &L, MsgRec *out, MsgHdr *hdr, int64_t cap,
                         hipStream_t s) {
  if (L.nsl == 0) return launch_compact(P, L, W, out, hdr, cap, 2, s);
  hipLaunchKernelGGL(k_bandflags, dim3(cdiv(L.nsl, 256)), dim3(256), 0, s, L);
  hipLaunchKernelGGL(k_bandscan, dim3(1), dim3(1024), 0, s, L);
  int hg = cdiv(L.nsl, 4);
  if (hg > 2048) hg = 2048;
  hipLaunchKernelGGL(k_heads, dim3(hg), dim3(256), 0, s, L);
  return launch_compact(P, L, W, out, hdr, cap, 2, s);
}

hipError_t launch_compact(const PlanDev &P, const Level &L, const Work &W, MsgRec *out, MsgHdr *hdr,
                          int64_t cap, int mode, hipStream_t s) {
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(256), 0, s, P, L, W, out, hdr, cap, mode);
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
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_gdef, dim3(grid), dim3(256), 0, s, P, A, W);
  hipLaunchKernelGGL(k_gdef_large, dim3(kGdefLargeGrid), dim3(64), 0, s, P, A, W);
  return hipGetLastError();
}

}  // namespace hd

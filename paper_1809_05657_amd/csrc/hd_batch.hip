// hd_batch.hip — one persistent launch for a batch of independent
// ApplyKernel calls (many arrays of uneven sizes and partition counts).
//
// Phases (the same device functions as the per-call kernels, so results are
// identical bit for bit), separated by grid-wide barriers:
//   runs -> band flags -> band scan (block 0) -> heads -> compact (block 0)
//   [-> level-2 stacking for 3-D arrays] -> pack + GDEF update -> unpack
//   -> user kernels (Jacobi / triangular / copy tiles of every box).
// The barrier spins with a bounded wait on the device clock: if a barrier
// does not complete within the limit (workgroups not co-resident), the
// kernel records an error and every workgroup leaves, so the launch always
// finishes.  The grid is sized to the co-resident capacity of the chip.
#include <hip/hip_runtime.h>

#include "hd_dev_data.hpp"
#include "hd_dev_meta.hpp"

namespace hd {

constexpr int kBWaves = 4;
constexpr int kBatchMaxB = 512;  // boundaries of one GDEF row update in a batch

// per-wave LDS: union of the runs scratch and the GDEF scratch
struct RunsLds {
  Ivl iv[kMaxCap];
  Run rr[kMaxRunsRow];
};
struct GdefLdsB {
  Ivl iv[kMaxCap];
  int32_t b[kBatchMaxB], u[kBatchMaxB], own[kBatchMaxB];
  uint64_t hold[kBatchMaxB];
};
union WaveLds {
  RunsLds r;
  GdefLdsB g;
};

// Grid barrier on a monotonically increasing counter (zeroed before the
// launch).  Returns false if the run was abandoned (timeout or earlier error).
__device__ inline bool grid_sync(unsigned *bar, unsigned nblk, unsigned &target, int32_t *err, int64_t limit) {
  __shared__ int s_ok;
  __syncthreads();
  target += nblk;
  if (threadIdx.x == 0) {
    __threadfence();
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t t0 = wall_clock64();
    int ok = 1;
    while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == -9 ||
          wall_clock64() - t0 > limit) {
        atomicCAS(err, 0, -9);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

template <int TH, int PW>
__global__ __launch_bounds__(256) void k_batch(BatchArgs B) {
  __shared__ WaveLds s_lds[kBWaves];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const unsigned nblk = gridDim.x;
  const int gw = blockIdx.x * kBWaves + wv, nw = gridDim.x * kBWaves;
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, gs = (int64_t)gridDim.x * blockDim.x;
  unsigned target = 0;
  WaveLds &my = s_lds[wv];
  int32_t *err = B.W.err;
  int ph = 0;
  auto stamp = [&]() {
    if (blockIdx.x == 0 && threadIdx.x == 0) B.clk[ph] = wall_clock64();
    ++ph;
  };
  stamp();
  // runs of every use row
  for (int s = gw; s < B.P.nsl1; s += nw) dev_runs(B.P, B.A, B.W, s, my.r.iv, my.r.rr);
  if (!grid_sync(B.bar, nblk, target, err, B.spin_limit)) return;
  stamp();
  for (int c = gw; c * 64 < B.L1.nsl; c += nw) dev_bandflags(B.L1, c * 64 + lane);
  if (!grid_sync(B.bar, nblk, target, err, B.spin_limit)) return;
  stamp();
  if (blockIdx.x == 0 && B.L1.nsl) dev_bandscan(B.L1);
  if (!grid_sync(B.bar, nblk, target, err, B.spin_limit)) return;
  stamp();
  {
    const int nb = B.L1.nsl ? *B.L1.nb : 0;
    for (int b = gw; b < nb; b += nw) dev_heads(B.L1, b);
  }
  if (!grid_sync(B.bar, nblk, target, err, B.spin_limit)) return;
  stamp();
  if (!B.P.has3d) {
    if (blockIdx.x == 0) dev_compact(B.P, B.L1, B.W, B.tab, B.hdr, B.tab_cap, 0);
  } else {
    if (blockIdx.x == 0) dev_compact(B.P, B.L1, B.W, B.tab, B.hdr, B.tab_cap, 1);
    if (!grid_sync(B.bar, nblk, target, err, B.spin_limit)) return;
    stamp();
    for (int c = gw; c * 64 < B.L2.nsl; c += nw) dev_bandflags(B.L2, c * 64 + lane);
    if (!grid_sync(B.bar, nblk, target, err, B.spin_limit)) return;
    stamp();
    if (blockIdx.x == 0 && B.L2.nsl) dev_bandscan(B.L2);
    if (!grid_sync(B.bar, nblk, target, err, B.spin_limit)) return;
    stamp();
    {
      const int nb = B.L2.nsl ? *B.L2.nb : 0;
      for (int b = gw; b < nb; b += nw) dev_heads(B.L2, b);
    }
    if (!grid_sync(B.bar, nblk, target, err, B.spin_limit)) return;
    stamp();
    if (blockIdx.x == 0) dev_compact(B.P, B.L2, B.W, B.tab, B.hdr, B.tab_cap, 2);
  }
  if (!grid_sync(B.bar, nblk, target, err, B.spin_limit)) return;
  stamp();
  // pack + unpack in one pass, and the GDEF update (metadata only,
  // independent of the data)
  const int64_t nmsg = B.hdr->nmsg, words = B.hdr->bytes >> 2;
  {
    int m = 0;
    for (int64_t q = gt; q * PW < words; q += gs)
#pragma unroll
      for (int e = 0; e < PW; ++e)
        if (q * PW + e < words) dev_pack_word(B.tab, nmsg, B.A, B.stg, 2, q * PW + e, m);
  }
  {
    GdefLds S{my.g.iv, my.g.b, my.g.u, my.g.own, my.g.hold};
    for (int t = gw; t < B.P.ngrow; t += nw)
      if (!dev_gdef_row_fast(B.P, B.A, B.W, t)) dev_gdef_row(B.P, B.A, B.W, t, S, kBatchMaxB);
  }
  if (!grid_sync(B.bar, nblk, target, err, B.spin_limit)) return;
  stamp();
  // user kernels: one wave per tile
  for (int64_t t = gw; t < B.ntiles; t += nw) {
    const WorkBox bx = B.wb[find_box(B.wb, B.nbox, t)];
    if (bx.kind == 1)
      dev_jacobi_tile<TH, false>(bx, t - bx.tile0, B.A);
    else if (bx.kind == 5)
      dev_jacobi_tile<TH, true>(bx, t - bx.tile0, B.A);
    else if (bx.kind == 2)
      dev_copy_tile(bx, t - bx.tile0, B.A);
  }
  stamp();
}

__global__ void k_zero_bar(unsigned *bar) {
  if (threadIdx.x == 0) *bar = 0u;
}

typedef void (*batch_kernel_t)(BatchArgs);

static batch_kernel_t pick(int th, int pw) {
  if (th == 4) return pw == 4 ? k_batch<4, 4> : k_batch<4, 1>;
  if (th == 16) return pw == 4 ? k_batch<16, 4> : k_batch<16, 1>;
  return pw == 4 ? k_batch<8, 4> : k_batch<8, 1>;
}

int batch_max_blocks(int th, int pw) {
  int dev = 0, ncu = 0, occ = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)pick(th, pw), 256, 0) != hipSuccess)
    return -1;
  if (occ < 1) occ = 1;
  if (occ > 2) occ = 2;
  return ncu * occ;
}

// the step as two nodes on one stream: zero the barrier, run the batch
hipError_t launch_batch(const BatchArgs &a, int th, int pw, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_bar, dim3(1), dim3(64), 0, s, a.bar);
  hipLaunchKernelGGL(pick(th, pw), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

int batch_args_size() { return (int)sizeof(BatchArgs); }

}  // namespace hd

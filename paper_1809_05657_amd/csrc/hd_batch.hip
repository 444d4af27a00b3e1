// hd_batch.hip — one persistent launch for a batch of independent
// ApplyKernel calls (many arrays of uneven sizes and partition counts).
//
// Phases (the same device functions as the per-call kernels, so results are
// identical bit for bit), separated by grid-wide barriers:
//   runs -> band flags -> band scan (every block, redundantly) and heads,
//   with no barrier between them -> compaction (three
//   phases: chunk scans, then prefixes and padding in every block and the
//   writes, without a barrier between those two)
//   [3-D arrays: level-1 compaction in block 0, then level-2 stacking]
//   -> pack + unpack (one pass) with the GDEF update.
// The user kernels (Jacobi / triangular / copy tiles of every box) follow
// as a second launch in the same graph, one wave per tile as in the
// per-call kernels: the persistent grid keeps only a few waves per CU
// (its workgroups must all be resident for the barriers), too few loads in
// flight for the stencils, while a one-wave launch fills every CU.
// The barrier spins with a bounded wait on the device clock: if a barrier
// does not complete within the limit (workgroups not co-resident), the
// kernel records an error and every workgroup leaves, so the launch always
// finishes.  The grid is sized to the co-resident capacity of the chip.
#include <hip/hip_runtime.h>

#include "hd_dev_data.hpp"
#include "hd_dev_jacobi.hpp"
#include "hd_dev_meta.hpp"

namespace hd {

constexpr int kBWaves = 4;
// per-wave scratch of a batch, smaller than the per-call kernels' so that
// four workgroups fit a CU: boundaries of one GDEF row update, runs of one
// use row, items of a band held in LDS (longer lists are searched in global
// memory; more boundaries or runs than this raise HD_ECAPACITY)
constexpr int kBatchMaxB = 256;
constexpr int kBatchRuns = 64;
constexpr int kBatchHeads = 64;

// per-wave LDS: union of the runs scratch and the GDEF scratch
struct RunsLds {
  Ivl iv[kMaxCap];
  Run rr[kBatchRuns];
};
struct GdefLdsB {
  Ivl iv[kMaxCap];
  int32_t b[kBatchMaxB], u[kBatchMaxB], own[kBatchMaxB];
  uint64_t hold[kBatchMaxB];
};
struct HeadsLds {
  Item p[kBatchHeads], w[kBatchHeads];
};
// runs of up to 8 per row found one row per lane
constexpr int kBatchLaneRuns = 8;
struct LaneRunsLds {
  int32_t lr[4 * kBatchLaneRuns * 64];
};
union WaveLds {
  RunsLds r;
  GdefLdsB g;
  HeadsLds h;
  LaneRunsLds l;
};

// Grid barrier on a monotonically increasing counter (zeroed before the
// launch).  Returns false if the run was abandoned (timeout or earlier error).
// One thread per workgroup arrives with a release increment (after the
// workgroup barrier, so it publishes the whole workgroup's writes), polls
// with relaxed loads and then takes one acquire fence: an acquire on every
// poll would invalidate the XCD's L2 once per poll, slowing every other
// workgroup on it.
__device__ inline bool grid_sync(unsigned *bar, unsigned nblk, unsigned &target, int32_t *err, int64_t limit) {
  __shared__ int s_ok;
  __syncthreads();
  target += nblk;
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t t0 = wall_clock64();
    int ok = 1;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == -9 ||
          wall_clock64() - t0 > limit) {
        atomicCAS(err, 0, -9);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// the three compaction phases (modes 0 and 2): a grid barrier after the
// chunk scans; phase 2 runs in every workgroup, so phase 3 follows at once
__device__ inline bool batch_compact(const BatchArgs &B, const Level &L, int mode, unsigned nblk, unsigned &target,
                                     int32_t *err, int &ph, int64_t *lds) {
  dev_compact_p1(L, B.cs, mode);
  if (!grid_sync(B.bar, nblk, target, err, B.spin_limit)) return false;
  if (blockIdx.x == 0 && threadIdx.x == 0) B.clk[ph] = wall_clock64();
  ++ph;
  dev_compact_p2(B.P, L, B.W, B.hdr, B.tab_cap, B.cs, (int)nblk, mode, lds);
  if (blockIdx.x == 0 && threadIdx.x == 0) B.clk[ph] = wall_clock64();
  ++ph;
  dev_compact_p3(B.P, L, B.W, B.tab, B.tab_cap, B.cs, mode, lds + 2 * kCompactCarr);
  return true;
}

__global__ __launch_bounds__(256) void k_batch(BatchArgs B) {
  __shared__ WaveLds s_lds[kBWaves];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const unsigned nblk = gridDim.x;
  const int gw = blockIdx.x * kBWaves + wv, nw = gridDim.x * kBWaves;
  unsigned target = 0;
  WaveLds &my = s_lds[wv];
  // workgroup-wide scratch of the single-workgroup phases (no wave uses its
  // own scratch at the same time)
  int64_t *lds = reinterpret_cast<int64_t *>(s_lds);
  static_assert(sizeof(WaveLds) * kBWaves >= 4 * kCompactCarr * sizeof(int64_t), "compaction scratch");
  int32_t *err = B.W.err;
  int ph = 0;
  auto stamp = [&]() {
    if (blockIdx.x == 0 && threadIdx.x == 0) B.clk[ph] = wall_clock64();
    ++ph;
  };
  stamp();
  // runs of every use row: 64 rows per wave, one per lane where the row is
  // simple, the others by the whole wave
  for (int c = gw; c * 64 < B.P.nsl1; c += nw) {
    const int s = c * 64 + lane;
    const bool done = s >= B.P.nsl1 || dev_runs_lane<kBatchLaneRuns>(B.P, B.A, B.W, s, my.l.lr);
    uint64_t left = __ballot(!done);
    wave_lds_sync();
    while (left) {
      const int l = __ffsll((unsigned long long)left) - 1;
      left &= left - 1;
      dev_runs(B.P, B.A, B.W, c * 64 + l, my.r.iv, my.r.rr, kBatchRuns);
    }
  }
  if (!grid_sync(B.bar, nblk, target, err, B.spin_limit)) return;
  stamp();
  for (int c = gw; c * 64 < B.L1.nsl; c += nw) dev_bandflags(B.L1, c * 64 + lane);
  if (!grid_sync(B.bar, nblk, target, err, B.spin_limit)) return;
  stamp();
  // every workgroup scans the band flags itself: the scan is cheap, its
  // writes are the same values from every workgroup, and each workgroup's
  // heads then read what it wrote, so no grid barrier separates the scan
  // from the heads
  if (B.L1.nsl) dev_bandscan(B.L1);
  stamp();
  {
    const int nb = B.L1.nsl ? *B.L1.nb : 0;
    for (int b = gw; b < nb; b += nw) dev_heads(B.L1, b, nb, my.h.p, my.h.w, kBatchHeads);
    dev_compact_reset(B.P, B.cs);
  }
  if (!grid_sync(B.bar, nblk, target, err, B.spin_limit)) return;
  stamp();
  if (!B.P.has3d) {
    if (!batch_compact(B, B.L1, 0, nblk, target, err, ph, lds)) return;
  } else {
    if (blockIdx.x == 0) dev_compact(B.P, B.L1, B.W, B.tab, B.hdr, B.tab_cap, 1, lds);
    if (!grid_sync(B.bar, nblk, target, err, B.spin_limit)) return;
    stamp();
    for (int c = gw; c * 64 < B.L2.nsl; c += nw) dev_bandflags(B.L2, c * 64 + lane);
    if (!grid_sync(B.bar, nblk, target, err, B.spin_limit)) return;
    stamp();
    if (B.L2.nsl) dev_bandscan(B.L2);
    stamp();
    {
      const int nb = B.L2.nsl ? *B.L2.nb : 0;
      for (int b = gw; b < nb; b += nw) dev_heads(B.L2, b, nb, my.h.p, my.h.w, kBatchHeads);
      dev_compact_reset(B.P, B.cs);
    }
    if (!grid_sync(B.bar, nblk, target, err, B.spin_limit)) return;
    stamp();
    if (!batch_compact(B, B.L2, 2, nblk, target, err, ph, lds)) return;
  }
  if (!grid_sync(B.bar, nblk, target, err, B.spin_limit)) return;
  stamp();
  // pack + unpack in one pass, and the GDEF update (metadata only,
  // independent of the data)
  {
    // (message, span) pairs per workgroup, as the per-call pack kernel
    const int64_t nmsg = B.hdr->nmsg, words = B.hdr->bytes >> 2;
    if (nmsg > 0) {
      int64_t S = (words + nmsg * 1024 - 1) / (nmsg * 1024);
      const int64_t smax = (int64_t)nblk / nmsg > 1 ? (int64_t)nblk / nmsg : 1;
      if (S > smax) S = smax;
      if (S < 1) S = 1;
      for (int64_t q = blockIdx.x; q < nmsg * S; q += nblk) {
        const int64_t m = q / S, sub = q % S;
        const MsgRec r = B.tab[m];
        const int64_t nw8 = r.bytes >> 2;
        const int64_t a0 = nw8 * sub / S, a1 = nw8 * (sub + 1) / S;
        if (nw8 < (int64_t(1) << 31))
          dev_pack_span<int32_t>(r, B.A, B.stg, 2, (int32_t)a0, (int32_t)a1);
        else
          dev_pack_span<int64_t>(r, B.A, B.stg, 2, a0, a1);
      }
    }
  }
  {
    // rows the definitions tile: one lane per row
    for (int c = gw; c * 64 < B.P.ngfull; c += nw) {
      const int t = c * 64 + lane;
      if (t < B.P.ngfull) dev_gdef_full_lane(B.P, B.A, B.W, t);
    }
    // the other rows 64 at a time: small rows one per lane (a row with no
    // definition and no holder-adding run is left as it is), the larger
    // ones by the whole wave, one after the other
    GdefLds S{my.g.iv, my.g.b, my.g.u, my.g.own, my.g.hold};
    const int nrest = B.P.ngrow - B.P.ngfull;
    for (int c = gw; c * 64 < nrest; c += nw) {
      const int t0 = B.P.ngfull + c * 64;
      const bool done = c * 64 + lane >= nrest || dev_gdef_small_lane(B.P, B.A, B.W, t0 + lane);
      uint64_t m = __ballot(!done);
      while (m) {
        const int t = t0 + __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        if (!dev_gdef_row_fast(B.P, B.A, B.W, t)) dev_gdef_row(B.P, B.A, B.W, t, S, kBatchMaxB);
      }
    }
  }
  // the user kernels follow in their own launch (stream order makes the
  // unpacked halos visible to them)
}

__global__ void k_zero_bar(unsigned *bar) {
  if (threadIdx.x == 0) *bar = 0u;
}

// The user kernels of a batch: one wave per tile; the tile's box from the
// per-tile table (both tables read-only, indices uniform per workgroup).
template <int TH, bool HF>
__global__ __launch_bounds__(64) void k_batch_tiles(const WorkBox *__restrict__ wb, const int32_t *__restrict__ tbox,
                                                    const ArrDev *__restrict__ A, int64_t ntiles) {
  const int64_t t = xcd_remap(blockIdx.x, ntiles);
  const WorkBox bx = wb[tbox[t]];
  if (bx.kind == 1)
    dev_jacobi_tile<TH, false, HF>(bx, t - bx.tile0, A);
  else if (bx.kind == 5)
    dev_jacobi_tile<TH, true, HF>(bx, t - bx.tile0, A);
  else if (bx.kind == 2)
    dev_copy_tile(bx, t - bx.tile0, A);
}

// The same tiles four waves at a time, stacked down a tile of 16 rows
// (halo rows shared through LDS when the box's rows can be read as float4,
// the per-box choice uniform over the workgroup); a copy box's tiles go
// four to a workgroup, one per wave.
__global__ __launch_bounds__(256) void k_batch_stack(const WorkBox *__restrict__ wb, const int32_t *__restrict__ tbox,
                                                     const ArrDev *__restrict__ A, int64_t ntiles) {
  const int64_t t = xcd_remap(blockIdx.x, ntiles);
  const WorkBox bx = wb[tbox[t]];
  const int64_t lt = t - bx.tile0;
  if (bx.kind == 2) {
    const int64_t ct = 4 * lt + (threadIdx.x >> 6);
    if (ct < copy_tiles(bx, A[bx.ain].esize)) dev_copy_tile(bx, ct, A);
    return;
  }
  const bool vec = ((bx.lo[2] & 3) == 0) && ((A[bx.ain].n[2] & 3) == 0) && ((A[bx.ain].rs[bx.dev] & 3) == 0) &&
                   ((A[bx.aout].rs[bx.dev] & 3) == 0);
  if (bx.kind == 1) {
    if (vec)
      dev_stack_tile<4, 4, 0, true>(bx, lt, A, Coef9{});
    else
      dev_stack_tile<4, 4, 0, false>(bx, lt, A, Coef9{});
  } else if (bx.kind == 5) {
    if (vec)
      dev_stack_tile<4, 4, 1, true>(bx, lt, A, Coef9{});
    else
      dev_stack_tile<4, 4, 1, false>(bx, lt, A, Coef9{});
  }
}

typedef void (*tiles_kernel_t)(const WorkBox *, const int32_t *, const ArrDev *, int64_t);

// th: rows per wave; hf: 1 one-wave tiles numbered along rows first, 0 down
// columns first, 2 four waves of 4 rows stacked (th is 4; more rows per wave
// in this kernel leave one wave per SIMD)
static tiles_kernel_t pick_tiles(int th, int hf) {
  if (hf == 2) return k_batch_stack;
  if (th == 4) return hf ? k_batch_tiles<4, true> : k_batch_tiles<4, false>;
  if (th == 16) return hf ? k_batch_tiles<16, true> : k_batch_tiles<16, false>;
  return hf ? k_batch_tiles<8, true> : k_batch_tiles<8, false>;
}

int batch_max_blocks(int max_per_cu) {
  int dev = 0, ncu = 0, occ = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)k_batch, 256, 0) != hipSuccess) return -1;
  if (occ < 1) occ = 1;
  if (occ > max_per_cu) occ = max_per_cu;
  // the compaction keeps one chunk per workgroup
  return ncu * occ < kCompactCarr ? ncu * occ : kCompactCarr;
}

// the step as three nodes on one stream: zero the barrier, run the
// persistent metadata + communication kernel, then the user kernels
hipError_t launch_batch(const BatchArgs &a, int th, int hf, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_bar, dim3(1), dim3(64), 0, s, a.bar);
  hipLaunchKernelGGL(k_batch, dim3(grid), dim3(256), 0, s, a);
  if (a.ntiles > 0)
    hipLaunchKernelGGL(pick_tiles(th, hf), dim3((unsigned)a.ntiles), dim3(hf == 2 ? 256 : 64), 0, s, a.wb, a.tbox,
                       (const ArrDev *)a.A, a.ntiles);
  return hipGetLastError();
}

int batch_args_size() { return (int)sizeof(BatchArgs); }

}  // namespace hd

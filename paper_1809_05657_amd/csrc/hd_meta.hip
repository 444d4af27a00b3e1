// hd_meta.hip — per-phase kernels of the communication-set derivation
// (Sec. 2.2, Eq. 1-2) and the GDEF update (Eq. 3-4); the device code is in
// hd_dev_meta.hpp and shared with the persistent batched kernel.
//
// Every kernel here runs one-wave workgroups: the derivation of call k+1
// overlaps the user kernel of call k, and a one-wave workgroup finds a free
// slot on a CU that kernel keeps busy, where a large workgroup waits until
// many slots free up at once.
#include <hip/hip_runtime.h>

#include "hd_dev_meta.hpp"

namespace hd {

constexpr int kGdefMaxB = 1024;



// One wave per use row (a measurement alternative; see launch_runs).
template <int CAP>
__global__ __launch_bounds__(64) void k_runs_wave(PlanDev P, const ArrDev *__restrict__ A, Work W) {
  __shared__ Ivl s_iv[CAP];
  __shared__ Run s_run[kMaxRunsRow];
  const int s = blockIdx.x;
  if (s >= P.nsl1) return;
  const int nr = dev_runs_find(P, A, W, s, s_iv, s_run);
  dev_runs_store(P, W, s, s_run, nr);
}

// 64 use rows per one-wave workgroup: rows with few intervals, segments
// and runs one per lane; the wave then takes the other rows of its 64 one
// at a time.  The runs of each row, sorted, go to the row's slot.
template <int CAP>
__global__ __launch_bounds__(64) void k_runs(PlanDev P, const ArrDev *__restrict__ A, Work W) {
  __shared__ Ivl s_iv[CAP];
  __shared__ Run s_run[kMaxRunsRow];
  __shared__ int32_t s_lr[4 * kRunSlot * 64];
  const int s = blockIdx.x * 64 + threadIdx.x;
  const bool done = s >= P.nsl1 || dev_runs_lane<kRunSlot>(P, A, W, s, s_lr);
  uint64_t left = __ballot(!done);
  while (left) {
    const int l = __ffsll((unsigned long long)left) - 1;
    left &= left - 1;
    const int r = blockIdx.x * 64 + l;
    const int nr = dev_runs_find(P, A, W, r, s_iv, s_run);
    dev_runs_store(P, W, r, s_run, nr);
    wave_lds_sync();
  }
}

// One wave per 64 slices: band-start flags from the stored items -> chunk
// masks.
__global__ __launch_bounds__(64) void k_bandflags(Level L) { dev_bandflags(L, blockIdx.x * 64 + threadIdx.x); }

// One workgroup (one wave for small levels): exclusive scan of the band
// counts, band -> first slice.
template <int NT>
__global__ __launch_bounds__(NT) void k_bandscan(Level L) { dev_bandscan(L); }

// Heads of every band, one wave per band.
__global__ __launch_bounds__(64) void k_heads(Level L) {
  __shared__ Item s_p[kHeadLds], s_w[kHeadLds];
  const int nb = *L.nb;
  for (int b = blockIdx.x; b < nb; b += gridDim.x) dev_heads(L, b, nb, s_p, s_w);
}

// One wave: the message table (or the level-2 items).
__global__ __launch_bounds__(64) void k_compact(PlanDev P, Level L, Work W, MsgRec *out, MsgHdr *hdr,
                                                 int64_t out_cap, int mode) {
  __shared__ int64_t s[2 * kCompactCarr];
  dev_compact(P, L, W, out, hdr, out_cap, mode, s);
}

__global__ __launch_bounds__(256) void k_compact_wg(PlanDev P, Level L, Work W, MsgRec *out, MsgHdr *hdr,
                                                     int64_t out_cap, int mode) {
  __shared__ int64_t s[2 * kCompactCarr];
  dev_compact(P, L, W, out, hdr, out_cap, mode, s);
}

// The first nfw workgroups copy the rows the definitions tile, one lane
// per row; the others take 64 of the other rows each, one per lane where
// the row is small (dev_gdef_small_lane), and list the rest (count in
// *cnt, one atomic per wave) for k_gdef_large.
__global__ __launch_bounds__(64) void k_gdef(PlanDev P, ArrDev *__restrict__ A, Work W, int32_t *cnt, int nfw) {
  if ((int)blockIdx.x < nfw) {
    const int t = blockIdx.x * 64 + threadIdx.x;
    if (t < P.ngfull) dev_gdef_full_lane(P, A, W, t);
    return;
  }
  const int t = P.ngfull + ((int)blockIdx.x - nfw) * 64 + (int)threadIdx.x;
  const bool done = t >= P.ngrow || dev_gdef_small_lane(P, A, W, t);
  const uint64_t m = __ballot(!done);
  if (m) {
    int base = 0;
    if (threadIdx.x == 0) base = atomicAdd(cnt, __popcll(m));
    base = __shfl(base, 0);
    if (!done) W.ovf_list[base + __popcll(m & lanemask_lt())] = t;
  }
}

// The other form: the first nfw workgroups as above, then one wave per row,
// register-only up to 64 boundaries; larger rows are listed (count in
// *cnt) for k_gdef_large.
__global__ __launch_bounds__(64) void k_gdef_wave(PlanDev P, ArrDev *__restrict__ A, Work W, int32_t *cnt, int nfw) {
  if ((int)blockIdx.x < nfw) {
    const int t = blockIdx.x * 64 + threadIdx.x;
    if (t < P.ngfull) dev_gdef_full_lane(P, A, W, t);
    return;
  }
  const int g = (int)gridDim.x - nfw;
  for (int t = P.ngfull + (int)blockIdx.x - nfw; t < P.ngrow; t += g)
    if (!dev_gdef_row_fast(P, A, W, t) && threadIdx.x == 0) W.ovf_list2[atomicAdd(cnt, 1)] = t;
}

// The listed rows, one wave each, register-only; a row with more than 64
// boundaries goes to the second list (count in *cnt2) for k_gdef_large.
constexpr int kGdefListGrid = 2048;
__global__ __launch_bounds__(64) void k_gdef_list(PlanDev P, ArrDev *__restrict__ A, Work W, const int32_t *cnt,
                                                  int32_t *cnt2) {
  const int n = *cnt;
  for (int q = blockIdx.x; q < n; q += gridDim.x) {
    const int t = W.ovf_list[q];
    if (!dev_gdef_row_fast(P, A, W, t) && threadIdx.x == 0) W.ovf_list2[atomicAdd(cnt2, 1)] = t;
  }
}

// The rows of the second list, one wave each with LDS scratch (such rows
// are rare, so the grid is small).  Each list has two counters that
// alternate between calls:
// this launch clears the other one, which the previous launch (finished,
// same stream) read and the next k_gdef appends to, so no workgroup has to
// wait for the others before a counter is reset.
constexpr int kGdefLargeGrid = 32;
__global__ __launch_bounds__(64) void k_gdef_large(PlanDev P, ArrDev *__restrict__ A, Work W, const int32_t *cnt2,
                                                   int32_t *other, int32_t *other2) {
  __shared__ Ivl s_iv[kMaxCap];
  __shared__ int32_t s_b[kGdefMaxB], s_u[kGdefMaxB], s_own[kGdefMaxB];
  __shared__ uint64_t s_hold[kGdefMaxB];
  GdefLds S{s_iv, s_b, s_u, s_own, s_hold};
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *other = 0;
    *other2 = 0;
  }
  const int n = *cnt2;
  for (int q = blockIdx.x; q < n; q += gridDim.x) dev_gdef_row(P, A, W, W.ovf_list2[q], S, kGdefMaxB);
}


// ------------------------------------------------------ small instances
// Bands leave most calls with few slices and cells.  One workgroup then
// derives the whole communication set (runs, band flags, band scan, heads,
// compaction: one launch instead of five, each phase a few dependent loads
// long), and each GDEF cell is updated by one wave.
constexpr int kDerive1Max = 64;  // slices (and level-2 groups) of the small form

// Two launches per call.  k_runs1: the runs, one wave per slice (the
// intervals in lanes, runs by ballot).  k_tail1:
// workgroup 0 turns the runs into the message table (band flags, band scan,
// heads shared out band by band over its waves with item lists of up to
// kHead1 items staged in LDS, compaction) while the other workgroups update
// GDEF (both only read the runs), so the table and the update finish
// together.
constexpr int kDerive1Waves = 8, kHead1 = 32;
// k_runs1: one wave per workgroup and one workgroup per slice.  Each slice
// is a short chain of dependent global loads (slice record, the cell's list,
// the runs' store).  The kernel runs beside the previous call's user
// kernel, which holds most of every SIMD's registers: a one-wave workgroup
// of about 48 VGPRs fits in what is left, where a workgroup of several
// waves on one CU waits until that CU drains.  The spill pool's top is
// reset by the compaction that consumes the runs (and at initialisation).
template <int CAP>
__global__ __launch_bounds__(64) void k_runs1(PlanDev P, const ArrDev *__restrict__ A, Work W) {
  __shared__ __align__(16) Ivl s_iv[CAP];
  __shared__ __align__(16) Run s_rr[kMaxRunsRow];
  if (W.skip && *W.skip) return;  // the plan's stored runs are current
  for (int sl = blockIdx.x; sl < P.nsl1; sl += gridDim.x) {
    const int nr = dev_runs_find(P, A, W, sl, s_iv, s_rr);
    dev_runs_store(P, W, sl, s_rr, nr);
    wave_lds_sync();
  }
}


__global__ __launch_bounds__(64 * kDerive1Waves) void k_tail1(PlanDev P, ArrDev *__restrict__ A, Work W, Level L1,
                                                            Level L2, MsgRec *out, MsgHdr *hdr, int64_t cap,
                                                            int has3d) {
  // workgroup 0: the heads' scratch (2 * kHead1 items per wave), then the
  // compaction's; the others: one wave's LDS form of the GDEF update
  __shared__ __align__(16) char s_buf[sizeof(Ivl) * kMaxCap + (3 * 4 + 8) * kGdefMaxB];
  __shared__ int32_t s_def[kDerive1Waves];
  __shared__ int32_t s_ndef;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (blockIdx.x > 0) {
    // one cell per wave in registers; the LDS scratch serves one wave, so
    // the cells that need it (more than 64 boundaries) are updated after
    // the others by wave 0, one after the other
    Ivl *iv = reinterpret_cast<Ivl *>(s_buf);
    int32_t *b = reinterpret_cast<int32_t *>(s_buf + sizeof(Ivl) * kMaxCap);
    const GdefLds S{iv, b, b + kGdefMaxB, b + 2 * kGdefMaxB, reinterpret_cast<uint64_t *>(b + 3 * kGdefMaxB)};
    const int nw = (gridDim.x - 1) * kDerive1Waves;
    for (int t0 = (blockIdx.x - 1) * kDerive1Waves; t0 < P.ngrow; t0 += nw) {
      if (threadIdx.x == 0) s_ndef = 0;
      __syncthreads();
      const int t = t0 + wv;
      if (t < P.ngrow && !dev_gdef_row_fast(P, A, W, t) && lane == 0) s_def[atomicAdd(&s_ndef, 1)] = t;
      __syncthreads();
      if (wv == 0)
        for (int k = 0; k < s_ndef; ++k) dev_gdef_row(P, A, W, s_def[k], S, kGdefMaxB);
      __syncthreads();
    }
    return;
  }
  if (W.skip && *W.skip) return;  // the plan's stored table is current
  for (int lv = 1; lv <= (has3d ? 2 : 1); ++lv) {
    const Level &L = lv == 1 ? L1 : L2;
    if (L.nsl > 0) {
      if (wv == 0) dev_bandflags(L, lane);
      __syncthreads();
      dev_bandscan(L);
      const int nb = *L.nb;
      Item *sp = reinterpret_cast<Item *>(s_buf + wv * 2 * kHead1 * sizeof(Item));
      for (int b = wv; b < nb; b += kDerive1Waves) dev_heads(L, b, nb, sp, sp + kHead1, kHead1);
      __syncthreads();
    }
    dev_compact(P, L, W, out, hdr, cap, lv == 1 ? (has3d ? 1 : 0) : 2, reinterpret_cast<int64_t *>(s_buf));
  }
}

// The GDEF update of cell t, one wave: the cell's first row holds its list;
// the task applies the cell's edits to it in registers, or through LDS when
// the row has more than 64 boundaries.  No task waits for another.
__device__ inline void gdef_task(const PlanDev &P, ArrDev *__restrict__ A, const Work &W, int t, GdefLds S) {
  if (!dev_gdef_row_fast(P, A, W, t)) dev_gdef_row(P, A, W, t, S, kGdefMaxB);
}

__global__ __launch_bounds__(64) void k_gdef_tasks(PlanDev P, ArrDev *__restrict__ A, Work W) {
  __shared__ Ivl s_iv[kMaxCap];
  __shared__ int32_t s_b[kGdefMaxB], s_u[kGdefMaxB], s_own[kGdefMaxB];
  __shared__ uint64_t s_hold[kGdefMaxB];
  GdefLds S{s_iv, s_b, s_u, s_own, s_hold};
  for (int t = blockIdx.x; t < P.ngrow; t += gridDim.x) gdef_task(P, A, W, t, S);
}

// Band lists copied to the first rows of cells that split a band: one
// wave per record.
__global__ __launch_bounds__(64) void k_mat(const MatRec *__restrict__ M, int n, ArrDev *__restrict__ A) {
  const int lane = threadIdx.x & 63;
  for (int q = blockIdx.x; q < n; q += gridDim.x) {
    const MatRec m = M[q];
    ArrDev &a = A[m.arr];
    const int c = a.cnt[m.src];
    for (int e = lane; e < c; e += 64) a.ivl[m.dst * a.cap + e] = a.ivl[m.src * a.cap + e];
    if (lane == 0) a.cnt[m.dst] = c;
  }
}

// Plan cache, second step (Sec. 4.2: compare the GDEF sections themselves
// when the history does not decide).  One workgroup; snap holds, per slice
// of the plan's small-form instance, the list its runs were derived from
// (kMaxCap entries a slice, scnt the counts).  compare: *skip = 1 when every
// slice's current list equals its snapshot (the plan's table and runs are
// then current; *hits counts such calls); otherwise, or without compare,
// *skip = 0 and the snapshot is refreshed from the current lists, which the
// call's derivation is about to read.
__global__ __launch_bounds__(512) void k_snap(PlanDev P, const ArrDev *__restrict__ A, Ivl *__restrict__ snap,
                                              int32_t *__restrict__ scnt, int32_t *skip, int32_t *hits,
                                              int compare) {
  __shared__ int s_diff;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (threadIdx.x == 0) s_diff = compare ? 0 : 1;
  __syncthreads();
  if (compare) {
    bool diff = false;
    for (int s = wv; s < P.nsl1; s += nw) {
      const SliceRec r = P.srec[s];
      const ArrDev &a = A[r.arr];
      const int n = a.cnt[r.grow];
      bool d = n != scnt[s];
      for (int e = lane; !d && e < n; e += 64) {
        const Ivl x = a.ivl[r.grow * a.cap + e], y = snap[(int64_t)s * kMaxCap + e];
        d = x.start != y.start || x.owner != y.owner || x.holders != y.holders;
      }
      diff = diff || d;
    }
    if (diff) s_diff = 1;
  }
  __syncthreads();
  const bool same = s_diff == 0;
  if (threadIdx.x == 0) {
    *skip = same ? 1 : 0;
    if (same) *hits += 1;
  }
  if (same) return;
  for (int s = wv; s < P.nsl1; s += nw) {
    const SliceRec r = P.srec[s];
    const ArrDev &a = A[r.arr];
    const int n = a.cnt[r.grow];
    for (int e = lane; e < n; e += 64) snap[(int64_t)s * kMaxCap + e] = a.ivl[r.grow * a.cap + e];
    if (lane == 0) scnt[s] = n;
  }
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

hipError_t launch_snap(const PlanDev &P, const ArrDev *A, Ivl *snap, int32_t *scnt, int32_t *skip, int32_t *hits,
                       bool compare, hipStream_t s) {
  hipLaunchKernelGGL(k_snap, dim3(1), dim3(512), 0, s, P, A, snap, scnt, skip, hits, compare ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_mat(const MatRec *m, int n, ArrDev *A, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mat, dim3(n < 4096 ? n : 4096), dim3(64), 0, s, m, n, A);
  return hipGetLastError();
}


hipError_t launch_compact(const PlanDev &P, const Level &L, const Work &W, MsgRec *out, MsgHdr *hdr,
                          int64_t cap, int mode, hipStream_t s) {
  // one wave for tables of a few thousand bands at most; a full workgroup
  // when the level has many slices (and so possibly many bands)
  const int nt = L.nsl <= 8192 ? 64 : 256;
  if (nt == 64)
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(64), 0, s, P, L, W, out, hdr, cap, mode);
  else
    hipLaunchKernelGGL(k_compact_wg, dim3(1), dim3(256), 0, s, P, L, W, out, hdr, cap, mode);
  return hipGetLastError();
}

static void launch_heads(const Level &L, hipStream_t s) {
  const int hg = L.nsl < 256 ? L.nsl : 256;
  hipLaunchKernelGGL(k_heads, dim3(hg), dim3(64), 0, s, L);
}

static void launch_bands(const Level &L, hipStream_t s) {
  hipLaunchKernelGGL(k_bandflags, dim3(cdiv(L.nsl, 64)), dim3(64), 0, s, L);
  if (L.nsl <= 8192)
    hipLaunchKernelGGL(k_bandscan<64>, dim3(1), dim3(64), 0, s, L);
  else if (L.nsl <= (1 << 18))
    hipLaunchKernelGGL(k_bandscan<256>, dim3(1), dim3(256), 0, s, L);
  else  // levels of 3-D arrays (a slice per use row of every plane)
    hipLaunchKernelGGL(k_bandscan<1024>, dim3(1), dim3(1024), 0, s, L);
  launch_heads(L, s);
}

// level 1: runs (the only step that reads GDEF), then band flags, band
// scan, heads, compaction (mode 0: the final messages; mode 1: the level-2
// items of 3-D arrays)
// Levels of fewer use rows than g_runs_wave_max use one wave per row.  A
// wave per row finishes the runs sooner on its own (25 vs 70 us on the
// 8192-row Jacobi level next to the stencil kernel), but its many small
// workgroups slow the stencil kernel they overlap more than that gains, so
// the default (0) is the lane form everywhere.
int g_runs_wave_max = 0;

hipError_t launch_runs(const PlanDev &P, const ArrDev *A, const Work &W, int row_cap, hipStream_t s) {
  if (P.nsl1 == 0) return hipSuccess;
  // LDS for the row's intervals sized to the row capacity
  if (P.nsl1 < g_runs_wave_max) {
    if (row_cap <= 64)
      hipLaunchKernelGGL(k_runs_wave<64>, dim3(P.nsl1), dim3(64), 0, s, P, A, W);
    else
      hipLaunchKernelGGL(k_runs_wave<kMaxCap>, dim3(P.nsl1), dim3(64), 0, s, P, A, W);
  } else if (row_cap <= 64) {
    hipLaunchKernelGGL(k_runs<64>, dim3(cdiv(P.nsl1, 64)), dim3(64), 0, s, P, A, W);
  } else {
    hipLaunchKernelGGL(k_runs<kMaxCap>, dim3(cdiv(P.nsl1, 64)), dim3(64), 0, s, P, A, W);
  }
  return hipGetLastError();
}

hipError_t launch_level1_tail(const PlanDev &P, const Work &W, const Level &L, MsgRec *out, MsgHdr *hdr, int64_t cap,
                              int mode, hipStream_t s) {
  if (P.nsl1 > 0) launch_bands(L, s);
  return launch_compact(P, L, W, out, hdr, cap, mode, s);
}

hipError_t launch_level1(const PlanDev &P, const ArrDev *A, const Work &W, const Level &L, MsgRec *out,
                         MsgHdr *hdr, int64_t cap, int mode, int row_cap, hipStream_t s) {
  const hipError_t e = launch_runs(P, A, W, row_cap, s);
  if (e != hipSuccess) return e;
  return launch_level1_tail(P, W, L, out, hdr, cap, mode, s);
}

// level 2 (rectangles of consecutive planes stacked into boxes)
hipError_t launch_level2(const PlanDev &P, const Work &W, const Level &L, MsgRec *out, MsgHdr *hdr, int64_t cap,
                         hipStream_t s) {
  if (L.nsl > 0) launch_bands(L, s);
  return launch_compact(P, L, W, out, hdr, cap, 2, s);
}

hipError_t launch_init_rows(Ivl *ivl, int32_t *cnt, int64_t rows, int cap, hipStream_t s) {
  int grid = cdiv(rows, 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_init_rows, dim3(grid), dim3(256), 0, s, ivl, cnt, rows, cap);
  return hipGetLastError();
}

// The two-launch derivation of small instances (with the GDEF update unless
// gdef is false); returns hipErrorNotSupported for larger ones (the caller
// then takes the per-phase form).
hipError_t launch_derive1(const PlanDev &P, ArrDev *A, const Work &W, const Level &L1, const Level &L2,
                          MsgRec *out, MsgHdr *hdr, int64_t cap, int row_cap, bool gdef, hipStream_t s) {
  if (P.nsl1 > kDerive1Max || P.ngrp > kDerive1Max) return hipErrorNotSupported;
  if (P.nsl1 > 0) {
    if (row_cap <= 64)
      hipLaunchKernelGGL(k_runs1<64>, dim3(P.nsl1), dim3(64), 0, s, P, A, W);
    else
      hipLaunchKernelGGL(k_runs1<kMaxCap>, dim3(P.nsl1), dim3(64), 0, s, P, A, W);
  }
  const int gw = gdef && P.ngrow > 0 ? (P.ngrow + kDerive1Waves - 1) / kDerive1Waves : 0;
  hipLaunchKernelGGL(k_tail1, dim3(1 + (gw < 1024 ? gw : 1024)), dim3(64 * kDerive1Waves), 0, s, P, A, W, L1, L2,
                     out, hdr, cap, P.has3d ? 1 : 0);
  return hipGetLastError();
}

// Every GDEF update of the runtime goes through here, in stream order (the
// meta stream waits for the second internal stream before it launches
// another), so the counter parity alternates launch by launch.
static int g_ovf_parity = 0;
hipError_t launch_gdef(const PlanDev &P, ArrDev *A, const Work &W, hipStream_t s) {
  if (P.ngrow == 0) return hipSuccess;
  const int p = g_ovf_parity;
  g_ovf_parity ^= 1;
  int32_t *cur = W.ovf_cnt + p, *other = W.ovf_cnt + (1 - p);
  int32_t *cur2 = W.ovf_cnt + 2 + p, *other2 = W.ovf_cnt + 2 + (1 - p);
  const int nfw = cdiv(P.ngfull, 64);
  const int rest = P.ngrow - P.ngfull;
  if (P.ngrow <= 4096) {
    // few cells: one launch, one wave per cell
    {
      const int grid = P.ngrow;
      hipLaunchKernelGGL(k_gdef_tasks, dim3(grid), dim3(64), 0, s, P, A, W);
    }
    return hipGetLastError();
  }
  if (P.gdef_lane) {
    hipLaunchKernelGGL(k_gdef, dim3(nfw + cdiv(rest, 64)), dim3(64), 0, s, P, A, W, cur, nfw);
    hipLaunchKernelGGL(k_gdef_list, dim3(kGdefListGrid), dim3(64), 0, s, P, A, W, (const int32_t *)cur, cur2);
  } else {
    const int grid = nfw + (rest < (1 << 20) ? rest : (1 << 20));
    hipLaunchKernelGGL(k_gdef_wave, dim3(grid), dim3(64), 0, s, P, A, W, cur2, nfw);
  }
  hipLaunchKernelGGL(k_gdef_large, dim3(kGdefLargeGrid), dim3(64), 0, s, P, A, W, (const int32_t *)cur2, other, other2);
  return hipGetLastError();
}

}  // namespace hd

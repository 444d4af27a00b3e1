// hd_meta.hip — communication-set derivation and GDEF update on gfx950.
//
// Paper: Sec. 2.2, Eq. 1-2 (messages = GDEF intersected with LUSE, taken
// right before the kernel) and Eq. 3-4 (GDEF update: receivers become
// holders, a definition makes the definer the owner and only holder).
// Sec. 4.2 merges adjacent sections; here the merge is made canonical:
//   runs   maximal innermost-dimension runs with one source, per (row, dst);
//   level 1 runs identical on consecutive rows of a plane stack into rects;
//   level 2 rects identical on consecutive planes stack into boxes;
//   order  (argument, lower corner row-major, destination).
//
// Pipeline per call (all device-resident, no host readback):
//   k_runs       one wave per use row: intersect the row's GDEF interval list
//                with every destination's use segments (wave ballot + prefix
//                popcount compaction), sort runs by (col, dst)
//   k_bandflags  one lane per slice: a band starts where the item list or the
//                adjacency changes (ballot -> 64-bit chunk mask)
//   k_bandscan   one workgroup: exclusive scan of band counts, band -> slice
//   k_heads      one lane per band: items not continued from the previous
//                slice are heads; their extent is found by walking bands
//   k_compact    one workgroup: scan of head counts and bytes -> message table
//                in canonical order with pack offsets (or level-1 output)
//   k_gdef       one wave per touched row: apply holder additions and
//                definitions to the row's interval list, re-merge
#include <hip/hip_runtime.h>

#include "hd_internal.hpp"

namespace hd {

__device__ inline uint64_t lanemask_lt() {
  const unsigned lane = threadIdx.x & 63;
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

__device__ inline void set_err(int32_t *err, int code) { atomicCAS(err, 0, code); }

__device__ inline bool item_eq(const Item &x, const Item &y) {
  return x.src == y.src && x.dst == y.dst && x.a0 == y.a0 && x.a1 == y.a1 && x.b0 == y.b0 && x.b1 == y.b1;
}
// order inside a slice: (b0, a0, dst)
__device__ inline bool item_less(const Item &x, const Item &y) {
  if (x.b0 != y.b0) return x.b0 < y.b0;
  if (x.a0 != y.a0) return x.a0 < y.a0;
  return x.dst < y.dst;
}
__device__ inline bool contains(const Item *it, int cnt, const Item &q) {
  int lo = 0, hi = cnt;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (item_less(it[mid], q))
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo < cnt && item_eq(it[lo], q);
}

// --------------------------------------------------------------- k_runs
constexpr int kRunWaves = 4;

__global__ __launch_bounds__(256) void k_runs(PlanDev P, const ArrDev *__restrict__ A, Work W) {
  __shared__ Ivl s_iv[kRunWaves][kMaxCap];
  __shared__ Item s_run[kRunWaves][kMaxRunsRow];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  Ivl *iv = s_iv[wv];
  Item *rr = s_run[wv];
  for (int s = blockIdx.x * kRunWaves + wv; s < P.nsl1; s += gridDim.x * kRunWaves) {
    const int aidx = P.grp_aidx[P.grp1[s]];
    const ArrDev &a = A[P.carr[aidx].arr];
    const int64_t grow = P.grow1[s];
    const int n = a.cnt[grow];
    const int W2 = (int)a.n[2];
    const Ivl *row = a.ivl + grow * (int64_t)a.cap;
    for (int i = lane; i < n; i += 64) iv[i] = row[i];
    wave_lds_sync();
    int nr = 0;
    const int sg1 = P.seg0[s] + P.nseg[s];
    for (int sg = P.seg0[s]; sg < sg1; ++sg) {
      const Seg S = P.useg[sg];
      const uint64_t bit = 1ull << S.dst;
      auto need = [&](int i) -> bool {
        const int st = iv[i].start, en = (i + 1 < n) ? iv[i + 1].start : W2;
        return max(st, S.c0) < min(en, S.c1) && !(iv[i].holders & bit);
      };
      for (int base = 0; base < n; base += 64) {
        const int i = base + lane;
        bool start = false;
        int src = 0;
        if (i < n) {
          src = iv[i].owner;
          start = need(i) && !(i > 0 && iv[i - 1].owner == src && need(i - 1));
        }
        const uint64_t m = __ballot(start);
        if (start) {
          int j = i + 1;
          while (j < n && iv[j].owner == src && need(j)) ++j;
          const int c0 = max(iv[i].start, S.c0);
          const int c1 = min((j < n) ? iv[j].start : W2, S.c1);
          const int k = nr + __popcll(m & lanemask_lt());
          if (k < kMaxRunsRow) rr[k] = Item{src, S.dst, c0, c1, 0, 0, 0, 0};
        }
        nr += __popcll(m);
      }
    }
    if (nr > kMaxRunsRow) {
      if (lane == 0) set_err(W.err, -8);
      nr = 0;
    }
    wave_lds_sync();
    int off = 0;
    if (lane == 0 && nr) {
      off = atomicAdd(W.run_top, nr);
      if ((int64_t)off + nr > W.run_cap) {
        set_err(W.err, -8);
        off = -1;
      }
    }
    off = __shfl(off, 0);
    if (off < 0) nr = 0;
    // rank sort by (col, dst): keys are unique (runs of one dst are disjoint)
    for (int i = lane; i < nr; i += 64) {
      const Item x = rr[i];
      int rank = 0;
      for (int j = 0; j < nr; ++j) {
        const Item y = rr[j];
        rank += (y.a0 < x.a0) || (y.a0 == x.a0 && y.dst < x.dst);
      }
      W.runs[off + rank] = x;
    }
    if (lane == 0) {
      W.roff[s] = nr ? off : 0;
      W.rcnt[s] = nr;
    }
    wave_lds_sync();
  }
}

// ----------------------------------------------------------- k_bandflags
__global__ __launch_bounds__(256) void k_bandflags(Level L) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  bool st = false;
  if (s < L.nsl) {
    if (s == 0 || L.grp[s] != L.grp[s - 1] || L.pos[s] != L.pos[s - 1] + 1) {
      st = true;
    } else {
      const int c = L.icnt[s];
      if (c != L.icnt[s - 1]) {
        st = true;
      } else {
        const Item *x = L.items + L.ioff[s];
        const Item *y = L.items + L.ioff[s - 1];
        for (int k = 0; k < c; ++k)
          if (!item_eq(x[k], y[k])) {
            st = true;
            break;
          }
      }
    }
  }
  const uint64_t m = __ballot(st);
  const int chunk = s >> 6;
  if ((threadIdx.x & 63) == 0 && chunk * 64 < L.nsl) {
    L.bmask[chunk] = m;
    L.bcnt[chunk] = __popcll(m);
  }
}

// ------------------------------------------------------------ block scans
// Exclusive scan of one value per thread over a 1024-thread block; returns
// the exclusive prefix and writes the block total to *total.
template <typename T>
__device__ T block_exscan(T v, T *total) {
  __shared__ T s_w[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) s_w[wv] = x;
  __syncthreads();
  if (wv == 0) {
    T w = lane < 16 ? s_w[lane] : T(0);
#pragma unroll
    for (int d = 1; d < 16; d <<= 1) {
      T y = __shfl_up(w, d);
      if (lane >= d) w += y;
    }
    if (lane < 16) s_w[lane] = w;
  }
  __syncthreads();
  const T wbase = wv ? s_w[wv - 1] : T(0);
  *total = s_w[15];
  __syncthreads();
  return wbase + x - v;
}

// ----------------------------------------------------------- k_bandscan
constexpr int kScanIt = 4;

__global__ __launch_bounds__(1024) void k_bandscan(Level L) {
  const int nchunk = (L.nsl + 63) / 64;
  int carry = 0;
  for (int base = 0; base < nchunk; base += 1024 * kScanIt) {
    int v[kScanIt];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < kScanIt; ++k) {
      const int c = base + threadIdx.x * kScanIt + k;
      v[k] = c < nchunk ? L.bcnt[c] : 0;
      sum += v[k];
    }
    int tot;
    int ex = block_exscan<int>(sum, &tot) + carry;
#pragma unroll
    for (int k = 0; k < kScanIt; ++k) {
      const int c = base + threadIdx.x * kScanIt + k;
      if (c < nchunk) L.bbase[c] = ex;
      ex += v[k];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) *L.nb = carry;
  __syncthreads();
  for (int c = threadIdx.x; c < nchunk; c += 1024) {
    uint64_t m = L.bmask[c];
    int b = L.bbase[c];
    while (m) {
      const int bit = __ffsll((long long)m) - 1;
      L.bandslice[b++] = c * 64 + bit;
      m &= m - 1;
    }
  }
  if (threadIdx.x == 0) L.bandslice[carry] = L.nsl;
}

// --------------------------------------------------------------- k_heads
__device__ inline int band_of(const Level &L, int s) {
  const int c = s >> 6;
  return L.bbase[c] + __popcll(L.bmask[c] & ((1ull << (s & 63)) - 1ull));
}

__global__ __launch_bounds__(256) void k_heads(Level L, int32_t *err) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int nb = *L.nb;
  if (b >= nb) return;
  const int s0 = L.bandslice[b], s1 = L.bandslice[b + 1];
  const bool adj = s0 > 0 && L.grp[s0 - 1] == L.grp[s0] && L.pos[s0 - 1] + 1 == L.pos[s0];
  const Item *cur = L.items + L.ioff[s0];
  const int cc = L.icnt[s0];
  const Item *prv = adj ? L.items + L.ioff[s0 - 1] : nullptr;
  const int pc = adj ? L.icnt[s0 - 1] : 0;
  int nh = 0;
  for (int k = 0; k < cc; ++k)
    if (!(adj && contains(prv, pc, cur[k]))) ++nh;
  int off = 0;
  if (nh) {
    off = atomicAdd(L.head_top, nh);
    if ((int64_t)off + nh > L.head_cap) {
      set_err(err, -8);
      nh = 0;
    }
  }
  L.hoff[b] = off;
  L.hcnt[b] = nh;
  int h = 0;
  for (int k = 0; k < cc && h < nh; ++k) {
    const Item it = cur[k];
    if (adj && contains(prv, pc, it)) continue;
    int e = s1;
    while (e < L.nsl && L.grp[e] == L.grp[e - 1] && L.pos[e] == L.pos[e - 1] + 1 &&
           contains(L.items + L.ioff[e], L.icnt[e], it))
      e = L.bandslice[band_of(L, e) + 1];
    Item o = it;
    o.pos0 = L.pos[s0];
    o.pos1 = L.pos[e - 1] + 1;
    L.heads[off + h] = o;
    ++h;
  }
}

// ------------------------------------------------------------- k_compact
// mode 0: level-1 heads are the final messages (all arrays at most 2-D)
// mode 1: level-1 heads become the level-2 items (per-group lists)
// mode 2: level-2 heads are the final messages
__device__ inline int64_t head_volume(const Item &h, int mode) {
  if (mode == 0) return (int64_t)(h.pos1 - h.pos0) * (h.a1 - h.a0);
  return (int64_t)(h.pos1 - h.pos0) * (h.b1 - h.b0) * (h.a1 - h.a0);
}

__global__ __launch_bounds__(1024) void k_compact(PlanDev P, Level L, Work W, MsgRec *out, MsgHdr *hdr,
                                                  int64_t out_cap, int mode) {
  __shared__ int64_t s_carry_b;
  __shared__ int s_carry_n;
  const int nb = L.nsl ? *L.nb : 0;
  if (threadIdx.x == 0) {
    s_carry_b = 0;
    s_carry_n = 0;
  }
  __syncthreads();
  for (int j = 0; j < P.ncarr; ++j) {
    const CallArr ca = P.carr[j];
    const int sa = mode == 2 ? ca.grp0 : ca.slice0;
    const int sb = mode == 2 ? ca.grp1 : ca.slice1;
    if (sa >= sb) continue;
    const int b0 = band_of(L, sa);
    const int b1 = sb < L.nsl ? band_of(L, sb) : nb;
    if (threadIdx.x == 0 && mode != 1) s_carry_b = (s_carry_b + ca.esize - 1) / ca.esize * ca.esize;
    __syncthreads();
    for (int base = b0; base < b1; base += 1024 * kScanIt) {
      int cn[kScanIt];
      int64_t by[kScanIt];
      int sn = 0;
      int64_t sbyt = 0;
#pragma unroll
      for (int k = 0; k < kScanIt; ++k) {
        const int b = base + threadIdx.x * kScanIt + k;
        cn[k] = 0;
        by[k] = 0;
        if (b < b1) {
          cn[k] = L.hcnt[b];
          if (mode != 1)
            for (int h = 0; h < cn[k]; ++h) by[k] += head_volume(L.heads[L.hoff[b] + h], mode) * ca.esize;
        }
        sn += cn[k];
        sbyt += by[k];
      }
      const int cn0 = s_carry_n;
      const int64_t cb0 = s_carry_b;
      int totn;
      int64_t totb;
      int exn = block_exscan<int>(sn, &totn) + cn0;
      int64_t exb = block_exscan<int64_t>(sbyt, &totb) + cb0;
#pragma unroll
      for (int k = 0; k < kScanIt; ++k) {
        const int b = base + threadIdx.x * kScanIt + k;
        if (b >= b1) break;
        const Item *hs = L.heads + L.hoff[b];
        const int s0 = L.bandslice[b];
        if (mode == 1) {
          const int g = L.grp[s0];
          const bool gstart = s0 == 0 || L.grp[s0 - 1] != g;
          if (gstart) W.goff[g] = exn;
          for (int h = 0; h < cn[k]; ++h) {
            if (exn + h < W.l1_cap) {
              Item it = hs[h];
              // rows of the stacked run become the item's b-range
              W.l1out[exn + h] = Item{it.src, it.dst, it.a0, it.a1, it.pos0, it.pos1, 0, 0};
            }
          }
        } else {
          int64_t ob = exb;
          for (int h = 0; h < cn[k]; ++h) {
            const Item it = hs[h];
            MsgRec r;
            r.aidx = j;
            r.arr = ca.arr;
            r.src = it.src;
            r.dst = it.dst;
            if (mode == 0) {
              const int plane = P.grp_plane[L.grp[s0]];
              r.lo[0] = plane;
              r.hi[0] = plane + 1;
              r.lo[1] = it.pos0;
              r.hi[1] = it.pos1;
            } else {
              r.lo[0] = it.pos0;
              r.hi[0] = it.pos1;
              r.lo[1] = it.b0;
              r.hi[1] = it.b1;
            }
            r.lo[2] = it.a0;
            r.hi[2] = it.a1;
            r.argpos = ca.argpos;
            r.esize = ca.esize;
            r.off = ob;
            r.bytes = head_volume(it, mode) * ca.esize;
            ob += r.bytes;
            if (exn + h < out_cap) out[exn + h] = r;
          }
        }
        exn += cn[k];
        exb += by[k];
      }
      if (threadIdx.x == 0) {
        s_carry_n += totn;
        s_carry_b += totb;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  if (mode == 1) {
    // per-group counts from consecutive offsets (every group has >= 1 band)
    for (int g = threadIdx.x; g < P.ngrp; g += 1024) {
      const int e = (g + 1 < P.ngrp) ? W.goff[g + 1] : s_carry_n;
      W.gcnt[g] = e - W.goff[g];
    }
    if (threadIdx.x == 0) {
      if (s_carry_n > W.l1_cap) set_err(W.err, -8);
      *L.head_top = 0;  // the next level reuses the head pool
    }
  } else if (threadIdx.x == 0) {
    if (s_carry_n > out_cap) set_err(W.err, -8);
    hdr->nmsg = s_carry_n < out_cap ? s_carry_n : out_cap;
    hdr->bytes = s_carry_b;
    *L.head_top = 0;  // pools are free for the next call
    *W.run_top = 0;
  }
}

// Every row starts as one interval [0, n2) owned and held by the host.
__global__ void k_init_rows(Ivl *ivl, int32_t *cnt, int64_t rows, int cap) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < rows; g += (int64_t)gridDim.x * blockDim.x) {
    ivl[g * cap] = Ivl{0, kHost, 1ull << kHost};
    cnt[g] = 1;
  }
}

// ---------------------------------------------------------------- k_gdef
// One wave per touched row.  Edits: holder additions from the row's runs
// (every receiver of an element becomes a holder) then definitions (owner =
// definer, holders = {definer} [+ host for Write]).
__global__ __launch_bounds__(64) void k_gdef(PlanDev P, ArrDev *__restrict__ A, Work W) {
  __shared__ Ivl s_iv[kMaxCap];
  __shared__ int32_t s_b[kMaxBoundaries];
  __shared__ int32_t s_u[kMaxBoundaries];
  __shared__ int32_t s_own[kMaxBoundaries];
  __shared__ uint64_t s_hold[kMaxBoundaries];
  const int lane = threadIdx.x;
  for (int t = blockIdx.x; t < P.ngrow; t += gridDim.x) {
    const int aidx = P.gr_aidx[t];
    ArrDev &a = A[P.carr[aidx].arr];
    const int64_t grow = P.gr_row[t];
    const int n = a.cnt[grow];
    const int W2 = (int)a.n[2];
    Ivl *row = a.ivl + grow * (int64_t)a.cap;
    const int sl = P.gr_slice[t];
    const Item *runs = sl >= 0 ? W.runs + W.roff[sl] : nullptr;
    const int nrun = sl >= 0 ? W.rcnt[sl] : 0;
    const Seg *ds = P.dseg + P.gr_dseg0[t];
    const int nds = P.gr_ndseg[t];
    const int nbnd = n + 2 * (nrun + nds);
    if (nbnd > kMaxBoundaries) {
      if (lane == 0) set_err(W.err, -8);
      continue;
    }
    for (int i = lane; i < n; i += 64) {
      s_iv[i] = row[i];
      s_b[i] = row[i].start;
    }
    for (int e = lane; e < nrun; e += 64) {
      s_b[n + 2 * e] = runs[e].a0;
      s_b[n + 2 * e + 1] = runs[e].a1 < W2 ? runs[e].a1 : 0;
    }
    for (int e = lane; e < nds; e += 64) {
      s_b[n + 2 * nrun + 2 * e] = ds[e].c0;
      s_b[n + 2 * nrun + 2 * e + 1] = ds[e].c1 < W2 ? ds[e].c1 : 0;
    }
    wave_lds_sync();
    // stable rank sort of the boundaries
    for (int i = lane; i < nbnd; i += 64) {
      const int x = s_b[i];
      int r = 0;
      for (int j = 0; j < nbnd; ++j) {
        const int y = s_b[j];
        r += (y < x) || (y == x && j < i);
      }
      s_u[r] = x;
    }
    wave_lds_sync();
    // unique, in place into s_b
    int nu = 0;
    for (int base = 0; base < nbnd; base += 64) {
      const int i = base + lane;
      const bool keep = i < nbnd && (i == 0 || s_u[i] != s_u[i - 1]);
      const int x = i < nbnd ? s_u[i] : 0;
      const uint64_t m = __ballot(keep);
      wave_lds_sync();
      if (keep) s_b[nu + __popcll(m & lanemask_lt())] = x;
      nu += __popcll(m);
      wave_lds_sync();
    }
    // state of every elementary segment
    for (int k = lane; k < nu; k += 64) {
      const int x = s_b[k];
      int lo = 0, hi = n - 1;  // last interval with start <= x
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_iv[mid].start <= x)
          lo = mid;
        else
          hi = mid - 1;
      }
      int own = s_iv[lo].owner;
      uint64_t hol = s_iv[lo].holders;
      for (int e = 0; e < nrun; ++e)
        if (runs[e].a0 <= x && x < runs[e].a1) hol |= 1ull << runs[e].dst;
      for (int e = 0; e < nds; ++e)
        if (ds[e].c0 <= x && x < ds[e].c1) {
          own = ds[e].dst;
          hol = (1ull << ds[e].dst) | ((ds[e].flags & 1) ? (1ull << kHost) : 0ull);
        }
      s_own[k] = own;
      s_hold[k] = hol;
    }
    wave_lds_sync();
    // merge equal neighbours and write the new list
    int nn = 0;
    for (int base = 0; base < nu; base += 64) {
      const int k = base + lane;
      const bool keep = k < nu && (k == 0 || s_own[k] != s_own[k - 1] || s_hold[k] != s_hold[k - 1]);
      const uint64_t m = __ballot(keep);
      if (keep) {
        const int p = nn + __popcll(m & lanemask_lt());
        if (p < a.cap) row[p] = Ivl{s_b[k], s_own[k], s_hold[k]};
      }
      nn += __popcll(m);
    }
    if (lane == 0) {
      if (nn > a.cap) {
        set_err(W.err, -8);
      } else {
        a.cnt[grow] = nn;
      }
    }
    wave_lds_sync();
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
  int grid = P.ngrow < 16384 ? P.ngrow : 16384;
  hipLaunchKernelGGL(k_gdef, dim3(grid), dim3(64), 0, s, P, A, W);
  return hipGetLastError();
}

}  // namespace hd

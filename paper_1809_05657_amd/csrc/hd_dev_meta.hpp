// hd_dev_meta.hpp — device functions of the communication-set derivation and
// the GDEF update, shared by the per-phase kernels (hd_meta.hip) and the
// persistent batched kernel (hd_batch.hip) so both compute identical results.
//
// Paper: Sec. 2.2, Eq. 1-2 (messages = GDEF intersected with LUSE, taken
// right before the kernel) and Eq. 3-4 (GDEF update: receivers become
// holders, a definition makes the definer the owner and only holder).
// Sec. 4.2 merges adjacent sections; here the merge is made canonical:
//   runs    maximal innermost-dimension runs with one source, per (row, dst);
//   level 1 runs identical on consecutive rows of a plane stack into rects;
//   level 2 rects identical on consecutive planes stack into boxes;
//   order   (argument, lower corner row-major, destination).
//
// Steps (all device-resident, no host readback):
//   dev_runs       one wave per use row: intersect the row's GDEF interval
//                  list with every destination's use segments (wave ballot +
//                  prefix popcount compaction), rank-sort runs by (col, dst)
//   dev_bandflags  one lane per slice: a band starts where the item list or
//                  the adjacency changes (ballot -> 64-bit chunk mask)
//   dev_bandscan   one workgroup: exclusive scan of band counts, band -> slice
//   dev_heads      one lane per band: items not continued from the previous
//                  slice are heads; their extent is found by walking bands
//   dev_compact    one workgroup: scan of head counts and bytes -> message
//                  table in canonical order with pack offsets (or level-1 list)
//   dev_gdef_row   one wave per touched row: apply holder additions and
//                  definitions to the row's interval list, re-merge
#pragma once
#include <hip/hip_runtime.h>

#include "hd_internal.hpp"

namespace hd {

__device__ inline uint64_t lanemask_lt() {
  const unsigned lane = threadIdx.x & 63;
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Orders the LDS accesses of the lanes of one wave: the LDS executes a
// wave's operations in issue order, so a wavefront-scope fence (which keeps
// the compiler from moving LDS accesses across it) is enough; a wider scope
// would also wait for every outstanding global memory operation.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ inline void set_err(int32_t *err, int code) { atomicCAS(err, 0, code); }

// End (exclusive) of slice s's positions.
__device__ inline int pend_of(const Level &L, int s) { return L.pend ? L.pend[s] : L.pos[s] + 1; }

// Value of v in lane l (l the same in every lane).
__device__ inline int lane_read(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

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

// ------------------------------------------------------------------- runs
// One wave (all 64 lanes) finds the runs of use row s and leaves them in rr
// in discovery order: by use segment (destination, then column; the
// planner merges each destination's segments of a row, so they are
// disjoint and sorted), then by column.  That order is a function of the
// run set alone, so two rows have the same runs iff their rr lists are
// equal.  iv (at least the row capacity) and rr (maxr runs) are LDS
// scratch private to the wave.  Returns the run count (0 after a capacity
// error, which is recorded).

__device__ inline int dev_runs_find(const PlanDev &P, const ArrDev *__restrict__ A, const Work &W, int s, Ivl *iv,
                                    Run *rr, int maxr = kMaxRunsRow) {
  const int lane = threadIdx.x & 63;
  const SliceRec sr = P.srec[s];
  const ArrDev &a = A[sr.arr];
  const Ivl *row = a.ivl + sr.grow * (int64_t)a.cap;
  const int W2 = (int)a.n[2];
  // the first 64 intervals are read together with the count (the row's
  // capacity bounds the read) and with the first 64 use segments (one per
  // lane, read back with lane reads)
  Ivl v0{};
  if (lane < a.cap) v0 = row[lane];
  Seg mine{0, 0, 0, 0};
  if (lane < sr.nseg) mine = P.useg[sr.seg0 + lane];
  const int n = a.cnt[sr.grow];
  if (lane < n) iv[lane] = v0;
  for (int i = 64 + lane; i < n; i += 64) iv[i] = row[i];
  wave_lds_sync();
  int nr = 0;
  for (int sb = 0; sb < sr.nseg; sb += 64) {
    if (sb > 0) {
      mine = Seg{0, 0, 0, 0};
      if (sb + lane < sr.nseg) mine = P.useg[sr.seg0 + sb + lane];
    }
    const int sn = min(64, sr.nseg - sb);
    for (int q = 0; q < sn; ++q) {
      const int sdst = lane_read(mine.dst, q), sc0 = lane_read(mine.c0, q), sc1 = lane_read(mine.c1, q);
      const uint64_t bit = 1ull << sdst;
      auto need = [&](int i) -> bool {
        const int st = iv[i].start, en = (i + 1 < n) ? iv[i + 1].start : W2;
        return max(st, sc0) < min(en, sc1) && !(iv[i].holders & bit);
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
          const int c0 = max(iv[i].start, sc0);
          const int c1 = min((j < n) ? iv[j].start : W2, sc1);
          const int k = nr + __popcll(m & lanemask_lt());
          if (k < maxr) rr[k] = Run{src, sdst, c0, c1};
        }
        nr += __popcll(m);
      }
    }
  }
  if (nr > maxr) {
    if (lane == 0) set_err(W.err, -8);
    nr = 0;
  }
  wave_lds_sync();
  return nr;
}

// One use row per lane, for rows with at most kLaneIvl intervals, kLaneSeg
// use segments and LR runs (LR <= kRunSlot; the common case: a few owners
// per row): the intervals sit in registers, the runs are found in the same
// order as by the wave (by segment, then column; consecutive needed
// intervals of one owner merge), staged in the lane's own column of lr
// ([4 * LR][64]: src, dst, a0, a1) and stored rank-sorted by (col, dst) into
// the row's slot, exactly as the wave stores them.  Returns false, writing
// nothing, for any other row.
constexpr int kLaneIvl = 8, kLaneSeg = 8;
template <int LR = kRunSlot>
__device__ inline bool dev_runs_lane(const PlanDev &P, const ArrDev *__restrict__ A, const Work &W, int s,
                                     int32_t *lr) {
  static_assert(LR <= kRunSlot, "runs beyond the row's slot take the wave path");
  const int lane = threadIdx.x & 63;
  const SliceRec sr = P.srec[s];
  if (sr.nseg > kLaneSeg) return false;
  // the segments, the row's count and its first intervals (bounded by the
  // row's capacity) are all requested before any is used
  Seg segs[kLaneSeg];
#pragma unroll
  for (int q = 0; q < kLaneSeg; ++q) segs[q] = q < sr.nseg ? P.useg[sr.seg0 + q] : Seg{0, 0, 0, 0};
  const ArrDev &a = A[sr.arr];
  const Ivl *row = a.ivl + sr.grow * (int64_t)a.cap;
  Ivl v8[kLaneIvl];
#pragma unroll
  for (int i = 0; i < kLaneIvl; ++i) v8[i] = i < a.cap ? row[i] : Ivl{0, 0, 0ull};
  const int n = a.cnt[sr.grow];
  if (n > kLaneIvl) return false;
  const int W2 = (int)a.n[2];
  int st[kLaneIvl + 1], ow[kLaneIvl];
  uint64_t ho[kLaneIvl];
#pragma unroll
  for (int i = 0; i < kLaneIvl; ++i) {
    st[i] = W2;
    ow[i] = -1;
    ho[i] = ~0ull;
    if (i < n) {
      st[i] = v8[i].start;
      ow[i] = v8[i].owner;
      ho[i] = v8[i].holders;
    }
  }
  st[kLaneIvl] = W2;
  int nr = 0;
  bool over = false;
  auto emit = [&](int src, int dst, int a0, int a1) {
    if (nr < LR) {
      lr[(4 * nr + 0) * 64 + lane] = src;
      lr[(4 * nr + 1) * 64 + lane] = dst;
      lr[(4 * nr + 2) * 64 + lane] = a0;
      lr[(4 * nr + 3) * 64 + lane] = a1;
    } else {
      over = true;
    }
    ++nr;
  };
#pragma unroll
  for (int q = 0; q < kLaneSeg; ++q) {
    if (q < sr.nseg) {
      const Seg S = segs[q];
      const uint64_t bit = 1ull << S.dst;
      int cs = -1, c0 = 0, c1 = 0;
#pragma unroll
      for (int i = 0; i < kLaneIvl; ++i) {
        const int en = st[i + 1];
        const bool nd = i < n && max(st[i], S.c0) < min(en, S.c1) && !(ho[i] & bit);
        if (nd && cs == ow[i]) {
          c1 = min(en, S.c1);
        } else {
          if (cs >= 0) emit(cs, S.dst, c0, c1);
          cs = -1;
          if (nd) {
            cs = ow[i];
            c0 = max(st[i], S.c0);
            c1 = min(en, S.c1);
          }
        }
      }
      if (cs >= 0) emit(cs, S.dst, c0, c1);
    }
  }
  if (over) return false;
  const int off = s * kRunSlot;
  for (int i = 0; i < nr; ++i) {
    const int xa = lr[(4 * i + 2) * 64 + lane], xd = lr[(4 * i + 1) * 64 + lane];
    int rank = 0;
    for (int j = 0; j < nr; ++j) {
      const int ya = lr[(4 * j + 2) * 64 + lane], yd = lr[(4 * j + 1) * 64 + lane];
      rank += (ya < xa) || (ya == xa && yd < xd);
    }
    W.runs[off + rank] = Item{lr[(4 * i) * 64 + lane], xd, xa, lr[(4 * i + 3) * 64 + lane], 0, 0, 0, 0};
  }
  W.roff[s] = nr ? off : 0;
  W.rcnt[s] = nr;
  return true;
}

// Stores the runs of slice s sorted by (col, dst) (rank sort; the keys are
// unique because the runs of one destination are disjoint): the row's own
// slot, or the spill pool after all slots.
__device__ inline void dev_runs_store(const PlanDev &P, const Work &W, int s, const Run *rr, int nr) {
  const int lane = threadIdx.x & 63;
  int off = s * kRunSlot;
  if (nr > kRunSlot) {
    const int64_t pool0 = (int64_t)P.nsl1 * kRunSlot;
    if (lane == 0) {
      off = atomicAdd(W.run_top, nr);
      if (pool0 + off + nr > W.run_cap) {
        set_err(W.err, -8);
        off = -1;
      } else {
        off += (int)pool0;
      }
    }
    off = __shfl(off, 0);
    if (off < 0) nr = 0;
  }
  for (int i = lane; i < nr; i += 64) {
    const Run x = rr[i];
    int rank = 0;
    for (int j = 0; j < nr; ++j) {
      const Run y = rr[j];
      rank += (y.a0 < x.a0) || (y.a0 == x.a0 && y.dst < x.dst);
    }
    W.runs[off + rank] = Item{x.src, x.dst, x.a0, x.a1, 0, 0, 0, 0};
  }
  if (lane == 0) {
    W.roff[s] = nr ? off : 0;
    W.rcnt[s] = nr;
  }
}

__device__ inline void dev_runs(const PlanDev &P, const ArrDev *__restrict__ A, const Work &W, int s, Ivl *iv,
                                Run *rr, int maxr = kMaxRunsRow) {
  const int nr = dev_runs_find(P, A, W, s, iv, rr, maxr);
  dev_runs_store(P, W, s, rr, nr);
  wave_lds_sync();
}

// -------------------------------------------------------------- band flags
// Called by whole waves; s = 64 * chunk + lane.
__device__ inline void dev_bandflags(const Level &L, int s) {
  bool st = false;
  if (s < L.nsl) {
    if (s == 0) {
      st = true;
    } else {
      // every index is read in one round; the item lists are compared four
      // pairs at a time (loads issued together)
      const int g0 = L.grp[s], g1 = L.grp[s - 1], p0 = L.pos[s];
      const int c = L.icnt[s], cp = L.icnt[s - 1];
      const Item *x = L.items + L.ioff[s];
      const Item *y = L.items + L.ioff[s - 1];
      st = g0 != g1 || p0 != pend_of(L, s - 1) || c != cp;
      for (int k = 0; k < c && !st; k += 4) {
        Item xa[4], ya[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (k + q < c) {
            xa[q] = x[k + q];
            ya[q] = y[k + q];
          }
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (k + q < c && !item_eq(xa[q], ya[q])) st = true;
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
// Exclusive scan of one value per thread over the whole workgroup (at most
// 16 waves); returns the exclusive prefix, writes the total to *total.
template <typename T>
__device__ T block_exscan(T v, T *total) {
  __shared__ T s_w[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  T x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) s_w[wv] = x;
  __syncthreads();
  if (wv == 0) {
    T w = lane < nw ? s_w[lane] : T(0);
#pragma unroll
    for (int d = 1; d < 16; d <<= 1) {
      T y = __shfl_up(w, d);
      if (lane >= d) w += y;
    }
    if (lane < nw) s_w[lane] = w;
  }
  __syncthreads();
  const T wbase = wv ? s_w[wv - 1] : T(0);
  *total = s_w[nw - 1];
  __syncthreads();
  return wbase + x - v;
}

constexpr int kScanIt = 4;

// ---------------------------------------------------------------- band scan
__device__ inline void dev_bandscan(const Level &L) {
  const int nchunk = (L.nsl + 63) / 64;
  const int nt = blockDim.x;
  int carry = 0;
  for (int base = 0; base < nchunk; base += nt * kScanIt) {
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
  for (int c = threadIdx.x; c < nchunk; c += nt) {
    uint64_t m = L.bmask[c];
    int b = L.bbase[c];
    while (m) {
      const int bit = __ffsll((long long)m) - 1;
      L.bandslice[b++] = c * 64 + bit;
      m &= m - 1;
    }
  }
  if (threadIdx.x == 0) L.bandslice[carry] = L.nsl;
  __syncthreads();
}

// -------------------------------------------------------------------- heads
__device__ inline int band_of(const Level &L, int s) {
  const int c = s >> 6;
  return L.bbase[c] + __popcll(L.bmask[c] & ((1ull << (s & 63)) - 1ull));
}

// One wave per band b (nb bands); lanes take the items of the band's first
// slice.  An item not continued from the previous (adjacent) slice is a
// head; its extent is found by walking the following bands while their
// first slice holds it: the wave walks all its heads together, band by
// band, reading each band's items once into LDS (sp: the previous slice,
// sw: the band being walked; hcap items each, larger lists are searched in
// global memory).  Heads keep the item order and are stored at their items'
// positions.
constexpr int kHeadLds = 128;

__device__ inline void lds_items(Item *dst, const Item *src, int cnt, int hcap) {
  const int lane = threadIdx.x & 63;
  if (cnt <= hcap)
    for (int k = lane; k < cnt; k += 64) dst[k] = src[k];
}

__device__ inline void dev_heads(const Level &L, int b, int nb, Item *sp, Item *sw, int hcap = kHeadLds) {
  const int lane = threadIdx.x & 63;
  const int s0 = L.bandslice[b], s1 = L.bandslice[b + 1];
  const bool adj = s0 > 0 && L.grp[s0 - 1] == L.grp[s0] && pend_of(L, s0 - 1) == L.pos[s0];
  const int off = L.ioff[s0];
  const Item *cur = L.items + off;
  const int cc = L.icnt[s0];
  const Item *prv = adj ? L.items + L.ioff[s0 - 1] : nullptr;
  const int pc = adj ? L.icnt[s0 - 1] : 0;
  const int p0 = L.pos[s0];
  // the next 64 bands, one per lane: does the band continue the slice before
  // it (same group, next position), its first slice's item count and
  // offset, and the slice after it; read back with lane reads in the walk
  const int bl = b + 1 + lane;
  int n_cont = 0, n_tc = 0, n_to = 0, n_end = L.nsl;
  if (bl < nb) {
    const int t0 = L.bandslice[bl];
    n_end = L.bandslice[bl + 1];
    if (t0 < L.nsl) {
      n_cont = L.grp[t0] == L.grp[t0 - 1] && L.pos[t0] == pend_of(L, t0 - 1);
      n_tc = L.icnt[t0];
      n_to = L.ioff[t0];
    }
  }
  lds_items(sp, prv, pc, hcap);
  wave_lds_sync();
  int nh = 0;
  int64_t vol = 0;
  for (int base = 0; base < cc; base += 64) {
    const int k = base + lane;
    Item it{};
    bool head = false;
    if (k < cc) {
      it = cur[k];
      head = !(adj && (pc <= hcap ? contains(sp, pc, it) : contains(prv, pc, it)));
    }
    const uint64_t m = __ballot(head);
    int e = s1;
    bool go = head;
    for (int bb = b + 1; __ballot(go) != 0ull; ++bb) {
      const int q = bb - b - 1;
      int cont, tc, toff, tend;
      if (q < 64) {
        cont = lane_read(n_cont, q);
        tc = lane_read(n_tc, q);
        toff = lane_read(n_to, q);
        tend = lane_read(n_end, q);
      } else {
        const int t0 = bb < nb ? L.bandslice[bb] : L.nsl;
        cont = bb < nb && t0 < L.nsl && L.grp[t0] == L.grp[t0 - 1] && L.pos[t0] == pend_of(L, t0 - 1);
        tc = cont ? L.icnt[t0] : 0;
        toff = cont ? L.ioff[t0] : 0;
        tend = cont ? L.bandslice[bb + 1] : L.nsl;
      }
      if (!cont) break;
      const Item *ti = L.items + toff;
      wave_lds_sync();
      lds_items(sw, ti, tc, hcap);
      wave_lds_sync();
      if (go) {
        if (tc <= hcap ? contains(sw, tc, it) : contains(ti, tc, it))
          e = tend;
        else
          go = false;
      }
    }
    if (head) {
      it.pos0 = p0;
      it.pos1 = pend_of(L, e - 1);
      L.heads[off + nh + __popcll(m & lanemask_lt())] = it;
      vol += (int64_t)(it.pos1 - it.pos0) * (it.a1 - it.a0) * max(1, it.b1 - it.b0);
    }
    nh += __popcll(m);
  }
  wave_lds_sync();
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) vol += __shfl_xor(vol, d);
  if (lane == 0) {
    const int g = L.grp[s0];
    const int j = L.grp_carr ? L.grp_carr[g] : g;
    L.hoff[b] = off;
    L.hcnt[b] = nh;
    L.bcarr[b] = j;
    L.hbytes[b] = vol * L.carr[j].esize;
  }
}

// ------------------------------------------------------------------ compact
// mode 0: level-1 heads are the final messages (all arrays at most 2-D)
// mode 1: level-1 heads become the level-2 items (per-group lists)
// mode 2: level-2 heads are the final messages
__device__ inline int64_t head_volume(const Item &h, int mode) {
  if (mode == 0) return (int64_t)(h.pos1 - h.pos0) * (h.a1 - h.a0);
  return (int64_t)(h.pos1 - h.pos0) * (h.b1 - h.b0) * (h.a1 - h.a0);
}

// Writes the heads of band b as messages (modes 0, 2) starting at message
// exn and byte offset ob, or as level-2 items (mode 1) starting at exn.
__device__ inline void compact_band(const PlanDev &P, const Level &L, const Work &W, MsgRec *out, int64_t out_cap,
                                    int mode, int b, int exn, int64_t ob) {
  const int j = L.bcarr[b];
  const int cnt = L.hcnt[b];
  const Item *hs = L.heads + L.hoff[b];
  const int s0 = L.bandslice[b];
  if (mode == 1) {
    const int g = L.grp[s0];
    const bool gstart = s0 == 0 || L.grp[s0 - 1] != g;
    if (gstart) W.goff[g] = exn;
    for (int h = 0; h < cnt; ++h) {
      if (exn + h < W.l1_cap) {
        const Item it = hs[h];
        // rows of the stacked run become the item's b-range
        W.l1out[exn + h] = Item{it.src, it.dst, it.a0, it.a1, it.pos0, it.pos1, 0, 0};
      }
    }
    return;
  }
  const CallArr ca = P.carr[j];
  const int plane = mode == 0 ? P.grp_plane[L.grp[s0]] : 0;
  for (int h = 0; h < cnt; ++h) {
    const Item it = hs[h];
    MsgRec r;
    r.aidx = j;
    r.arr = ca.arr;
    r.src = it.src;
    r.dst = it.dst;
    if (mode == 0) {
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

// lds: 2 * kCompactCarr int64 of LDS scratch
__device__ inline void dev_compact(const PlanDev &P, const Level &L, const Work &W, MsgRec *out, MsgHdr *hdr,
                                   int64_t out_cap, int mode, int64_t *lds) {
  // one workgroup: (A) a flat exclusive scan of head counts and bytes over
  // all bands; (B) the alignment padding at the first band of every
  // call-array (pack offsets are aligned to the element size), in call-array
  // order; (C) every band writes its heads at its offsets
  int64_t *s_raw = lds;                 // byte prefix at the call-array's first band, -1: none
  int64_t *s_pad = lds + kCompactCarr;  // padding inserted up to and including that call-array
  __shared__ int64_t s_carry_b, s_total_b;
  __shared__ int s_carry_n;
  const int nt = blockDim.x;
  const int nb = L.nsl ? *L.nb : 0;
  const int ncarr = P.ncarr < kCompactCarr ? P.ncarr : kCompactCarr;
  for (int j = threadIdx.x; j < ncarr; j += nt) s_raw[j] = -1;
  if (threadIdx.x == 0) {
    s_carry_b = 0;
    s_carry_n = 0;
    if (P.ncarr > kCompactCarr) set_err(W.err, -8);
  }
  __syncthreads();
  for (int base = 0; base < nb; base += nt * kScanIt) {
    int cn[kScanIt];
    int64_t by[kScanIt];
    bool first[kScanIt];
    int jj[kScanIt];
    int sn = 0;
    int64_t sbyt = 0;
#pragma unroll
    for (int k = 0; k < kScanIt; ++k) {
      const int b = base + threadIdx.x * kScanIt + k;
      cn[k] = 0;
      by[k] = 0;
      first[k] = false;
      jj[k] = 0;
      if (b < nb) {
        cn[k] = L.hcnt[b];
        jj[k] = L.bcarr[b];
        if (mode != 1) by[k] = L.hbytes[b];
        first[k] = b == 0 || L.bcarr[b - 1] != jj[k];
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
      if (b >= nb) break;
      L.nofs[b] = exn;
      L.bofs[b] = exb;
      if (first[k] && jj[k] < kCompactCarr) s_raw[jj[k]] = exb;
      exn += cn[k];
      exb += by[k];
    }
    if (threadIdx.x == 0) {
      s_carry_n += totn;
      s_carry_b += totb;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int64_t pad = 0;
    for (int j = 0; j < ncarr; ++j) {
      if (s_raw[j] >= 0 && mode != 1) {
        const int64_t at = s_raw[j] + pad, e = P.carr[j].esize;
        pad += (at + e - 1) / e * e - at;
      }
      s_pad[j] = pad;
    }
    s_total_b = s_carry_b + pad;
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += nt) {
    const int j = L.bcarr[b];
    compact_band(P, L, W, out, out_cap, mode, b, L.nofs[b], L.bofs[b] + (j < kCompactCarr ? s_pad[j] : 0));
  }
  __syncthreads();
  if (mode == 1) {
    // per-group counts from consecutive offsets (every group has >= 1 band)
    for (int g = threadIdx.x; g < P.ngrp; g += nt) {
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
    hdr->bytes = s_total_b;
    *L.head_top = 0;  // pools are free for the next call
    *W.run_top = 0;
  }
  __syncthreads();
}

// Compaction by all workgroups of a persistent launch (modes 0 and 2), in
// three phases separated by grid barriers.  cs: scratch of 6 * kCompactCarr
// int64: chunk totals (count, bytes), chunk prefixes (count, bytes), and per
// call-array the local byte prefix of its first band and that band's chunk
// (-1: no band; reset by dev_compact_reset before the heads phase).
// Workgroup w owns bands [nb * w / G, nb * (w + 1) / G), G <= kCompactCarr.
struct CScratch {
  int64_t *tot_n, *tot_b, *pre_n, *pre_b, *first_b, *first_c;
  __device__ CScratch(int64_t *cs)
      : tot_n(cs), tot_b(cs + kCompactCarr), pre_n(cs + 2 * kCompactCarr), pre_b(cs + 3 * kCompactCarr),
        first_b(cs + 4 * kCompactCarr), first_c(cs + 5 * kCompactCarr) {}
};

__device__ inline void dev_compact_reset(const PlanDev &P, int64_t *cs) {
  CScratch c(cs);
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < kCompactCarr; j += gridDim.x * blockDim.x) c.first_c[j] = -1;
}

// phase 1: scan of the workgroup's own chunk of bands
__device__ inline void dev_compact_p1(const Level &L, int64_t *cs, int mode) {
  CScratch c(cs);
  __shared__ int64_t s_cb;
  __shared__ int s_cn;
  const int nb = L.nsl ? *L.nb : 0;
  const int G = gridDim.x, w = blockIdx.x, nt = blockDim.x;
  const int b0 = (int)((int64_t)nb * w / G), b1 = (int)((int64_t)nb * (w + 1) / G);
  if (threadIdx.x == 0) {
    s_cb = 0;
    s_cn = 0;
  }
  __syncthreads();
  for (int base = b0; base < b1; base += nt) {
    const int b = base + threadIdx.x;
    int cn = 0;
    int64_t by = 0;
    int j = -1;
    bool first = false;
    if (b < b1) {
      cn = L.hcnt[b];
      j = L.bcarr[b];
      by = mode != 1 ? L.hbytes[b] : 0;
      first = b == 0 || L.bcarr[b - 1] != j;
    }
    int tn;
    int64_t tb;
    const int exn = block_exscan<int>(cn, &tn) + s_cn;
    const int64_t exb = block_exscan<int64_t>(by, &tb) + s_cb;
    if (b < b1) {
      L.nofs[b] = exn;
      L.bofs[b] = exb;
      if (first && j < kCompactCarr) {
        c.first_b[j] = exb;
        c.first_c[j] = w;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      s_cn += tn;
      s_cb += tb;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    c.tot_n[w] = s_cn;
    c.tot_b[w] = s_cb;
  }
}

// phase 2 (one workgroup): chunk prefixes, padding per call-array, totals
// lds: 4 * kCompactCarr int64 of LDS scratch
// Every workgroup runs phase 2 itself (the same values from each, so the
// shared writes agree) and keeps the call-arrays' padding in its own LDS
// (lds + 2 * kCompactCarr) for phase 3, so no grid barrier separates the
// two phases.
__device__ inline void dev_compact_p2(const PlanDev &P, const Level &L, const Work &W, MsgHdr *hdr, int64_t out_cap,
                                      int64_t *cs, int nchunk, int mode, int64_t *lds) {
  // all threads load into LDS and scan; one thread walks the call-arrays in
  // order over LDS values only
  int64_t *s_n = lds, *s_b = lds + kCompactCarr, *s_at = lds + 2 * kCompactCarr, *s_e = lds + 3 * kCompactCarr;
  __shared__ int64_t s_tn, s_tb;
  CScratch c(cs);
  const int nt = blockDim.x;
  const int ncarr = P.ncarr < kCompactCarr ? P.ncarr : kCompactCarr;
  for (int w = threadIdx.x; w < nchunk; w += nt) {
    s_n[w] = c.tot_n[w];
    s_b[w] = c.tot_b[w];
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    // one wave scans the chunk totals in place (inclusive per 64, carried)
    int64_t cn = 0, cb = 0;
    for (int base = 0; base < nchunk; base += 64) {
      const int w = base + (int)threadIdx.x;
      int64_t xn = w < nchunk ? s_n[w] : 0, xb = w < nchunk ? s_b[w] : 0;
      const int64_t vn = xn, vb = xb;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int64_t yn = __shfl_up(xn, d), yb = __shfl_up(xb, d);
        if ((int)threadIdx.x >= d) {
          xn += yn;
          xb += yb;
        }
      }
      if (w < nchunk) {
        c.pre_n[w] = cn + xn - vn;
        c.pre_b[w] = cb + xb - vb;
      }
      cn += __shfl(xn, 63);
      cb += __shfl(xb, 63);
    }
    if (threadIdx.x == 0) {
      s_tn = cn;
      s_tb = cb;
    }
  }
  __syncthreads();
  // raw byte position of every call-array's first band (-1: no band)
  for (int j = threadIdx.x; j < ncarr; j += nt) {
    const int64_t fc = c.first_c[j];
    s_at[j] = fc >= 0 ? c.first_b[j] + c.pre_b[fc] : -1;
    s_e[j] = P.carr[j].esize;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t pad = 0;
    for (int j = 0; j < ncarr; ++j) {
      if (s_at[j] >= 0 && mode != 1) {
        const int64_t at = s_at[j] + pad, e = s_e[j];
        pad += (at + e - 1) / e * e - at;
      }
      s_at[j] = pad;  // the padding of the call-arrays up to j, for the bands of j
    }
    const int64_t n = s_tn;
    if (P.ncarr > kCompactCarr || n > out_cap) set_err(W.err, -8);
    hdr->nmsg = n < out_cap ? n : out_cap;
    hdr->bytes = s_tb + pad;
    *L.head_top = 0;
    *W.run_top = 0;
  }
  __syncthreads();
}

// phase 3: every workgroup writes the messages of its chunk; pad: the
// call-arrays' padding that phase 2 left in this workgroup's LDS
__device__ inline void dev_compact_p3(const PlanDev &P, const Level &L, const Work &W, MsgRec *out, int64_t out_cap,
                                      int64_t *cs, int mode, const int64_t *pad) {
  CScratch c(cs);
  const int nb = L.nsl ? *L.nb : 0;
  const int G = gridDim.x, w = blockIdx.x;
  const int b0 = (int)((int64_t)nb * w / G), b1 = (int)((int64_t)nb * (w + 1) / G);
  const int64_t pn = c.pre_n[w], pb = c.pre_b[w];
  for (int b = b0 + threadIdx.x; b < b1; b += blockDim.x) {
    const int j = L.bcarr[b];
    compact_band(P, L, W, out, out_cap, mode, b, (int)(L.nofs[b] + pn),
                 L.bofs[b] + pb + (j < kCompactCarr ? pad[j] : 0));
  }
}

// --------------------------------------------------------------- GDEF row
// One wave per touched row.  Edits: holder additions from the row's runs
// (every receiver of an element becomes a holder) then definitions (owner =
// definer, holders = {definer} [+ host for Write]).  LDS scratch private to
// the wave: iv[kMaxCap], b[maxb], u[maxb], own[maxb], hold[maxb].
// State of the elementary segment starting at x: old interval (lanes 0..n-1
// hold the old list), then holder additions, then definitions.
// Runs and definitions of the row sit one per lane (lane e: run e, def e);
// the loops read them with lane reads, so no global load is serialised.
struct RowEdits {
  int nrun, ra0, ra1, rdst;
  int nds, dc0, dc1, ddst, dfl;
};

__device__ inline void gdef_state(int x, int n, int st, int ow, uint64_t ho, const RowEdits &E, int &own,
                                  uint64_t &hol) {
  // last interval with start <= x (old starts in lanes 0..n-1, start[0] = 0);
  // binary lifting with every lane active at every shuffle
  int lo = 0;
#pragma unroll
  for (int step = 32; step >= 1; step >>= 1) {
    const int cand = lo + step;
    const int v = __shfl(st, cand & 63);
    if (cand < n && v <= x) lo = cand;
  }
  own = __shfl(ow, lo);
  hol = __shfl(ho, lo);
  for (int e = 0; e < E.nrun; ++e) {
    const int a0 = lane_read(E.ra0, e), a1 = lane_read(E.ra1, e), d = lane_read(E.rdst, e);
    if (a0 <= x && x < a1) hol |= 1ull << d;
  }
  for (int e = 0; e < E.nds; ++e) {
    const int c0 = lane_read(E.dc0, e), c1 = lane_read(E.dc1, e), d = lane_read(E.ddst, e);
    if (c0 <= x && x < c1) {
      own = d;
      hol = (1ull << d) | ((lane_read(E.dfl, e) & 1) ? (1ull << kHost) : 0ull);
    }
  }
}

// Register-only update of one row (one wave, no LDS): every boundary of the
// old list and of the edits sits in one lane.  Returns false (row untouched)
// when the row has more than 64 boundaries; the caller then uses dev_gdef_row.
// A row the definitions tile (touching spans of one device already merged by
// the planner): the definitions are the new list.  One lane per row.

__device__ inline void dev_gdef_full_lane(const PlanDev &P, ArrDev *__restrict__ A, const Work &W, int t) {
  const GRowRec gr = P.grec[t];
  const ArrDev &a = A[gr.arr];
  const int nds = gr.ndseg;
  if (nds > a.cap) {
    set_err(W.err, -8);
    return;
  }
  Ivl *row = a.ivl + gr.grow * (int64_t)a.cap;
  const Seg *ds = P.dseg + gr.dseg0;
  for (int e = 0; e < nds; ++e) {
    const Seg d = ds[e];
    row[e] = Ivl{d.c0, d.dst, (1ull << d.dst) | ((d.flags & 1) ? (1ull << kHost) : 0ull)};
  }
  a.cnt[gr.grow] = nds;
}

// Lane-per-row update of a small row (at most kGL old intervals, kGR
// holder-adding runs and kGD definitions): the boundaries and the state at
// each (the old interval containing it, holders added by the runs covering
// it, then the definitions covering it) as in the wave form, in registers.
// Returns false, leaving the row alone, when the row is larger or the
// definitions tile it (other paths take those rows).  A row with neither
// runs nor definitions keeps its (already merged) list.
constexpr int kGL = 4, kGR = 4, kGD = 2, kGB = kGL + 2 * (kGR + kGD);

struct SmallRow {
  int n, nrun, nds;
  int st[kGL], ow[kGL];
  uint64_t ho[kGL];
  int ra0[kGR], ra1[kGR], rd[kGR];
  int dc0[kGD], dc1[kGD], dd[kGD];
  uint64_t dh[kGD];
};

__device__ inline void small_state(const SmallRow &R, int x, int &own, uint64_t &hol) {
  own = R.ow[0];
  hol = R.ho[0];
#pragma unroll
  for (int k = 1; k < kGL; ++k)
    if (k < R.n && R.st[k] <= x) {
      own = R.ow[k];
      hol = R.ho[k];
    }
#pragma unroll
  for (int e = 0; e < kGR; ++e)
    if (e < R.nrun && R.ra0[e] <= x && x < R.ra1[e]) hol |= 1ull << R.rd[e];
#pragma unroll
  for (int e = 0; e < kGD; ++e)
    if (e < R.nds && R.dc0[e] <= x && x < R.dc1[e]) {
      own = R.dd[e];
      hol = R.dh[e];
    }
}

__device__ inline bool dev_gdef_small_lane(const PlanDev &P, ArrDev *__restrict__ A, const Work &W, int t) {
  const GRowRec gr = P.grec[t];
  if (gr.full) return false;
  const int sl = gr.slice;
  SmallRow R;
  R.nds = gr.ndseg;
  R.nrun = sl >= 0 ? W.rcnt[sl] : 0;
  if (R.nrun == 0 && R.nds == 0) return true;
  ArrDev &a = A[gr.arr];
  const int64_t grow = gr.grow;
  R.n = a.cnt[grow];
  if (R.n > kGL || R.nrun > kGR || R.nds > kGD) return false;
  Ivl *row = a.ivl + grow * (int64_t)a.cap;
  const int roff = sl >= 0 ? W.roff[sl] : 0;
  const int W2 = (int)a.n[2];
#pragma unroll
  for (int k = 0; k < kGL; ++k) {
    Ivl v{0x7fffffff, 0, 0ull};
    if (k < R.n) v = row[k];
    R.st[k] = v.start;
    R.ow[k] = v.owner;
    R.ho[k] = v.holders;
  }
#pragma unroll
  for (int e = 0; e < kGR; ++e) {
    R.ra0[e] = R.ra1[e] = R.rd[e] = 0;
    if (e < R.nrun) {
      const Item r = W.runs[roff + e];
      R.ra0[e] = r.a0;
      R.ra1[e] = r.a1;
      R.rd[e] = r.dst;
    }
  }
#pragma unroll
  for (int e = 0; e < kGD; ++e) {
    R.dc0[e] = R.dc1[e] = R.dd[e] = 0;
    R.dh[e] = 0ull;
    if (e < R.nds) {
      const Seg d = P.dseg[gr.dseg0 + e];
      R.dc0[e] = d.c0;
      R.dc1[e] = d.c1;
      R.dd[e] = d.dst;
      R.dh[e] = (1ull << d.dst) | ((d.flags & 1) ? (1ull << kHost) : 0ull);
    }
  }
  // boundaries: old starts, run starts / ends, definition starts / ends (an
  // end at the row's width is the wrap to 0, already a start)
  int b[kGB];
  bool ok[kGB];
#pragma unroll
  for (int k = 0; k < kGL; ++k) {
    b[k] = R.st[k];
    ok[k] = k < R.n;
  }
#pragma unroll
  for (int e = 0; e < kGR; ++e) {
    b[kGL + 2 * e] = R.ra0[e];
    b[kGL + 2 * e + 1] = R.ra1[e] < W2 ? R.ra1[e] : 0;
    ok[kGL + 2 * e] = ok[kGL + 2 * e + 1] = e < R.nrun;
  }
#pragma unroll
  for (int e = 0; e < kGD; ++e) {
    b[kGL + 2 * kGR + 2 * e] = R.dc0[e];
    b[kGL + 2 * kGR + 2 * e + 1] = R.dc1[e] < W2 ? R.dc1[e] : 0;
    ok[kGL + 2 * kGR + 2 * e] = ok[kGL + 2 * kGR + 2 * e + 1] = e < R.nds;
  }
  // a boundary stays if it is the first of its value and the state there
  // differs from the state at the next smaller boundary value
  bool keep[kGB];
  int nn = 0;
#pragma unroll
  for (int j = 0; j < kGB; ++j) {
    bool first = ok[j];
    int pv = -1;
#pragma unroll
    for (int i = 0; i < kGB; ++i) {
      if (!ok[i]) continue;
      if (i < j && b[i] == b[j]) first = false;
      if (b[i] < b[j] && b[i] > pv) pv = b[i];
    }
    bool k = first;
    if (first && pv >= 0) {
      int o0, o1;
      uint64_t h0, h1;
      small_state(R, b[j], o0, h0);
      small_state(R, pv, o1, h1);
      k = o0 != o1 || h0 != h1;
    }
    keep[j] = k;
    nn += k ? 1 : 0;
  }
  if (nn > a.cap) {
    set_err(W.err, -8);
    return true;
  }
#pragma unroll
  for (int j = 0; j < kGB; ++j) {
    if (!keep[j]) continue;
    int r = 0;
#pragma unroll
    for (int i = 0; i < kGB; ++i) r += (keep[i] && b[i] < b[j]) ? 1 : 0;
    int o;
    uint64_t h;
    small_state(R, b[j], o, h);
    row[r] = Ivl{b[j], o, h};
  }
  a.cnt[grow] = nn;
  return true;
}

__device__ inline bool dev_gdef_row_fast(const PlanDev &P, ArrDev *__restrict__ A, const Work &W, int t) {
  const int lane = threadIdx.x & 63;
  const GRowRec gr = P.grec[t];
  ArrDev &a = A[gr.arr];
  const int64_t grow = gr.grow;
  Ivl *row = a.ivl + grow * (int64_t)a.cap;
  const Seg *ds = P.dseg + gr.dseg0;
  const int nds = gr.ndseg;
  const int sl = gr.slice;
  // every load that depends only on the row record is issued at once: the
  // count, the first 64 old intervals (the row's capacity bounds the read),
  // the run location and the first 64 definitions
  Ivl v{0x7fffffff, 0, 0ull};
  if (!gr.full && lane < a.cap) v = row[lane];
  const int n = gr.full ? 0 : a.cnt[grow];
  const int nrun = sl >= 0 ? W.rcnt[sl] : 0;
  const int roff = sl >= 0 ? W.roff[sl] : 0;
  Seg d{0, 0, 0, 0};
  if (lane < nds) d = ds[lane];
  if (gr.full) {
    // the definitions tile the row (touching spans of one device already
    // merged by the planner): they are the new list
    if (nds > a.cap) {
      if (lane == 0) set_err(W.err, -8);
      return true;
    }
    for (int e = lane; e < nds; e += 64) {
      const Seg de = e < 64 ? d : ds[e];
      row[e] = Ivl{de.c0, de.dst, (1ull << de.dst) | ((de.flags & 1) ? (1ull << kHost) : 0ull)};
    }
    if (lane == 0) a.cnt[grow] = nds;
    return true;
  }
  const int W2 = (int)a.n[2];
  const int nb = n + 2 * (nrun + nds);
  if (nb > 64) return false;
  const int st = lane < n ? v.start : 0x7fffffff;
  const int ow = lane < n ? v.owner : 0;
  const uint64_t ho = lane < n ? v.holders : 0ull;
  // edits one per lane
  RowEdits E{nrun, 0, 0, 0, nds, d.c0, d.c1, d.dst, d.flags};
  if (lane < nrun) {
    const Item r = W.runs[roff + lane];
    E.ra0 = r.a0;
    E.ra1 = r.a1;
    E.rdst = r.dst;
  }
  // boundaries: old starts, then run ends, then definition ends (an end at
  // the row's width is the wrap to 0, already a start)
  // (every lane takes part in the shuffles; the source lanes are in range)
  const int er = ((lane - n) >> 1) & 63, ed = ((lane - n - 2 * nrun) >> 1) & 63;
  const int a0 = __shfl(E.ra0, er), a1 = __shfl(E.ra1, er);
  const int c0 = __shfl(E.dc0, ed), c1 = __shfl(E.dc1, ed);
  int b = 0x7fffffff;
  if (lane < n) {
    b = st;
  } else if (lane < n + 2 * nrun) {
    b = ((lane - n) & 1) ? (a1 < W2 ? a1 : 0) : a0;
  } else if (lane < nb) {
    b = ((lane - n - 2 * nrun) & 1) ? (c1 < W2 ? c1 : 0) : c0;
  }
  // first occurrence of each value, and its predecessor value
  bool first = lane < nb;
  int pv = -1;
  for (int j = 0; j < nb; ++j) {
    const int y = lane_read(b, j);
    if (j < lane && y == b) first = false;
    if (y < b && y > pv) pv = y;
  }
  int own = 0, pown = 0;
  uint64_t hol = 0, phol = 0;
  // both calls are made by every lane (they contain shuffles)
  gdef_state(first ? b : 0, n, st, ow, ho, E, own, hol);
  gdef_state(pv < 0 ? 0 : pv, n, st, ow, ho, E, pown, phol);
  const bool keep = first && (pv < 0 || own != pown || hol != phol);
  int idx = 0;
  for (int j = 0; j < nb; ++j) {
    const int y = lane_read(b, j);
    const int kj = lane_read((int)keep, j);
    if (kj && y < b) ++idx;
  }
  const int nn = __popcll(__ballot(keep));
  if (nn > a.cap) {
    if (lane == 0) set_err(W.err, -8);
    return true;
  }
  if (keep) row[idx] = Ivl{b, own, hol};
  if (lane == 0) a.cnt[grow] = nn;
  return true;
}

struct GdefLds {
  Ivl *iv;
  int32_t *b, *u, *own;
  uint64_t *hold;
};

__device__ inline void dev_gdef_row(const PlanDev &P, ArrDev *__restrict__ A, const Work &W, int t, GdefLds S,
                                    int maxb) {
  const int lane = threadIdx.x & 63;
  const GRowRec gr = P.grec[t];
  ArrDev &a = A[gr.arr];
  const int64_t grow = gr.grow;
  const int n = a.cnt[grow];
  const int W2 = (int)a.n[2];
  Ivl *row = a.ivl + grow * (int64_t)a.cap;
  const int sl = gr.slice;
  const Item *runs = sl >= 0 ? W.runs + W.roff[sl] : nullptr;
  const int nrun = sl >= 0 ? W.rcnt[sl] : 0;
  const Seg *ds = P.dseg + gr.dseg0;
  const int nds = gr.ndseg;
  const int nbnd = n + 2 * (nrun + nds);
  if (nbnd > maxb) {
    if (lane == 0) set_err(W.err, -8);
    return;
  }
  for (int i = lane; i < n; i += 64) {
    S.iv[i] = row[i];
    S.b[i] = row[i].start;
  }
  for (int e = lane; e < nrun; e += 64) {
    S.b[n + 2 * e] = runs[e].a0;
    S.b[n + 2 * e + 1] = runs[e].a1 < W2 ? runs[e].a1 : 0;
  }
  for (int e = lane; e < nds; e += 64) {
    S.b[n + 2 * nrun + 2 * e] = ds[e].c0;
    S.b[n + 2 * nrun + 2 * e + 1] = ds[e].c1 < W2 ? ds[e].c1 : 0;
  }
  wave_lds_sync();
  // stable rank sort of the boundaries
  for (int i = lane; i < nbnd; i += 64) {
    const int x = S.b[i];
    int r = 0;
    for (int j = 0; j < nbnd; ++j) {
      const int y = S.b[j];
      r += (y < x) || (y == x && j < i);
    }
    S.u[r] = x;
  }
  wave_lds_sync();
  // unique, in place into b
  int nu = 0;
  for (int base = 0; base < nbnd; base += 64) {
    const int i = base + lane;
    const bool keep = i < nbnd && (i == 0 || S.u[i] != S.u[i - 1]);
    const int x = i < nbnd ? S.u[i] : 0;
    const uint64_t m = __ballot(keep);
    wave_lds_sync();
    if (keep) S.b[nu + __popcll(m & lanemask_lt())] = x;
    nu += __popcll(m);
    wave_lds_sync();
  }
  // state of every elementary segment
  for (int k = lane; k < nu; k += 64) {
    const int x = S.b[k];
    int lo = 0, hi = n - 1;  // last interval with start <= x
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (S.iv[mid].start <= x)
        lo = mid;
      else
        hi = mid - 1;
    }
    int own = S.iv[lo].owner;
    uint64_t hol = S.iv[lo].holders;
    for (int e = 0; e < nrun; ++e)
      if (runs[e].a0 <= x && x < runs[e].a1) hol |= 1ull << runs[e].dst;
    for (int e = 0; e < nds; ++e)
      if (ds[e].c0 <= x && x < ds[e].c1) {
        own = ds[e].dst;
        hol = (1ull << ds[e].dst) | ((ds[e].flags & 1) ? (1ull << kHost) : 0ull);
      }
    S.own[k] = own;
    S.hold[k] = hol;
  }
  wave_lds_sync();
  // merge equal neighbours and write the new list
  int nn = 0;
  Ivl *wrow = a.ivl + grow * (int64_t)a.cap;
  for (int base = 0; base < nu; base += 64) {
    const int k = base + lane;
    const bool keep = k < nu && (k == 0 || S.own[k] != S.own[k - 1] || S.hold[k] != S.hold[k - 1]);
    const uint64_t m = __ballot(keep);
    if (keep) {
      const int p = nn + __popcll(m & lanemask_lt());
      if (p < a.cap) wrow[p] = Ivl{S.b[k], S.own[k], S.hold[k]};
    }
    nn += __popcll(m);
  }
  if (lane == 0) {
    if (nn > a.cap)
      set_err(W.err, -8);
    else
      a.cnt[grow] = nn;
  }
  wave_lds_sync();
}

}  // namespace hd

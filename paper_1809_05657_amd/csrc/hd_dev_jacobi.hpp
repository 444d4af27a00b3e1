// hd_dev_jacobi.hpp — the 2-D 5-point Jacobi / lower-triangular tile
// (Sec. 5.1 formula: A[i][j] = (((B[i][j-1] + B[i][j+1]) + B[i-1][j]) +
// B[i+1][j]) / 4 on interior cells, A = B on the array boundary), shared by
// the per-call kernels (hd_jacobi.hip) and the persistent batched kernel,
// and the 3 x 3 convolution tile on the same tiling.
#pragma once
#include <hip/hip_runtime.h>

#include "hd_dev_common.hpp"

namespace hd {

// ------------------------------------------------------------ jacobi / tri
// One wave computes a tile of TH rows x 256 columns of one box; each lane
// owns 4 consecutive columns, the left / right neighbours come from the
// adjacent lanes (lanes 0 and 63 load the tile's edge columns).  HF: tiles
// are numbered along a row of tiles first (consecutive waves cover
// consecutive 1 KiB pieces of the same rows); otherwise down a column of
// tiles first (consecutive waves share halo rows).
template <int TH, bool HF>
__device__ inline void tile_pos(const WorkBox &B, int64_t lt, int &tx, int &ty) {
  if (HF) {
    const int ntx = (B.hi[2] - B.lo[2] + 255) / 256;
    tx = (int)(lt % ntx);
    ty = (int)(lt / ntx);
  } else {
    const int nty = (B.hi[1] - B.lo[1] + TH - 1) / TH;
    ty = (int)(lt % nty);
    tx = (int)(lt / nty);
  }
}

// One row of the lane's 4 columns with its left / right neighbour column
// (zero when the row is outside the array or past rlim; such rows are never
// used).  Called by whole waves (the neighbours come from adjacent lanes).
__device__ inline void load_row(gcf *__restrict__ in, int64_t rs, int r, int rlim, int c, int N1, int N2, bool vec,
                                f4 &v, float &Lh, float &Rh) {
  const int lane = threadIdx.x & 63;
  f4 x = {0.f, 0.f, 0.f, 0.f};
  float l = 0.f, rr = 0.f;
  if (r >= 0 && r < N1 && r <= rlim) {
    gcf *p = in + (int64_t)r * rs;
    if (vec && c + 4 <= N2) {
      x = *(gcf4 *)(p + c);
    } else {
      if (c < N2) x.x = p[c];
      if (c + 1 < N2) x.y = p[c + 1];
      if (c + 2 < N2) x.z = p[c + 2];
      if (c + 3 < N2) x.w = p[c + 3];
    }
    if (lane == 0 && c >= 1 && c - 1 < N2) l = p[c - 1];
    if (lane == 63 && c + 4 < N2) rr = p[c + 4];
  }
  const float lw = __shfl_up(x.w, 1);
  const float rx = __shfl_down(x.x, 1);
  Lh = lane == 0 ? l : lw;
  Rh = lane == 63 ? rr : rx;
  v = x;
}

// Rows r0-1 .. r0+TH of the lane's 4 columns (rows past r1 or outside the
// array read as zero and are never used).
template <int TH>
__device__ inline void load_rows(gcf *__restrict__ in, int64_t rs, int r0, int r1, int c, int N1, int N2, bool vec,
                                 f4 *v, float *Lh, float *Rh) {
#pragma unroll
  for (int k = 0; k < TH + 2; ++k) load_row(in, rs, r0 - 1 + k, r1, c, N1, N2, vec, v[k], Lh[k], Rh[k]);
}

__device__ inline void store4(gwf *q, const float *o, const bool *wr, bool vec) {
  if (vec && wr[0] && wr[1] && wr[2] && wr[3]) {
    f4 ov = {o[0], o[1], o[2], o[3]};
    __builtin_nontemporal_store(ov, (gwf4 *)(q));
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (wr[e]) q[e] = o[e];
  }
}

// ------------------------------------------------- unaligned rows (coalesced)
// When a row cannot be read as float4 (row length or box start not a
// multiple of 4), lane l takes columns tc + 64 e + l (e = 0..3) instead of
// four consecutive ones, so every load and store covers 256 consecutive
// bytes.  A cell's left / right neighbours come from the adjacent lane, from
// lane 63 / 0 of the neighbouring group, or from the tile's edge columns.
struct RowI {
  float x[4], l[4], r[4];
};

__device__ inline RowI load_row_i(gcf *__restrict__ in, int64_t rs, int r, int rlim, int tc, int N1, int N2) {
  const int lane = threadIdx.x & 63;
  RowI q;
  float el = 0.f, er = 0.f;
  const bool ok = r >= 0 && r < N1 && r <= rlim;
  gcf *p = in + (int64_t)r * rs;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int col = tc + 64 * e + lane;
    q.x[e] = ok && col < N2 ? p[col] : 0.f;
  }
  if (ok && lane == 0 && tc >= 1) el = p[tc - 1];
  if (ok && lane == 63 && tc + 256 < N2) er = p[tc + 256];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const float up = __shfl_up(q.x[e], 1), dn = __shfl_down(q.x[e], 1);
    float prev = el, next = er;
    if (e > 0) prev = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q.x[e > 0 ? e - 1 : 0]), 63));
    if (e < 3) next = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q.x[e < 3 ? e + 1 : 3]), 0));
    q.l[e] = lane > 0 ? up : prev;
    q.r[e] = lane < 63 ? dn : next;
  }
  return q;
}

template <int TH, bool TRI, bool HF>
__device__ inline void dev_jacobi_tile_i(const WorkBox &B, int tx, int r0, int r1, gcf *__restrict__ in,
                                         gwf *__restrict__ out, int64_t rsi, int64_t rso, int N1, int N2) {
  const int lane = threadIdx.x & 63;
  const int tc = B.lo[2] + tx * 256;
  RowI v[TH + 2];
#pragma unroll
  for (int k = 0; k < TH + 2; ++k) v[k] = load_row_i(in, rsi, r0 - 1 + k, r1, tc, N1, N2);
#pragma unroll
  for (int k = 1; k <= TH; ++k) {
    const int i = r0 + k - 1;
    if (i >= r1) break;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = tc + 64 * e + lane;
      bool interior, write = j < B.hi[2];
      if (TRI) {
        write = write && j <= i;
        interior = j >= 1 && j < i && i <= N1 - 2;
      } else {
        interior = i >= 1 && i <= N1 - 2 && j >= 1 && j <= N2 - 2;
      }
      float s = v[k].l[e] + v[k].r[e];
      s = s + v[k - 1].x[e];
      s = s + v[k + 1].x[e];
      if (write) out[(int64_t)i * rso + j] = interior ? s * 0.25f : v[k].x[e];
    }
  }
}

template <int TH, bool TRI, bool HF = true>
__device__ inline void dev_jacobi_tile(const WorkBox &B, int64_t lt, const ArrDev *__restrict__ A) {
  const int lane = threadIdx.x & 63;
  int tx, ty;
  tile_pos<TH, HF>(B, lt, tx, ty);
  const int r0 = B.lo[1] + ty * TH;
  const int r1 = min(r0 + TH, B.hi[1]);
  // triangular kernel: a tile entirely above the diagonal writes nothing
  if (TRI && B.lo[2] + tx * 256 > r1 - 1) return;
  const int c = B.lo[2] + tx * 256 + 4 * lane;
  const ArrDev &ai = A[B.ain];
  gcf *__restrict__ in = (gcf *)ai.buf[B.dev];
  gwf *__restrict__ out = (gwf *)A[B.aout].buf[B.dev];
  const int N1 = (int)ai.n[1], N2 = (int)ai.n[2];
  const int64_t rsi = ai.rs[B.dev], rso = A[B.aout].rs[B.dev];
  const bool vec = ((N2 & 3) == 0) && ((B.lo[2] & 3) == 0);
  if (!vec) {
    dev_jacobi_tile_i<TH, TRI, HF>(B, tx, r0, r1, in, out, rsi, rso, N1, N2);
    return;
  }
  f4 v[TH + 2];
  float Lh[TH + 2], Rh[TH + 2];
  load_rows<TH>(in, rsi, r0, r1, c, N1, N2, vec, v, Lh, Rh);
#pragma unroll
  for (int k = 1; k <= TH; ++k) {
    const int i = r0 + k - 1;
    if (i >= r1) break;
    const f4 up = v[k - 1], cu = v[k], dn = v[k + 1];
    const float cv[6] = {Lh[k], cu.x, cu.y, cu.z, cu.w, Rh[k]};
    const float uv[4] = {up.x, up.y, up.z, up.w};
    const float dv[4] = {dn.x, dn.y, dn.z, dn.w};
    float o[4];
    bool wr[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = c + e;
      bool interior, write = j < B.hi[2];
      if (TRI) {
        write = write && j <= i;
        interior = j >= 1 && j < i && i <= N1 - 2;
      } else {
        interior = i >= 1 && i <= N1 - 2 && j >= 1 && j <= N2 - 2;
      }
      float s = cv[e] + cv[e + 2];
      s = s + uv[e];
      s = s + dv[e];
      o[e] = interior ? s * 0.25f : cv[e + 1];
      wr[e] = write;
    }
    store4(out + (int64_t)i * rso + c, o, wr, vec);
  }
}

// ------------------------------------------------------------ convolution
// 2-D convolution with the eight neighbours (Sec. 5.1), weights w[0..8] over
// the 3 x 3 window row by row: the first product rounded, then one fused
// multiply-add per further cell in the same order; the array boundary is
// copied.  Same tiles as the Jacobi kernel.
struct Coef9 {
  float w[9];
};

template <int TH, bool HF = true>
__device__ inline void dev_conv_tile(const WorkBox &B, int64_t lt, const ArrDev *__restrict__ A, const Coef9 &W) {
  const int lane = threadIdx.x & 63;
  int tx, ty;
  tile_pos<TH, HF>(B, lt, tx, ty);
  const int r0 = B.lo[1] + ty * TH;
  const int r1 = min(r0 + TH, B.hi[1]);
  const int c = B.lo[2] + tx * 256 + 4 * lane;
  const ArrDev &ai = A[B.ain];
  gcf *__restrict__ in = (gcf *)ai.buf[B.dev];
  gwf *__restrict__ out = (gwf *)A[B.aout].buf[B.dev];
  const int N1 = (int)ai.n[1], N2 = (int)ai.n[2];
  const int64_t rsi = ai.rs[B.dev], rso = A[B.aout].rs[B.dev];
  const bool vec = ((N2 & 3) == 0) && ((B.lo[2] & 3) == 0);
  f4 v[TH + 2];
  float Lh[TH + 2], Rh[TH + 2];
  load_rows<TH>(in, rsi, r0, r1, c, N1, N2, vec, v, Lh, Rh);
#pragma unroll
  for (int k = 1; k <= TH; ++k) {
    const int i = r0 + k - 1;
    if (i >= r1) break;
    const f4 up = v[k - 1], cu = v[k], dn = v[k + 1];
    const float row[3][6] = {{Lh[k - 1], up.x, up.y, up.z, up.w, Rh[k - 1]},
                             {Lh[k], cu.x, cu.y, cu.z, cu.w, Rh[k]},
                             {Lh[k + 1], dn.x, dn.y, dn.z, dn.w, Rh[k + 1]}};
    float o[4];
    bool wr[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = c + e;
      const bool interior = i >= 1 && i <= N1 - 2 && j >= 1 && j <= N2 - 2;
      float acc = W.w[0] * row[0][e];
      acc = __builtin_fmaf(W.w[1], row[0][e + 1], acc);
      acc = __builtin_fmaf(W.w[2], row[0][e + 2], acc);
      acc = __builtin_fmaf(W.w[3], row[1][e], acc);
      acc = __builtin_fmaf(W.w[4], row[1][e + 1], acc);
      acc = __builtin_fmaf(W.w[5], row[1][e + 2], acc);
      acc = __builtin_fmaf(W.w[6], row[2][e], acc);
      acc = __builtin_fmaf(W.w[7], row[2][e + 1], acc);
      acc = __builtin_fmaf(W.w[8], row[2][e + 2], acc);
      o[e] = interior ? acc : row[1][e + 1];
      wr[e] = j < B.hi[2];
    }
    store4(out + (int64_t)i * rso + c, o, wr, vec);
  }
}

// ---------------------------------------------------------------- strips
// Tall strips (TS rows x 256 columns, one wave): the rows stream through a
// register window in chunks of C rows, the next chunk's loads issued before
// the current chunk is computed, so each input row is read once per strip
// (plus two halo rows per strip) with a small register footprint.
// OP: 0 Jacobi, 1 lower-triangular Jacobi, 2 3 x 3 convolution (weights W).
template <int OP>
__device__ inline void strip_row(int i, int c, int N1, int N2, int64_t rso, const WorkBox &B, const f4 &up, const f4 &cu,
                                 const f4 &dn, float Lu, float Ru, float Lc, float Rc, float Ld, float Rd,
                                 const Coef9 &W, gwf *__restrict__ out, bool vec) {
  float o[4];
  bool wr[4];
  const float cv[6] = {Lc, cu.x, cu.y, cu.z, cu.w, Rc};
  if (OP == 2) {
    const float uv[6] = {Lu, up.x, up.y, up.z, up.w, Ru};
    const float dv[6] = {Ld, dn.x, dn.y, dn.z, dn.w, Rd};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = c + e;
      const bool interior = i >= 1 && i <= N1 - 2 && j >= 1 && j <= N2 - 2;
      float acc = W.w[0] * uv[e];
      acc = __builtin_fmaf(W.w[1], uv[e + 1], acc);
      acc = __builtin_fmaf(W.w[2], uv[e + 2], acc);
      acc = __builtin_fmaf(W.w[3], cv[e], acc);
      acc = __builtin_fmaf(W.w[4], cv[e + 1], acc);
      acc = __builtin_fmaf(W.w[5], cv[e + 2], acc);
      acc = __builtin_fmaf(W.w[6], dv[e], acc);
      acc = __builtin_fmaf(W.w[7], dv[e + 1], acc);
      acc = __builtin_fmaf(W.w[8], dv[e + 2], acc);
      o[e] = interior ? acc : cv[e + 1];
      wr[e] = j < B.hi[2];
    }
  } else {
    const float uv[4] = {up.x, up.y, up.z, up.w};
    const float dv[4] = {dn.x, dn.y, dn.z, dn.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = c + e;
      bool interior, write = j < B.hi[2];
      if (OP == 1) {
        write = write && j <= i;
        interior = j >= 1 && j < i && i <= N1 - 2;
      } else {
        interior = i >= 1 && i <= N1 - 2 && j >= 1 && j <= N2 - 2;
      }
      float s = cv[e] + cv[e + 2];
      s = s + uv[e];
      s = s + dv[e];
      o[e] = interior ? s * 0.25f : cv[e + 1];
      wr[e] = write;
    }
  }
  store4(out + (int64_t)i * rso + c, o, wr, vec);
}

template <int TS, int C, int OP, bool HF>
__device__ inline void dev_strip(const WorkBox &B, int64_t lt, const ArrDev *__restrict__ A, const Coef9 &W) {
  const int lane = threadIdx.x & 63;
  int tx, ty;
  tile_pos<TS, HF>(B, lt, tx, ty);
  const int r0 = B.lo[1] + ty * TS;
  const int r1 = min(r0 + TS, B.hi[1]);
  if (OP == 1 && B.lo[2] + tx * 256 > r1 - 1) return;
  const int c = B.lo[2] + tx * 256 + 4 * lane;
  const ArrDev &ai = A[B.ain];
  gcf *__restrict__ in = (gcf *)ai.buf[B.dev];
  gwf *__restrict__ out = (gwf *)A[B.aout].buf[B.dev];
  const int N1 = (int)ai.n[1], N2 = (int)ai.n[2];
  const int64_t rsi = ai.rs[B.dev], rso = A[B.aout].rs[B.dev];
  const bool vec = ((N2 & 3) == 0) && ((B.lo[2] & 3) == 0);
  // window: rows base-1 .. base+C
  f4 v[C + 2];
  float L[C + 2], R[C + 2];
  load_rows<C>(in, rsi, r0, r1, c, N1, N2, vec, v, L, R);
  for (int base = r0; base < r1; base += C) {
    f4 nv[C];
    float nL[C], nR[C];
    if (base + C < r1) {
#pragma unroll
      for (int k = 0; k < C; ++k) load_row(in, rsi, base + C + 1 + k, r1, c, N1, N2, vec, nv[k], nL[k], nR[k]);
    }
#pragma unroll
    for (int k = 1; k <= C; ++k) {
      const int i = base + k - 1;
      if (i >= r1) break;
      strip_row<OP>(i, c, N1, N2, rso, B, v[k - 1], v[k], v[k + 1], L[k - 1], R[k - 1], L[k], R[k], L[k + 1], R[k + 1], W,
                    out, vec);
    }
    v[0] = v[C];
    v[1] = v[C + 1];
    L[0] = L[C];
    L[1] = L[C + 1];
    R[0] = R[C];
    R[1] = R[C + 1];
#pragma unroll
    for (int k = 0; k < C; ++k) {
      v[k + 2] = nv[k];
      L[k + 2] = nL[k];
      R[k + 2] = nR[k];
    }
  }
}

// ------------------------------------------------------- stacked waves
// W waves stacked down one tile of W*TH rows x 256 columns: each wave loads
// its own TH rows once; the row above its first and the row below its last
// come from the neighbouring waves through LDS (the top and bottom waves
// load the tile's two halo rows), so a tile reads W*TH + 2 rows instead of
// W*(TH + 2).  Tiles run along rows of tiles.  VEC: every box of the launch
// has rows that can be read as float4 (row length and box start multiples
// of 4); otherwise each wave takes the coalesced per-wave path (no LDS).
// OP: 0 Jacobi, 1 lower-triangular Jacobi, 2 3 x 3 convolution.
template <int W, int TH, int OP, bool VEC>
__device__ inline void dev_stack_tile_p(const WorkBox &B, int64_t lt, gcf *__restrict__ in, int64_t rsi,
                                        gwf *__restrict__ out, int64_t rso, int N1, int N2, const Coef9 &Wt) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int tx, ty;
  tile_pos<W * TH, true>(B, lt, tx, ty);
  const int t0 = B.lo[1] + ty * (W * TH);
  const int t1 = min(t0 + W * TH, B.hi[1]);
  // triangular kernel: a tile entirely above the diagonal writes nothing
  // (the whole workgroup leaves together, before the barrier)
  if (OP == 1 && B.lo[2] + tx * 256 > t1 - 1) return;
  const int c = B.lo[2] + tx * 256 + 4 * lane;
  const int r0 = t0 + wv * TH;
  if (!VEC) {
    if (r0 >= t1) return;
    const int r1 = min(r0 + TH, t1);
    if (OP != 2) {
      dev_jacobi_tile_i<TH, OP == 1, true>(B, tx, r0, r1, in, out, rsi, rso, N1, N2);
    } else {
      f4 v[TH + 2];
      float L[TH + 2], R[TH + 2];
      load_rows<TH>(in, rsi, r0, r1, c, N1, N2, false, v, L, R);
#pragma unroll
      for (int k = 1; k <= TH; ++k) {
        const int i = r0 + k - 1;
        if (i >= r1) break;
        strip_row<2>(i, c, N1, N2, rso, B, v[k - 1], v[k], v[k + 1], L[k - 1], R[k - 1], L[k], R[k], L[k + 1], R[k + 1],
                     Wt, out, false);
      }
    }
    return;
  }
  // [0]: each wave's first row, [1]: its last row; the convolution also
  // needs those rows' left / right neighbour columns
  __shared__ f4 sv[2][W][64];
  __shared__ float sl[OP == 2 ? 2 : 1][W][64], sr[OP == 2 ? 2 : 1][W][64];
  f4 v[TH + 2];
  float L[TH + 2], R[TH + 2];
  // A full tile away from the array boundary (the common case, uniform over
  // the workgroup): every row and halo column exists, every cell is interior
  // and written, so no per-lane guard is needed.
  const int tc = B.lo[2] + tx * 256;
  if (OP != 1 && t0 >= 1 && t0 + W * TH <= min(B.hi[1], N1 - 1) && tc >= 1 && tc + 256 <= min(B.hi[2], N2 - 1)) {
    gcf *p = in + (int64_t)(r0 - 1) * rsi + c;
#pragma unroll
    for (int k = 1; k <= TH; ++k) v[k] = *(gcf4 *)(p + (int64_t)k * rsi);
    if (wv == 0) v[0] = *(gcf4 *)(p);
    if (wv == W - 1) v[TH + 1] = *(gcf4 *)(p + (int64_t)(TH + 1) * rsi);
    const int k0 = OP == 2 ? 0 : 1, k1 = OP == 2 ? TH + 1 : TH;
    float le[TH + 2], ri[TH + 2];
#pragma unroll
    for (int k = 0; k < TH + 2; ++k) le[k] = ri[k] = 0.f;
    if (lane == 0) {
#pragma unroll
      for (int k = k0; k <= k1; ++k)
        if ((k > 0 && k <= TH) || (k == 0 && wv == 0) || (k == TH + 1 && wv == W - 1)) le[k] = p[(int64_t)k * rsi - 1];
    }
    if (lane == 63) {
#pragma unroll
      for (int k = k0; k <= k1; ++k)
        if ((k > 0 && k <= TH) || (k == 0 && wv == 0) || (k == TH + 1 && wv == W - 1)) ri[k] = p[(int64_t)k * rsi + 4];
    }
#pragma unroll
    for (int k = k0; k <= k1; ++k) {
      if ((k == 0 && wv != 0) || (k == TH + 1 && wv != W - 1)) continue;
      const float lw = __shfl_up(v[k].w, 1), rx = __shfl_down(v[k].x, 1);
      L[k] = lane == 0 ? le[k] : lw;
      R[k] = lane == 63 ? ri[k] : rx;
    }
    sv[0][wv][lane] = v[1];
    sv[1][wv][lane] = v[TH];
    if (OP == 2) {
      sl[0][wv][lane] = L[1];
      sr[0][wv][lane] = R[1];
      sl[OP == 2 ? 1 : 0][wv][lane] = L[TH];
      sr[OP == 2 ? 1 : 0][wv][lane] = R[TH];
    }
    __syncthreads();
    if (wv > 0) {
      v[0] = sv[1][wv - 1][lane];
      if (OP == 2) {
        L[0] = sl[OP == 2 ? 1 : 0][wv - 1][lane];
        R[0] = sr[OP == 2 ? 1 : 0][wv - 1][lane];
      }
    }
    if (wv < W - 1) {
      v[TH + 1] = sv[0][wv + 1][lane];
      if (OP == 2) {
        L[TH + 1] = sl[0][wv + 1][lane];
        R[TH + 1] = sr[0][wv + 1][lane];
      }
    }
    gwf *q = out + (int64_t)r0 * rso + c;
#pragma unroll
    for (int k = 1; k <= TH; ++k) {
      const f4 up = v[k - 1], cu = v[k], dn = v[k + 1];
      const float cv[6] = {L[k], cu.x, cu.y, cu.z, cu.w, R[k]};
      float o[4];
      if (OP == 2) {
        const float uv[6] = {L[k - 1], up.x, up.y, up.z, up.w, R[k - 1]};
        const float dv[6] = {L[k + 1], dn.x, dn.y, dn.z, dn.w, R[k + 1]};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float acc = Wt.w[0] * uv[e];
          acc = __builtin_fmaf(Wt.w[1], uv[e + 1], acc);
          acc = __builtin_fmaf(Wt.w[2], uv[e + 2], acc);
          acc = __builtin_fmaf(Wt.w[3], cv[e], acc);
          acc = __builtin_fmaf(Wt.w[4], cv[e + 1], acc);
          acc = __builtin_fmaf(Wt.w[5], cv[e + 2], acc);
          acc = __builtin_fmaf(Wt.w[6], dv[e], acc);
          acc = __builtin_fmaf(Wt.w[7], dv[e + 1], acc);
          acc = __builtin_fmaf(Wt.w[8], dv[e + 2], acc);
          o[e] = acc;
        }
      } else {
        const float uv[4] = {up.x, up.y, up.z, up.w};
        const float dv[4] = {dn.x, dn.y, dn.z, dn.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float t = cv[e] + cv[e + 2];
          t = t + uv[e];
          t = t + dv[e];
          o[e] = t * 0.25f;
        }
      }
      const f4 ov = {o[0], o[1], o[2], o[3]};
      __builtin_nontemporal_store(ov, (gwf4 *)(q + (int64_t)(k - 1) * rso));
    }
    return;
  }
  // rows up to t1 are read (t1 itself is the halo below the tile's last row);
  // rows outside the array or past t1 read as zero and are never used
#pragma unroll
  for (int k = 1; k <= TH; ++k) load_row(in, rsi, r0 - 1 + k, t1, c, N1, N2, true, v[k], L[k], R[k]);
  if (wv == 0) load_row(in, rsi, r0 - 1, t1, c, N1, N2, true, v[0], L[0], R[0]);
  if (wv == W - 1) load_row(in, rsi, r0 + TH, t1, c, N1, N2, true, v[TH + 1], L[TH + 1], R[TH + 1]);
  sv[0][wv][lane] = v[1];
  sv[1][wv][lane] = v[TH];
  if (OP == 2) {
    sl[0][wv][lane] = L[1];
    sr[0][wv][lane] = R[1];
    sl[OP == 2 ? 1 : 0][wv][lane] = L[TH];
    sr[OP == 2 ? 1 : 0][wv][lane] = R[TH];
  }
  __syncthreads();
  if (wv > 0) {
    v[0] = sv[1][wv - 1][lane];
    if (OP == 2) {
      L[0] = sl[OP == 2 ? 1 : 0][wv - 1][lane];
      R[0] = sr[OP == 2 ? 1 : 0][wv - 1][lane];
    }
  }
  if (wv < W - 1) {
    v[TH + 1] = sv[0][wv + 1][lane];
    if (OP == 2) {
      L[TH + 1] = sl[0][wv + 1][lane];
      R[TH + 1] = sr[0][wv + 1][lane];
    }
  }
#pragma unroll
  for (int k = 1; k <= TH; ++k) {
    const int i = r0 + k - 1;
    if (i >= t1) break;
    strip_row<OP>(i, c, N1, N2, rso, B, v[k - 1], v[k], v[k + 1], L[k - 1], R[k - 1], L[k], R[k], L[k + 1], R[k + 1], Wt,
                  out, true);
  }
}

template <int W, int TH, int OP, bool VEC>
__device__ inline void dev_stack_tile(const WorkBox &B, int64_t lt, const ArrDev *__restrict__ A, const Coef9 &Wt) {
  const ArrDev &ai = A[B.ain], &ao = A[B.aout];
  dev_stack_tile_p<W, TH, OP, VEC>(B, lt, (gcf *)ai.buf[B.dev], ai.rs[B.dev], (gwf *)ao.buf[B.dev], ao.rs[B.dev],
                                   (int)ai.n[1], (int)ai.n[2], Wt);
}


__host__ __device__ inline int64_t jacobi_tiles(const WorkBox &B, int th) {
  const int64_t h = B.hi[1] - B.lo[1], w = B.hi[2] - B.lo[2];
  if (h <= 0 || w <= 0 || B.hi[0] <= B.lo[0]) return 0;
  return ((h + th - 1) / th) * ((w + 255) / 256);
}

}  // namespace hd

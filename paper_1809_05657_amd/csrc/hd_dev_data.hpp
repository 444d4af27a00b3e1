// hd_dev_data.hpp — device functions of the data path (pack / unpack and the
// built-in user kernels), shared by the per-call kernels (hd_data.hip) and
// the persistent batched kernel (hd_batch.hip), so both perform the same
// operations in the same order.
//
// Built-in kernels (device d reads its own buffers and writes its work box
// of the output; buffers are full-extent and row-major):
//   jacobi2d   A[i][j] = (((B[i][j-1] + B[i][j+1]) + B[i-1][j]) + B[i+1][j]) / 4
//              on interior cells (Sec. 5.1), A = B on the array boundary
//   tri2d      the same update on 1 <= j < i <= n-2, copy on the other cells
//              with j <= i; cells with j > i are not written
//   copy       out = in (raw 4- or 8-byte elements)
//   stencil3d7 acc = c0*u; acc = fma(c_e, u[x+e], acc) for e = -i,+i,-j,+j,-k,+k
//              on interior cells, copy on the boundary
// FP32 throughout, no contraction beyond the explicit fused multiply-adds.
#pragma once
#include <hip/hip_runtime.h>

#include "hd_dev_common.hpp"
#include "hd_dev_jacobi.hpp"

namespace hd {

// ------------------------------------------------------------ pack / unpack
__device__ inline int find_msg(const MsgRec *__restrict__ M, int64_t n, int64_t byteoff) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (M[mid].off <= byteoff)
      lo = mid;
    else
      hi = mid - 1;
  }
  return (int)lo;
}

// Packed word w of the staging buffer <-> element word of the section in the
// source (pack) or destination (unpack) endpoint's buffer, at the same global
// coordinates.  Sections are row-major inside each box.  m caches the message
// of the previous word.  mode 0 packs, 1 unpacks, 2 does both in one pass
// (the word read from the source goes to the staging buffer and to the
// destination).  Mode 2 is safe within one table: a message reads cells its
// source owns and writes cells its destination does not hold, and the owner
// of a cell always holds it, so no word is written and read in the same pass.
__device__ inline void dev_pack_word(const MsgRec *__restrict__ M, int64_t n, const ArrDev *__restrict__ A,
                                     uint32_t *__restrict__ stg, int unpack, int64_t w, int &m) {
  if (!(M[m].off <= 4 * w && 4 * w < M[m].off + M[m].bytes)) m = find_msg(M, n, 4 * w);
  const MsgRec &r = M[m];
  const int64_t lw = w - (r.off >> 2);
  if (4 * lw >= r.bytes) return;  // alignment padding between arrays
  const int k = r.esize >> 2;
  const int64_t wid = (int64_t)(r.hi[2] - r.lo[2]) * k;
  const int64_t rows = r.hi[1] - r.lo[1];
  const int64_t c = lw % wid, t = lw / wid;
  const int64_t rr = t % rows, p = t / rows;
  const ArrDev &a = A[r.arr];
  const int64_t gs = HD_EOFF(a, r.src, r.lo[0] + p, r.lo[1] + rr, r.lo[2]) * k + c;
  const int64_t gd = HD_EOFF(a, r.dst, r.lo[0] + p, r.lo[1] + rr, r.lo[2]) * k + c;
  if (unpack == 0) {
    stg[w] = reinterpret_cast<const uint32_t *>(a.buf[r.src])[gs];
  } else if (unpack == 1) {
    reinterpret_cast<uint32_t *>(a.buf[r.dst])[gd] = stg[w];
  } else {
    const uint32_t v = reinterpret_cast<const uint32_t *>(a.buf[r.src])[gs];
    stg[w] = v;
    reinterpret_cast<uint32_t *>(a.buf[r.dst])[gd] = v;
  }
}

// Words [b0, b1) of message r (row-major inside its box), 4 per thread per
// iteration; one workgroup of 256 threads.  IT: index type of the word
// arithmetic (32-bit whenever the message has fewer than 2^31 words).
template <typename IT>
__device__ inline void dev_pack_span(const MsgRec &r, const ArrDev *__restrict__ A, uint32_t *__restrict__ stg,
                                     int mode, IT b0, IT b1) {
  const ArrDev &a = A[r.arr];
  const IT k = (IT)(r.esize >> 2);
  const IT wid = (IT)(r.hi[2] - r.lo[2]) * k, rows = (IT)(r.hi[1] - r.lo[1]);
  // source and destination windows have their own strides
  const int64_t rps = a.rs[r.src] * k, pps = a.ps[r.src] * k;
  const int64_t rpd = a.rs[r.dst] * k, ppd = a.ps[r.dst] * k;
  const int64_t bs = HD_EOFF(a, r.src, r.lo[0], r.lo[1], r.lo[2]) * k;
  const int64_t bd = HD_EOFF(a, r.dst, r.lo[0], r.lo[1], r.lo[2]) * k;
  const uint32_t *__restrict__ src = reinterpret_cast<const uint32_t *>(a.buf[r.src]);
  uint32_t *__restrict__ dst = reinterpret_cast<uint32_t *>(a.buf[r.dst]);
  uint32_t *__restrict__ sp = stg + (r.off >> 2);
  for (IT q = b0 + (IT)threadIdx.x; q < b1; q += 4 * 256) {
    int64_t gs[4], gd[4];
    bool ok[4];
    uint32_t v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const IT lw = q + (IT)(e * 256);
      ok[e] = lw < b1;
      const IT c = lw % wid, t = lw / wid;
      const IT rr = t % rows, p = t / rows;
      gs[e] = bs + (int64_t)p * pps + (int64_t)rr * rps + (int64_t)c;
      gd[e] = bd + (int64_t)p * ppd + (int64_t)rr * rpd + (int64_t)c;
      if (ok[e]) v[e] = mode == 1 ? sp[lw] : src[gs[e]];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (!ok[e]) continue;
      const IT lw = q + (IT)(e * 256);
      if (mode != 1) sp[lw] = v[e];
      if (mode != 0) dst[gd[e]] = v[e];
    }
  }
}

// Grid-stride over the words of the whole table (the count is device-resident).
__device__ inline void dev_pack(const MsgRec *__restrict__ M, const MsgHdr *__restrict__ H,
                                const ArrDev *__restrict__ A, uint32_t *__restrict__ stg, int unpack, int64_t first,
                                int64_t stride) {
  const int64_t n = H->nmsg;
  const int64_t words = H->bytes >> 2;
  int m = 0;
  for (int64_t w = first; w < words; w += stride) dev_pack_word(M, n, A, stg, unpack, w, m);
}

// --------------------------------------------------------------------- copy
// One wave: 16 rows x 256 words of one plane of the box.
__device__ inline void dev_copy_tile(const WorkBox &B, int64_t lt, const ArrDev *__restrict__ A) {
  const int lane = threadIdx.x & 63;
  const ArrDev &ai = A[B.ain];
  const int k = ai.esize >> 2;
  const int h = B.hi[1] - B.lo[1];
  const int64_t wwords = (int64_t)(B.hi[2] - B.lo[2]) * k;
  const int nty = (h + 15) / 16;
  const int ntx = (int)((wwords + 255) / 256);
  const int ty = (int)(lt % nty);
  const int64_t rest = lt / nty;
  const int tx = (int)(rest % ntx);
  const int p = B.lo[0] + (int)(rest / ntx);
  const ArrDev &ao = A[B.aout];
  const uint32_t *__restrict__ in = reinterpret_cast<const uint32_t *>(ai.buf[B.dev]);
  uint32_t *__restrict__ out = reinterpret_cast<uint32_t *>(ao.buf[B.dev]);
  const int64_t c0 = (int64_t)B.lo[2] * k + (int64_t)tx * 256 + 4 * lane;
  const int64_t cend = (int64_t)B.hi[2] * k;
  // window columns start at multiples of 4, so with row strides of a
  // multiple of 4 words an aligned column gives aligned words
  const bool vec = (c0 & 3) == 0 && ((ai.rs[B.dev] * k) & 3) == 0 && ((ao.rs[B.dev] * k) & 3) == 0;
  const int rb = B.lo[1] + ty * 16;
  const int64_t wc0 = (int64_t)B.lo[2] * k + (int64_t)tx * 256;
  if (rb + 16 <= B.hi[1] && wc0 + 256 <= cend && vec) {
    // a whole tile (wave-uniform test): all sixteen rows' loads in flight
    // before the first store
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    typedef const u4 __attribute__((address_space(1))) guint4;
    typedef u4 __attribute__((address_space(1))) gwuint4;
    u4 v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = *(guint4 *)((gcf *)in + HD_EOFF(ai, B.dev, p, rb + q, 0) * k + c0);
#pragma unroll
    for (int q = 0; q < 16; ++q) *(gwuint4 *)((gwf *)out + HD_EOFF(ao, B.dev, p, rb + q, 0) * k + c0) = v[q];
    return;
  }
  for (int r = rb; r < min(rb + 16, B.hi[1]); ++r) {
    const int64_t bi = HD_EOFF(ai, B.dev, p, r, 0) * k, bo = HD_EOFF(ao, B.dev, p, r, 0) * k;
    if (vec && c0 + 4 <= cend) {
      *reinterpret_cast<uint4 *>(out + bo + c0) = *reinterpret_cast<const uint4 *>(in + bi + c0);
    } else {
      for (int e = 0; e < 4; ++e)
        if (c0 + e < cend) out[bo + c0 + e] = in[bi + c0 + e];
    }
  }
}

__host__ __device__ inline int64_t copy_tiles(const WorkBox &B, int esize) {
  const int64_t d = B.hi[0] - B.lo[0], h = B.hi[1] - B.lo[1], w = B.hi[2] - B.lo[2];
  if (d <= 0 || h <= 0 || w <= 0) return 0;
  return d * ((h + 15) / 16) * ((w * (esize / 4) + 255) / 256);
}

// ------------------------------------------------------------- stencil3d
// The forward march: one wave computes a pair of rows (j, j + 1) of 256
// columns (4 per lane) over a segment of planes (B.seg, kS3dSeg when
// unset), marching in i with the rows of the planes around i in registers
// (s3d_march_rows below), so each plane of the input is read from memory
// about once; the adjoint marches one row per wave the same way.  Four
// consecutive row pairs per workgroup share their j-neighbour rows in
// cache.  (Plane tiles that issue all of a tile's row loads at once, as
// the 2-D kernel does, measured slower on the 512^3 workload: 900 vs 580 us
// forward, 2600 vs 1730 us adjoint.)
constexpr int kS3dSeg = 32;
// planes between a row's load and its use in the forward march (two planes
// ahead measured no faster than one)
constexpr int kS3dDist = 1;

// Four consecutive elements of a row at columns [c, c + 4) (zeros outside
// the row); vec: rows are 16-byte aligned and c is a multiple of 4.
__device__ inline f4 ld_row4(const float *__restrict__ row, int c, int n2, bool vec) {
  f4 x = {0.f, 0.f, 0.f, 0.f};
  if (vec) {
    if (c < n2) x = *reinterpret_cast<const f4 *>(row + c);
  } else {
    if (c >= 0 && c < n2) x.x = row[c];
    if (c + 1 >= 0 && c + 1 < n2) x.y = row[c + 1];
    if (c + 2 >= 0 && c + 2 < n2) x.z = row[c + 2];
    if (c + 3 >= 0 && c + 3 < n2) x.w = row[c + 3];
  }
  return x;
}

// Row (i, j) of a full-extent array, or null outside the array.
__device__ inline const float *row_ptr(const float *__restrict__ u, int i, int j, int n0, int n1, int n2) {
  if (i < 0 || i >= n0 || j < 0 || j >= n1) return nullptr;
  return u + ((int64_t)i * n1 + j) * n2;
}

// A row chunk with its left / right neighbour columns (valid in lanes 0 / 63).
struct RowQ {
  f4 v;
  float l, r;
};

__device__ inline RowQ ld_rowq(const float *__restrict__ row, int c, int n2, bool vec, int lane) {
  RowQ q;
  q.v = {0.f, 0.f, 0.f, 0.f};
  q.l = q.r = 0.f;
  if (!row) return q;
  q.v = ld_row4(row, c, n2, vec);
  if (lane == 0 && c >= 1 && c - 1 < n2) q.l = row[c - 1];
  if (lane == 63 && c + 4 >= 0 && c + 4 < n2) q.r = row[c + 4];
  return q;
}

__device__ inline f4 ld_rowv(const float *__restrict__ row, int c, int n2, bool vec) {
  if (!row) return f4{0.f, 0.f, 0.f, 0.f};
  return ld_row4(row, c, n2, vec);
}

__device__ inline float f4at(const f4 &v, int e) { return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w; }

// Tiles of a box: rows x 256-column chunks x plane segments, rows fastest.
// Columns start at the box's low column rounded down to a multiple of 4.
__host__ __device__ inline int seg_of(const WorkBox &B) { return B.seg > 0 ? B.seg : kS3dSeg; }

__host__ __device__ inline int64_t march_tiles(int lo0, int hi0, int lo1, int hi1, int lo2, int hi2, int seg) {
  if (hi0 <= lo0 || hi1 <= lo1 || hi2 <= lo2) return 0;
  const int64_t kb = lo2 & ~3;
  return (int64_t)((hi0 - lo0 + seg - 1) / seg) * ((hi2 - kb + 255) / 256) * (hi1 - lo1);
}

// the forward march takes two rows per wave (rows j, j + 1 of a row pair)
__host__ __device__ inline int64_t s3d_tiles(const WorkBox &B) {
  const int pairs = (B.hi[1] - B.lo[1] + 1) / 2;
  return march_tiles(B.lo[0], B.hi[0], 0, pairs, B.lo[2], B.hi[2], seg_of(B));
}

// Geometry of one wave's row chunk for the marching kernels: columns
// [c, c + 4) of lane `lane`, and the halo column (c - 1 for lane 0, c + 4 for
// lane 63).  Every row load of the march is unconditional: plane, row and
// column indices are clamped into the array, so each load is in bounds, and
// a value read through a clamped index only ever feeds a boundary cell,
// whose output is its own input (or a column the chunk does not write).
// Loads for the next plane therefore never sit behind branches, and the
// waits before a plane's arithmetic cover only that plane's loads.
struct MarchRow {
  int c, n2;
  uint32_t uc, hc;  // c and the halo column as unsigned offsets: a uniform
                    // row base plus a zero-extended 32-bit lane offset is
                    // the scalar-base form of a global load
};

// c0: the chunk's first column (wave-uniform)
__device__ inline MarchRow march_row(int c0, int n2, int lane) {
  MarchRow m;
  m.c = c0 + 4 * lane;
  m.n2 = n2;
  const int h = lane == 0 ? m.c - 1 : m.c + 4;
  m.hc = (uint32_t)(h < 0 ? 0 : h >= n2 ? n2 - 1 : h);
  m.uc = (uint32_t)(m.c < 0 ? 0 : m.c);
  return m;
}

// row (i, j) with both indices clamped into the array
__device__ inline gcf *grow_clamp(gcf *u, int i, int j, int n0, int n1, int n2) {
  i = i < 0 ? 0 : i >= n0 ? n0 - 1 : i;
  j = j < 0 ? 0 : j >= n1 ? n1 - 1 : j;
  return u + ((int64_t)i * n1 + j) * n2;
}

// FULL: the row length is a multiple of 4 and the chunk's 256 columns lie
// in the row (one float4 per lane); otherwise clamped loads
template <bool FULL>
__device__ inline f4 mrd4(gcf *row, const MarchRow &m) {
  if constexpr (FULL) {
    return *(gcf4 *)(row + m.uc);
  } else {
    f4 x;
    float *px = reinterpret_cast<float *>(&x);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = m.c + e;
      px[e] = row[k < 0 ? 0 : k >= m.n2 ? m.n2 - 1 : k];
    }
    return x;
  }
}

// a row chunk with the lane's halo column (lanes 0 and 63 use it)
struct MRow {
  f4 v;
  float h;
};

template <bool FULL>
__device__ inline MRow mrdq(gcf *row, const MarchRow &m) {
  MRow q;
  q.v = mrd4<FULL>(row, m);
  q.h = row[m.hc];
  return q;
}

// One plane step of the 7-point stencil for lane's four columns: pm / pp
// the row j of planes i -+ 1, cu (with its halo column) plane i, jm / jp the
// rows j -+ 1 of plane i; iint: plane i and row j are interior.
__device__ inline void s3d_point(const Coef7 &cf, const WorkBox &B, const MarchRow &m, int lane, bool iint,
                                 const f4 &pm, const MRow &cu, const f4 &pp, const f4 &jm, const f4 &jp, gwf *q,
                                 bool wfull) {
  const float lw = __shfl_up(cu.v.w, 1), rx = __shfl_down(cu.v.x, 1);
  const float kl[4] = {lane == 0 ? cu.h : lw, cu.v.x, cu.v.y, cu.v.z};
  const float kr[4] = {cu.v.y, cu.v.z, cu.v.w, lane == 63 ? cu.h : rx};
  float o[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int k = m.c + e;
    const float x = f4at(cu.v, e);
    float acc = cf.c[0] * x;
    acc = __builtin_fmaf(cf.c[1], f4at(pm, e), acc);
    acc = __builtin_fmaf(cf.c[2], f4at(pp, e), acc);
    acc = __builtin_fmaf(cf.c[3], f4at(jm, e), acc);
    acc = __builtin_fmaf(cf.c[4], f4at(jp, e), acc);
    acc = __builtin_fmaf(cf.c[5], kl[e], acc);
    acc = __builtin_fmaf(cf.c[6], kr[e], acc);
    o[e] = iint && k >= 1 && k <= m.n2 - 2 ? acc : x;
  }
  if (wfull) {
    __builtin_nontemporal_store(f4{o[0], o[1], o[2], o[3]}, (gwf4 *)(q + m.c));
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = m.c + e;
      if (k >= B.lo[2] && k < B.hi[2]) q[k] = o[e];
    }
  }
}

// The march over planes [i0, i1) of one chunk of the row pair j, j + 1,
// with the loads for plane i + D issued before plane i is computed.  Each
// row of the pair is the other's j-neighbour, so a plane costs four row
// loads for two output rows (rows j - 1 and j + 2 besides the pair).  The
// rows live in rings of registers: each row of the pair for planes
// i - 1 .. i + 1 + D (NR slots), rows j - 1 and j + 2 for planes i .. i + D
// (NJ slots); the loop is unrolled U = lcm(NR, NJ) times so that every slot
// is a fixed set of registers and nothing is copied between slots (a copy
// of a slot still being loaded would wait for that load).  two: row j + 1
// lies in the box (else it is read as a neighbour only).
template <bool FULL, int D>
__device__ inline void s3d_march_rows(const WorkBox &B, const Coef7 &cf, gcf *u, gwf *out, int N0, int N1, int N2,
                                      int i0, int i1, int j, bool two, int c0, bool wfull) {
  static_assert(D == 1 || D == 2, "prefetch distance");
  constexpr int NR = D == 1 ? 4 : 6, NJ = D == 1 ? 2 : 3, U = D == 1 ? 4 : 6;
  const int lane = threadIdx.x & 63;
  const MarchRow m = march_row(c0, N2, lane);
  const bool jint0 = j >= 1 && j <= N1 - 2, jint1 = j + 1 >= 1 && j + 1 <= N1 - 2;
  MRow R0[NR], R1[NR];
  f4 JM[NJ], JP[NJ];
  // slot of plane p: (p - i0 + 1) % NR for the pair, (p - i0) % NJ for
  // rows j - 1 and j + 2
#pragma unroll
  for (int q = 0; q < D + 2; ++q) {
    R0[q] = mrdq<FULL>(grow_clamp(u, i0 - 1 + q, j, N0, N1, N2), m);
    R1[q] = mrdq<FULL>(grow_clamp(u, i0 - 1 + q, j + 1, N0, N1, N2), m);
  }
#pragma unroll
  for (int q = 0; q < D; ++q) {
    JM[q] = mrd4<FULL>(grow_clamp(u, i0 + q, j - 1, N0, N1, N2), m);
    JP[q] = mrd4<FULL>(grow_clamp(u, i0 + q, j + 2, N0, N1, N2), m);
  }
  for (int ib = i0; ib < i1; ib += U) {
#pragma unroll
    for (int s = 0; s < U; ++s) {
      const int i = ib + s;
      if (i >= i1) break;
      // rows for plane i + D (past the segment's end they are read and not
      // used)
      R0[(s + 2 + D) % NR] = mrdq<FULL>(grow_clamp(u, i + 1 + D, j, N0, N1, N2), m);
      R1[(s + 2 + D) % NR] = mrdq<FULL>(grow_clamp(u, i + 1 + D, j + 1, N0, N1, N2), m);
      JM[(s + D) % NJ] = mrd4<FULL>(grow_clamp(u, i + D, j - 1, N0, N1, N2), m);
      JP[(s + D) % NJ] = mrd4<FULL>(grow_clamp(u, i + D, j + 2, N0, N1, N2), m);
      const bool iint = i >= 1 && i <= N0 - 2;
      gwf *q = out + ((int64_t)i * N1 + j) * N2;
      s3d_point(cf, B, m, lane, iint && jint0, R0[s % NR].v, R0[(s + 1) % NR], R0[(s + 2) % NR].v, JM[s % NJ],
                R1[(s + 1) % NR].v, q, wfull);
      if (two)
        s3d_point(cf, B, m, lane, iint && jint1, R1[s % NR].v, R1[(s + 1) % NR], R1[(s + 2) % NR].v,
                  R0[(s + 1) % NR].v, JP[s % NJ], q + N2, wfull);
    }
  }
}

// lt: the wave's tile within box B (wave-uniform): row pair, then column
// chunk, then plane segment
__device__ inline void dev_s3d_march(const WorkBox &B, int64_t lt, const ArrDev *__restrict__ A, const Coef7 &cf) {
  const int pairs = (B.hi[1] - B.lo[1] + 1) / 2;
  const int kb = B.lo[2] & ~3;
  const int nk = (B.hi[2] - kb + 255) / 256;
  const int j = B.lo[1] + 2 * (int)(lt % pairs);
  const bool two = j + 1 < B.hi[1];
  const int64_t rest = lt / pairs;
  const int c0 = kb + (int)(rest % nk) * 256;
  const int seg = seg_of(B);
  const int i0 = B.lo[0] + (int)(rest / nk) * seg;
  const int i1 = min(i0 + seg, B.hi[0]);
  const ArrDev &ai = A[B.ain];
  gcf *u = (gcf *)ai.buf[B.dev];
  gwf *out = (gwf *)A[B.aout].buf[B.dev];
  const int N0 = (int)ai.n[0], N1 = (int)ai.n[1], N2 = (int)ai.n[2];
  const bool vec = (N2 & 3) == 0;
  const bool wfull = vec && c0 >= B.lo[2] && c0 + 256 <= B.hi[2];
  if (vec && c0 + 256 <= N2)
    s3d_march_rows<true, kS3dDist>(B, cf, u, out, N0, N1, N2, i0, i1, j, two, c0, wfull);
  else
    s3d_march_rows<false, 1>(B, cf, u, out, N0, N1, N2, i0, i1, j, two, c0, wfull);
}

}  // namespace hd

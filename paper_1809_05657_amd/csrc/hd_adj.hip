// hd_adj.hip — adjoint of one ApplyKernel step of the 7-point stencil, with
// the reverse halo exchange (the cotangent of a halo element is added to its
// owner's value).
//
// Forward (per interior cell y): u1[y] = c0 u[y] + c1 u[y-ei] + c2 u[y+ei]
//   + c3 u[y-ej] + c4 u[y+ej] + c5 u[y-ek] + c6 u[y+ek]; boundary: u1 = u.
// Reverse: du[x] = sum over outputs y that read x of c_e * du1[y], plus
// du1[x] on the boundary; dc_e = sum over interior y of du1[y] * u[y + off_e].
//
// Distributed form: device d only knows du1 on its own work box W_d, so it
// computes the part of du coming from its own outputs on W_d +- 1 (its use
// region); the values on halo cells are partial sums that belong to the
// owner of the cell.  The reverse messages are the use-region messages with
// source and destination swapped; the owner adds the partial sums it
// receives to its own, in message-table order (deterministic).
#include <hip/hip_runtime.h>

#include "hd_dev_data.hpp"

namespace hd {

struct AdjArgs {
  const WorkBox *wb;  // work boxes W_d (ain = du1 array, aout = du array, ain2 = u array)
  int nbox;
  int64_t ntiles;     // tiles over the extended boxes
  Coef7 cf;
  double *part;       // [gridDim.x][8] coefficient-gradient partials
};

// tiles of the extended box W +- 1 (clipped), marched like the forward
// kernel: one wave per (row, 256 columns, segment of planes), four rows per
// workgroup.  The column tiles cover the box's own columns; the extended
// column on either side is one extra cell of lane 0 / lane 63 (it gets a
// contribution from its one neighbour inside the box only).
__host__ __device__ inline void ext_box(const WorkBox &B, const int64_t *n, int *lo, int *hi) {
  for (int q = 0; q < 3; ++q) {
    lo[q] = B.lo[q] - 1 < 0 ? 0 : B.lo[q] - 1;
    hi[q] = B.hi[q] + 1 > n[q] ? (int)n[q] : B.hi[q] + 1;
  }
}

// y is an interior cell of the array inside the work box (one coordinate)
__device__ inline bool adj_in(int y, int lo, int hi, int n) { return y >= 1 && y <= n - 2 && y >= lo && y < hi; }

// row flags of the march: rows j, j -+ 1 interior in the box; row j owned, interior
struct AdjRow {
  bool rj, rjm, rjp, jown, jint;
};

// Every du1 value enters the adjoint only through the outputs the device
// owns: the term c_e du1[y] reaches x = y + off_e, and du1[y] u[y + off_e]
// enters dc_e, exactly when y is an interior cell of the work box.  So each
// du1 value is masked once by that flag of its own position (a bit mask,
// all ones or zero), after which every term is an unconditional fused
// multiply-add: a masked value adds a zero product, which leaves the sums
// bitwise unchanged, and a value read through a clamped index is always
// masked.  The flags split into a column part, fixed per lane for the whole
// march (VGPR bit masks), and a plane / row part, uniform across the wave.
struct AdjMask {
  uint32_t kz[4];  // column of element e is inside the box and interior
  uint32_t kh;     // the same for the halo column (lane 0: left, lane 63: right)
  uint32_t cpa[4]; // boundary copy on a boundary plane: row and column owned
  uint32_t cpb[4]; // boundary copy on an interior plane: owned, not interior
};

__device__ inline float msk(float v, uint32_t m) { return __uint_as_float(__float_as_uint(v) & m); }
__device__ inline uint32_t ones(bool b) { return b ? 0xffffffffu : 0u; }

// One plane of the adjoint for lane's four columns of row j: gpm / gpp the
// du1 row j of planes i -+ 1, gcu (with its halo column) plane i, gjm / gjp
// du1 rows j -+ 1 of plane i, wcu (with its halo column) the u row j of
// plane i.  Writes du of the extended box's cells (terms in the order
// e = 0..6, then du1[x] itself when x is an owned boundary cell) and adds
// the coefficient gradient terms u[y] du1[y - off_e] to cb.
__device__ inline void adj_point(const Coef7 &cf, const WorkBox &B, const int *lo, const int *hi, const MarchRow &m,
                                 int lane, int i, int N0, const AdjRow &R, const AdjMask &M, const f4 &gpm,
                                 const MRow &gcu, const f4 &gpp, const f4 &gjm, const f4 &gjp, const MRow &wcu,
                                 gwf *q, bool wfull, bool xl, bool xr, double *cb) {
  const bool pi = adj_in(i, B.lo[0], B.hi[0], N0), pim = adj_in(i - 1, B.lo[0], B.hi[0], N0),
             pip = adj_in(i + 1, B.lo[0], B.hi[0], N0);
  const bool iown = i >= B.lo[0] && i < B.hi[0], iint = i >= 1 && i <= N0 - 2;
  const uint32_t rc = ones(pi && R.rj), rp = ones(pip && R.rj), rm = ones(pim && R.rj), rjp = ones(pi && R.rjp),
                 rjm = ones(pi && R.rjm);
  float zx[4], zp[4], zm[4], zjp[4], zjm[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    zx[e] = msk(f4at(gcu.v, e), M.kz[e] & rc);
    zp[e] = msk(f4at(gpp, e), M.kz[e] & rp);
    zm[e] = msk(f4at(gpm, e), M.kz[e] & rm);
    zjp[e] = msk(f4at(gjp, e), M.kz[e] & rjp);
    zjm[e] = msk(f4at(gjm, e), M.kz[e] & rjm);
  }
  const float zh = msk(gcu.h, M.kh & rc);
  const float zlw = __shfl_up(zx[3], 1), zrx = __shfl_down(zx[0], 1);
  const float zkl[4] = {lane == 0 ? zh : zlw, zx[0], zx[1], zx[2]};
  const float zkr[4] = {zx[1], zx[2], zx[3], lane == 63 ? zh : zrx};
  float o[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float acc = __builtin_fmaf(cf.c[0], zx[e], 0.f);
    acc = __builtin_fmaf(cf.c[1], zp[e], acc);
    acc = __builtin_fmaf(cf.c[2], zm[e], acc);
    acc = __builtin_fmaf(cf.c[3], zjp[e], acc);
    acc = __builtin_fmaf(cf.c[4], zjm[e], acc);
    acc = __builtin_fmaf(cf.c[5], zkr[e], acc);
    acc = __builtin_fmaf(cf.c[6], zkl[e], acc);
    const uint32_t cp = iown ? (iint ? M.cpb[e] : M.cpa[e]) : 0u;
    o[e] = acc + msk(f4at(gcu.v, e), cp);
    // u[y] du1[y - off_e]: the FP64 product of two FP32 values is exact, so
    // the fused form rounds exactly like a product followed by an add
    const double uy = (double)f4at(wcu.v, e);
    cb[0] = __builtin_fma(uy, (double)zx[e], cb[0]);
    cb[1] = __builtin_fma(uy, (double)zp[e], cb[1]);
    cb[2] = __builtin_fma(uy, (double)zm[e], cb[2]);
    cb[3] = __builtin_fma(uy, (double)zjp[e], cb[3]);
    cb[4] = __builtin_fma(uy, (double)zjm[e], cb[4]);
    cb[5] = __builtin_fma(uy, (double)zkr[e], cb[5]);
    cb[6] = __builtin_fma(uy, (double)zkl[e], cb[6]);
  }
  if (wfull) {
    *(gwf4 *)(q + m.c) = f4{o[0], o[1], o[2], o[3]};
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = m.c + e;
      if (k >= lo[2] && k < hi[2]) q[k] = o[e];
    }
  }
  // the extended column next to the box (outside it, so never owned): only
  // the term of its neighbour inside the box reaches it
  if (xl) {
    q[m.c - 1] = __builtin_fmaf(cf.c[5], zx[0], 0.f);
    cb[5] = __builtin_fma((double)wcu.h, (double)zx[0], cb[5]);
  }
  if (xr) {
    q[m.c + 4] = __builtin_fmaf(cf.c[6], zx[3], 0.f);
    cb[6] = __builtin_fma((double)wcu.h, (double)zx[3], cb[6]);
  }
}

// The adjoint march over planes [i0, i1) of one row chunk of the extended
// box, with the loads for plane i + 1 issued before plane i is computed.
// Rings of registers as in the forward march: du1 row j of planes
// i - 1 .. i + 2 (four slots), du1 rows j -+ 1 and the u row j of planes
// i, i + 1 (two slots each); the loop is unrolled four times so that every
// slot is a fixed set of registers.  Every load is unconditional with
// clamped indices; a value read through a clamped index is always masked.
template <bool FULL>
__device__ inline void adj_march(const Coef7 &cf, const WorkBox &B, const int *lo, const int *hi, gcf *g1, gcf *u,
                                 gwf *g0, int N0, int N1, int N2, int i0, int i1, int j, int c0, bool wfull,
                                 bool xl, bool xr, double *cb) {
  const int lane = threadIdx.x & 63;
  const MarchRow m = march_row(c0, N2, lane);
  AdjRow R;
  R.rj = adj_in(j, B.lo[1], B.hi[1], N1);
  R.rjm = adj_in(j - 1, B.lo[1], B.hi[1], N1);
  R.rjp = adj_in(j + 1, B.lo[1], B.hi[1], N1);
  R.jown = j >= B.lo[1] && j < B.hi[1];
  R.jint = j >= 1 && j <= N1 - 2;
  AdjMask M;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int k = m.c + e;
    const bool kown = k >= B.lo[2] && k < B.hi[2], kint = k >= 1 && k <= N2 - 2;
    M.kz[e] = ones(adj_in(k, B.lo[2], B.hi[2], N2));
    M.cpa[e] = ones(R.jown && kown);
    M.cpb[e] = ones(R.jown && kown && !(R.jint && kint));
  }
  M.kh = ones(adj_in(lane == 0 ? m.c - 1 : m.c + 4, B.lo[2], B.hi[2], N2));
  MRow G[4], W[2];
  f4 JM[2], JP[2];
  // slot of plane p: (p - i0 + 1) & 3 for G, (p - i0) & 1 for the others
  G[0] = mrdq<FULL>(grow_clamp(g1, i0 - 1, j, N0, N1, N2), m);
  G[1] = mrdq<FULL>(grow_clamp(g1, i0, j, N0, N1, N2), m);
  G[2] = mrdq<FULL>(grow_clamp(g1, i0 + 1, j, N0, N1, N2), m);
  JM[0] = mrd4<FULL>(grow_clamp(g1, i0, j - 1, N0, N1, N2), m);
  JP[0] = mrd4<FULL>(grow_clamp(g1, i0, j + 1, N0, N1, N2), m);
  W[0] = mrdq<FULL>(grow_clamp(u, i0, j, N0, N1, N2), m);
  for (int ib = i0; ib < i1; ib += 4) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int i = ib + s;
      if (i >= i1) break;
      G[(s + 3) & 3] = mrdq<FULL>(grow_clamp(g1, i + 2, j, N0, N1, N2), m);
      JM[(s + 1) & 1] = mrd4<FULL>(grow_clamp(g1, i + 1, j - 1, N0, N1, N2), m);
      JP[(s + 1) & 1] = mrd4<FULL>(grow_clamp(g1, i + 1, j + 1, N0, N1, N2), m);
      W[(s + 1) & 1] = mrdq<FULL>(grow_clamp(u, i + 1, j, N0, N1, N2), m);
      adj_point(cf, B, lo, hi, m, lane, i, N0, R, M, G[s & 3].v, G[(s + 1) & 3], G[(s + 2) & 3].v, JM[s & 1],
                JP[s & 1], W[s & 1], g0 + ((int64_t)i * N1 + j) * N2, wfull, xl, xr, cb);
    }
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_s3d_adj(AdjArgs a, const ArrDev *__restrict__ A) {
  __shared__ double s_red[4][8];
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double cb[7] = {0, 0, 0, 0, 0, 0, 0};
  const int64_t nwg = (a.ntiles + 3) >> 2;
  const int64_t t = xcd_remap(blockIdx.x, nwg) * 4 + wv;
  if (t < a.ntiles) {
    const WorkBox B = a.wb[find_box(a.wb, a.nbox, t)];
    const ArrDev &ag = A[B.ain], &ao = A[B.aout], &au = A[B.ain2];
    int lo[3], hi[3];
    ext_box(B, ag.n, lo, hi);
    const int64_t lt = t - B.tile0;
    const int jrows = hi[1] - lo[1];
    const int kb = B.lo[2] & ~3;
    const int nk = (B.hi[2] - kb + 255) / 256;
    const int j = lo[1] + (int)(lt % jrows);
    const int64_t rest = lt / jrows;
    const int tk = (int)(rest % nk);
    const int c0 = kb + tk * 256;
    // extended columns outside the column tiles
    const bool xl = lane == 0 && tk == 0 && lo[2] < kb;
    const bool xr = lane == 63 && tk == nk - 1 && hi[2] > kb + nk * 256;
    const int seg = seg_of(B);
    const int i0 = lo[0] + (int)(rest / nk) * seg;
    const int i1 = min(i0 + seg, hi[0]);
    const int N0 = (int)ag.n[0], N1 = (int)ag.n[1], N2 = (int)ag.n[2];
    const bool vec = (N2 & 3) == 0;
    gcf *g1 = (gcf *)ag.buf[B.dev];
    gcf *u = (gcf *)au.buf[B.dev];
    gwf *g0 = (gwf *)ao.buf[B.dev];
    const bool wfull = vec && c0 >= lo[2] && c0 + 256 <= hi[2];
    if (vec && c0 + 256 <= N2)
      adj_march<true>(a.cf, B, lo, hi, g1, u, g0, N0, N1, N2, i0, i1, j, c0, wfull, xl, xr, cb);
    else
      adj_march<false>(a.cf, B, lo, hi, g1, u, g0, N0, N1, N2, i0, i1, j, c0, wfull, xl, xr, cb);
  }
  // fixed-order reduction of the FP64 coefficient partials of this workgroup
#pragma unroll
  for (int e = 0; e < 7; ++e) {
    double v = cb[e];
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    cb[e] = v;
  }
  if (lane == 0)
    for (int e = 0; e < 7; ++e) s_red[wv][e] = cb[e];
  __syncthreads();
  if (threadIdx.x < 7) {
    const int e = threadIdx.x;
    a.part[blockIdx.x * 8 + e] = ((s_red[0][e] + s_red[1][e]) + s_red[2][e]) + s_red[3][e];
  }
}

// cbar[e] += sum of the workgroup partials, one workgroup per coefficient:
// thread t sums partials t, t + 256, ... in increasing order, then a
// pairwise tree over the threads; the order depends only on the count, so
// the result is reproducible.
__device__ inline void cbar_final(const double *part, int64_t nblk, double *cbar, int e) {
  __shared__ double s[256];
  const int t = threadIdx.x;
  double v = 0.0;
  for (int64_t b = t; b < nblk; b += 256) v += part[b * 8 + e];
  s[t] = v;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (t < h) s[t] = s[t] + s[t + h];
    __syncthreads();
  }
  if (t == 0) cbar[e] += s[0];
}

__device__ inline bool msg_has(const MsgRec &r, int64_t p, int64_t q, int64_t c) {
  return p >= r.lo[0] && p < r.hi[0] && q >= r.lo[1] && q < r.hi[1] && c >= r.lo[2] && c < r.hi[2];
}

// The reverse exchange in one pass over the words of the reverse messages:
// each thread copies its word, the partial sum held by the message's user
// (the forward destination), into the staging buffer (the wire), and the
// thread of the first message (in table order) that carries a cell adds
// every contribution to that cell, in table order, to the owner's value,
// reading the partials where the users hold them (the same values the
// staging words carry).  Each cell scans the message table twice, so the
// table is staged in LDS when it is small, and the buffers are read through
// global-address pointers (flat loads would also be waited for by every
// LDS read).  Workgroups past the first npack sum the coefficient partials
// instead, one per coefficient.
constexpr int kUnpackLdsMsgs = 128;

__global__ __launch_bounds__(256) void k_unpack_add(const MsgRec *__restrict__ M, const MsgHdr *__restrict__ H,
                                                    const ArrDev *__restrict__ A, uint32_t *__restrict__ stg,
                                                    int npack, const double *part, int64_t nblk, double *cbar) {
  if ((int)blockIdx.x >= npack) {
    cbar_final(part, nblk, cbar, (int)blockIdx.x - npack);
    return;
  }
  __shared__ MsgRec s_m[kUnpackLdsMsgs];
  const int64_t n = H->nmsg, words = H->bytes >> 2;
  const bool in_lds = n <= kUnpackLdsMsgs;
  if (in_lds)
    for (int i = threadIdx.x; i < n; i += blockDim.x) s_m[i] = M[i];
  __syncthreads();
  const MsgRec *T = in_lds ? s_m : M;
  gwf *sg = (gwf *)stg;
  int m = 0;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += (int64_t)npack * blockDim.x) {
    if (!(T[m].off <= 4 * w && 4 * w < T[m].off + T[m].bytes)) m = find_msg(T, n, 4 * w);
    const MsgRec &r = T[m];
    const int64_t lw = w - (r.off >> 2);
    if (4 * lw >= r.bytes) continue;
    const int64_t wid = r.hi[2] - r.lo[2], rows = r.hi[1] - r.lo[1];
    const int64_t c = r.lo[2] + lw % wid, t = lw / wid, q = r.lo[1] + t % rows, p = r.lo[0] + t / rows;
    const ArrDev &a = A[r.arr];
    const float mine = ((gcf *)a.buf[r.dst])[HD_EOFF(a, r.dst, p, q, c)];
    sg[w] = mine;
    bool first = true;
    for (int64_t m2 = 0; m2 < m; ++m2)
      if (T[m2].src == r.src && T[m2].arr == r.arr && msg_has(T[m2], p, q, c)) {
        first = false;
        break;
      }
    if (!first) continue;
    gwf *own = (gwf *)a.buf[r.src];
    const int64_t g = HD_EOFF(a, r.src, p, q, c);
    float v = own[g] + mine;
    for (int64_t m2 = m + 1; m2 < n; ++m2) {
      const MsgRec &e = T[m2];
      if (e.src != r.src || e.arr != r.arr || !msg_has(e, p, q, c)) continue;
      v = v + ((gcf *)a.buf[e.dst])[HD_EOFF(a, e.dst, p, q, c)];
    }
    own[g] = v;
  }
}

int64_t adj_tiles(const WorkBox &B, const int64_t *n) {
  int lo[3], hi[3];
  ext_box(B, n, lo, hi);
  return march_tiles(lo[0], hi[0], lo[1], hi[1], B.lo[2], B.hi[2], seg_of(B));
}

hipError_t launch_adjoint(const WorkBox *wb, int nbox, int64_t ntiles, const float *coef, double *part,
                          double *cbar, const MsgRec *M, const MsgHdr *H, const ArrDev *A, uint32_t *stg,
                          int64_t bound_words, hipStream_t s) {
  AdjArgs a;
  a.wb = wb;
  a.nbox = nbox;
  a.ntiles = ntiles;
  for (int e = 0; e < 7; ++e) a.cf.c[e] = coef[e];
  a.part = part;
  int64_t nwg = 0;
  if (ntiles > 0) {
    nwg = (ntiles + 3) / 4;
    hipLaunchKernelGGL(k_s3d_adj, dim3((unsigned)nwg), dim3(256), 0, s, a, A);
  }
  int grid = (int)((bound_words + 255) / 256);
  if (grid > 4096) grid = 4096;
  if (grid < 1) grid = 1;
  // seven more workgroups reduce the coefficient partials
  const int ncb = cbar && nwg > 0 ? 7 : 0;
  hipLaunchKernelGGL(k_unpack_add, dim3(grid + ncb), dim3(256), 0, s, M, H, A, stg, grid, part, nwg, cbar);
  return hipGetLastError();
}

}  // namespace hd

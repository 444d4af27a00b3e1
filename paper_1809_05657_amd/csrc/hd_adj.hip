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

__device__ inline bool in_box(const WorkBox &B, int i, int j, int k) {
  return i >= B.lo[0] && i < B.hi[0] && j >= B.lo[1] && j < B.hi[1] && k >= B.lo[2] && k < B.hi[2];
}

// tiles of the extended box W +- 1 (clipped): one wave per (plane, row) x 256
// columns, 4 rows per workgroup
__host__ __device__ inline void ext_box(const WorkBox &B, const int64_t *n, int *lo, int *hi) {
  for (int q = 0; q < 3; ++q) {
    lo[q] = B.lo[q] - 1 < 0 ? 0 : B.lo[q] - 1;
    hi[q] = B.hi[q] + 1 > n[q] ? (int)n[q] : B.hi[q] + 1;
  }
}

__global__ __launch_bounds__(256) void k_s3d_adj(AdjArgs a, const ArrDev *__restrict__ A) {
  __shared__ double s_red[4][8];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double cb[7] = {0, 0, 0, 0, 0, 0, 0};
  const int64_t t = blockIdx.x;
  const WorkBox B = a.wb[find_box(a.wb, a.nbox, t)];
  const ArrDev &ag = A[B.ain], &ao = A[B.aout], &au = A[B.ain2];
  int lo[3], hi[3];
  ext_box(B, ag.n, lo, hi);
  const int h = hi[1] - lo[1], w = hi[2] - lo[2];
  const int nty = (h + 3) / 4, ntx = (w + 255) / 256;
  const int64_t lt = t - B.tile0;
  const int ty = (int)(lt % nty);
  const int64_t rest = lt / nty;
  const int tx = (int)(rest % ntx);
  const int i = lo[0] + (int)(rest / ntx);
  const int j = lo[1] + ty * 4 + wv;
  const int N0 = (int)ag.n[0], N1 = (int)ag.n[1], N2 = (int)ag.n[2];
  const int64_t si = (int64_t)N1 * N2, sj = N2;
  if (j < hi[1]) {
    const float *__restrict__ g1 = reinterpret_cast<const float *>(ag.buf[B.dev]);
    const float *__restrict__ u = reinterpret_cast<const float *>(au.buf[B.dev]);
    float *__restrict__ g0 = reinterpret_cast<float *>(ao.buf[B.dev]);
    // neighbour y = x - off_e for e = 0..6 with off = (0, -ei, +ei, -ej, +ej, -ek, +ek)
    const int di[7] = {0, 1, -1, 0, 0, 0, 0}, dj[7] = {0, 0, 0, 1, -1, 0, 0}, dk[7] = {0, 0, 0, 0, 0, 1, -1};
    const int64_t offs[7] = {0, -si, si, -sj, sj, -1, 1};
    const int c0 = lo[2] + tx * 256 + 4 * lane;
#pragma unroll
    for (int e4 = 0; e4 < 4; ++e4) {
      const int k = c0 + e4;
      if (k >= hi[2]) break;
      const int64_t x = (int64_t)i * si + (int64_t)j * sj + k;
      float acc = 0.f;
#pragma unroll
      for (int e = 0; e < 7; ++e) {
        const int yi = i + di[e], yj = j + dj[e], yk = k + dk[e];
        const bool yint = yi >= 1 && yi <= N0 - 2 && yj >= 1 && yj <= N1 - 2 && yk >= 1 && yk <= N2 - 2;
        if (yint && in_box(B, yi, yj, yk)) acc = __builtin_fmaf(a.cf.c[e], g1[x - offs[e]], acc);
      }
      const bool xint = i >= 1 && i <= N0 - 2 && j >= 1 && j <= N1 - 2 && k >= 1 && k <= N2 - 2;
      const bool xown = in_box(B, i, j, k);
      if (xown && !xint) acc = acc + g1[x];
      g0[x] = acc;
      if (xown && xint) {
        const double gy = (double)g1[x];
#pragma unroll
        for (int e = 0; e < 7; ++e) cb[e] += gy * (double)u[x + offs[e]];
      }
    }
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
__global__ __launch_bounds__(256) void k_cbar_final(const double *part, int64_t nblk, double *cbar) {
  __shared__ double s[256];
  const int e = blockIdx.x, t = threadIdx.x;
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

// reverse pack: the partial sums at the halo cells of the device that holds
// them (the forward destination) go to the staging buffer
__global__ __launch_bounds__(256) void k_rev_pack(const MsgRec *__restrict__ M, const MsgHdr *__restrict__ H,
                                                  const ArrDev *__restrict__ A, uint32_t *__restrict__ stg) {
  const int64_t n = H->nmsg, words = H->bytes >> 2;
  int m = 0;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += (int64_t)gridDim.x * blockDim.x) {
    if (!(M[m].off <= 4 * w && 4 * w < M[m].off + M[m].bytes)) m = find_msg(M, n, 4 * w);
    const MsgRec &r = M[m];
    const int64_t lw = w - (r.off >> 2);
    if (4 * lw >= r.bytes) continue;
    const int64_t wid = r.hi[2] - r.lo[2], rows = r.hi[1] - r.lo[1];
    const int64_t c = lw % wid, t = lw / wid, rr = t % rows, p = t / rows;
    const ArrDev &a = A[r.arr];
    const int64_t g = ((r.lo[0] + p) * a.n[1] + r.lo[1] + rr) * a.n[2] + r.lo[2] + c;
    stg[w] = reinterpret_cast<const uint32_t *>(a.buf[r.dst])[g];
  }
}

__device__ inline bool msg_has(const MsgRec &r, int64_t p, int64_t q, int64_t c) {
  return p >= r.lo[0] && p < r.hi[0] && q >= r.lo[1] && q < r.hi[1] && c >= r.lo[2] && c < r.hi[2];
}

// ordered scatter-add into the owners: the thread of the first message (in
// table order) that carries a cell adds every contribution to that cell, in
// table order, to the owner's value
__global__ __launch_bounds__(256) void k_unpack_add(const MsgRec *__restrict__ M, const MsgHdr *__restrict__ H,
                                                    const ArrDev *__restrict__ A, const float *__restrict__ stg) {
  const int64_t n = H->nmsg, words = H->bytes >> 2;
  int m = 0;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += (int64_t)gridDim.x * blockDim.x) {
    if (!(M[m].off <= 4 * w && 4 * w < M[m].off + M[m].bytes)) m = find_msg(M, n, 4 * w);
    const MsgRec &r = M[m];
    const int64_t lw = w - (r.off >> 2);
    if (4 * lw >= r.bytes) continue;
    const int64_t wid = r.hi[2] - r.lo[2], rows = r.hi[1] - r.lo[1];
    const int64_t c = r.lo[2] + lw % wid, t = lw / wid, q = r.lo[1] + t % rows, p = r.lo[0] + t / rows;
    bool first = true;
    for (int64_t m2 = 0; m2 < m; ++m2)
      if (M[m2].src == r.src && M[m2].arr == r.arr && msg_has(M[m2], p, q, c)) {
        first = false;
        break;
      }
    if (!first) continue;
    const ArrDev &a = A[r.arr];
    float *own = reinterpret_cast<float *>(a.buf[r.src]);
    const int64_t g = (p * a.n[1] + q) * a.n[2] + c;
    float v = own[g];
    for (int64_t m2 = m; m2 < n; ++m2) {
      const MsgRec &s = M[m2];
      if (s.src != r.src || s.arr != r.arr || !msg_has(s, p, q, c)) continue;
      const int64_t sw = s.hi[2] - s.lo[2], sr = s.hi[1] - s.lo[1];
      const int64_t idx = ((p - s.lo[0]) * sr + (q - s.lo[1])) * sw + (c - s.lo[2]);
      v = v + stg[(s.off >> 2) + idx];
    }
    own[g] = v;
  }
}

int64_t adj_tiles(const WorkBox &B, const int64_t *n) {
  int lo[3], hi[3];
  ext_box(B, n, lo, hi);
  const int64_t d = hi[0] - lo[0], h = hi[1] - lo[1], w = hi[2] - lo[2];
  if (d <= 0 || h <= 0 || w <= 0) return 0;
  return d * ((h + 3) / 4) * ((w + 255) / 256);
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
  if (ntiles > 0) {
    hipLaunchKernelGGL(k_s3d_adj, dim3(ntiles), dim3(256), 0, s, a, A);
    if (cbar) hipLaunchKernelGGL(k_cbar_final, dim3(7), dim3(256), 0, s, part, ntiles, cbar);
  }
  int grid = (int)((bound_words + 255) / 256);
  if (grid > 4096) grid = 4096;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_rev_pack, dim3(grid), dim3(256), 0, s, M, H, A, stg);
  hipLaunchKernelGGL(k_unpack_add, dim3(grid), dim3(256), 0, s, M, H, A, (const float *)stg);
  return hipGetLastError();
}

}  // namespace hd

// hd_data.hip — data-path kernels of the HDArray runtime on gfx950:
// pack / unpack of the message table (Sec. 3.1: the section copies around
// the wire), the built-in user kernels run over every logical device of a
// partition in one launch (Sec. 3.2 GEMM, Sec. 5.1 Jacobi), and reductions
// (Table 2 Reduce).
//
// Built-in kernels (each device d reads its own buffers and writes its work
// box of the output, both full-extent, row-major):
//   jacobi2d   A[i][j] = (((B[i][j-1] + B[i][j+1]) + B[i-1][j]) + B[i+1][j]) / 4
//              on interior cells, A = B on the array boundary (fp32, no FMA)
//   tri2d      the same update on 1 <= j < i <= n-2, copy on the other cells
//              with j <= i; cells with j > i are not written
//   copy       out = in (raw 4- or 8-byte elements)
//   stencil3d7 acc = c0*u; acc = fma(c_e, u[x+e], acc) for e = -i,+i,-j,+j,-k,+k
//              on interior cells, copy on the boundary
//   matmul     C[i][j] = sum_k A[i][k] * B[k][j] over the rows/cols of the box
#include <hip/hip_runtime.h>

#include "hd_internal.hpp"

namespace hd {

typedef float f4 __attribute__((ext_vector_type(4)));

static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Flat tile index so that each XCD (workgroups are dealt round-robin over the
// 8 XCDs) walks a contiguous range of tiles: neighbouring tiles, which share
// halo rows, then hit the same L2.
__device__ inline int64_t xcd_remap(int64_t bid, int64_t ntiles) {
  const int64_t q = ntiles >> 3, r = ntiles & 7;
  const int64_t x = bid & 7, k = bid >> 3;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

__device__ inline int find_box(const WorkBox *__restrict__ wb, int nbox, int64_t t) {
  int lo = 0, hi = nbox - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wb[mid].tile0 <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

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
// coordinates.  Sections are row-major inside each box.
__global__ __launch_bounds__(256) void k_pack(const MsgRec *__restrict__ M, const MsgHdr *__restrict__ H,
                                              const ArrDev *__restrict__ A, uint32_t *__restrict__ stg,
                                              int unpack) {
  const int64_t n = H->nmsg;
  const int64_t words = H->bytes >> 2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int m = 0;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += stride) {
    if (!(M[m].off <= 4 * w && 4 * w < M[m].off + M[m].bytes)) m = find_msg(M, n, 4 * w);
    const MsgRec &r = M[m];
    const int64_t lw = w - (r.off >> 2);
    if (4 * lw >= r.bytes) continue;  // alignment padding between arrays
    const int k = r.esize >> 2;
    const int64_t wid = (int64_t)(r.hi[2] - r.lo[2]) * k;
    const int64_t rows = r.hi[1] - r.lo[1];
    const int64_t c = lw % wid, t = lw / wid;
    const int64_t rr = t % rows, p = t / rows;
    const ArrDev &a = A[r.arr];
    const int64_t g = (((int64_t)r.lo[0] + p) * a.n[1] + r.lo[1] + rr) * a.n[2] * k + (int64_t)r.lo[2] * k + c;
    if (!unpack)
      stg[w] = reinterpret_cast<const uint32_t *>(a.buf[r.src])[g];
    else
      reinterpret_cast<uint32_t *>(a.buf[r.dst])[g] = stg[w];
  }
}

// ---------------------------------------------------------------- jacobi2d
template <int TH, bool TRI>
__global__ __launch_bounds__(64) void k_jacobi(const WorkBox *__restrict__ wb, int nbox,
                                               const ArrDev *__restrict__ A, int aout, int ain, int64_t ntiles) {
  const int lane = threadIdx.x;
  const int64_t t = xcd_remap(blockIdx.x, ntiles);
  const WorkBox B = wb[find_box(wb, nbox, t)];
  const int64_t lt = t - B.tile0;
  const int h = B.hi[1] - B.lo[1];
  const int nty = (h + TH - 1) / TH;
  const int ty = (int)(lt % nty), tx = (int)(lt / nty);
  const int r0 = B.lo[1] + ty * TH;
  const int r1 = min(r0 + TH, B.hi[1]);
  const int c = B.lo[2] + tx * 256 + 4 * lane;
  const ArrDev &ai = A[ain];
  const float *__restrict__ in = reinterpret_cast<const float *>(ai.buf[B.dev]);
  float *__restrict__ out = reinterpret_cast<float *>(A[aout].buf[B.dev]);
  const int N1 = (int)ai.n[1], N2 = (int)ai.n[2];
  const bool vec = ((N2 & 3) == 0) && ((B.lo[2] & 3) == 0);
  f4 v[TH + 2];
  float Lh[TH + 2], Rh[TH + 2];
#pragma unroll
  for (int k = 0; k < TH + 2; ++k) {
    const int r = r0 - 1 + k;
    f4 x = {0.f, 0.f, 0.f, 0.f};
    float l = 0.f, rr = 0.f;
    if (r >= 0 && r < N1 && r <= r1) {
      const float *p = in + (int64_t)r * N2;
      if (vec && c + 4 <= N2) {
        x = *reinterpret_cast<const f4 *>(p + c);
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
    Lh[k] = lane == 0 ? l : lw;
    Rh[k] = lane == 63 ? rr : rx;
    v[k] = x;
  }
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
    float *q = out + (int64_t)i * N2 + c;
    if (vec && wr[0] && wr[1] && wr[2] && wr[3]) {
      f4 ov = {o[0], o[1], o[2], o[3]};
      __builtin_nontemporal_store(ov, reinterpret_cast<f4 *>(q));
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (wr[e]) q[e] = o[e];
    }
  }
}

// -------------------------------------------------------------------- copy
// out = in over each device's box; 2-D tiles of 256 words x 16 rows per plane.
__global__ __launch_bounds__(64) void k_copy(const WorkBox *__restrict__ wb, int nbox, const ArrDev *__restrict__ A,
                                             int aout, int ain, int64_t ntiles) {
  const int lane = threadIdx.x;
  const int64_t t = xcd_remap(blockIdx.x, ntiles);
  const WorkBox B = wb[find_box(wb, nbox, t)];
  const ArrDev &ai = A[ain];
  const int k = ai.esize >> 2;
  const int64_t lt = t - B.tile0;
  const int h = B.hi[1] - B.lo[1];
  const int64_t wwords = (int64_t)(B.hi[2] - B.lo[2]) * k;
  const int nty = (h + 15) / 16;
  const int ntx = (int)((wwords + 255) / 256);
  const int ty = (int)(lt % nty);
  const int64_t rest = lt / nty;
  const int tx = (int)(rest % ntx);
  const int p = B.lo[0] + (int)(rest / ntx);
  const uint32_t *__restrict__ in = reinterpret_cast<const uint32_t *>(ai.buf[B.dev]);
  uint32_t *__restrict__ out = reinterpret_cast<uint32_t *>(A[aout].buf[B.dev]);
  const int64_t rowwords = ai.n[2] * k;
  const int64_t c0 = (int64_t)B.lo[2] * k + (int64_t)tx * 256 + 4 * lane;
  const int64_t cend = (int64_t)B.hi[2] * k;
  const bool vec = (rowwords & 3) == 0 && (c0 & 3) == 0;
  for (int r = B.lo[1] + ty * 16; r < min(B.lo[1] + ty * 16 + 16, B.hi[1]); ++r) {
    const int64_t base = ((int64_t)p * ai.n[1] + r) * rowwords;
    if (vec && c0 + 4 <= cend) {
      *reinterpret_cast<uint4 *>(out + base + c0) = *reinterpret_cast<const uint4 *>(in + base + c0);
    } else {
      for (int e = 0; e < 4; ++e)
        if (c0 + e < cend) out[base + c0 + e] = in[base + c0 + e];
    }
  }
}

// -------------------------------------------------------------- stencil3d7
// One wave per (plane, row) x 256 columns; 4 rows per workgroup.
struct Coef7 {
  float c[7];
};

__global__ __launch_bounds__(256) void k_s3d(const WorkBox *__restrict__ wb, int nbox, const ArrDev *__restrict__ A,
                                             int aout, int ain, int64_t ntiles, Coef7 cf) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t t = xcd_remap(blockIdx.x, ntiles);
  const WorkBox B = wb[find_box(wb, nbox, t)];
  const int64_t lt = t - B.tile0;
  const int h = B.hi[1] - B.lo[1];
  const int w = B.hi[2] - B.lo[2];
  const int nty = (h + 3) / 4, ntx = (w + 255) / 256;
  const int ty = (int)(lt % nty);
  const int64_t rest = lt / nty;
  const int tx = (int)(rest % ntx);
  const int i = B.lo[0] + (int)(rest / ntx);
  const int j = B.lo[1] + ty * 4 + wv;
  if (j >= B.hi[1]) return;
  const ArrDev &ai = A[ain];
  const float *__restrict__ u = reinterpret_cast<const float *>(ai.buf[B.dev]);
  float *__restrict__ out = reinterpret_cast<float *>(A[aout].buf[B.dev]);
  const int N0 = (int)ai.n[0], N1 = (int)ai.n[1], N2 = (int)ai.n[2];
  const int64_t si = (int64_t)N1 * N2, sj = N2;
  const int c = B.lo[2] + tx * 256 + 4 * lane;
  const int64_t x0 = (int64_t)i * si + (int64_t)j * sj;
  const bool rowint = i >= 1 && i <= N0 - 2 && j >= 1 && j <= N1 - 2;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int k = c + e;
    if (k >= B.hi[2]) break;
    const int64_t x = x0 + k;
    float r;
    if (rowint && k >= 1 && k <= N2 - 2) {
      float acc = cf.c[0] * u[x];
      acc = __builtin_fmaf(cf.c[1], u[x - si], acc);
      acc = __builtin_fmaf(cf.c[2], u[x + si], acc);
      acc = __builtin_fmaf(cf.c[3], u[x - sj], acc);
      acc = __builtin_fmaf(cf.c[4], u[x + sj], acc);
      acc = __builtin_fmaf(cf.c[5], u[x - 1], acc);
      acc = __builtin_fmaf(cf.c[6], u[x + 1], acc);
      r = acc;
    } else {
      r = u[x];
    }
    out[x] = r;
  }
}

// ------------------------------------------------------------------ matmul
// First correct version: 64x64 tiles of C, 256 threads with 4x4 each, K in
// steps of 16 staged through LDS.
__global__ __launch_bounds__(256) void k_mm_simple(const WorkBox *__restrict__ wb, int nbox,
                                                   const ArrDev *__restrict__ A, int aa, int ab, int ac,
                                                   int64_t ntiles) {
  __shared__ float sA[16][64 + 4];
  __shared__ float sB[16][64 + 4];
  const int64_t t = xcd_remap(blockIdx.x, ntiles);
  const WorkBox Bx = wb[find_box(wb, nbox, t)];
  const int64_t lt = t - Bx.tile0;
  const int h = Bx.hi[1] - Bx.lo[1], w = Bx.hi[2] - Bx.lo[2];
  const int nty = (h + 63) / 64;
  const int ty = (int)(lt % nty), tx = (int)(lt / nty);
  (void)w;
  const int i0 = Bx.lo[1] + ty * 64, j0 = Bx.lo[2] + tx * 64;
  const ArrDev &ma = A[aa], &mb = A[ab], &mc = A[ac];
  const float *__restrict__ a = reinterpret_cast<const float *>(ma.buf[Bx.dev]);
  const float *__restrict__ b = reinterpret_cast<const float *>(mb.buf[Bx.dev]);
  float *__restrict__ cc = reinterpret_cast<float *>(mc.buf[Bx.dev]);
  const int K = (int)ma.n[2], M = (int)mb.n[2];
  const int tr = threadIdx.x / 16, tcn = threadIdx.x % 16;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int q = threadIdx.x; q < 16 * 64; q += 256) {
      const int kk = q / 64, ii = q % 64;
      const int gi = i0 + ii, gk = k0 + kk;
      sA[kk][ii] = (gi < Bx.hi[1] && gk < K) ? a[(int64_t)gi * K + gk] : 0.f;
      const int gj = j0 + ii;
      sB[kk][ii] = (gj < Bx.hi[2] && gk < K) ? b[(int64_t)gk * M + gj] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float av[4], bv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        av[e] = sA[kk][tr * 4 + e];
        bv[e] = sB[kk][tcn * 4 + e];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = __builtin_fmaf(av[x], bv[y], acc[x][y]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int gi = i0 + tr * 4 + x, gj = j0 + tcn * 4 + y;
      if (gi < Bx.hi[1] && gj < Bx.hi[2]) cc[(int64_t)gi * M + gj] = acc[x][y];
    }
}

// ------------------------------------------------------------------ reduce
// Partial results per (box, block) in a fixed order, combined by one thread
// in (device, block) order, so the result is reproducible run to run.
constexpr int kRedBlocks = 64;

template <int TYPE, int OP>  // TYPE 0 f32, 1 i32, 2 f64
__global__ __launch_bounds__(256) void k_reduce_part(const WorkBox *__restrict__ wb, const ArrDev *__restrict__ A,
                                                     int arr, double *pf, uint32_t *pi) {
  __shared__ double sf[256];
  __shared__ uint32_t si[256];
  const WorkBox B = wb[blockIdx.y];
  const ArrDev &a = A[arr];
  const int64_t h = B.hi[1] - B.lo[1], w = B.hi[2] - B.lo[2], d = B.hi[0] - B.lo[0];
  const int64_t tot = h * w * d;
  double f = OP == 0 ? 0.0 : OP == 1 ? 1.0 : OP == 2 ? -__builtin_inf() : __builtin_inf();
  uint32_t iv = OP == 0 ? 0u : OP == 1 ? 1u : OP == 2 ? 0x80000000u : 0x7fffffffu;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < tot; q += (int64_t)gridDim.x * 256) {
    const int64_t cc = q % w, rr = (q / w) % h, pp = q / (w * h);
    const int64_t x = ((B.lo[0] + pp) * a.n[1] + B.lo[1] + rr) * a.n[2] + B.lo[2] + cc;
    if (TYPE == 1) {
      const int32_t v = reinterpret_cast<const int32_t *>(a.buf[B.dev])[x];
      if (OP == 0) iv += (uint32_t)v;
      if (OP == 1) iv *= (uint32_t)v;
      if (OP == 2 && v > (int32_t)iv) iv = (uint32_t)v;
      if (OP == 3 && v < (int32_t)iv) iv = (uint32_t)v;
    } else {
      const double v = TYPE == 0 ? (double)reinterpret_cast<const float *>(a.buf[B.dev])[x]
                                 : reinterpret_cast<const double *>(a.buf[B.dev])[x];
      if (OP == 0) f += v;
      if (OP == 1) f *= v;
      if (OP == 2 && v > f) f = v;
      if (OP == 3 && v < f) f = v;
    }
  }
  sf[threadIdx.x] = f;
  si[threadIdx.x] = iv;
  __syncthreads();
  if (threadIdx.x == 0) {
    double F = sf[0];
    uint32_t I = si[0];
    for (int k = 1; k < 256; ++k) {
      if (TYPE == 1) {
        const uint32_t v = si[k];
        if (OP == 0) I += v;
        if (OP == 1) I *= v;
        if (OP == 2 && (int32_t)v > (int32_t)I) I = v;
        if (OP == 3 && (int32_t)v < (int32_t)I) I = v;
      } else {
        const double v = sf[k];
        if (OP == 0) F += v;
        if (OP == 1) F *= v;
        if (OP == 2 && v > F) F = v;
        if (OP == 3 && v < F) F = v;
      }
    }
    pf[blockIdx.y * kRedBlocks + blockIdx.x] = F;
    pi[blockIdx.y * kRedBlocks + blockIdx.x] = I;
  }
}

template <int TYPE, int OP>
__global__ void k_reduce_final(int nbox, const double *pf, const uint32_t *pi, void *res) {
  double F = OP == 0 ? 0.0 : OP == 1 ? 1.0 : OP == 2 ? -__builtin_inf() : __builtin_inf();
  uint32_t I = OP == 0 ? 0u : OP == 1 ? 1u : OP == 2 ? 0x80000000u : 0x7fffffffu;
  for (int k = 0; k < nbox * kRedBlocks; ++k) {
    if (TYPE == 1) {
      const uint32_t v = pi[k];
      if (OP == 0) I += v;
      if (OP == 1) I *= v;
      if (OP == 2 && (int32_t)v > (int32_t)I) I = v;
      if (OP == 3 && (int32_t)v < (int32_t)I) I = v;
    } else {
      const double v = pf[k];
      if (OP == 0) F += v;
      if (OP == 1) F *= v;
      if (OP == 2 && v > F) F = v;
      if (OP == 3 && v < F) F = v;
    }
  }
  if (TYPE == 0) *reinterpret_cast<float *>(res) = (float)F;
  if (TYPE == 1) *reinterpret_cast<int32_t *>(res) = (int32_t)I;
  if (TYPE == 2) *reinterpret_cast<double *>(res) = F;
}

// ------------------------------------------------------------- launchers
hipError_t launch_pack(const MsgRec *M, const MsgHdr *H, const ArrDev *A, uint32_t *stg, int64_t bound_words,
                       int unpack, hipStream_t s) {
  int grid = cdiv(bound_words, 256);
  if (grid > 4096) grid = 4096;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_pack, dim3(grid), dim3(256), 0, s, M, H, A, stg, unpack);
  return hipGetLastError();
}

// tile counts per box for each kernel shape
int64_t tiles_for(int kind, const int32_t *lo, const int32_t *hi, int esize, int th) {
  const int64_t d = hi[0] - lo[0], h = hi[1] - lo[1], w = hi[2] - lo[2];
  if (d <= 0 || h <= 0 || w <= 0) return 0;
  switch (kind) {
    case 1:  // jacobi / tri
      return (int64_t)cdiv(h, th) * cdiv(w, 256);
    case 2:  // copy
      return d * cdiv(h, 16) * cdiv(w * (esize / 4), 256);
    case 3:  // stencil3d
      return d * cdiv(h, 4) * cdiv(w, 256);
    case 4:  // matmul
      return (int64_t)cdiv(h, 64) * cdiv(w, 64);
  }
  return 0;
}

hipError_t launch_user(int kind, int th, const WorkBox *wb, int nbox, const ArrDev *A, const int *args,
                       int64_t ntiles, const float *coef, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  switch (kind) {
    case 1:  // jacobi2d (args: out, in)
      if (th == 8)
        hipLaunchKernelGGL((k_jacobi<8, false>), dim3(ntiles), dim3(64), 0, s, wb, nbox, A, args[0], args[1], ntiles);
      else if (th == 32)
        hipLaunchKernelGGL((k_jacobi<32, false>), dim3(ntiles), dim3(64), 0, s, wb, nbox, A, args[0], args[1], ntiles);
      else
        hipLaunchKernelGGL((k_jacobi<16, false>), dim3(ntiles), dim3(64), 0, s, wb, nbox, A, args[0], args[1], ntiles);
      break;
    case 5:  // tri2d
      hipLaunchKernelGGL((k_jacobi<16, true>), dim3(ntiles), dim3(64), 0, s, wb, nbox, A, args[0], args[1], ntiles);
      break;
    case 2:
      hipLaunchKernelGGL(k_copy, dim3(ntiles), dim3(64), 0, s, wb, nbox, A, args[0], args[1], ntiles);
      break;
    case 3: {
      Coef7 c;
      for (int e = 0; e < 7; ++e) c.c[e] = coef[e];
      hipLaunchKernelGGL(k_s3d, dim3(ntiles), dim3(256), 0, s, wb, nbox, A, args[0], args[1], ntiles, c);
    } break;
    case 4:  // matmul (A, B, C)
      hipLaunchKernelGGL(k_mm_simple, dim3(ntiles), dim3(256), 0, s, wb, nbox, A, args[0], args[1], args[2], ntiles);
      break;
  }
  return hipGetLastError();
}

template <int TYPE, int OP>
static void red2(const WorkBox *wb, int nbox, const ArrDev *A, int arr, double *pf, uint32_t *pi, void *res,
                 hipStream_t s) {
  hipLaunchKernelGGL((k_reduce_part<TYPE, OP>), dim3(kRedBlocks, nbox), dim3(256), 0, s, wb, A, arr, pf, pi);
  hipLaunchKernelGGL((k_reduce_final<TYPE, OP>), dim3(1), dim3(1), 0, s, nbox, pf, pi, res);
}
template <int TYPE>
static void red1(int op, const WorkBox *wb, int nbox, const ArrDev *A, int arr, double *pf, uint32_t *pi, void *res,
                 hipStream_t s) {
  switch (op) {
    case 0: red2<TYPE, 0>(wb, nbox, A, arr, pf, pi, res, s); break;
    case 1: red2<TYPE, 1>(wb, nbox, A, arr, pf, pi, res, s); break;
    case 2: red2<TYPE, 2>(wb, nbox, A, arr, pf, pi, res, s); break;
    default: red2<TYPE, 3>(wb, nbox, A, arr, pf, pi, res, s); break;
  }
}
hipError_t launch_reduce(int type, int op, const WorkBox *wb, int nbox, const ArrDev *A, int arr, double *pf,
                         uint32_t *pi, void *res, hipStream_t s) {
  if (type == 0) red1<0>(op, wb, nbox, A, arr, pf, pi, res, s);
  else if (type == 1) red1<1>(op, wb, nbox, A, arr, pf, pi, res, s);
  else red1<2>(op, wb, nbox, A, arr, pf, pi, res, s);
  return hipGetLastError();
}

int reduce_blocks() { return kRedBlocks; }

}  // namespace hd

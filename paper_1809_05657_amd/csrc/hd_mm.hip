// hd_mm.hip — the GEMM user kernel of Sec. 3.2 (C = A x B, alpha = 1,
// beta = 0) on the gfx950 FP32 matrix cores, over every logical device of
// a partition in one launch.  Device d computes its work box of C from its
// own buffers of A (rows of the box, all columns) and B (all rows, columns of
// the box) — exactly LUSE of use(A,(0,*)) use(B,(*,0)).
//
// Tiling: a 256-thread workgroup owns a 128 x 128 tile of C; its four waves
// own 64 x 64 each as 2 x 2 tiles of v_mfma_f32_32x32x2f32 (16 accumulators
// per lane per tile).  K advances in steps of 16 through double-buffered LDS
// (A stored k-major so each MFMA operand fetch is 32 consecutive words).
// MFMA operand layout (32x32x2, wave64): lane l supplies A[l%32][l/32] and
// B[l/32][l%32]; accumulator register r of lane l is C[8(r/4) + 4(l/32) +
// r%4][l%32].
#include <hip/hip_runtime.h>

#include "hd_internal.hpp"

namespace hd {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

__device__ inline int64_t xcd_remap_mm(int64_t bid, int64_t ntiles) {
  const int64_t q = ntiles >> 3, r = ntiles & 7;
  const int64_t x = bid & 7, k = bid >> 3;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// LDS row strides: B rows are written as float4 (stride a multiple of 4
// words); A is written transposed, one word per lane, where 32 lanes hold
// 8 rows x 4 k values: a stride of 2 mod 32 words puts them in 32 different
// banks (a stride of 4 mod 32 gave two-way conflicts).
constexpr int BM = 128, BN = 128, BK = 16, LDP = BM + 4, LDA = BM + 2;

__global__ __launch_bounds__(256) void k_mm_mfma(const WorkBox *__restrict__ wb, int nbox,
                                                 const ArrDev *__restrict__ A, int64_t ntiles) {
  __shared__ float sA[2][BK][LDA];
  __shared__ float sB[2][BK][LDP];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t t = xcd_remap_mm(blockIdx.x, ntiles);
  int lo = 0, hi = nbox - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wb[mid].tile0 <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  const WorkBox Bx = wb[lo];
  const int aa = Bx.ain, ab = Bx.ain2, ac = Bx.aout;
  const int64_t lt = t - Bx.tile0;
  const int h = Bx.hi[1] - Bx.lo[1];
  const int nty = (h + BM - 1) / BM;
  const int ty = (int)(lt % nty), tx = (int)(lt / nty);
  const int i0 = Bx.lo[1] + ty * BM, j0 = Bx.lo[2] + tx * BN;
  const ArrDev &ma = A[aa], &mb = A[ab], &mc = A[ac];
  const float *__restrict__ a = reinterpret_cast<const float *>(ma.buf[Bx.dev]);
  const float *__restrict__ b = reinterpret_cast<const float *>(mb.buf[Bx.dev]);
  float *__restrict__ c = reinterpret_cast<float *>(mc.buf[Bx.dev]);
  const int K = (int)ma.n[2], M = (int)mb.n[2];
  const int ihi = Bx.hi[1], jhi = Bx.hi[2];
  const bool avec = (K & 3) == 0, bvec = (M & 3) == 0 && (j0 & 3) == 0;

  // global -> register staging: each thread moves 2 float4 of A and 2 of B
  f4 ra[2], rb[2];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int v = tid + 256 * q;  // 512 float4 per operand tile
      // A tile: 128 rows x 16 k -> row v/4, k (v%4)*4
      {
        const int ii = i0 + v / 4, kk = k0 + (v % 4) * 4;
        f4 x = {0.f, 0.f, 0.f, 0.f};
        if (ii < ihi) {
          const float *p = a + (int64_t)ii * K + kk;
          if (avec && kk + 4 <= K) {
            x = *reinterpret_cast<const f4 *>(p);
          } else {
            if (kk < K) x.x = p[0];
            if (kk + 1 < K) x.y = p[1];
            if (kk + 2 < K) x.z = p[2];
            if (kk + 3 < K) x.w = p[3];
          }
        }
        ra[q] = x;
      }
      // B tile: 16 k x 128 cols -> k v/32, col (v%32)*4
      {
        const int kk = k0 + v / 32, jj = j0 + (v % 32) * 4;
        f4 x = {0.f, 0.f, 0.f, 0.f};
        if (kk < K) {
          const float *p = b + (int64_t)kk * M + jj;
          if (bvec && jj + 4 <= jhi) {
            x = *reinterpret_cast<const f4 *>(p);
          } else {
            if (jj < jhi) x.x = p[0];
            if (jj + 1 < jhi) x.y = p[1];
            if (jj + 2 < jhi) x.z = p[2];
            if (jj + 3 < jhi) x.w = p[3];
          }
        }
        rb[q] = x;
      }
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int v = tid + 256 * q;
      const int ii = v / 4, kk = (v % 4) * 4;
      sA[buf][kk + 0][ii] = ra[q].x;
      sA[buf][kk + 1][ii] = ra[q].y;
      sA[buf][kk + 2][ii] = ra[q].z;
      sA[buf][kk + 3][ii] = ra[q].w;
      const int k2 = v / 32, jj = (v % 32) * 4;
      *reinterpret_cast<f4 *>(&sB[buf][k2][jj]) = rb[q];
    }
  };

  f16v acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[x][y][r] = 0.f;

  const int wi = (wv >> 1) * 64, wj = (wv & 1) * 64;
  const int lr = lane & 31, lk = lane >> 5;
  gload(0);
  lstore(0);
  __syncthreads();
  int cur = 0;
  for (int k0 = 0; k0 < K; k0 += BK) {
    const bool more = k0 + BK < K;
    if (more) gload(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      const float a0 = sA[cur][kk + lk][wi + lr];
      const float a1 = sA[cur][kk + lk][wi + 32 + lr];
      const float b0 = sB[cur][kk + lk][wj + lr];
      const float b1 = sB[cur][kk + lk][wj + 32 + lr];
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (more) {
      lstore(cur ^ 1);
      __syncthreads();
      cur ^= 1;
    }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ii = i0 + wi + 32 * x + 8 * (r >> 2) + 4 * lk + (r & 3);
        const int jj = j0 + wj + 32 * y + lr;
        if (ii < ihi && jj < jhi) c[(int64_t)ii * M + jj] = acc[x][y][r];
      }
}

int64_t mm_tiles(const int32_t *lo, const int32_t *hi) {
  const int64_t h = hi[1] - lo[1], w = hi[2] - lo[2];
  if (h <= 0 || w <= 0 || hi[0] <= lo[0]) return 0;
  return ((h + BM - 1) / BM) * ((w + BN - 1) / BN);
}

hipError_t launch_mm(const WorkBox *wb, int nbox, const ArrDev *A, int64_t ntiles, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mm_mfma, dim3(ntiles), dim3(256), 0, s, wb, nbox, A, ntiles);
  return hipGetLastError();
}

}  // namespace hd

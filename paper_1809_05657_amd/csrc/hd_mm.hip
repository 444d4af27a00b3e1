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

// Global-memory pointers: loads through them are global (not flat)
// instructions, which count only against the vector-memory counter, so the
// waits for LDS reads in the MFMA loop do not also wait for the next tile's
// global loads.
typedef const float __attribute__((address_space(1))) gfloat;
typedef const f4 __attribute__((address_space(1))) gf4;
typedef float __attribute__((address_space(1))) gfloat_w;

// FULL: every box of the launch is a multiple of the tile in rows and
// columns, K is a multiple of BK and rows of A and B are float4-aligned, so
// no load or store needs a bounds check (the host checks this per plan).
template <bool FULL>
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
  gfloat *__restrict__ a = (gfloat *)ma.buf[Bx.dev];
  gfloat *__restrict__ b = (gfloat *)mb.buf[Bx.dev];
  gfloat_w *__restrict__ c = (gfloat_w *)mc.buf[Bx.dev];
  const int K = (int)ma.n[2], M = (int)mb.n[2];
  const int ihi = Bx.hi[1], jhi = Bx.hi[2];
  const bool avec = (K & 3) == 0, bvec = (M & 3) == 0 && (j0 & 3) == 0;

  // global -> register staging: each thread moves 2 float4 of A and 2 of B
  f4 ra[2], rb[2];
  // FULL: thread tid loads A rows tid/4 and 64 + tid/4 at k (tid%4)*4, and B
  // rows tid/32 and 8 + tid/32 at column (tid%32)*4; the pointers advance by
  // one K step per call
  gfloat *pa = a + (int64_t)(i0 + tid / 4) * K + (tid % 4) * 4;
  gfloat *pb = b + (int64_t)(tid / 32) * M + j0 + (tid % 32) * 4;
  auto gload = [&](int k0) {
    if constexpr (FULL) {
      ra[0] = *(gf4 *)pa;
      ra[1] = *(gf4 *)(pa + (int64_t)64 * K);
      rb[0] = *(gf4 *)pb;
      rb[1] = *(gf4 *)(pb + (int64_t)8 * M);
      pa += BK;
      pb += (int64_t)BK * M;
      return;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int v = tid + 256 * q;  // 512 float4 per operand tile
      // A tile: 128 rows x 16 k -> row v/4, k (v%4)*4
      {
        const int ii = i0 + v / 4, kk = k0 + (v % 4) * 4;
        f4 x = {0.f, 0.f, 0.f, 0.f};
        if (ii < ihi) {
          gfloat *p = a + (int64_t)ii * K + kk;
          if (avec && kk + 4 <= K) {
            x = *(gf4 *)p;
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
          gfloat *p = b + (int64_t)kk * M + jj;
          if (bvec && jj + 4 <= jhi) {
            x = *(gf4 *)p;
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
  // the operands of k pair kk + 2 are read from LDS before the MFMAs of
  // pair kk are issued
  auto mma = [&](int buf) {
    float oa[2][2], ob[2][2];
    auto rd = [&](int kk, int s) {
      oa[s][0] = sA[buf][kk + lk][wi + lr];
      oa[s][1] = sA[buf][kk + lk][wi + 32 + lr];
      ob[s][0] = sB[buf][kk + lk][wj + lr];
      ob[s][1] = sB[buf][kk + lk][wj + 32 + lr];
    };
    rd(0, 0);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      const int s = (kk >> 1) & 1;
      if (kk + 2 < BK) rd(kk + 2, s ^ 1);
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(oa[s][0], ob[s][0], acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(oa[s][0], ob[s][1], acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(oa[s][1], ob[s][0], acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(oa[s][1], ob[s][1], acc[1][1], 0, 0, 0);
    }
    // instruction order: two LDS reads, then (two LDS reads, four MFMAs)
    // per k pair, so each wave has the next pair's reads in flight while
    // its MFMAs issue
    __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
#pragma unroll
    for (int kk = 0; kk < BK - 2; kk += 2) {
      __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
  };
  // one barrier per K step: the tile read from one buffer while the next
  // is stored to the other (every wave has finished reading a buffer before
  // the barrier that precedes its next store)
  gload(0);
  lstore(0);
  __syncthreads();
  int cur = 0;
  for (int k0 = BK; k0 < K; k0 += BK) {
    gload(k0);
    // keep the next tile's global loads ahead of this tile's MFMAs (the
    // scheduler would otherwise sink them to just before their LDS stores)
    __builtin_amdgcn_sched_barrier(0);
    mma(cur);
    lstore(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  mma(cur);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ii = i0 + wi + 32 * x + 8 * (r >> 2) + 4 * lk + (r & 3);
        const int jj = j0 + wj + 32 * y + lr;
        if (FULL || (ii < ihi && jj < jhi)) c[(int64_t)ii * M + jj] = acc[x][y][r];
      }
}

int64_t mm_tiles(const int32_t *lo, const int32_t *hi) {
  const int64_t h = hi[1] - lo[1], w = hi[2] - lo[2];
  if (h <= 0 || w <= 0 || hi[0] <= lo[0]) return 0;
  return ((h + BM - 1) / BM) * ((w + BN - 1) / BN);
}

bool mm_full(const int32_t *lo, const int32_t *hi, int64_t K, int64_t M) {
  return (hi[1] - lo[1]) % BM == 0 && (hi[2] - lo[2]) % BN == 0 && K >= BK && K % BK == 0 && M % 4 == 0 &&
         lo[2] % 4 == 0;
}

hipError_t launch_mm(bool full, const WorkBox *wb, int nbox, const ArrDev *A, int64_t ntiles, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (full)
    hipLaunchKernelGGL(k_mm_mfma<true>, dim3(ntiles), dim3(256), 0, s, wb, nbox, A, ntiles);
  else
    hipLaunchKernelGGL(k_mm_mfma<false>, dim3(ntiles), dim3(256), 0, s, wb, nbox, A, ntiles);
  return hipGetLastError();
}

}  // namespace hd

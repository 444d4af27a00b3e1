// hd_data.hip — per-call data-path kernels of the HDArray runtime on gfx950:
// pack / unpack of the message table (the section copies around the wire,
// Sec. 3.1), the built-in user kernels over every logical device of a
// partition in one launch (device code in hd_dev_data.hpp, matmul in
// hd_mm.hip), and reductions (Table 2 Reduce).
#include <hip/hip_runtime.h>

#include "hd_dev_data.hpp"

namespace hd {

static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
int64_t mm_tiles(const int32_t *lo, const int32_t *hi);
hipError_t launch_mm(bool full, const WorkBox *wb, int nbox, const ArrDev *A, int64_t ntiles, hipStream_t s);
hipError_t launch_jacobi(bool tri, int th, int waves, int order, bool vec, const WorkBox *wb, int nbox, const ArrDev *A,
                         int64_t ntiles, hipStream_t s);
hipError_t launch_conv(int th, int waves, int order, bool vec, const WorkBox *wb, int nbox, const ArrDev *A, int64_t ntiles,
                       const float *coef, hipStream_t s);

// Pack / unpack (mode 0 / 1) or both in one pass (mode 2).  Every message is
// cut into S equal spans (S from the average message size, so that the
// workgroups share the volume); workgroups take (message, span) pairs, so the
// record is read once per span and no word searches the table.
__global__ __launch_bounds__(256) void k_pack(const MsgRec *__restrict__ M, const MsgHdr *__restrict__ H,
                                              const ArrDev *__restrict__ A, uint32_t *__restrict__ stg, int mode) {
  const int64_t nmsg = H->nmsg;
  if (nmsg <= 0) return;
  const int64_t words = H->bytes >> 2;
  const int64_t G = gridDim.x;
  int64_t S = (words + nmsg * 256 - 1) / (nmsg * 256);
  const int64_t smax = G / nmsg > 1 ? G / nmsg : 1;
  if (S > smax) S = smax;
  if (S < 1) S = 1;
  for (int64_t q = blockIdx.x; q < nmsg * S; q += G) {
    const int64_t m = q / S, sub = q % S;
    const MsgRec r = M[m];
    const int64_t nw = r.bytes >> 2;
    const int64_t b0 = nw * sub / S, b1 = nw * (sub + 1) / S;
    if (nw < (int64_t(1) << 31))
      dev_pack_span<int32_t>(r, A, stg, mode, (int32_t)b0, (int32_t)b1);
    else
      dev_pack_span<int64_t>(r, A, stg, mode, b0, b1);
  }
}

__global__ __launch_bounds__(64) void k_copy(const WorkBox *__restrict__ wb, int nbox, const ArrDev *__restrict__ A,
                                             int64_t ntiles) {
  const int64_t t = xcd_remap(blockIdx.x, ntiles);
  const WorkBox B = wb[find_box(wb, nbox, t)];
  dev_copy_tile(B, t - B.tile0, A);
}

// Four waves (four consecutive rows) per workgroup.  The march is bound by
// the loads in flight, so the register budget is held to six waves per SIMD
// (78 VGPRs, no spills; the unconstrained build takes 83 and fits five):
// 307 against 351 us per 512^3 launch.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_s3d(const WorkBox *__restrict__ wb, int nbox, const ArrDev *__restrict__ A,
                                             int64_t ntiles, Coef7 cf) {
  const int64_t nwg = (ntiles + 3) >> 2;
  // the wave's tile index, made explicitly wave-uniform so that the box
  // lookup and the march's geometry live in scalar registers
  const int64_t t = xcd_remap(blockIdx.x, nwg) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (t >= ntiles) return;
  const WorkBox B = wb[find_box(wb, nbox, t)];
  dev_s3d_march(B, t - B.tile0, A, cf);
}

// ------------------------------------------------------- device-pointer I/O
// Copies the rows of every box between an external dense full-extent array
// and the device buffers of array arr (to_ext: buffers -> external).  One
// wave per row; box tile0 counts rows.
__global__ __launch_bounds__(256) void k_ext_copy(const WorkBox *__restrict__ wb, int nbox, int64_t rows,
                                                  const ArrDev *__restrict__ A, int arr, uint32_t *__restrict__ ext,
                                                  int to_ext) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows) return;
  const WorkBox B = wb[find_box(wb, nbox, r)];
  const ArrDev &a = A[arr];
  const int64_t lr = r - B.tile0;
  const int h = B.hi[1] - B.lo[1];
  const int64_t p = B.lo[0] + lr / h, q = B.lo[1] + lr % h;
  const int k = a.esize >> 2;
  const int64_t base = ((p * a.n[1] + q) * a.n[2] + B.lo[2]) * k;  // dense external array
  const int64_t bb = HD_EOFF(a, B.dev, p, q, B.lo[2]) * k;          // the device's window
  const int64_t words = (int64_t)(B.hi[2] - B.lo[2]) * k;
  uint32_t *buf = reinterpret_cast<uint32_t *>(a.buf[B.dev]);
  if (to_ext) {
    for (int64_t w = lane; w < words; w += 64) ext[base + w] = buf[bb + w];
  } else {
    for (int64_t w = lane; w < words; w += 64) buf[bb + w] = ext[base + w];
  }
}

hipError_t launch_ext_copy(const WorkBox *wb, int nbox, int64_t rows, const ArrDev *A, int arr, void *ext, int to_ext,
                           hipStream_t s) {
  if (rows <= 0 || nbox <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ext_copy, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, wb, nbox, rows, A, arr,
                     reinterpret_cast<uint32_t *>(ext), to_ext);
  return hipGetLastError();
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
    const int64_t x = HD_EOFF(a, B.dev, B.lo[0] + pp, B.lo[1] + rr, B.lo[2] + cc);
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
  // up to 4 workgroups per CU; fewer when the table cannot be that large
  // (a workgroup per 256 words: one word per thread and pass)
  int grid = cdiv(bound_words, 256);
  if (grid > 1024) grid = 1024;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_pack, dim3(grid), dim3(256), 0, s, M, H, A, stg, unpack);
  return hipGetLastError();
}

// tiles of one work box for a kernel kind (th: rows per Jacobi tile)
int64_t tiles_for(int kind, const WorkBox &B, int esize, int th) {
  switch (kind) {
    case 1:
    case 5:
    case 6:
      return jacobi_tiles(B, th);
    case 2:
      return copy_tiles(B, esize);
    case 3:
      return s3d_tiles(B);
    case 4:
      return mm_tiles(B.lo, B.hi);
  }
  return 0;
}

// vec: every box's rows can be read as float4 (row length and box start
// multiples of 4), used by the stacked 2-D stencil shape; for the matmul,
// every box is whole tiles (no bounds checks).
hipError_t launch_user(int kind, int th, int waves, int order, bool vec, const WorkBox *wb, int nbox, const ArrDev *A,
                       int64_t ntiles, const float *coef, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  switch (kind) {
    case 1:
    case 5:
      return launch_jacobi(kind == 5, th, waves, order, vec, wb, nbox, A, ntiles, s);
    case 6:
      return launch_conv(th, waves, order, vec, wb, nbox, A, ntiles, coef, s);
    case 2:
      hipLaunchKernelGGL(k_copy, dim3(ntiles), dim3(64), 0, s, wb, nbox, A, ntiles);
      break;
    case 3: {
      Coef7 c;
      for (int e = 0; e < 7; ++e) c.c[e] = coef ? coef[e] : 0.f;
      hipLaunchKernelGGL(k_s3d, dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, s, wb, nbox, A, ntiles, c);
    } break;
    case 4:
      return launch_mm(vec, wb, nbox, A, ntiles, s);
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

// ------------------------------------------------- reduce without allocation
// Scratch of the no-allocation reduce: the device-side result (first 256
// bytes), then the FP64 partials and the 32-bit integer partials of every
// (box, block) pair.  One copy per GPU, held until the process ends; calls on
// one GPU share it, so overlapping calls race.  In host code `scratch` is only
// a host-side stand-in: its device address comes from hipGetSymbolAddress.
constexpr int64_t kScratchBytes = 64 * 1024;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
static void *g_scratch_ptr[kScratchDevices] = {};

// Looks up this GPU's copy of the scratch array; called once per device at
// set-up, with that device current.
hipError_t reduce_scratch_init(int device) {
  if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
  if (g_scratch_ptr[device]) return hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

// Bytes of scratch one reduce over nbox boxes needs, and the maximum.
int64_t reduce_scratch_need(int nbox) { return 256 + (int64_t)nbox * kRedBlocks * (8 + 4); }
int64_t reduce_scratch_max() { return kScratchBytes; }

// The reduce kernels of launch_reduce with the partials and the result in
// this device's scratch; *res_dev receives the result's device address.
hipError_t launch_reduce_scratch(int device, int type, int op, const WorkBox *wb, int nbox, const ArrDev *A, int arr,
                                 void **res_dev, hipStream_t s) {
  if (device < 0 || device >= kScratchDevices || !g_scratch_ptr[device]) return hipErrorNotInitialized;
  if (reduce_scratch_need(nbox) > kScratchBytes) return hipErrorInvalidValue;
  char *base = static_cast<char *>(g_scratch_ptr[device]);
  double *pf = reinterpret_cast<double *>(base + 256);
  uint32_t *pi = reinterpret_cast<uint32_t *>(base + 256 + (int64_t)nbox * kRedBlocks * 8);
  *res_dev = base;
  return launch_reduce(type, op, wb, nbox, A, arr, pf, pi, base, s);
}

}  // namespace hd

// hdarray.cpp — host side of the MI355X HDArray runtime: the C ABI of
// include/hdarray.h, the planner that turns partitions, offsets and absolute
// sections into per-row use / def segments (Sec. 3, Table 1-2), the plan
// cache, and the enqueue of one ApplyKernel on two HIP streams:
//   meta stream: communication-set derivation (Eq. 1-2) and GDEF update
//                (Eq. 3-4) — metadata only, overlapping the previous kernel;
//   data stream: pack + unpack in one pass (the wire is the staging buffer
//                on one GPU),
//                the user kernel over all logical devices in one launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <map>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/hdarray.h"
#include "hd_internal.hpp"

namespace hd {
hipError_t launch_compact(const PlanDev &P, const Level &L, const Work &W, MsgRec *out, MsgHdr *hdr, int64_t cap,
                          int mode, hipStream_t s);
hipError_t launch_gdef(const PlanDev &P, ArrDev *A, const Work &W, hipStream_t s);
hipError_t launch_derive1(const PlanDev &P, ArrDev *A, const Work &W, const Level &L1, const Level &L2,
                          MsgRec *out, MsgHdr *hdr, int64_t cap, int row_cap, bool gdef, hipStream_t s);
extern int g_runs_wave_max;
hipError_t launch_runs(const PlanDev &P, const ArrDev *A, const Work &W, int row_cap, hipStream_t s);
hipError_t launch_level1_tail(const PlanDev &P, const Work &W, const Level &L, MsgRec *out, MsgHdr *hdr, int64_t cap,
                              int mode, hipStream_t s);
hipError_t launch_level1(const PlanDev &P, const ArrDev *A, const Work &W, const Level &L, MsgRec *out,
                         MsgHdr *hdr, int64_t cap, int mode, int row_cap, hipStream_t s);
hipError_t launch_level2(const PlanDev &P, const Work &W, const Level &L, MsgRec *out, MsgHdr *hdr, int64_t cap,
                         hipStream_t s);
hipError_t launch_pack(const MsgRec *M, const MsgHdr *H, const ArrDev *A, uint32_t *stg, int64_t bound_words,
                       int unpack, hipStream_t s);
int64_t tiles_for(int kind, const WorkBox &B, int esize, int th);
bool mm_full(const int32_t *lo, const int32_t *hi, int64_t K, int64_t M);
hipError_t launch_ext_copy(const WorkBox *wb, int nbox, int64_t rows, const ArrDev *A, int arr, void *ext,
                           int to_ext, hipStream_t s);
hipError_t launch_stack_args(int op, int th, const StackArgs &a, int64_t ntiles, const float *coef, hipStream_t s);
hipError_t launch_user(int kind, int th, int waves, int order, bool vec, const WorkBox *wb, int nbox, const ArrDev *A,
                       int64_t ntiles, const float *coef, hipStream_t s);
hipError_t launch_reduce(int type, int op, const WorkBox *wb, int nbox, const ArrDev *A, int arr, double *pf,
                         uint32_t *pi, void *res, hipStream_t s);
hipError_t launch_init_rows(Ivl *ivl, int32_t *cnt, int64_t rows, int cap, hipStream_t s);
int reduce_blocks();
hipError_t reduce_scratch_init(int device);
int64_t reduce_scratch_need(int nbox);
int64_t reduce_scratch_max();
hipError_t launch_reduce_scratch(int device, int type, int op, const WorkBox *wb, int nbox, const ArrDev *A, int arr,
                                 void **res_dev, hipStream_t s);
int batch_max_blocks(int max_per_cu);
hipError_t launch_batch(const BatchArgs &a, int th, int hf, int grid, hipStream_t s);
hipError_t launch_mat(const MatRec *m, int n, ArrDev *A, hipStream_t s);
hipError_t launch_snap(const PlanDev &P, const ArrDev *A, Ivl *snap, int32_t *scnt, int32_t *skip, int32_t *hits,
                       bool compare, hipStream_t s);
int64_t adj_tiles(const WorkBox &B, const int64_t *n);
hipError_t launch_adjoint(const WorkBox *wb, int nbox, int64_t ntiles, const float *coef, double *part,
                          double *cbar, const MsgRec *M, const MsgHdr *H, const ArrDev *A, uint32_t *stg,
                          int64_t bound_words, hipStream_t s);
}  // namespace hd

using namespace hd;

// ---------------------------------------------------------------- state
struct Shape {
  int kind;  // 0 box (normalised, half-open), 1 trapezoid (2-D)
  int64_t lo[3], hi[3];
  int64_t c[8];
};

struct hd_array {
  int id;
  int type;  // 0 f32, 1 i32, 2 f64
  int esize;
  int dim;
  int64_t n[3];
  int64_t N;
  std::string sym;
  char *host;
  char *host_dev;
  // per device: a window of the array (a box covering every element the
  // device ever holds or its kernels read).  mem: the allocation; buf: the
  // window's origin shifted back to element (0, 0, 0), the address kernels
  // index with p * ps + r * rs + c.  A full window (wfull) is the whole array
  // with the dense strides n2 / n1 * n2; other windows start at a column that
  // is a multiple of 4 and have a row stride that is a multiple of 4.
  char *buf[kMaxDev] = {};
  char *mem[kMaxDev] = {};
  int64_t wlo[kMaxDev][3] = {}, whi[kMaxDev][3] = {};
  int64_t rs[kMaxDev] = {}, ps[kMaxDev] = {};
  bool wfull[kMaxDev] = {};
  Ivl *ivl;
  int32_t *cnt;
  int cap;
  // GDEF history since the last call that defined the whole array (no use
  // of it in that call): (plan id, call-array) pairs; empty + hist_ok false
  // when unknown.  Equal histories mean equal GDEF (the update is a
  // deterministic function of the state before and the plan).
  std::vector<uint64_t> hist;
  bool hist_ok = false;
  // GDEF bands: sorted plane / row breakpoints (with 0 and n); all rows of
  // planes [pbrk[i], pbrk[i+1]) x rows [rbrk[k], rbrk[k+1]) have the list
  // stored at the band's first row (the other rows' storage is stale);
  // bver counts their changes
  std::vector<int64_t> pbrk, rbrk;
  uint64_t bver = 0;
};

struct Partition {
  int dim, ndev;
  int64_t lo[kMaxDev][3], hi[kMaxDev][3];
};

struct Kernel {
  std::string name;
  int builtin;  // 1 jacobi2d, 2 copy, 3 stencil3d7, 4 matmul, 5 tri2d, 6 conv2d9
  int noff[8][2];
  int32_t off[8][2][64][3];
  std::map<std::tuple<int, int, int, int>, std::vector<Shape>> abs;  // (part, arr, dev, uod)
  int64_t version;
};

struct CallArray {
  hd_array *a;
  int argpos;
  std::vector<Shape> use[64];
  std::vector<Shape> def[64];
  int def_flags = 0;
  bool no_holders = false;  // receivers do not become holders (adjoint partial sums)
};

// The device data of a plan for one set of GDEF bands of its arrays.
struct PlanInst {
  PlanDev P;
  void *mem = nullptr;
};

struct Plan {
  PlanDev P;          // the instance selected for the current call
  void *mem = nullptr;  // work boxes
  int nsl1 = 0, ngrp = 0, ngrow = 0, has3d = 0;
  int64_t nsl_max = 0;  // slices of the finest instance (one per use row)
  // the call's arrays with their shapes; per call-array the (endpoint,
  // shape) lists and the plan's own plane / row breakpoints
  std::vector<CallArray> cas;
  std::vector<std::vector<std::pair<int, const Shape *>>> uses, defs;
  std::vector<std::vector<int64_t>> pbp, rbp;
  std::map<std::vector<int64_t>, PlanInst *> insts;
  PlanInst *cur = nullptr;
  std::vector<int64_t> cur_key;
  // device lists of band copies per (instance, array bands): {records, count}
  std::map<std::vector<int64_t>, std::pair<void *, int>> mats;
  // the arrays' band versions at the last selection, and its copy list
  std::vector<uint64_t> sel_ver;
  const MatRec *sel_mat = nullptr;
  int sel_nmat = 0;
  PlanInst *last_inst = nullptr;  // instance of the plan cache's last derivation
  int64_t stg_bound = 0;  // bytes
  // user kernel
  int ukind = 0, th = 8;
  WorkBox *wb = nullptr;
  // stencil kinds: the work boxes for 4, 8 and 16 rows per tile, and the
  // key of the tile-shape tuning shared by plans with the same boxes
  WorkBox *wbj[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  std::vector<WorkBox> hwbj[5];  // host copies (for launches that pass the boxes by value)
  bool vec = false;  // every work box's rows can be read as float4 (matmul:
                     // every box is whole tiles, no bounds checks needed)
  int64_t ntj[5] = {0, 0, 0, 0, 0};
  std::vector<int64_t> tkey;
  // device-pointer Write / Read plans: the partition's regions as boxes whose
  // tile0 counts rows (in the third box slot, unused by those plans)
  int xn = -1;
  int64_t xrows = 0;
  // plan cache (Sec. 4.2): per call-array the array id and whether the call
  // defines the whole array without using it; the plan's own message table
  // and runs, and the GDEF histories they were derived under
  uint64_t uid = 0;
  bool apply = false;
  std::vector<int> ca_arr;
  std::vector<char> ca_full;
  int64_t pcap = 0;
  MsgRec *ptab = nullptr;
  MsgHdr *phdr = nullptr;
  Item *pruns = nullptr;
  int32_t *proff = nullptr, *prcnt = nullptr;
  hipEvent_t ev_ready = nullptr, ev_used = nullptr;
  bool used_pending = false, have = false;
  std::vector<uint64_t> last_key;
  // second step: the lists the last small-form derivation read, and its instance
  Ivl *snap = nullptr;
  int32_t *scnt = nullptr;
  const PlanInst *snap_inst = nullptr;
  // adjoint plans: extended-box tiles and coefficient partials
  bool adjoint = false;
  double *part = nullptr;
  int nbox = 0;
  int64_t ntiles = 0;
};

struct CallArray;
struct RecCall;
struct Batch;

// Stencil tile shapes tried on real calls, each timed kTuneReps times in
// interleaved order; the one with the least median time is kept.  The shape
// never changes a result.
constexpr int kTuneN = 4, kTuneReps = 8;
// (rows per wave, waves per workgroup, order): one wave per tile with the
// tiles of an XCD along rows (order 1) or down columns (0), or four waves
// stacked down a tile of 4 x rows (halo rows shared through LDS)
constexpr int kTuneCand[kTuneN][3] = {{4, 4, 1}, {8, 4, 1}, {4, 1, 1}, {4, 1, 0}};
struct TuneState {
  int next = 0;
  bool done = false;
  int best = 0;
  hipEvent_t ev[2 * kTuneN * kTuneReps] = {};
};

struct Runtime {
  bool inited = false;
  int device = 0;
  hipStream_t data = nullptr, meta = nullptr;
  hd_alloc_fn ualloc = nullptr;
  hd_free_fn ufree = nullptr;
  void *uctx = nullptr;
  int row_cap = 64;
  bool serial = false;  // metadata work on the data stream (measurement aid)
  bool fused = true;    // small plan instances: the derivation in one wave
  int jacobi_order = 1;  // with a fixed shape: 1 tiles along rows, 0 down columns
  int jacobi_rows = 0;   // HD_JACOBI_ROWS / HD_JACOBI_WAVES fix the stencil tile shape;
  int jacobi_waves = 0;  // otherwise it is tuned per work-box geometry
  int s3d_seg = 0;       // planes per wave of the 3-D stencil kernels (0: default)
  // buffer windows: whole arrays by default (measured faster for the 2-D
  // stencils); --hd-windows=compact keeps per device only a box around what
  // it holds or reads (column origin and row stride multiples of win_align)
  bool win_full = true;
  int win_align = 4;
  std::map<std::vector<int64_t>, struct TuneState> tunes;
  std::vector<hd_array *> arrays;
  std::vector<Partition> parts;
  std::vector<Kernel> kernels;
  std::unordered_map<std::string, int> kidx;
  ArrDev *d_arrs = nullptr;
  std::vector<ArrDev> h_arrs;
  int arr_cap = 0;
  std::map<std::vector<int64_t>, Plan *> plans;
  // workspace
  Work W{};
  int64_t ws_nsl = 0, ws_ngrp = 0, ws_items = 0;
  uint64_t *bmask = nullptr;
  int32_t *bcnt = nullptr, *bbase = nullptr, *bandslice = nullptr, *hoff = nullptr, *hcnt = nullptr;
  int64_t *hbytes = nullptr, *bofs = nullptr;
  int32_t *bcarr = nullptr, *nofs = nullptr;
  Item *heads = nullptr;
  int32_t *counters = nullptr;  // [0] run_top [1] head_top [2] nb [3] err
  int64_t *cscratch = nullptr;  // compaction scratch of the batched kernel
  MsgRec *tab[2] = {nullptr, nullptr};
  MsgHdr *hdr[2] = {nullptr, nullptr};
  hipEvent_t ev_cs[2] = {nullptr, nullptr}, ev_free[2] = {nullptr, nullptr};
  bool free_pending[2] = {false, false};
  int parity = 0, last_tab = -1;
  MsgRec *last_ptab = nullptr;  // plan-owned table of the last call (plan cache on)
  MsgHdr *last_phdr = nullptr;
  bool plan_cache = false;
  uint64_t next_uid = 1;
  char *staging = nullptr;
  int64_t staging_cap = 0;
  double *red_pf = nullptr;
  uint32_t *red_pi = nullptr;
  void *red_res_dev = nullptr;
  char *red_res_host = nullptr;
  hd_stats_t stats{};
  // batch recording
  bool recording = false;
  std::vector<struct RecCall> rec;
  std::vector<struct Batch *> batches;
  int64_t ws_epoch = 0;
  int last_batch = -1;
  hipEvent_t ev_meta = nullptr, ev_data = nullptr;
  hipStream_t cap = nullptr;
  // GDEF updates run on a second internal stream beside the rest of the
  // derivation (they need only its runs)
  hipStream_t meta2 = nullptr;
  hipEvent_t ev_runs = nullptr, ev_gdef = nullptr;
  bool system_events = false;
  unsigned sync_ev = 0, time_ev = 0, free_ev = 0;
  double *adj_cbar = nullptr;
  // opt-in phase timing
  int prof = 0;  // bit p: time phase p
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_pending;
};

static Runtime R;
static thread_local int g_last_error = 0;

static int fail(int code) {
  g_last_error = code;
  return code;
}

#define HIPCK(x)                                                                              \
  do {                                                                                        \
    hipError_t _e = (x);                                                                      \
    if (_e != hipSuccess) {                                                                   \
      fprintf(stderr, "hdarray: HIP error %s at %s:%d\n", hipGetErrorString(_e), __FILE__, __LINE__); \
      return fail(HD_EHIP);                                                                   \
    }                                                                                         \
  } while (0)

static void *dalloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  R.stats.allocs++;
  if (R.ualloc) return R.ualloc(bytes, R.uctx);
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}
static void dfree(void *p) {
  if (!p) return;
  if (R.ufree)
    R.ufree(p, R.uctx);
  else
    (void)hipFree(p);
}

static void normalise(int dim, const int64_t *v, int64_t fill, int64_t *out) {
  out[0] = out[1] = fill;
  if (dim == 1) out[2] = v[0];
  if (dim == 2) {
    out[1] = v[0];
    out[2] = v[1];
  }
  if (dim == 3) {
    out[0] = v[0];
    out[1] = v[1];
    out[2] = v[2];
  }
}

static int64_t floordiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) q--;
  return q;
}

// ------------------------------------------------------------ array table
static int push_arrdev(hd_array *a) {
  ArrDev &d = R.h_arrs[a->id];
  memset(&d, 0, sizeof(d));
  for (int k = 0; k < 3; ++k) d.n[k] = a->n[k];
  d.esize = a->esize;
  d.cap = a->cap;
  d.ivl = a->ivl;
  d.cnt = a->cnt;
  for (int e = 0; e < kMaxDev; ++e) {
    d.buf[e] = a->buf[e];
    d.rs[e] = a->buf[e] ? a->rs[e] : a->n[2];
    d.ps[e] = a->buf[e] ? a->ps[e] : a->n[1] * a->n[2];
  }
  d.buf[kHost] = a->host_dev;
  d.rs[kHost] = a->n[2];
  d.ps[kHost] = a->n[1] * a->n[2];
  HIPCK(hipMemcpyAsync(R.d_arrs + a->id, &d, sizeof(ArrDev), hipMemcpyHostToDevice, R.meta));
  HIPCK(hipStreamSynchronize(R.meta));
  return HD_OK;
}

// Make device dev's window of a cover [lo, hi) (clipped to the array), or
// the whole array with dense strides when full (3-D arrays always: the 3-D
// stencil, its adjoint and the matmul index with the array's extents).  A
// window only grows: the new one is the union of the old and the request,
// the old contents are copied over and the old allocation freed.  Kernels
// in flight may use the old buffer, so the device is drained first.
static int ensure_window(hd_array *a, int dev, const int64_t *lo, const int64_t *hi, bool full) {
  if (dev < 0 || dev >= kMaxDev) return HD_OK;
  if (a->n[0] > 1 || R.win_full) full = true;
  if (a->wfull[dev]) return HD_OK;
  int64_t nlo[3], nhi[3];
  for (int q = 0; q < 3; ++q) {
    nlo[q] = full ? 0 : std::max<int64_t>(lo[q], 0);
    nhi[q] = full ? a->n[q] : std::min<int64_t>(hi[q], a->n[q]);
    if (nlo[q] >= nhi[q]) return HD_OK;  // nothing to hold
  }
  if (a->mem[dev]) {
    bool inside = !full;
    for (int q = 0; q < 3; ++q) {
      if (nlo[q] < a->wlo[dev][q] || nhi[q] > a->whi[dev][q]) inside = false;
      nlo[q] = std::min(nlo[q], a->wlo[dev][q]);
      nhi[q] = std::max(nhi[q], a->whi[dev][q]);
    }
    if (inside) return HD_OK;
  }
  int64_t rs, ps;
  if (full) {
    rs = a->n[2];
    ps = a->n[1] * a->n[2];
  } else {
    const int64_t g = R.win_align;
    nlo[2] = nlo[2] / g * g;
    rs = (nhi[2] - nlo[2] + g - 1) / g * g;
    ps = rs * (nhi[1] - nlo[1]);
  }
  const size_t es = a->esize;
  const size_t bytes = (size_t)((nhi[0] - nlo[0]) * ps) * es;
  HIPCK(hipDeviceSynchronize());
  char *p = (char *)dalloc(bytes);
  if (!p) return fail(HD_ENOMEM);
  HIPCK(hipMemset(p, 0, bytes));
  char *org = (char *)((uintptr_t)p - (uintptr_t)((nlo[0] * ps + nlo[1] * rs + nlo[2]) * (int64_t)es));
  if (a->mem[dev]) {
    const int64_t *ol = a->wlo[dev], *oh = a->whi[dev];
    const int64_t ors = a->rs[dev], ops = a->ps[dev];
    for (int64_t q = ol[0]; q < oh[0]; ++q)
      HIPCK(hipMemcpy2D(org + (q * ps + ol[1] * rs + ol[2]) * es, rs * es,
                        a->buf[dev] + (q * ops + ol[1] * ors + ol[2]) * es, ors * es, (oh[2] - ol[2]) * es,
                        oh[1] - ol[1], hipMemcpyDeviceToDevice));
    HIPCK(hipDeviceSynchronize());
    dfree(a->mem[dev]);
  }
  a->mem[dev] = p;
  a->buf[dev] = org;
  for (int q = 0; q < 3; ++q) {
    a->wlo[dev][q] = nlo[q];
    a->whi[dev][q] = nhi[q];
  }
  a->rs[dev] = rs;
  a->ps[dev] = ps;
  a->wfull[dev] = full;
  return push_arrdev(a);
}

static int ensure_full(hd_array *a, int dev) {
  const int64_t z[3] = {0, 0, 0};
  return ensure_window(a, dev, z, a->n, true);
}

// ------------------------------------------------------------- init/exit
extern "C" int hdarray_init(int argc, char **argv, const char *kpath, const char *dpath) {
  (void)kpath;
  (void)dpath;
  if (R.inited) return R.device;
  for (int i = 0; i < argc && argv; ++i) {
    if (argv[i] && !strncmp(argv[i], "--hd-row-cap=", 13)) {
      int c = atoi(argv[i] + 13);
      if (c >= 4 && c <= kMaxCap) R.row_cap = c;
    }
    if (argv[i] && !strcmp(argv[i], "--hd-windows=compact")) R.win_full = false;
    if (argv[i] && !strcmp(argv[i], "--hd-windows=full")) R.win_full = true;
  }
  if (const char *e = getenv("HD_SERIAL")) R.serial = atoi(e) != 0;
  if (const char *e = getenv("HD_FUSED_META")) R.fused = atoi(e) != 0;
  if (const char *e = getenv("HD_JACOBI_ROWS")) {
    const int v = atoi(e);
    if (v == 4 || v == 8 || v == 16 || v == 32 || v == 64) R.jacobi_rows = v;
  }
  if (const char *e = getenv("HD_S3D_SEG")) {
    const int v = atoi(e);
    if (v >= 1 && v <= 4096) R.s3d_seg = v;
  }
  if (const char *e = getenv("HD_JACOBI_WAVES")) {
    const int v = atoi(e);
    if (v == 1 || v == 4) R.jacobi_waves = v;
  }
  if (const char *e = getenv("HD_JACOBI_ORDER")) R.jacobi_order = atoi(e) != 0;
  g_runs_wave_max = 0;
  if (const char *e = getenv("HD_RUNS_WAVE_MAX")) g_runs_wave_max = atoi(e);
  int dev = 0;
  HIPCK(hipGetDevice(&dev));
  R.device = dev;
  HIPCK(hipStreamCreateWithFlags(&R.meta, hipStreamNonBlocking));
  HIPCK(hipStreamCreateWithFlags(&R.cap, hipStreamNonBlocking));
  HIPCK(hipStreamCreateWithFlags(&R.meta2, hipStreamNonBlocking));
  // events order work between the runtime's streams on this one device, so
  // a device-scope release is enough (the default system-scope one also
  // writes caches back for the host); timing events need no fence at all
  if (const char *e = getenv("HD_EVENT_SCOPE")) R.system_events = !strcmp(e, "system");
  R.sync_ev = hipEventDisableTiming | (R.system_events ? 0u : (unsigned)hipEventReleaseToDevice);
  R.free_ev = hipEventDisableTiming | (R.system_events ? 0u : (unsigned)hipEventDisableSystemFence);
  R.time_ev = R.system_events ? 0u : (unsigned)hipEventDisableSystemFence;
  HIPCK(hipEventCreateWithFlags(&R.ev_runs, R.sync_ev));
  HIPCK(hipEventCreateWithFlags(&R.ev_gdef, R.sync_ev));
  HIPCK(hipEventCreateWithFlags(&R.ev_meta, R.sync_ev));
  HIPCK(hipEventCreateWithFlags(&R.ev_data, R.sync_ev));
  for (int k = 0; k < 2; ++k) {
    HIPCK(hipEventCreateWithFlags(&R.ev_cs[k], R.sync_ev));
    HIPCK(hipEventCreateWithFlags(&R.ev_free[k], R.sync_ev));
  }
  R.arr_cap = 4096;
  R.h_arrs.assign(R.arr_cap, ArrDev{});
  R.d_arrs = (ArrDev *)dalloc(sizeof(ArrDev) * R.arr_cap);
  R.counters = (int32_t *)dalloc(64);
  R.cscratch = (int64_t *)dalloc(sizeof(int64_t) * 6 * kCompactCarr);
  if (!R.cscratch) return fail(HD_ENOMEM);
  if (!R.d_arrs || !R.counters) return fail(HD_ENOMEM);
  HIPCK(hipMemset(R.counters, 0, 64));
  R.W.run_top = R.counters + 0;
  R.W.err = R.counters + 3;
  // [8]: the plan cache's second-step decision for the current call, [9]: its hits
  R.W.skip = nullptr;
  // [4], [5]: rows listed past the one-lane GDEF update; [6], [7]: rows for
  // the LDS update; each pair alternates between calls
  R.W.ovf_cnt = R.counters + 4;
  R.stats.allocs++;
  HIPCK(hipHostMalloc((void **)&R.red_res_host, 64, hipHostMallocDefault));
  // this GPU's copy of the no-allocation reduce's static scratch
  HIPCK(reduce_scratch_init(dev));
  R.red_res_dev = dalloc(64);
  R.red_pf = (double *)dalloc(sizeof(double) * kMaxDev * 64 * 4);
  R.red_pi = (uint32_t *)dalloc(sizeof(uint32_t) * kMaxDev * 64 * 4);
  R.inited = true;
  return dev;
}

static void free_ws();
static void free_batches();
static void free_plan_buffers(Plan *pl);
static void plan_free(Plan *pl);

extern "C" void hdarray_exit(void) {
  if (!R.inited) return;
  (void)hipStreamSynchronize(R.meta);
  (void)hipStreamSynchronize(R.meta2);
  (void)hipStreamSynchronize(R.data);
  for (auto &kv : R.plans) plan_free(kv.second);
  R.plans.clear();
  free_batches();
  for (hd_array *a : R.arrays) {
    if (!a) continue;
    for (int e = 0; e < kMaxDev; ++e) dfree(a->mem[e]);
    dfree(a->ivl);
    dfree(a->cnt);
    (void)hipHostFree(a->host);
    delete a;
  }
  R.arrays.clear();
  free_ws();
  dfree(R.d_arrs);
  dfree(R.counters);
  dfree(R.cscratch);
  dfree(R.red_res_dev);
  dfree(R.red_pf);
  dfree(R.red_pi);
  (void)hipHostFree(R.red_res_host);
  for (int k = 0; k < 2; ++k) {
    (void)hipEventDestroy(R.ev_cs[k]);
    (void)hipEventDestroy(R.ev_free[k]);
  }
  for (auto &p : R.prof_pending) {
    (void)hipEventDestroy(p.second.first);
    (void)hipEventDestroy(p.second.second);
  }
  for (hipEvent_t e : R.ev_pool) (void)hipEventDestroy(e);
  for (auto &kv : R.tunes)
    for (hipEvent_t e : kv.second.ev)
      if (e) (void)hipEventDestroy(e);
  R.tunes.clear();
  (void)hipEventDestroy(R.ev_meta);
  (void)hipEventDestroy(R.ev_data);
  (void)hipEventDestroy(R.ev_runs);
  (void)hipEventDestroy(R.ev_gdef);
  (void)hipStreamDestroy(R.cap);
  (void)hipStreamDestroy(R.meta2);
  (void)hipStreamDestroy(R.meta);
  hd_alloc_fn ua = R.ualloc;
  hd_free_fn uf = R.ufree;
  void *uc = R.uctx;
  hipStream_t ds = R.data;
  R = Runtime();
  R.ualloc = ua;
  R.ufree = uf;
  R.uctx = uc;
  R.data = ds;
}

extern "C" void hdarray_show_device_info(int dev_id) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev_id) != hipSuccess) {
    g_last_error = HD_EHIP;
    return;
  }
  printf("HDArray device %d: %s (%s), %d CUs, %.1f GiB HBM, wavefront %d, LDS/CU %zu KiB\n", dev_id, p.name,
         p.gcnArchName, p.multiProcessorCount, p.totalGlobalMem / 1073741824.0, p.warpSize,
         (size_t)p.maxSharedMemoryPerMultiProcessor / 1024);
}

extern "C" int hdarray_set_stream(void *s) {
  R.data = (hipStream_t)s;
  return HD_OK;
}

extern "C" int hdarray_set_allocator(hd_alloc_fn a, hd_free_fn f, void *ctx) {
  if ((a == nullptr) != (f == nullptr)) return fail(HD_EINVAL);
  R.ualloc = a;
  R.ufree = f;
  R.uctx = ctx;
  return HD_OK;
}

extern "C" int hdarray_last_error(void) { return g_last_error; }

extern "C" const char *hdarray_error_string(int code) {
  switch (code) {
    case HD_OK: return "ok";
    case HD_EINVAL: return "invalid argument";
    case HD_EBOUNDS: return "section outside the array";
    case HD_ERACE: return "def sections of different devices overlap";
    case HD_EKERNEL: return "unknown kernel";
    case HD_ENOMEM: return "out of memory";
    case HD_EHIP: return "HIP runtime error";
    case HD_ESTATE: return "runtime not initialised";
    case HD_ECAPACITY: return "GDEF row list or work pool capacity exceeded";
    case HD_ENOPLAN: return "no-allocation call needs the plan an earlier call on the same array and partition built";
  }
  return "unknown error";
}

// ---------------------------------------------------------------- create
extern "C" hd_array_t *hdarray_create(const char *sym, const char *type, const void *uA, int dim,
                                      const int64_t *sizes) {
  if (!R.inited) {
    fail(HD_ESTATE);
    return nullptr;
  }
  if (dim < 1 || dim > 3 || !type || !sizes) {
    fail(HD_EINVAL);
    return nullptr;
  }
  int t;
  if (!strcmp(type, "float"))
    t = 0;
  else if (!strcmp(type, "int"))
    t = 1;
  else if (!strcmp(type, "double"))
    t = 2;
  else {
    fail(HD_EINVAL);
    return nullptr;
  }
  if ((int)R.arrays.size() >= R.arr_cap) {
    fail(HD_ENOMEM);
    return nullptr;
  }
  hd_array *a = new hd_array();
  a->id = (int)R.arrays.size();
  a->type = t;
  a->esize = t == 2 ? 8 : 4;
  a->dim = dim;
  a->sym = sym ? sym : "";
  normalise(dim, sizes, 1, a->n);
  for (int k = 0; k < 3; ++k)
    if (a->n[k] < 1 || a->n[k] > (1ll << 31) - 1) {
      delete a;
      fail(HD_EINVAL);
      return nullptr;
    }
  a->N = a->n[0] * a->n[1] * a->n[2];
  // every row starts with the same list (the host owns and holds it all)
  a->pbrk = {0, a->n[0]};
  a->rbrk = {0, a->n[1]};
  size_t bytes = (size_t)a->N * a->esize;
  R.stats.allocs++;
  if (hipHostMalloc((void **)&a->host, bytes, hipHostMallocDefault) != hipSuccess) {
    delete a;
    fail(HD_ENOMEM);
    return nullptr;
  }
  if (uA)
    memcpy(a->host, uA, bytes);
  else
    memset(a->host, 0, bytes);
  void *hd = nullptr;
  if (hipHostGetDevicePointer(&hd, a->host, 0) != hipSuccess) hd = a->host;
  a->host_dev = (char *)hd;
  a->cap = (int)std::min<int64_t>(R.row_cap, a->n[2]);
  if (a->cap < 4) a->cap = std::min<int64_t>(4, a->n[2]) > 0 ? 4 : 1;
  const int64_t rows = a->n[0] * a->n[1];
  a->ivl = (Ivl *)dalloc(sizeof(Ivl) * rows * a->cap);
  a->cnt = (int32_t *)dalloc(sizeof(int32_t) * rows);
  if (!a->ivl || !a->cnt) {
    fail(HD_ENOMEM);
    return nullptr;
  }
  // every row: one interval [0, n2) owned and held by the host (Sec. 2.1:
  // before any device writes, the host holds the only copy)
  if (launch_init_rows(a->ivl, a->cnt, rows, a->cap, R.meta) != hipSuccess) {
    fail(HD_EHIP);
    return nullptr;
  }
  R.arrays.push_back(a);
  if (push_arrdev(a) != HD_OK) return nullptr;
  return a;
}

extern "C" int hdarray_array_id(const hd_array_t *a) { return a ? a->id : -1; }

static hd_array *get_arr(hd_array_t *a) {
  if (!a || a->id < 0 || a->id >= (int)R.arrays.size() || R.arrays[a->id] != a) return nullptr;
  return a;
}

// ------------------------------------------------------------ partitions
static void block_factors(int P, int dim, int *f) {
  int best[3] = {P, 1, 1}, bs = P + 1, bm = P + 1;
  if (dim == 1) {
    f[0] = P;
    return;
  }
  for (int a = 1; a <= P; ++a) {
    if (P % a) continue;
    if (dim == 2) {
      int b = P / a;
      if (a < b) continue;
      int sp = a - b;
      if (sp < bs || (sp == bs && a < bm)) {
        bs = sp;
        bm = a;
        best[0] = a;
        best[1] = b;
      }
    } else {
      for (int b = 1; b <= P / a; ++b) {
        if ((P / a) % b) continue;
        int c = P / a / b;
        if (!(a >= b && b >= c)) continue;
        int sp = a - c;
        if (sp < bs || (sp == bs && a < bm)) {
          bs = sp;
          bm = a;
          best[0] = a;
          best[1] = b;
          best[2] = c;
        }
      }
    }
  }
  for (int k = 0; k < dim; ++k) f[k] = best[k];
}

extern "C" int hdarray_partition(hd_part_t type, int dim, const int64_t *sizes, const int64_t *rlo,
                                 const int64_t *rhi, int ndev) {
  if (!R.inited) return fail(HD_ESTATE);
  if (dim < 1 || dim > 3 || ndev < 1 || ndev > kMaxDev || !sizes || !rlo || !rhi) return fail(HD_EINVAL);
  if (type < HD_ROW || type > HD_BLOCK) return fail(HD_EINVAL);
  for (int k = 0; k < dim; ++k)
    if (rlo[k] < 0 || rhi[k] > sizes[k] || rlo[k] > rhi[k]) return fail(HD_EBOUNDS);
  int f[3] = {1, 1, 1};
  if (type == HD_ROW)
    f[0] = ndev;
  else if (type == HD_COL)
    f[dim == 1 ? 0 : 1] = ndev;
  else
    block_factors(ndev, dim, f);
  Partition p{};
  p.dim = dim;
  p.ndev = ndev;
  for (int d = 0; d < ndev; ++d) {
    int g[3] = {0, 0, 0}, rem = d;
    for (int k = dim - 1; k >= 0; --k) {
      g[k] = rem % f[k];
      rem /= f[k];
    }
    int64_t lo[3], hi[3];
    for (int k = 0; k < dim; ++k) {
      const int64_t L = rlo[k], N = rhi[k] - rlo[k];
      lo[k] = L + (int64_t)g[k] * N / f[k];
      hi[k] = L + ((int64_t)g[k] + 1) * N / f[k];
    }
    normalise(dim, lo, 0, p.lo[d]);
    normalise(dim, hi, 1, p.hi[d]);
  }
  R.parts.push_back(p);
  return (int)R.parts.size() - 1;
}

extern "C" int hdarray_partition_manual(int dim, int ndev, const int64_t *lo, const int64_t *hi) {
  if (!R.inited) return fail(HD_ESTATE);
  if (dim < 1 || dim > 3 || ndev < 1 || ndev > kMaxDev || !lo || !hi) return fail(HD_EINVAL);
  Partition p{};
  p.dim = dim;
  p.ndev = ndev;
  for (int d = 0; d < ndev; ++d) {
    for (int k = 0; k < dim; ++k)
      if (lo[d * dim + k] < 0 || lo[d * dim + k] > hi[d * dim + k]) return fail(HD_EBOUNDS);
    normalise(dim, lo + d * dim, 0, p.lo[d]);
    normalise(dim, hi + d * dim, 1, p.hi[d]);
  }
  R.parts.push_back(p);
  return (int)R.parts.size() - 1;
}

extern "C" int hdarray_partition_region(int part, int dev, int64_t *lo3, int64_t *hi3) {
  if (part < 0 || part >= (int)R.parts.size()) return fail(HD_EINVAL);
  const Partition &p = R.parts[part];
  if (dev < 0 || dev >= p.ndev) return fail(HD_EINVAL);
  memcpy(lo3, p.lo[dev], sizeof(int64_t) * 3);
  memcpy(hi3, p.hi[dev], sizeof(int64_t) * 3);
  return HD_OK;
}

static bool part_dev_empty(const Partition &p, int d) {
  for (int k = 0; k < 3; ++k)
    if (p.lo[d][k] >= p.hi[d][k]) return true;
  return false;
}

// --------------------------------------------------------------- kernels
extern "C" int hdarray_register_kernel(const char *kname, const char *builtin) {
  if (!R.inited) return fail(HD_ESTATE);
  if (!kname || !builtin) return fail(HD_EINVAL);
  int b = 0;
  if (!strcmp(builtin, "jacobi2d"))
    b = 1;
  else if (!strcmp(builtin, "copy"))
    b = 2;
  else if (!strcmp(builtin, "stencil3d7"))
    b = 3;
  else if (!strcmp(builtin, "matmul"))
    b = 4;
  else if (!strcmp(builtin, "tri2d"))
    b = 5;
  else if (!strcmp(builtin, "conv2d9"))
    b = 6;
  else
    return fail(HD_EKERNEL);
  if (R.kidx.count(kname)) return fail(HD_EINVAL);
  Kernel k;
  k.name = kname;
  k.builtin = b;
  memset(k.noff, 0, sizeof(k.noff));
  memset(k.off, 0, sizeof(k.off));
  k.version = 0;
  R.kernels.push_back(std::move(k));
  R.kidx[kname] = (int)R.kernels.size() - 1;
  return (int)R.kernels.size() - 1;
}

static Kernel *get_kernel(const char *kname) {
  if (!kname) return nullptr;
  auto it = R.kidx.find(kname);
  return it == R.kidx.end() ? nullptr : &R.kernels[it->second];
}

extern "C" int hdarray_set_offsets(const char *kname, int arg, int use_or_def, int noff, const int32_t *off) {
  Kernel *k = get_kernel(kname);
  if (!k) return fail(HD_EKERNEL);
  if (arg < 0 || arg >= 8 || use_or_def < 0 || use_or_def > 1 || noff < 0 || noff > 64 || (noff && !off))
    return fail(HD_EINVAL);
  k->noff[arg][use_or_def] = noff;
  for (int i = 0; i < noff; ++i)
    for (int j = 0; j < 3; ++j) k->off[arg][use_or_def][i][j] = off[i * 3 + j];
  k->version++;
  return HD_OK;
}

static int set_abs(const char *kname, int part, hd_array_t *ah, int dev, int dim, const int64_t *lo,
                   const int64_t *hi, int uod) {
  Kernel *k = get_kernel(kname);
  hd_array *a = get_arr(ah);
  if (!k) return fail(HD_EKERNEL);
  if (!a || part < 0 || part >= (int)R.parts.size() || dev < 0 || dev >= kMaxDev || dim != a->dim || !lo || !hi)
    return fail(HD_EINVAL);
  Shape s{};
  normalise(dim, lo, 0, s.lo);
  normalise(dim, hi, 1, s.hi);
  for (int j = 0; j < 3; ++j)
    if (s.lo[j] < 0 || s.hi[j] > a->n[j] || s.lo[j] > s.hi[j]) return fail(HD_EBOUNDS);
  k->abs[std::make_tuple(part, a->id, dev, uod)].push_back(s);
  k->version++;
  return HD_OK;
}

extern "C" int hdarray_set_absolute_use(const char *kname, int part, hd_array_t *a, int dev, int dim,
                                        const int64_t *lo, const int64_t *hi) {
  return set_abs(kname, part, a, dev, dim, lo, hi, 0);
}
extern "C" int hdarray_set_absolute_def(const char *kname, int part, hd_array_t *a, int dev, int dim,
                                        const int64_t *lo, const int64_t *hi) {
  return set_abs(kname, part, a, dev, dim, lo, hi, 1);
}

static int set_trap(const char *kname, int part, hd_array_t *ah, int dev, const int64_t *c, int uod) {
  Kernel *k = get_kernel(kname);
  hd_array *a = get_arr(ah);
  if (!k) return fail(HD_EKERNEL);
  if (!a || a->dim != 2 || part < 0 || part >= (int)R.parts.size() || dev < 0 || dev >= kMaxDev || !c)
    return fail(HD_EINVAL);
  if (c[0] != c[2] || c[4] != c[6] || c[0] > c[4]) return fail(HD_EINVAL);
  Shape s{};
  s.kind = 1;
  memcpy(s.c, c, sizeof(s.c));
  k->abs[std::make_tuple(part, a->id, dev, uod)].push_back(s);
  k->version++;
  return HD_OK;
}
extern "C" int hdarray_set_trapezoid_use(const char *kname, int part, hd_array_t *a, int dev,
                                         const int64_t *corners) {
  return set_trap(kname, part, a, dev, corners, 0);
}
extern "C" int hdarray_set_trapezoid_def(const char *kname, int part, hd_array_t *a, int dev,
                                         const int64_t *corners) {
  return set_trap(kname, part, a, dev, corners, 1);
}

extern "C" int hdarray_clear_sections(const char *kname, int part, hd_array_t *ah, int dev) {
  Kernel *k = get_kernel(kname);
  hd_array *a = get_arr(ah);
  if (!k) return fail(HD_EKERNEL);
  if (!a) return fail(HD_EINVAL);
  for (auto &kv : k->abs) {
    if (std::get<0>(kv.first) == part && std::get<1>(kv.first) == a->id && (dev < 0 || std::get<2>(kv.first) == dev))
      kv.second.clear();
  }
  k->version++;
  return HD_OK;
}

// ---------------------------------------------------------------- planner
// Row spans of a shape: calls fn(plane, row, c0, c1) with [c0, c1) clipped.
template <typename F>
static void shape_rows(const Shape &s, const int64_t *n, F fn) {
  if (s.kind == 0) {
    int64_t lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::max<int64_t>(s.lo[k], 0);
      hi[k] = std::min<int64_t>(s.hi[k], n[k]);
      if (lo[k] >= hi[k]) return;
    }
    for (int64_t p = lo[0]; p < hi[0]; ++p)
      for (int64_t r = lo[1]; r < hi[1]; ++r) fn(p, r, lo[2], hi[2]);
  } else {
    const int64_t r0 = s.c[0], r1 = s.c[4];
    for (int64_t r = std::max<int64_t>(r0, 0); r <= std::min<int64_t>(r1, n[1] - 1); ++r) {
      int64_t l, rt;
      if (r1 == r0) {
        l = s.c[1];
        rt = s.c[3];
      } else {
        l = s.c[1] + floordiv((r - r0) * (s.c[5] - s.c[1]), r1 - r0);
        rt = s.c[3] + floordiv((r - r0) * (s.c[7] - s.c[3]), r1 - r0);
      }
      l = std::max<int64_t>(l, 0);
      rt = std::min<int64_t>(rt, n[2] - 1);
      if (l <= rt) fn(0, r, l, rt + 1);
    }
  }
}

struct Span {
  int64_t row;
  int32_t e, c0, c1, flags;
};

// Per row, per endpoint: union of the spans (overlapping or touching merged).
static void merge_spans(std::vector<Span> &v) {
  std::sort(v.begin(), v.end(), [](const Span &a, const Span &b) {
    return std::tie(a.row, a.e, a.c0) < std::tie(b.row, b.e, b.c0);
  });
  size_t o = 0;
  for (size_t i = 0; i < v.size(); ++i) {
    if (o && v[o - 1].row == v[i].row && v[o - 1].e == v[i].e && v[i].c0 <= v[o - 1].c1) {
      v[o - 1].c1 = std::max(v[o - 1].c1, v[i].c1);
    } else {
      v[o++] = v[i];
    }
  }
  v.resize(o);
}

struct RecCall {
  std::vector<CallArray> cas;
  std::vector<WorkBox> boxes;
};


template <typename T>
static size_t push_blob(std::vector<char> &blob, const std::vector<T> &v) {
  size_t off = (blob.size() + 255) / 256 * 256;
  blob.resize(off + v.size() * sizeof(T) + 16);
  if (!v.empty()) memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
  return off;
}

static void free_ws() {
  dfree(R.W.roff);
  dfree(R.W.rcnt);
  dfree(R.W.runs);
  dfree(R.W.goff);
  dfree(R.W.gcnt);
  dfree(R.W.l1out);
  dfree(R.bmask);
  dfree(R.bcnt);
  dfree(R.bbase);
  dfree(R.bandslice);
  dfree(R.hoff);
  dfree(R.hcnt);
  dfree(R.hbytes);
  dfree(R.bofs);
  dfree(R.bcarr);
  dfree(R.nofs);
  R.hbytes = R.bofs = nullptr;
  R.bcarr = R.nofs = nullptr;
  dfree(R.heads);
  dfree(R.W.ovf_list);
  dfree(R.W.ovf_list2);
  R.W.ovf_list = R.W.ovf_list2 = nullptr;
  for (int k = 0; k < 2; ++k) {
    dfree(R.tab[k]);
    dfree(R.hdr[k]);
    R.tab[k] = nullptr;
    R.hdr[k] = nullptr;
  }
  dfree(R.staging);
  R.staging = nullptr;
  R.staging_cap = 0;
  R.W.roff = R.W.rcnt = R.W.goff = R.W.gcnt = nullptr;
  R.W.runs = R.W.l1out = nullptr;
  R.bmask = nullptr;
  R.bcnt = R.bbase = R.bandslice = R.hoff = R.hcnt = nullptr;
  R.heads = nullptr;
  R.ws_nsl = R.ws_ngrp = R.ws_items = 0;
}

static int ensure_ws(int64_t nsl, int64_t ngrp, int64_t items, int64_t stg, int64_t ngrow) {
  nsl = std::max<int64_t>(nsl, std::max<int64_t>(ngrp, ngrow));
  if (nsl <= R.ws_nsl && ngrp <= R.ws_ngrp && items <= R.ws_items && stg <= R.staging_cap) return HD_OK;
  HIPCK(hipStreamSynchronize(R.meta));
  HIPCK(hipStreamSynchronize(R.data));
  if (nsl > R.ws_nsl || ngrp > R.ws_ngrp || items > R.ws_items) {
    const int64_t ns = std::max(nsl, R.ws_nsl) + 64, ng = std::max(ngrp, R.ws_ngrp) + 64;
    const int64_t it = std::max(items, R.ws_items);
    // keep the staging buffer; release the rest
    char *stgsave = R.staging;
    int64_t stgcap = R.staging_cap;
    R.staging = nullptr;
    free_ws();
    R.staging = stgsave;
    R.staging_cap = stgcap;
    const int64_t nch = ns / 64 + 2;
    R.W.roff = (int32_t *)dalloc(4 * ns);
    R.W.rcnt = (int32_t *)dalloc(4 * ns);
    R.W.runs = (Item *)dalloc(sizeof(Item) * it);
    R.W.run_cap = it;
    R.W.goff = (int32_t *)dalloc(4 * ng);
    R.W.gcnt = (int32_t *)dalloc(4 * ng);
    R.W.l1out = (Item *)dalloc(sizeof(Item) * it);
    R.W.l1_cap = it;
    R.bmask = (uint64_t *)dalloc(8 * nch);
    R.bcnt = (int32_t *)dalloc(4 * nch);
    R.bbase = (int32_t *)dalloc(4 * nch);
    R.bandslice = (int32_t *)dalloc(4 * (ns + 1));
    R.hoff = (int32_t *)dalloc(4 * ns);
    R.hcnt = (int32_t *)dalloc(4 * ns);
    R.hbytes = (int64_t *)dalloc(8 * ns);
    R.bofs = (int64_t *)dalloc(8 * ns);
    R.bcarr = (int32_t *)dalloc(4 * ns);
    R.nofs = (int32_t *)dalloc(4 * ns);
    R.heads = (Item *)dalloc(sizeof(Item) * it);
    R.W.ovf_list = (int32_t *)dalloc(4 * ns);
    R.W.ovf_list2 = (int32_t *)dalloc(4 * ns);
    for (int k = 0; k < 2; ++k) {
      R.tab[k] = (MsgRec *)dalloc(sizeof(MsgRec) * it);
      R.hdr[k] = (MsgHdr *)dalloc(sizeof(MsgHdr));
      if (R.hdr[k]) HIPCK(hipMemset(R.hdr[k], 0, sizeof(MsgHdr)));
    }
    if (!R.W.roff || !R.W.rcnt || !R.W.runs || !R.W.goff || !R.W.gcnt || !R.W.l1out || !R.bmask || !R.bcnt ||
        !R.bbase || !R.bandslice || !R.hoff || !R.hcnt || !R.hbytes || !R.bofs || !R.bcarr || !R.nofs || !R.heads || !R.W.ovf_list || !R.W.ovf_list2 || !R.tab[0] || !R.tab[1] || !R.hdr[0] ||
        !R.hdr[1])
      return fail(HD_ENOMEM);
    HIPCK(hipMemset(R.W.roff, 0, 4 * ns));
    HIPCK(hipMemset(R.W.rcnt, 0, 4 * ns));
    R.ws_nsl = ns;
    R.ws_ngrp = ng;
    R.ws_items = it;
    R.ws_epoch++;
    R.last_tab = -1;
    R.free_pending[0] = R.free_pending[1] = false;
  }
  if (stg > R.staging_cap) {
    dfree(R.staging);
    R.staging = (char *)dalloc(stg);
    if (!R.staging) return fail(HD_ENOMEM);
    R.staging_cap = stg;
    R.ws_epoch++;
  }
  return HD_OK;
}

// Columns [c0, c1) of shape s on row r of plane p, clipped to the array
// (the same rows and columns as shape_rows).
static bool shape_seg(const Shape &s, const int64_t *n, int64_t p, int64_t r, int32_t &c0, int32_t &c1) {
  if (s.kind == 0) {
    if (p < std::max<int64_t>(s.lo[0], 0) || p >= std::min<int64_t>(s.hi[0], n[0])) return false;
    if (r < std::max<int64_t>(s.lo[1], 0) || r >= std::min<int64_t>(s.hi[1], n[1])) return false;
    const int64_t a = std::max<int64_t>(s.lo[2], 0), b = std::min<int64_t>(s.hi[2], n[2]);
    if (a >= b) return false;
    c0 = (int32_t)a;
    c1 = (int32_t)b;
    return true;
  }
  const int64_t r0 = s.c[0], r1 = s.c[4];
  if (p != 0 || r < std::max<int64_t>(r0, 0) || r > std::min<int64_t>(r1, n[1] - 1)) return false;
  int64_t l, rt;
  if (r1 == r0) {
    l = s.c[1];
    rt = s.c[3];
  } else {
    l = s.c[1] + floordiv((r - r0) * (s.c[5] - s.c[1]), r1 - r0);
    rt = s.c[3] + floordiv((r - r0) * (s.c[7] - s.c[3]), r1 - r0);
  }
  l = std::max<int64_t>(l, 0);
  rt = std::min<int64_t>(rt, n[2] - 1);
  if (l > rt) return false;
  c0 = (int32_t)l;
  c1 = (int32_t)(rt + 1);
  return true;
}

// Plane and row breakpoints of a shape: its segment is the same on every
// row between two consecutive ones (a box: its faces; a trapezoid: every
// row unless both edges are vertical).
static void shape_breaks(const Shape &s, const int64_t *n, std::vector<int64_t> &pb, std::vector<int64_t> &rb) {
  auto clip = [](int64_t v, int64_t hi) { return std::min<int64_t>(std::max<int64_t>(v, 0), hi); };
  if (s.kind == 0) {
    pb.push_back(clip(s.lo[0], n[0]));
    pb.push_back(clip(s.hi[0], n[0]));
    rb.push_back(clip(s.lo[1], n[1]));
    rb.push_back(clip(s.hi[1], n[1]));
    return;
  }
  const int64_t a = clip(s.c[0], n[1]), b = clip(s.c[4] + 1, n[1]);
  if (s.c[1] == s.c[5] && s.c[3] == s.c[7]) {
    rb.push_back(a);
    rb.push_back(b);
  } else {
    for (int64_t r = a; r <= b; ++r) rb.push_back(r);
  }
}

// Sorted, unique breakpoints including 0 and n.
static void norm_breaks(std::vector<int64_t> &v, int64_t n) {
  v.push_back(0);
  v.push_back(n);
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
}

static std::vector<int64_t> merge_breaks(const std::vector<int64_t> &x, const std::vector<int64_t> &y) {
  std::vector<int64_t> v;
  v.reserve(x.size() + y.size());
  std::merge(x.begin(), x.end(), y.begin(), y.end(), std::back_inserter(v));
  v.erase(std::unique(v.begin(), v.end()), v.end());
  return v;
}

// The segments of (plane p, row r) for every endpoint of a shape list,
// merged per endpoint (overlapping or touching segments joined) and ordered
// by (endpoint, column).
static void row_segs(const std::vector<std::pair<int, const Shape *>> &sh, const int64_t *n, int64_t p, int64_t r,
                     int flags, std::vector<Seg> &out) {
  out.clear();
  for (const auto &es : sh) {
    int32_t c0, c1;
    if (shape_seg(*es.second, n, p, r, c0, c1)) out.push_back(Seg{es.first, c0, c1, flags});
  }
  std::sort(out.begin(), out.end(), [](const Seg &a, const Seg &b) { return std::tie(a.dst, a.c0) < std::tie(b.dst, b.c0); });
  size_t o = 0;
  for (size_t i = 0; i < out.size(); ++i) {
    if (o && out[o - 1].dst == out[i].dst && out[i].c0 <= out[o - 1].c1)
      out[o - 1].c1 = std::max(out[o - 1].c1, out[i].c1);
    else
      out[o++] = out[i];
  }
  out.resize(o);
}

static void free_inst(PlanInst *in) {
  if (!in) return;
  dfree(in->mem);
  delete in;
}

// Device data of one plan instance: the call's slices and GDEF cells for the
// given plane / row bands of every call-array (each band uniform in the
// arrays' GDEF and in the call's sections).
static PlanInst *build_inst(Plan *pl, const std::vector<std::vector<int64_t>> &PB,
                            const std::vector<std::vector<int64_t>> &QB) {
  std::vector<CallArr> carr(pl->cas.size());
  std::vector<int32_t> grp1, pos1, pend1, seg0, nseg, grp_aidx, grp_plane, grp2, pos2, pend2;
  std::vector<int64_t> grow1;
  std::vector<Seg> useg, dseg, us, ds;
  std::vector<SliceRec> srec;
  std::vector<GRowRec> grec;
  PlanInst *in = new PlanInst();
  PlanDev &P = in->P;
  memset(&P, 0, sizeof(P));
  P.ncarr = (int)pl->cas.size();
  int has3d = 0;
  for (size_t j = 0; j < pl->cas.size(); ++j) {
    const CallArray &ca = pl->cas[j];
    hd_array *a = ca.a;
    CallArr &C = carr[j];
    C.arr = a->id;
    C.argpos = ca.argpos;
    C.esize = a->esize;
    C.is3d = a->n[0] > 1;
    for (int k = 0; k < 3; ++k) C.n[k] = a->n[k];
    has3d |= C.is3d;
    C.slice0 = (int32_t)grow1.size();
    C.grp0 = (int32_t)grp_aidx.size();
    const std::vector<int64_t> &pb = PB[j], &qb = QB[j];
    for (size_t ip = 0; ip + 1 < pb.size(); ++ip) {
      const int64_t pa = pb[ip], pe = pb[ip + 1];
      bool open = false;
      for (size_t ir = 0; ir + 1 < qb.size(); ++ir) {
        const int64_t ra = qb[ir], re = qb[ir + 1];
        const int64_t grow = pa * a->n[1] + ra;
        row_segs(pl->uses[j], a->n, pa, ra, 0, us);
        row_segs(pl->defs[j], a->n, pa, ra, ca.def_flags, ds);
        int32_t slice = -1;
        if (!us.empty()) {
          if (!open) {
            grp_aidx.push_back((int32_t)j);
            grp_plane.push_back((int32_t)pa);
            grp2.push_back((int32_t)j);
            pos2.push_back((int32_t)pa);
            pend2.push_back((int32_t)pe);
            open = true;
          }
          slice = (int32_t)grow1.size();
          grp1.push_back((int32_t)grp_aidx.size() - 1);
          pos1.push_back((int32_t)ra);
          pend1.push_back((int32_t)re);
          grow1.push_back(grow);
          seg0.push_back((int32_t)useg.size());
          nseg.push_back((int32_t)us.size());
          useg.insert(useg.end(), us.begin(), us.end());
          srec.push_back(SliceRec{(int32_t)a->id, seg0.back(), (int32_t)us.size(), 0, grow});
        }
        if (us.empty() && ds.empty()) continue;
        GRowRec g{};
        g.arr = (int32_t)a->id;
        g.grow = grow;
        g.slice = slice >= 0 && !ca.no_holders ? slice : -1;
        g.dseg0 = (int32_t)dseg.size();
        g.ndseg = (int32_t)ds.size();
        // definitions sorted by column that tile [0, n2), no holder additions
        bool full = !ds.empty() && g.slice < 0;
        if (full) {
          std::vector<Seg> v = ds;
          std::sort(v.begin(), v.end(), [](const Seg &x, const Seg &y) { return x.c0 < y.c0; });
          int64_t at = 0;
          for (const Seg &q : v) {
            if (q.c0 != at) full = false;
            at = q.c1;
          }
          if (at != a->n[2]) full = false;
          if (full) ds = v;
        }
        dseg.insert(dseg.end(), ds.begin(), ds.end());
        g.full = full ? 1 : 0;
        g.pad = 0;
        grec.push_back(g);
      }
    }
    C.slice1 = (int32_t)grow1.size();
    C.grp1 = (int32_t)grp_aidx.size();
  }
  P.has3d = has3d;
  P.nsl1 = (int32_t)grow1.size();
  P.ngrp = (int32_t)grp_aidx.size();
  // cells the definitions tile first (their update is a plain copy, one lane
  // per cell); the order of the other cells is kept
  std::stable_partition(grec.begin(), grec.end(), [](const GRowRec &g) { return g.full != 0; });
  P.ngrow = (int32_t)grec.size();
  P.ngfull = 0;
  for (const GRowRec &g : grec) P.ngfull += g.full ? 1 : 0;
  // GDEF update form of the other cells: when nearly all of them involve at
  // most two devices (row partitions, 3-D blocks split once along the row)
  // their lists stay short and one lane per cell updates them; cells shared
  // by more devices (2-D block partitions) are updated one wave per cell
  {
    int64_t small = 0, rest = 0;
    for (const GRowRec &g : grec) {
      if (g.full) continue;
      ++rest;
      int d0 = -1, d1 = -1;
      bool more = false;
      auto see = [&](int d) {
        if (d == d0 || d == d1) return;
        if (d0 < 0)
          d0 = d;
        else if (d1 < 0)
          d1 = d;
        else
          more = true;
      };
      if (g.slice >= 0)
        for (int e = 0; e < nseg[g.slice]; ++e) see(useg[seg0[g.slice] + e].dst);
      for (int e = 0; e < g.ndseg; ++e) see(dseg[g.dseg0 + e].dst);
      if (!more) ++small;
    }
    P.gdef_lane = rest > 0 && small * 10 >= rest * 9 ? 1 : 0;
  }
  // one device allocation for all instance arrays
  std::vector<char> blob;
  size_t o_carr = push_blob(blob, carr);
  size_t o_grp1 = push_blob(blob, grp1), o_pos1 = push_blob(blob, pos1), o_pend1 = push_blob(blob, pend1);
  size_t o_grow1 = push_blob(blob, grow1);
  size_t o_seg0 = push_blob(blob, seg0), o_nseg = push_blob(blob, nseg), o_useg = push_blob(blob, useg);
  size_t o_srec = push_blob(blob, srec);
  size_t o_ga = push_blob(blob, grp_aidx), o_gp = push_blob(blob, grp_plane);
  size_t o_g2 = push_blob(blob, grp2), o_p2 = push_blob(blob, pos2), o_pe2 = push_blob(blob, pend2);
  size_t o_grec = push_blob(blob, grec), o_ds = push_blob(blob, dseg);
  in->mem = dalloc(blob.size());
  if (!in->mem) {
    delete in;
    fail(HD_ENOMEM);
    return nullptr;
  }
  char *b = (char *)in->mem;
  P.carr = (const CallArr *)(b + o_carr);
  P.grp1 = (const int32_t *)(b + o_grp1);
  P.pos1 = (const int32_t *)(b + o_pos1);
  P.pend1 = (const int32_t *)(b + o_pend1);
  P.grow1 = (const int64_t *)(b + o_grow1);
  P.seg0 = (const int32_t *)(b + o_seg0);
  P.nseg = (const int32_t *)(b + o_nseg);
  P.useg = (const Seg *)(b + o_useg);
  P.srec = (const SliceRec *)(b + o_srec);
  P.grp_aidx = (const int32_t *)(b + o_ga);
  P.grp_plane = (const int32_t *)(b + o_gp);
  P.grp2 = (const int32_t *)(b + o_g2);
  P.pos2 = (const int32_t *)(b + o_p2);
  P.pend2 = (const int32_t *)(b + o_pe2);
  P.grec = (const GRowRec *)(b + o_grec);
  P.dseg = (const Seg *)(b + o_ds);

  if (hipMemcpy(in->mem, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
    free_inst(in);
    fail(HD_EHIP);
    return nullptr;
  }
  return in;
}

// Instance of a plan for the arrays' current bands (built on first use;
// may_build false: only an existing one, else HD_ENOPLAN).  A plan keeps at
// most kMaxInst instances; past that the others are dropped (after the
// streams are idle, so no queued work reads them).
constexpr size_t kMaxInst = 32;
static int copy_band_lists(Plan *pl, const std::vector<std::vector<int64_t>> &pb,
                           const std::vector<std::vector<int64_t>> &qb, const std::vector<int64_t> &ikey,
                           bool may_build);

// The band copies of the selected instance, then the band versions that
// let the next selection skip all this while no array's bands change.
static int select_done(Plan *pl, const std::vector<std::vector<int64_t>> &pb,
                       const std::vector<std::vector<int64_t>> &qb, const std::vector<int64_t> &key, bool may_build) {
  if (copy_band_lists(pl, pb, qb, key, may_build) != HD_OK) return g_last_error;
  for (const CallArray &ca : pl->cas) pl->sel_ver.push_back(ca.a->bver);
  return HD_OK;
}

// The stream of the metadata work (the data stream in serial mode).
static hipStream_t meta_stream() { return R.serial ? R.data : R.meta; }

// A cell of the instance that does not start one of its array's bands
// reads and writes its own first row, so the band's list is copied there
// first: the copies are queued on the metadata stream ahead of the call's
// derivation and GDEF update (repeating them is harmless: they read band
// representatives, which nothing in between writes).  Their device lists
// are kept per (instance, array bands); none are needed once the arrays'
// bands are the instance's, as in a repeated call.
static int copy_band_lists(Plan *pl, const std::vector<std::vector<int64_t>> &pb,
                           const std::vector<std::vector<int64_t>> &qb, const std::vector<int64_t> &ikey,
                           bool may_build) {
  std::vector<MatRec> mat;
  std::vector<int64_t> key = ikey;
  for (size_t j = 0; j < pl->cas.size(); ++j) {
    const hd_array *a = pl->cas[j].a;
    for (size_t ip = 0; ip + 1 < pb[j].size(); ++ip) {
      const int64_t pa = pb[j][ip];
      const int64_t pband = *(std::upper_bound(a->pbrk.begin(), a->pbrk.end(), pa) - 1);
      for (size_t ir = 0; ir + 1 < qb[j].size(); ++ir) {
        const int64_t ra = qb[j][ir];
        const int64_t rband = *(std::upper_bound(a->rbrk.begin(), a->rbrk.end(), ra) - 1);
        if (pband != pa || rband != ra)
          mat.push_back(MatRec{(int32_t)a->id, 0, pband * a->n[1] + rband, pa * a->n[1] + ra});
      }
    }
    key.push_back(-3);
    key.insert(key.end(), a->pbrk.begin(), a->pbrk.end());
    key.push_back(-4);
    key.insert(key.end(), a->rbrk.begin(), a->rbrk.end());
  }
  pl->sel_mat = nullptr;
  pl->sel_nmat = 0;
  if (mat.empty()) return HD_OK;
  auto it = pl->mats.find(key);
  if (it == pl->mats.end()) {
    if (!may_build) return fail(HD_ENOPLAN);
    if (pl->mats.size() >= kMaxInst) {
      // queued copies may still read the lists
      HIPCK(hipStreamSynchronize(R.meta));
      HIPCK(hipStreamSynchronize(R.data));
      for (auto &kv : pl->mats) dfree(kv.second.first);
      pl->mats.clear();
    }
    void *m = dalloc(sizeof(MatRec) * mat.size());
    if (!m) return fail(HD_ENOMEM);
    HIPCK(hipMemcpy(m, mat.data(), sizeof(MatRec) * mat.size(), hipMemcpyHostToDevice));
    it = pl->mats.emplace(key, std::make_pair(m, (int)mat.size())).first;
  }
  pl->sel_mat = (const MatRec *)it->second.first;
  pl->sel_nmat = it->second.second;
  HIPCK(launch_mat(pl->sel_mat, pl->sel_nmat, R.d_arrs, meta_stream()));
  return HD_OK;
}

static int select_inst(Plan *pl, bool may_build = true) {
  const size_t nc = pl->cas.size();
  // no array's bands changed since the last selection: same instance, same copies
  if (pl->cur && pl->sel_ver.size() == nc) {
    bool same = true;
    for (size_t j = 0; j < nc && same; ++j) same = pl->cas[j].a->bver == pl->sel_ver[j];
    if (same) {
      if (pl->sel_nmat > 0) HIPCK(launch_mat(pl->sel_mat, pl->sel_nmat, R.d_arrs, meta_stream()));
      return HD_OK;
    }
  }
  std::vector<std::vector<int64_t>> pb(nc), qb(nc);
  std::vector<int64_t> key;
  for (size_t j = 0; j < nc; ++j) {
    const hd_array *a = pl->cas[j].a;
    pb[j] = merge_breaks(a->pbrk, pl->pbp[j]);
    qb[j] = merge_breaks(a->rbrk, pl->rbp[j]);
    key.push_back(-1);
    key.insert(key.end(), pb[j].begin(), pb[j].end());
    key.push_back(-2);
    key.insert(key.end(), qb[j].begin(), qb[j].end());
  }
  pl->sel_ver.clear();
  if (pl->cur && key == pl->cur_key) return select_done(pl, pb, qb, key, may_build);
  PlanInst *in = nullptr;
  auto it = pl->insts.find(key);
  if (it != pl->insts.end()) {
    in = it->second;
  } else {
    if (!may_build) return fail(HD_ENOPLAN);
    if (pl->insts.size() >= kMaxInst) {
      HIPCK(hipStreamSynchronize(R.meta));
      HIPCK(hipStreamSynchronize(R.meta2));
      HIPCK(hipStreamSynchronize(R.data));
      for (auto &kv : pl->insts) free_inst(kv.second);
      pl->insts.clear();
      pl->cur = nullptr;
    }
    in = build_inst(pl, pb, qb);
    if (!in) return g_last_error;
    pl->insts[key] = in;
  }
  pl->cur = in;
  pl->cur_key = key;
  pl->P = in->P;
  pl->nsl1 = in->P.nsl1;
  pl->ngrp = in->P.ngrp;
  pl->ngrow = in->P.ngrow;
  return select_done(pl, pb, qb, key, may_build);
}

// After a call's GDEF update: the bands every call-array now holds, the old
// bands refined by the plan's (the call's cells).  They are never
// coarsened: a cell's first row holds its list, so a band that merged cells
// would make the next call copy lists back to the cells' first rows; with
// refinement only, the bands of arrays that a fixed set of plans touch
// settle after a few calls and later calls copy nothing.
static void advance_bands(const Plan *pl) {
  for (size_t j = 0; j < pl->cas.size(); ++j) {
    hd_array *a = pl->cas[j].a;
    const size_t np = a->pbrk.size(), nr = a->rbrk.size();
    a->pbrk = merge_breaks(a->pbrk, pl->pbp[j]);
    a->rbrk = merge_breaks(a->rbrk, pl->rbp[j]);
    if (a->pbrk.size() != np || a->rbrk.size() != nr) ++a->bver;
  }
}

// Builds a plan for one communication + GDEF update.  cas: the distinct
// arrays of the call in argument order with per-endpoint use and def
// shapes.  Checks the definitions for races, sizes the workspace for the
// finest instance (one cell per row), and selects the instance for the
// arrays' current bands.
static int build_plan(std::vector<CallArray> &cas, Plan *pl) {
  pl->ca_arr.clear();
  pl->ca_full.clear();
  pl->uid = R.next_uid++;
  int64_t stg = 0;
  int has3d = 0;
  int64_t nsl_max = 0, ngrp_max = 0, ngrow_max = 0, nseg_all = 0;
  pl->pbp.assign(cas.size(), {});
  pl->rbp.assign(cas.size(), {});
  for (size_t j = 0; j < cas.size(); ++j) {
    CallArray &ca = cas[j];
    hd_array *a = ca.a;
    has3d |= a->n[0] > 1;
    // use spans
    std::vector<Span> us;
    for (int e = 0; e < 64; ++e)
      for (const Shape &s : ca.use[e]) {
        shape_breaks(s, a->n, pl->pbp[j], pl->rbp[j]);
        shape_rows(s, a->n, [&](int64_t p, int64_t r, int64_t c0, int64_t c1) {
          us.push_back(Span{p * a->n[1] + r, e, (int32_t)c0, (int32_t)c1, 0});
        });
      }
    merge_spans(us);
    // def spans, race check across devices
    std::vector<Span> ds;
    for (int e = 0; e < 64; ++e)
      for (const Shape &s : ca.def[e]) {
        shape_breaks(s, a->n, pl->pbp[j], pl->rbp[j]);
        shape_rows(s, a->n, [&](int64_t p, int64_t r, int64_t c0, int64_t c1) {
          ds.push_back(Span{p * a->n[1] + r, e, (int32_t)c0, (int32_t)c1, ca.def_flags});
        });
      }
    merge_spans(ds);
    norm_breaks(pl->pbp[j], a->n[0]);
    norm_breaks(pl->rbp[j], a->n[1]);
    {
      std::vector<Span> byc = ds;
      std::sort(byc.begin(), byc.end(),
                [](const Span &x, const Span &y) { return std::tie(x.row, x.c0) < std::tie(y.row, y.c0); });
      for (size_t i = 1; i < byc.size(); ++i)
        if (byc[i].row == byc[i - 1].row && byc[i].c0 < byc[i - 1].c1 && byc[i].e != byc[i - 1].e)
          return fail(HD_ERACE);
    }
    // sizes of the finest instance: one slice per use row, one group per
    // plane with use rows, one cell per row with use or def spans
    std::vector<int64_t> urows, drows;
    for (const Span &s : us) {
      stg += (int64_t)(s.c1 - s.c0) * a->esize;
      if (urows.empty() || urows.back() != s.row) urows.push_back(s.row);
    }
    stg += 16;
    nseg_all += (int64_t)us.size();
    nsl_max += (int64_t)urows.size();
    {
      int64_t last = -1;
      for (int64_t r : urows)
        if (r / a->n[1] != last) {
          last = r / a->n[1];
          ++ngrp_max;
        }
    }
    for (const Span &s : ds)
      if (drows.empty() || drows.back() != s.row) drows.push_back(s.row);
    std::vector<int64_t> rows;
    std::set_union(urows.begin(), urows.end(), drows.begin(), drows.end(), std::back_inserter(rows));
    ngrow_max += (int64_t)rows.size();
    // a call that defines every row of the array whole and does not use it
    // leaves a GDEF that does not depend on the one before (plan cache)
    int64_t nfull = 0;
    if (urows.empty()) {
      size_t i = 0;
      while (i < ds.size()) {
        const int64_t row = ds[i].row;
        std::vector<Span> v;
        for (; i < ds.size() && ds[i].row == row; ++i) v.push_back(ds[i]);
        std::sort(v.begin(), v.end(), [](const Span &x, const Span &y) { return x.c0 < y.c0; });
        int64_t at = 0;
        bool full = true;
        for (const Span &q : v) {
          if (q.c0 != at) full = false;
          at = q.c1;
        }
        if (full && at == a->n[2]) ++nfull;
      }
    }
    pl->ca_arr.push_back(a->id);
    pl->ca_full.push_back(urows.empty() && nfull == a->n[0] * a->n[1] ? 1 : 0);
  }
  pl->has3d = has3d;
  pl->stg_bound = stg;
  pl->nsl_max = nsl_max;
  pl->cas = std::move(cas);
  pl->uses.assign(pl->cas.size(), {});
  pl->defs.assign(pl->cas.size(), {});
  for (size_t j = 0; j < pl->cas.size(); ++j)
    for (int e = 0; e < 64; ++e) {
      for (const Shape &s : pl->cas[j].use[e]) pl->uses[j].push_back({e, &s});
      for (const Shape &s : pl->cas[j].def[e]) pl->defs[j].push_back({e, &s});
    }
  // work boxes (filled by the caller)
  pl->mem = dalloc(sizeof(WorkBox) * 5 * kMaxDev + 256);
  if (!pl->mem) return fail(HD_ENOMEM);
  pl->wb = (WorkBox *)pl->mem;
  for (int k = 0; k < 5; ++k) pl->wbj[k] = pl->wb + k * kMaxDev;
  pl->nbox = 0;
  // workspace sizing for the finest instance: a slot of kRunSlot runs per
  // slice plus a spill pool
  const int64_t items = nsl_max * kRunSlot + std::max<int64_t>(int64_t(1) << 20, 4 * nseg_all);
  if (ensure_ws(nsl_max, ngrp_max, items, stg, ngrow_max) != HD_OK) return g_last_error;
  return select_inst(pl);
}

static Level make_level(int which, const PlanDev &P) {
  Level L{};
  if (which == 1) {
    L.nsl = P.nsl1;
    L.grp = P.grp1;
    L.pos = P.pos1;
    L.pend = P.pend1;
    L.ioff = R.W.roff;
    L.icnt = R.W.rcnt;
    L.items = R.W.runs;
  } else {
    L.nsl = P.ngrp;
    L.grp = P.grp2;
    L.pos = P.pos2;
    L.pend = P.pend2;
    L.ioff = R.W.goff;
    L.icnt = R.W.gcnt;
    L.items = R.W.l1out;
  }
  L.bmask = R.bmask;
  L.bcnt = R.bcnt;
  L.bbase = R.bbase;
  L.bandslice = R.bandslice;
  L.nb = R.counters + 2;
  L.hoff = R.hoff;
  L.hcnt = R.hcnt;
  L.hbytes = R.hbytes;
  L.bcarr = R.bcarr;
  L.nofs = R.nofs;
  L.bofs = R.bofs;
  L.grp_carr = which == 1 ? P.grp_aidx : nullptr;
  L.carr = P.carr;
  L.heads = R.heads;
  L.head_top = R.counters + 1;
  L.head_cap = R.ws_items;
  return L;
}

static hipEvent_t prof_event() {
  if (!R.ev_pool.empty()) {
    hipEvent_t e = R.ev_pool.back();
    R.ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, R.time_ev) != hipSuccess) return nullptr;
  return e;
}

struct PhaseTimer {
  int phase;
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s;
  PhaseTimer(int ph, hipStream_t st) : phase(ph), s(st) {
    if (!((R.prof >> ph) & 1)) return;
    a = prof_event();
    b = prof_event();
    if (a) (void)hipEventRecord(a, s);
  }
  ~PhaseTimer() {
    if (!a || !b) return;
    (void)hipEventRecord(b, s);
    R.prof_pending.push_back({phase, {a, b}});
  }
};

extern "C" int hdarray_set_stencil_shape(int rows, int waves, int order) {
  if (!R.inited) return fail(HD_ESTATE);
  if (!(rows == 0 || rows == 4 || rows == 8 || rows == 16 || rows == 32 || rows == 64)) return fail(HD_EINVAL);
  if (!(waves == 0 || waves == 1 || waves == 4)) return fail(HD_EINVAL);
  if (order != 0 && order != 1) return fail(HD_EINVAL);
  R.jacobi_rows = rows;
  R.jacobi_waves = waves;
  R.jacobi_order = order;
  return HD_OK;
}

extern "C" int hdarray_set_plan_cache(int on) {
  if (!R.inited) return fail(HD_ESTATE);
  R.plan_cache = on != 0;
  return HD_OK;
}

extern "C" int hdarray_profile(int enable) {
  R.prof = enable;
  return HD_OK;
}

extern "C" int hdarray_profile_read(hd_profile_t *out) {
  if (!out) return fail(HD_EINVAL);
  memset(out, 0, sizeof(*out));
  if (!R.inited) return fail(HD_ESTATE);
  HIPCK(hipStreamSynchronize(R.meta));
  HIPCK(hipStreamSynchronize(R.data));
  for (auto &p : R.prof_pending) {
    float ms = 0.f;
    HIPCK(hipEventElapsedTime(&ms, p.second.first, p.second.second));
    out->ms[p.first] += ms;
    out->count[p.first] += 1;
    R.ev_pool.push_back(p.second.first);
    R.ev_pool.push_back(p.second.second);
  }
  R.prof_pending.clear();
  return HD_OK;
}

// Enqueues communication (meta: derive; data: pack, unpack) and the GDEF
// update for a plan; the user kernel (if any) follows on the data stream.
// Tile shape of a stencil launch: fixed by the environment, or the next
// candidate of the tuning (with the event pair that times it), or the
// tuned best.  The tuning reads its events only once they have completed,
// so it never waits for the GPU.
static void stencil_shape(Plan *pl, int &th, int &waves, int &order, hipEvent_t &e0, hipEvent_t &e1) {
  e0 = e1 = nullptr;
  if (R.jacobi_rows || R.jacobi_waves) {
    th = R.jacobi_rows ? R.jacobi_rows : 4;
    waves = R.jacobi_waves ? R.jacobi_waves : 1;
    order = waves == 4 ? 1 : R.jacobi_order;
    return;
  }
  TuneState &ts = R.tunes[pl->tkey];
  int c = ts.best;
  if (!ts.done && ts.next < kTuneN * kTuneReps) {
    const int slot = ts.next++;
    c = slot % kTuneN;
    if (!ts.ev[2 * slot] && hipEventCreateWithFlags(&ts.ev[2 * slot], R.time_ev) != hipSuccess)
      ts.ev[2 * slot] = nullptr;
    if (!ts.ev[2 * slot + 1] && hipEventCreateWithFlags(&ts.ev[2 * slot + 1], R.time_ev) != hipSuccess)
      ts.ev[2 * slot + 1] = nullptr;
    if (ts.ev[2 * slot] && ts.ev[2 * slot + 1]) {
      e0 = ts.ev[2 * slot];
      e1 = ts.ev[2 * slot + 1];
    }
  } else if (!ts.done) {
    const int last = 2 * kTuneN * kTuneReps - 1;
    const bool ready = !ts.ev[last] || hipEventQuery(ts.ev[last]) == hipSuccess;
    (void)hipGetLastError();  // a not-ready query must not surface as an error of a later call
    if (ready) {
      // the candidate with the least median time over its calls (one fast
      // or slow call alone does not decide between shapes a few percent
      // apart)
      std::vector<float> t[kTuneN];
      for (int slot = 0; slot < kTuneN * kTuneReps; ++slot) {
        float ms = 0.f;
        if (!ts.ev[2 * slot] || !ts.ev[2 * slot + 1] ||
            hipEventElapsedTime(&ms, ts.ev[2 * slot], ts.ev[2 * slot + 1]) != hipSuccess)
          continue;
        t[slot % kTuneN].push_back(ms);
      }
      float best = 1e30f;
      for (int k = 0; k < kTuneN; ++k) {
        if (t[k].empty()) continue;
        std::sort(t[k].begin(), t[k].end());
        const float med = t[k][t[k].size() / 2];
        if (med < best) {
          best = med;
          ts.best = k;
        }
      }
      for (hipEvent_t &e : ts.ev)
        if (e) {
          (void)hipEventDestroy(e);
          e = nullptr;
        }
      ts.done = true;
    }
    c = ts.best;
  }
  th = kTuneCand[c][0];
  waves = kTuneCand[c][1];
  order = kTuneCand[c][2];
}

// ------------------------------------------------------------ plan cache
// Sec. 4.2: when the GDEF of every array of a call is the one the plan's
// last derivation saw, the communication sets are the same, so the plan's
// message table and runs are reused and only the GDEF update runs.  GDEF
// equality is decided on the host, exactly: each array keeps the list of
// (plan, call-array) updates since a call that defined all of it without
// using it; equal lists give equal GDEF.
static std::vector<uint64_t> plan_key(const Plan *pl) {
  std::vector<uint64_t> k;
  for (int id : pl->ca_arr) {
    const hd_array *a = R.arrays[id];
    if (!a || !a->hist_ok) return {};
    k.insert(k.end(), a->hist.begin(), a->hist.end());
    k.push_back(~0ull);
  }
  return k;
}

static void advance_hist(const Plan *pl) {
  for (size_t j = 0; j < pl->ca_arr.size(); ++j) {
    hd_array *a = R.arrays[pl->ca_arr[j]];
    const uint64_t tag = (pl->uid << 10) | j;
    if (pl->ca_full[j]) {
      a->hist.assign(1, tag);
      a->hist_ok = true;
    } else if (a->hist_ok) {
      if (a->hist.size() >= 8) {
        a->hist.clear();
        a->hist_ok = false;
      } else {
        a->hist.push_back(tag);
      }
    }
  }
}

// the plan's own table, runs and events (allocated on its first cached call)
// Snapshot of the lists a plan's small-form derivation last read (the plan
// cache's second step): one kMaxCap list per slice, at most kDerive1Slices.
constexpr int kDerive1Slices = 64;

static int plan_buffers(Plan *pl) {
  if (pl->ptab) return HD_OK;
  pl->snap = (Ivl *)dalloc(sizeof(Ivl) * kMaxCap * kDerive1Slices);
  pl->scnt = (int32_t *)dalloc(4 * kDerive1Slices);
  if (!pl->snap || !pl->scnt) return fail(HD_ENOMEM);
  pl->pcap = R.ws_items;
  pl->ptab = (MsgRec *)dalloc(sizeof(MsgRec) * pl->pcap);
  pl->phdr = (MsgHdr *)dalloc(sizeof(MsgHdr));
  pl->pruns = (Item *)dalloc(sizeof(Item) * pl->pcap);
  pl->proff = (int32_t *)dalloc(4 * (pl->nsl_max + 1));
  pl->prcnt = (int32_t *)dalloc(4 * (pl->nsl_max + 1));
  if (!pl->ptab || !pl->phdr || !pl->pruns || !pl->proff || !pl->prcnt) return fail(HD_ENOMEM);
  HIPCK(hipMemset(pl->phdr, 0, sizeof(MsgHdr)));
  HIPCK(hipEventCreateWithFlags(&pl->ev_ready, R.sync_ev));
  // the marker that the plan's stored table has been read by the pack: it
  // orders a later rewrite of the table after those reads (write after
  // read), so it carries no data and is recorded without a release fence
  // (measured: 9735-9762 -> 9906 steps/s with the plan cache on; the same
  // for the derive-every-step slots measured slower, 9190-9220 -> 8565-8595,
  // so those keep the device-scope release)
  HIPCK(hipEventCreateWithFlags(&pl->ev_used, R.free_ev));
  return HD_OK;
}

static void free_plan_buffers(Plan *pl) {
  dfree(pl->snap);
  dfree(pl->scnt);
  pl->snap = nullptr;
  pl->scnt = nullptr;
  pl->snap_inst = nullptr;
  dfree(pl->ptab);
  dfree(pl->phdr);
  dfree(pl->pruns);
  dfree(pl->proff);
  dfree(pl->prcnt);
  if (pl->ev_ready) (void)hipEventDestroy(pl->ev_ready);
  if (pl->ev_used) (void)hipEventDestroy(pl->ev_used);
  pl->ptab = nullptr;
  pl->phdr = nullptr;
  pl->pruns = nullptr;
  pl->proff = pl->prcnt = nullptr;
  pl->ev_ready = pl->ev_used = nullptr;
}

static void free_inst(PlanInst *in);
static void plan_free(Plan *pl) {
  if (!pl) return;
  free_plan_buffers(pl);
  for (auto &kv : pl->insts) free_inst(kv.second);
  pl->insts.clear();
  for (auto &kv : pl->mats) dfree(kv.second.first);
  pl->mats.clear();
  dfree(pl->mem);
  dfree(pl->part);
  delete pl;
}

static int enqueue_user(Plan *pl, const float *coef);

// Communication-set derivation and GDEF update of one call.  Only the runs
// read GDEF, so once they are found the GDEF update (which needs nothing
// else) runs on the second internal stream beside the rest of the
// derivation; the meta stream then waits for it, so the next call's runs
// see the updated GDEF.  ev_table (optional) marks the message table done.
static hipError_t derive_and_update(const PlanDev &P, const Work &W, const Level &L1, MsgRec *tab, MsgHdr *hdr,
                                    int64_t cap, int has3d, hipStream_t meta, hipEvent_t ev_table = nullptr) {
  hipError_t e;
  if (R.fused) {
    // small instances: two launches (runs; then the table and the GDEF
    // update side by side), no fork and no events
    e = launch_derive1(P, R.d_arrs, W, L1, make_level(2, P), tab, hdr, cap, R.row_cap, true, meta);
    if (e == hipSuccess) return ev_table ? hipEventRecord(ev_table, meta) : hipSuccess;
    if (e != hipErrorNotSupported) return e;
    (void)hipGetLastError();
  }
  e = launch_runs(P, R.d_arrs, W, R.row_cap, meta);
  if (e != hipSuccess) return e;
  const bool fork = meta != R.data;
  if (fork) {
    if ((e = hipEventRecord(R.ev_runs, meta)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(R.meta2, R.ev_runs, 0)) != hipSuccess) return e;
    if ((e = launch_gdef(P, R.d_arrs, W, R.meta2)) != hipSuccess) return e;
    if ((e = hipEventRecord(R.ev_gdef, R.meta2)) != hipSuccess) return e;
  }
  if ((e = launch_level1_tail(P, W, L1, tab, hdr, cap, has3d ? 1 : 0, meta)) != hipSuccess) return e;
  if (has3d) {
    Level L2 = make_level(2, P);
    if ((e = launch_level2(P, W, L2, tab, hdr, cap, meta)) != hipSuccess) return e;
  }
  if (ev_table && (e = hipEventRecord(ev_table, meta)) != hipSuccess) return e;
  if (fork) return hipStreamWaitEvent(meta, R.ev_gdef, 0);
  return launch_gdef(P, R.d_arrs, W, meta);
}

// A plain call with the plan cache on: derivation (on a miss) into the
// plan's own buffers, GDEF update from the plan's runs, pack from the
// plan's table.
static int enqueue_cached(Plan *pl, const float *coef) {
  const hipStream_t meta = R.serial ? R.data : R.meta;
  if (plan_buffers(pl) != HD_OK) return g_last_error;
  if (select_inst(pl) != HD_OK) return g_last_error;
  const std::vector<uint64_t> key = plan_key(pl);
  // equal histories give equal GDEF and so equal bands: the same instance
  const bool hit = pl->have && !key.empty() && key == pl->last_key && pl->cur == pl->last_inst;
  const PlanDev &P = pl->P;
  Work W = R.W;
  W.runs = pl->pruns;
  W.roff = pl->proff;
  W.rcnt = pl->prcnt;
  W.run_cap = pl->pcap;
  {
    PhaseTimer tm(0, meta);
    if (!hit) {
      // the data stream must be done with the table of this plan's last call
      if (pl->used_pending) HIPCK(hipStreamWaitEvent(meta, pl->ev_used, 0));
      Level L1 = make_level(1, P);
      L1.ioff = W.roff;
      L1.icnt = W.rcnt;
      L1.items = W.runs;
      // second step (Sec. 4.2): the history does not decide, so the slices'
      // lists are compared on the GPU with those the plan's last derivation
      // read (same instance); when equal the small-form derivation is left
      // out and the plan's table and runs are used.  A miss refreshes them.
      if (R.fused && P.nsl1 <= kDerive1Slices && P.ngrp <= kDerive1Slices) {
        HIPCK(launch_snap(P, R.d_arrs, pl->snap, pl->scnt, R.counters + 8, R.counters + 9, pl->snap_inst == pl->cur,
                          meta));
        pl->snap_inst = pl->cur;
        W.skip = R.counters + 8;
      } else {
        pl->snap_inst = nullptr;
      }
      HIPCK(derive_and_update(P, W, L1, pl->ptab, pl->phdr, pl->pcap, pl->has3d, meta, pl->ev_ready));
      R.stats.cache_misses++;
    } else {
      HIPCK(launch_gdef(P, R.d_arrs, W, meta));
      R.stats.cache_hits++;
    }
  }
  pl->last_key = key;
  pl->last_inst = pl->cur;
  pl->have = !key.empty();
  advance_hist(pl);
  advance_bands(pl);
  HIPCK(hipStreamWaitEvent(R.data, pl->ev_ready, 0));
  {
    PhaseTimer tm(1, R.data);
    HIPCK(launch_pack(pl->ptab, pl->phdr, R.d_arrs, (uint32_t *)R.staging, pl->stg_bound / 4 + 1, 2, R.data));
  }
  HIPCK(hipEventRecord(pl->ev_used, R.data));
  pl->used_pending = true;
  R.last_ptab = pl->ptab;
  R.last_phdr = pl->phdr;
  R.last_tab = -1;
  R.last_batch = -1;
  return enqueue_user(pl, coef);
}

static int enqueue(Plan *pl, const float *coef) {
  if (pl->apply && !pl->adjoint && R.plan_cache) return enqueue_cached(pl, coef);
  if (select_inst(pl) != HD_OK) return g_last_error;
  // every plan's GDEF update is a function of the plan and the GDEF before it
  advance_hist(pl);
  advance_bands(pl);
  R.last_ptab = nullptr;
  R.last_phdr = nullptr;
  const hipStream_t meta = R.serial ? R.data : R.meta;
  const int slot = R.parity;
  R.parity ^= 1;
  if (R.free_pending[slot]) HIPCK(hipStreamWaitEvent(meta, R.ev_free[slot], 0));
  const PlanDev &P = pl->P;
  Work W = R.W;
  {
  PhaseTimer tm(0, meta);
  // adjoint: the cotangent array is defined by the owners of the work boxes
  // first, so its use-region messages are exactly {(owner(x) -> d, x)}
  Level L1 = make_level(1, P);
  if (pl->adjoint) {
    HIPCK(launch_gdef(P, R.d_arrs, W, meta));
    bool done = false;
    if (R.fused) {
      const hipError_t e = launch_derive1(P, R.d_arrs, W, L1, make_level(2, P), R.tab[slot], R.hdr[slot], R.ws_items,
                                          R.row_cap, false, meta);
      if (e == hipSuccess)
        done = true;
      else if (e != hipErrorNotSupported)
        return fail(HD_EHIP);
      (void)hipGetLastError();
    }
    if (!done) {
      HIPCK(launch_level1(P, R.d_arrs, W, L1, R.tab[slot], R.hdr[slot], R.ws_items, pl->has3d ? 1 : 0, R.row_cap,
                          meta));
      if (pl->has3d) {
        Level L2 = make_level(2, P);
        HIPCK(launch_level2(P, W, L2, R.tab[slot], R.hdr[slot], R.ws_items, meta));
      }
    }
    HIPCK(hipEventRecord(R.ev_cs[slot], meta));
  } else {
    HIPCK(derive_and_update(P, W, L1, R.tab[slot], R.hdr[slot], R.ws_items, pl->has3d, meta, R.ev_cs[slot]));
  }
  }
  // data stream
  HIPCK(hipStreamWaitEvent(R.data, R.ev_cs[slot], 0));
  const int64_t bw = pl->stg_bound / 4 + 1;
  if (pl->adjoint) {
    {
      PhaseTimer tm(4, R.data);
      HIPCK(launch_adjoint(pl->wb, pl->nbox, pl->ntiles, coef, pl->part, R.adj_cbar, R.tab[slot], R.hdr[slot],
                           R.d_arrs, (uint32_t *)R.staging, bw, R.data));
    }
    HIPCK(hipEventRecord(R.ev_free[slot], R.data));
    R.free_pending[slot] = true;
    R.last_tab = slot;
    R.last_batch = -1;
    return HD_OK;
  }
  {
    // pack and unpack in one pass over the staging words (the phase-1 timer
    // covers both; phase 2 stays empty on this path)
    PhaseTimer tm(1, R.data);
    HIPCK(launch_pack(R.tab[slot], R.hdr[slot], R.d_arrs, (uint32_t *)R.staging, bw, 2, R.data));
  }
  HIPCK(hipEventRecord(R.ev_free[slot], R.data));
  R.free_pending[slot] = true;
  R.last_tab = slot;
  R.last_batch = -1;
  return enqueue_user(pl, coef);
}

// the user kernel of a call, on the data stream
static int enqueue_user(Plan *pl, const float *coef) {
  if (pl->ukind == 1 || pl->ukind == 5 || pl->ukind == 6) {
    int th = 8, waves = 1, order = 1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    stencil_shape(pl, th, waves, order, e0, e1);
    // tile height: rows per wave, times four for the stacked shape
    const int tr = waves == 4 && th < 32 ? 4 * th : th;
    const int q = tr == 4 ? 0 : tr == 8 ? 1 : tr == 16 ? 2 : tr == 32 ? 3 : 4;
    R.stats.stencil_rows = th;
    R.stats.stencil_waves = waves;
    R.stats.stencil_order = order;
    R.stats.stencil_vec = pl->vec ? 1 : 0;
    PhaseTimer tm(3, R.data);
    if (e0) HIPCK(hipEventRecord(e0, R.data));
    if (waves == 4 && th < 32 && pl->vec && pl->nbox <= kArgBoxes && !pl->hwbj[q].empty()) {
      // the stacked shape with the boxes and buffers passed by value
      const std::vector<WorkBox> &hb = pl->hwbj[q];
      StackArgs a{};
      a.nbox = (int32_t)hb.size();
      const hd_array *ai = R.arrays[hb[0].ain];
      a.N1 = (int32_t)ai->n[1];
      a.N2 = (int32_t)ai->n[2];
      for (size_t i = 0; i < hb.size(); ++i) {
        a.lo1[i] = hb[i].lo[1];
        a.lo2[i] = hb[i].lo[2];
        a.hi1[i] = hb[i].hi[1];
        a.hi2[i] = hb[i].hi[2];
        a.tile0[i] = hb[i].tile0;
        const hd_array *xi = R.arrays[hb[i].ain], *xo = R.arrays[hb[i].aout];
        a.in[i] = reinterpret_cast<const float *>(xi->buf[hb[i].dev]);
        a.out[i] = reinterpret_cast<float *>(xo->buf[hb[i].dev]);
        a.rsi[i] = xi->rs[hb[i].dev];
        a.rso[i] = xo->rs[hb[i].dev];
      }
      const int op = pl->ukind == 1 ? 0 : pl->ukind == 5 ? 1 : 2;
      HIPCK(launch_stack_args(op, th, a, pl->ntj[q], coef, R.data));
      R.stats.stencil_vec = 2;
    } else {
      HIPCK(launch_user(pl->ukind, th, waves, order, pl->vec, pl->wbj[q], pl->nbox, R.d_arrs, pl->ntj[q], coef,
                        R.data));
    }
    if (e1) HIPCK(hipEventRecord(e1, R.data));
  } else if (pl->ukind) {
    PhaseTimer tm(3, R.data);
    HIPCK(launch_user(pl->ukind, pl->th, 1, 1, pl->vec, pl->wb, pl->nbox, R.d_arrs, pl->ntiles, coef, R.data));
  }
  return HD_OK;
}

// ---------------------------------------------------------- apply kernel
struct KSpec {
  int nargs, out, nin, in[2], dim, nscal;
};
static bool kspec(int b, KSpec &s) {
  memset(&s, 0, sizeof(s));
  switch (b) {
    case 1:
    case 5:
      s = KSpec{2, 0, 1, {1, 0}, 2, 0};
      return true;
    case 2:
      s = KSpec{2, 0, 1, {1, 0}, 0, 0};
      return true;
    case 3:
      s = KSpec{2, 0, 1, {1, 0}, 3, 7};
      return true;
    case 4:
      s = KSpec{3, 2, 2, {0, 1}, 2, 0};
      return true;
    case 6:
      s = KSpec{2, 0, 1, {1, 0}, 2, 9};
      return true;
  }
  return false;
}

// LUSE_d / LDEF_d of one argument (Table 1 offsets composed with the work
// region, '*' = whole extent, clipped; or the absolute sections).
static void arg_region(const Kernel &k, int part, int arg, hd_array *a, int uod, int d, const int64_t *wlo,
                       const int64_t *whi, std::vector<Shape> &out) {
  bool absmode = false;
  for (const auto &kv : k.abs)
    if (std::get<0>(kv.first) == part && std::get<1>(kv.first) == a->id && std::get<3>(kv.first) == uod &&
        !kv.second.empty())
      absmode = true;
  if (absmode) {
    auto it = k.abs.find(std::make_tuple(part, a->id, d, uod));
    if (it != k.abs.end()) out.insert(out.end(), it->second.begin(), it->second.end());
    return;
  }
  for (int o = 0; o < k.noff[arg][uod]; ++o) {
    int32_t off3[3] = {0, 0, 0};
    bool star3[3] = {false, false, false};
    for (int j = 0; j < a->dim; ++j) {
      const int nj = 3 - a->dim + j;
      const int32_t v = k.off[arg][uod][o][j];
      if (v == HD_STAR)
        star3[nj] = true;
      else
        off3[nj] = v;
    }
    Shape s{};
    bool empty = false;
    for (int q = 0; q < 3; ++q) {
      if (star3[q]) {
        s.lo[q] = 0;
        s.hi[q] = a->n[q];
      } else {
        s.lo[q] = std::max<int64_t>(wlo[q] + off3[q], 0);
        s.hi[q] = std::min<int64_t>(whi[q] + off3[q], a->n[q]);
      }
      if (s.lo[q] >= s.hi[q]) empty = true;
    }
    if (!empty) out.push_back(s);
  }
}

static int user_kind(int builtin) {
  switch (builtin) {
    case 1: return 1;
    case 2: return 2;
    case 3: return 3;
    case 4: return 4;
    case 5: return 5;
    case 6: return 6;
  }
  return 0;
}

// Use / def shapes of every distinct array of a call (argument order) and
// the work boxes of its user kernel (tile prefixes left to the caller).
static int prepare_call(const Kernel &k, int part, const std::vector<hd_array *> &A, std::vector<CallArray> &cas,
                        std::vector<WorkBox> &wb) {
  const Partition &pt = R.parts[part];
  for (int i = 0; i < (int)A.size(); ++i) {
    bool seen = false;
    for (auto &c : cas)
      if (c.a == A[i]) seen = true;
    if (seen) continue;
    cas.emplace_back();
    cas.back().a = A[i];
    cas.back().argpos = i;
  }
  for (auto &c : cas)
    for (int i = 0; i < (int)A.size(); ++i) {
      if (A[i] != c.a) continue;
      for (int d = 0; d < pt.ndev; ++d) {
        if (part_dev_empty(pt, d)) continue;
        arg_region(k, part, i, c.a, 0, d, pt.lo[d], pt.hi[d], c.use[d]);
        arg_region(k, part, i, c.a, 1, d, pt.lo[d], pt.hi[d], c.def[d]);
      }
    }
  // every device touching an array gets a window covering its use and def
  // sections; the 2-D stencils also read, unused, the columns of their last
  // 256-column tile past the box, and the matmul and 3-D stencil index whole
  // arrays
  const bool stencil2d = k.builtin == 1 || k.builtin == 5 || k.builtin == 6;
  const bool whole = k.builtin == 3 || k.builtin == 4;
  for (auto &c : cas)
    for (int d = 0; d < kMaxDev; ++d) {
      int64_t lo[3] = {INT64_MAX, INT64_MAX, INT64_MAX}, hi[3] = {INT64_MIN, INT64_MIN, INT64_MIN};
      auto add = [&](const int64_t *l, const int64_t *h) {
        for (int q = 0; q < 3; ++q) {
          lo[q] = std::min(lo[q], l[q]);
          hi[q] = std::max(hi[q], h[q]);
        }
      };
      for (const auto *v : {&c.use[d], &c.def[d]})
        for (const Shape &sh : *v) {
          if (sh.kind == 0) {
            add(sh.lo, sh.hi);
          } else {
            const int64_t l[3] = {0, sh.c[0], std::min(sh.c[1], sh.c[5])};
            const int64_t h[3] = {1, sh.c[4] + 1, std::max(sh.c[3], sh.c[7]) + 1};
            add(l, h);
          }
        }
      const bool box = d < pt.ndev && !part_dev_empty(pt, d);
      if (box) {
        add(pt.lo[d], pt.hi[d]);
        if (stencil2d) {
          const int64_t w = pt.hi[d][2] - pt.lo[d][2];
          const int64_t l[3] = {pt.lo[d][0], pt.lo[d][1] - 1, pt.lo[d][2] - 1};
          const int64_t h[3] = {pt.hi[d][0], pt.hi[d][1] + 1, pt.lo[d][2] + (w + 255) / 256 * 256 + 4};
          add(l, h);
        }
      }
      if (lo[0] == INT64_MAX) continue;
      if (ensure_window(c.a, d, lo, hi, whole) != HD_OK) return g_last_error;
    }
  const int kind = user_kind(k.builtin);
  for (int d = 0; d < pt.ndev; ++d) {
    if (part_dev_empty(pt, d)) continue;
    WorkBox w{};
    w.dev = d;
    w.kind = kind;
    for (int q = 0; q < 3; ++q) {
      w.lo[q] = (int32_t)pt.lo[d][q];
      w.hi[q] = (int32_t)pt.hi[d][q];
    }
    if (k.builtin == 4) {
      w.ain = A[0]->id;
      w.ain2 = A[1]->id;
      w.aout = A[2]->id;
    } else {
      w.aout = A[0]->id;
      w.ain = A[1]->id;
      w.ain2 = A[1]->id;
    }
    wb.push_back(w);
  }
  return HD_OK;
}

extern "C" int hdarray_apply_kernel(const char *kname, int part, int nargs, const hd_arg_t *args) {
  if (!R.inited) return fail(HD_ESTATE);
  Kernel *k = get_kernel(kname);
  if (!k) return fail(HD_EKERNEL);
  if (part < 0 || part >= (int)R.parts.size()) return fail(HD_EINVAL);
  const Partition &pt = R.parts[part];
  KSpec ks;
  if (!kspec(k->builtin, ks)) return fail(HD_EKERNEL);
  // split arrays and scalars; arrays come first in built-in argument lists
  std::vector<hd_array *> A;
  std::vector<double> sc;
  for (int i = 0; i < nargs; ++i) {
    if (args[i].kind == HD_ARG_ARRAY) {
      hd_array *a = get_arr(args[i].v.array);
      if (!a || !sc.empty()) return fail(HD_EINVAL);
      A.push_back(a);
    } else if (args[i].kind == HD_ARG_FLOAT) {
      sc.push_back(args[i].v.f);
    } else if (args[i].kind == HD_ARG_INT) {
      sc.push_back((double)args[i].v.i);
    } else {
      return fail(HD_EINVAL);
    }
  }
  if ((int)A.size() != ks.nargs || (int)sc.size() < ks.nscal) return fail(HD_EINVAL);
  hd_array *ao = A[ks.out];
  for (int i = 0; i < ks.nin; ++i)
    if (A[ks.in[i]] == ao) return fail(HD_EINVAL);
  if (ao->type != 0 && k->builtin != 2) return fail(HD_EINVAL);
  if (ks.dim && ao->dim != ks.dim) return fail(HD_EINVAL);
  if (pt.dim != ao->dim) return fail(HD_EINVAL);
  switch (k->builtin) {
    case 1:
    case 2:
    case 3:
    case 6:
      if (memcmp(A[0]->n, A[1]->n, sizeof(A[0]->n)) || A[0]->esize != A[1]->esize) return fail(HD_EINVAL);
      if (k->builtin != 2 && A[1]->type != 0) return fail(HD_EINVAL);
      break;
    case 5:
      if (memcmp(A[0]->n, A[1]->n, sizeof(A[0]->n)) || A[1]->type != 0 || A[0]->n[1] != A[0]->n[2])
        return fail(HD_EINVAL);
      break;
    case 4:
      if (A[0]->type || A[1]->type || A[0]->dim != 2 || A[1]->dim != 2) return fail(HD_EINVAL);
      if (A[0]->n[2] != A[1]->n[1] || A[2]->n[1] != A[0]->n[1] || A[2]->n[2] != A[1]->n[2]) return fail(HD_EINVAL);
      break;
  }
  for (int d = 0; d < pt.ndev; ++d)
    for (int j = 0; j < 3; ++j)
      if (pt.hi[d][j] > ao->n[j]) return fail(HD_EBOUNDS);
  float coef[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int e = 0; e < 9 && e < (int)sc.size(); ++e) coef[e] = (float)sc[e];
  if (R.recording) {
    if (k->builtin != 1 && k->builtin != 2 && k->builtin != 5) return fail(HD_EINVAL);
    RecCall rc;
    if (prepare_call(*k, part, A, rc.cas, rc.boxes) != HD_OK) return g_last_error;
    R.rec.push_back(std::move(rc));
    return HD_OK;
  }
  // plan cache key
  std::vector<int64_t> key = {1, (int64_t)(k - &R.kernels[0]), part, k->version};
  for (hd_array *a : A) key.push_back(a->id);
  Plan *pl = nullptr;
  auto it = R.plans.find(key);
  if (it != R.plans.end()) {
    pl = it->second;
  } else {
    std::vector<CallArray> cas;
    std::vector<WorkBox> wb;
    if (prepare_call(*k, part, A, cas, wb) != HD_OK) return g_last_error;
    pl = new Plan();
    if (build_plan(cas, pl) != HD_OK) {
      plan_free(pl);
      return g_last_error;
    }
    pl->ukind = user_kind(k->builtin);
    pl->apply = true;
    pl->nbox = (int)wb.size();
    if (pl->ukind == 1 || pl->ukind == 5 || pl->ukind == 6) {
      // one set of work boxes per tile height (tile offsets differ)
      const int ths[5] = {4, 8, 16, 32, 64};
      for (int q = 0; q < 5; ++q) {
        int64_t t0 = 0;
        for (WorkBox &w : wb) {
          w.tile0 = t0;
          t0 += tiles_for(w.kind, w, R.arrays[w.aout]->esize, ths[q]);
        }
        pl->ntj[q] = t0;
        pl->hwbj[q] = wb;
        if (!wb.empty()) HIPCK(hipMemcpy(pl->wbj[q], wb.data(), sizeof(WorkBox) * wb.size(), hipMemcpyHostToDevice));
      }
      pl->vec = true;
      for (const WorkBox &w : wb)
        if ((w.lo[2] & 3) || (R.arrays[w.ain]->n[2] & 3)) pl->vec = false;
      pl->th = 8;
      pl->wb = pl->wbj[1];
      pl->ntiles = pl->ntj[1];
      pl->tkey = {pl->ukind, pl->nbox};
      for (const WorkBox &w : wb)
        for (int q = 0; q < 3; ++q) {
          pl->tkey.push_back(w.lo[q]);
          pl->tkey.push_back(w.hi[q]);
        }
    } else {
      int64_t t0 = 0;
      for (WorkBox &w : wb) {
        w.seg = R.s3d_seg;
        w.tile0 = t0;
        t0 += tiles_for(w.kind, w, R.arrays[w.aout]->esize, pl->th);
      }
      pl->ntiles = t0;
      if (pl->ukind == 4) {
        pl->vec = true;
        for (const WorkBox &w : wb)
          if (!mm_full(w.lo, w.hi, R.arrays[w.ain]->n[2], R.arrays[w.ain2]->n[2])) pl->vec = false;
      }
      if (!wb.empty()) HIPCK(hipMemcpy(pl->wb, wb.data(), sizeof(WorkBox) * wb.size(), hipMemcpyHostToDevice));
    }
    R.plans[key] = pl;
    R.stats.plans_built++;
  }
  R.stats.calls++;
  return enqueue(pl, coef);
}

// ---------------------------------------------------- write/read/reduce
static int part_boxes(int part, hd_array *a, std::vector<int> &devs) {
  if (part < 0 || part >= (int)R.parts.size()) return fail(HD_EINVAL);
  const Partition &pt = R.parts[part];
  if (pt.dim != a->dim) return fail(HD_EINVAL);
  for (int d = 0; d < pt.ndev; ++d) {
    if (part_dev_empty(pt, d)) continue;
    for (int k = 0; k < 3; ++k)
      if (pt.hi[d][k] > a->n[k]) return fail(HD_EBOUNDS);
    devs.push_back(d);
  }
  for (size_t x = 0; x < devs.size(); ++x)
    for (size_t y = x + 1; y < devs.size(); ++y) {
      bool ov = true;
      for (int k = 0; k < 3; ++k)
        if (pt.hi[devs[x]][k] <= pt.lo[devs[y]][k] || pt.hi[devs[y]][k] <= pt.lo[devs[x]][k]) ov = false;
      if (ov) return fail(HD_EINVAL);
    }
  return HD_OK;
}

static Shape part_shape(const Partition &pt, int d) {
  Shape s{};
  for (int k = 0; k < 3; ++k) {
    s.lo[k] = pt.lo[d][k];
    s.hi[k] = pt.hi[d][k];
  }
  return s;
}

// plan for an array-only communication (Read: use by the host; Reduce: use by
// each device of its region; Write: def by each device with the host)
static Plan *io_plan(int op, int part, hd_array *a) {
  std::vector<int64_t> key = {2, op, part, a->id};
  auto it = R.plans.find(key);
  if (it != R.plans.end()) return it->second;
  std::vector<int> devs;
  if (part_boxes(part, a, devs) != HD_OK) return nullptr;
  const Partition &pt = R.parts[part];
  std::vector<CallArray> cas(1);
  cas[0].a = a;
  cas[0].argpos = 0;
  for (int d : devs) {
    if (op == 0) cas[0].use[kHost].push_back(part_shape(pt, d));
    if (op == 1) cas[0].use[d].push_back(part_shape(pt, d));
    if (op == 2 || op == 3) cas[0].def[d].push_back(part_shape(pt, d));
  }
  cas[0].def_flags = op == 2 ? 1 : 0;
  for (int d : devs)
    if (ensure_window(a, d, pt.lo[d], pt.hi[d], false) != HD_OK) return nullptr;
  Plan *pl = new Plan();
  if (build_plan(cas, pl) != HD_OK) {
    plan_free(pl);
    return nullptr;
  }
  std::vector<WorkBox> wb;
  for (int d : devs) {
    WorkBox w{};
    w.dev = d;
    for (int q = 0; q < 3; ++q) {
      w.lo[q] = (int32_t)pt.lo[d][q];
      w.hi[q] = (int32_t)pt.hi[d][q];
    }
    wb.push_back(w);
  }
  pl->nbox = (int)wb.size();
  if (!wb.empty() && hipMemcpy(pl->wb, wb.data(), sizeof(WorkBox) * wb.size(), hipMemcpyHostToDevice) != hipSuccess) {
    fail(HD_EHIP);
    return nullptr;
  }
  R.plans[key] = pl;
  R.stats.plans_built++;
  return pl;
}

static int check_err() {
  int32_t e = 0;
  HIPCK(hipMemcpy(&e, R.counters + 3, 4, hipMemcpyDeviceToHost));
  if (e) {
    HIPCK(hipMemset(R.counters + 3, 0, 4));
    return fail(e);
  }
  return HD_OK;
}

extern "C" int hdarray_sync(void) {
  if (!R.inited) return fail(HD_ESTATE);
  HIPCK(hipStreamSynchronize(R.meta));
  HIPCK(hipStreamSynchronize(R.data));
  return check_err();
}

extern "C" int hdarray_write(hd_array_t *ah, const void *uA, int part) {
  if (!R.inited) return fail(HD_ESTATE);
  hd_array *a = get_arr(ah);
  if (!a || !uA) return fail(HD_EINVAL);
  Plan *pl = io_plan(2, part, a);
  if (!pl) return g_last_error;
  const Partition &pt = R.parts[part];
  // the host buffer may be in use by queued packs / unpacks
  HIPCK(hipStreamSynchronize(R.data));
  const size_t es = a->esize;
  for (int d = 0; d < pt.ndev; ++d) {
    if (part_dev_empty(pt, d)) continue;
    const int64_t *lo = pt.lo[d], *hi = pt.hi[d];
    for (int64_t p = lo[0]; p < hi[0]; ++p) {
      const size_t base = ((size_t)p * a->n[1] + lo[1]) * a->n[2] + lo[2];
      const size_t pitch = a->n[2] * es, w = (hi[2] - lo[2]) * es, rows = hi[1] - lo[1];
      for (size_t r = 0; r < rows; ++r)
        memcpy(a->host + (base + r * a->n[2]) * es, (const char *)uA + (base + r * a->n[2]) * es, w);
      char *dst = a->buf[d] + (p * a->ps[d] + lo[1] * a->rs[d] + lo[2]) * (int64_t)es;
      HIPCK(hipMemcpy2DAsync(dst, a->rs[d] * es, a->host + base * es, pitch, w, rows, hipMemcpyHostToDevice,
                             R.data));
    }
  }
  // GDEF: definitions by each device with the host as a second holder; no
  // communication (the plan has no use rows)
  pl->ukind = 0;
  if (select_inst(pl) != HD_OK) return g_last_error;
  HIPCK(launch_gdef(pl->P, R.d_arrs, R.W, meta_stream()));
  advance_hist(pl);
  advance_bands(pl);
  return HD_OK;
}

extern "C" int hdarray_read(hd_array_t *ah, void *uA, int part) {
  if (!R.inited) return fail(HD_ESTATE);
  hd_array *a = get_arr(ah);
  if (!a || !uA) return fail(HD_EINVAL);
  Plan *pl = io_plan(0, part, a);
  if (!pl) return g_last_error;
  if (enqueue(pl, nullptr) != HD_OK) return g_last_error;
  HIPCK(hipStreamSynchronize(R.data));
  HIPCK(hipStreamSynchronize(R.meta));
  int rc = check_err();
  if (rc != HD_OK) return rc;
  const Partition &pt = R.parts[part];
  const size_t es = a->esize;
  for (int d = 0; d < pt.ndev; ++d) {
    if (part_dev_empty(pt, d)) continue;
    const int64_t *lo = pt.lo[d], *hi = pt.hi[d];
    for (int64_t p = lo[0]; p < hi[0]; ++p)
      for (int64_t r = lo[1]; r < hi[1]; ++r) {
        const size_t base = ((size_t)p * a->n[1] + r) * a->n[2] + lo[2];
        memcpy((char *)uA + base * es, a->host + base * es, (hi[2] - lo[2]) * es);
      }
  }
  return HD_OK;
}

extern "C" int hdarray_reduce(hd_array_t *ah, void *res, hd_reduce_t op, int part) {
  if (!R.inited) return fail(HD_ESTATE);
  hd_array *a = get_arr(ah);
  if (!a || !res || op < HD_SUM || op > HD_MIN) return fail(HD_EINVAL);
  Plan *pl = io_plan(1, part, a);
  if (!pl) return g_last_error;
  if (enqueue(pl, nullptr) != HD_OK) return g_last_error;
  HIPCK(launch_reduce(a->type, op, pl->wb, pl->nbox, R.d_arrs, a->id, R.red_pf, R.red_pi, R.red_res_dev, R.data));
  HIPCK(hipMemcpyAsync(R.red_res_host, R.red_res_dev, 8, hipMemcpyDeviceToHost, R.data));
  HIPCK(hipStreamSynchronize(R.data));
  HIPCK(hipStreamSynchronize(R.meta));
  int rc = check_err();
  if (rc != HD_OK) return rc;
  memcpy(res, R.red_res_host, a->esize);
  return HD_OK;
}

// Reduce with no allocation: the plan of (array, partition) must exist (an
// earlier hdarray_reduce built it, with its workspace and device buffers);
// the partials and the device-side result go to the library's static scratch.
extern "C" int hdarray_reduce_noalloc(hd_array_t *ah, void *res, hd_reduce_t op, int part) {
  if (!R.inited) return fail(HD_ESTATE);
  hd_array *a = get_arr(ah);
  if (!a || !res || op < HD_SUM || op > HD_MIN) return fail(HD_EINVAL);
  const auto it = R.plans.find(std::vector<int64_t>{2, 1, part, a->id});
  if (it == R.plans.end()) return fail(HD_ENOPLAN);
  Plan *pl = it->second;
  if (reduce_scratch_need(pl->nbox) > reduce_scratch_max()) return fail(HD_ECAPACITY);
  // the instance for the arrays' current bands must exist too
  if (select_inst(pl, false) != HD_OK) return g_last_error;
  // phase timers may create events; they stay off for this call
  const int prof = R.prof;
  R.prof = 0;
  const int rc = enqueue(pl, nullptr);
  R.prof = prof;
  if (rc != HD_OK) return g_last_error;
  void *res_dev = nullptr;
  HIPCK(launch_reduce_scratch(R.device, a->type, op, pl->wb, pl->nbox, R.d_arrs, a->id, &res_dev, R.data));
  HIPCK(hipMemcpyAsync(R.red_res_host, res_dev, 8, hipMemcpyDeviceToHost, R.data));
  HIPCK(hipStreamSynchronize(R.data));
  HIPCK(hipStreamSynchronize(R.meta));
  const int rc2 = check_err();
  if (rc2 != HD_OK) return rc2;
  memcpy(res, R.red_res_host, a->esize);
  return HD_OK;
}

// ----------------------------------------------------------------- dumps
static void last_table(MsgRec **tab, MsgHdr **hdr);

extern "C" int hdarray_get_stats(hd_stats_t *st) {
  if (!st) return fail(HD_EINVAL);
  *st = R.stats;
  MsgRec *ltab = nullptr;
  MsgHdr *lhdr = nullptr;
  if (R.inited) last_table(&ltab, &lhdr);
  if (R.inited) {
    int32_t h = 0;
    HIPCK(hipStreamSynchronize(R.meta));
    HIPCK(hipMemcpy(&h, R.counters + 9, 4, hipMemcpyDeviceToHost));
    st->cache_gdef_hits = h;
  }
  if (lhdr) {
    if (hipStreamSynchronize(R.meta) != hipSuccess || hipStreamSynchronize(R.data) != hipSuccess)
      return fail(HD_EHIP);
    MsgHdr h{};
    HIPCK(hipMemcpy(&h, lhdr, sizeof(h), hipMemcpyDeviceToHost));
    st->last_messages = h.nmsg;
    st->last_bytes = h.bytes;
  }
  return HD_OK;
}

extern "C" int64_t hdarray_debug_messages(int64_t *out, int64_t cap) {
  if (!R.inited) return fail(HD_ESTATE);
  if (hdarray_sync() != HD_OK) return g_last_error;
  MsgRec *tab = nullptr;
  MsgHdr *hdr = nullptr;
  last_table(&tab, &hdr);
  if (!tab) return 0;
  MsgHdr h{};
  HIPCK(hipMemcpy(&h, hdr, sizeof(h), hipMemcpyDeviceToHost));
  std::vector<MsgRec> m(h.nmsg);
  if (h.nmsg) HIPCK(hipMemcpy(m.data(), tab, sizeof(MsgRec) * h.nmsg, hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < h.nmsg && i < cap; ++i) {
    int64_t *o = out + 12 * i;
    o[0] = m[i].argpos;
    o[1] = m[i].arr;
    o[2] = m[i].src;
    o[3] = m[i].dst;
    for (int k = 0; k < 3; ++k) {
      o[4 + k] = m[i].lo[k];
      o[7 + k] = m[i].hi[k];
    }
    o[10] = m[i].off;
    o[11] = m[i].bytes;
  }
  return h.nmsg;
}

extern "C" int64_t hdarray_debug_pack(void *out, int64_t cap) {
  if (!R.inited) return fail(HD_ESTATE);
  if (hdarray_sync() != HD_OK) return g_last_error;
  MsgRec *tab = nullptr;
  MsgHdr *hdr = nullptr;
  last_table(&tab, &hdr);
  if (!tab) return 0;
  MsgHdr h{};
  HIPCK(hipMemcpy(&h, hdr, sizeof(h), hipMemcpyDeviceToHost));
  const int64_t n = std::min(h.bytes, cap);
  if (n > 0) HIPCK(hipMemcpy(out, R.staging, n, hipMemcpyDeviceToHost));
  return h.bytes;
}

extern "C" int hdarray_debug_gdef(hd_array_t *ah, int8_t *owner, uint64_t *holders) {
  hd_array *a = get_arr(ah);
  if (!a) return fail(HD_EINVAL);
  if (hdarray_sync() != HD_OK) return g_last_error;
  const int64_t rows = a->n[0] * a->n[1];
  std::vector<int32_t> cnt(rows);
  std::vector<Ivl> iv((size_t)rows * a->cap);
  HIPCK(hipMemcpy(cnt.data(), a->cnt, 4 * rows, hipMemcpyDeviceToHost));
  HIPCK(hipMemcpy(iv.data(), a->ivl, sizeof(Ivl) * rows * a->cap, hipMemcpyDeviceToHost));
  for (int64_t g = 0; g < rows; ++g) {
    // the row's list is stored at its band's first row
    const int64_t p = g / a->n[1], r = g % a->n[1];
    const int64_t src = *(std::upper_bound(a->pbrk.begin(), a->pbrk.end(), p) - 1) * a->n[1] +
                        *(std::upper_bound(a->rbrk.begin(), a->rbrk.end(), r) - 1);
    const Ivl *L = iv.data() + src * a->cap;
    for (int i = 0; i < cnt[src]; ++i) {
      const int64_t e = (i + 1 < cnt[src]) ? L[i + 1].start : a->n[2];
      for (int64_t c = L[i].start; c < e; ++c) {
        if (owner) owner[g * a->n[2] + c] = (int8_t)L[i].owner;
        if (holders) holders[g * a->n[2] + c] = L[i].holders;
      }
    }
  }
  return HD_OK;
}

extern "C" int hdarray_debug_device_buffer(hd_array_t *ah, int dev, void *out) {
  hd_array *a = get_arr(ah);
  if (!a || !out || dev < 0 || dev > kHost) return fail(HD_EINVAL);
  if (hdarray_sync() != HD_OK) return g_last_error;
  if (dev == kHost) {
    memcpy(out, a->host, (size_t)a->N * a->esize);
    return HD_OK;
  }
  const size_t es = a->esize;
  memset(out, 0, (size_t)a->N * es);
  if (!a->buf[dev]) return HD_OK;
  const int64_t *lo = a->wlo[dev], *hi = a->whi[dev];
  for (int64_t p = lo[0]; p < hi[0]; ++p)
    HIPCK(hipMemcpy2D((char *)out + ((p * a->n[1] + lo[1]) * a->n[2] + lo[2]) * es, a->n[2] * es,
                      a->buf[dev] + (p * a->ps[dev] + lo[1] * a->rs[dev] + lo[2]) * es, a->rs[dev] * es,
                      (hi[2] - lo[2]) * es, hi[1] - lo[1], hipMemcpyDeviceToHost));
  return HD_OK;
}

extern "C" void *hdarray_device_ptr(hd_array_t *ah, int dev) {
  hd_array *a = get_arr(ah);
  if (!a || dev < 0 || dev >= kMaxDev) {
    fail(HD_EINVAL);
    return nullptr;
  }
  if (ensure_full(a, dev) != HD_OK) return nullptr;
  return a->buf[dev];
}

// ------------------------------------------------------------------ batch

struct Batch {
  Plan pl;
  std::vector<WorkBox> boxes;
  WorkBox *d_wb = nullptr;
  int32_t *d_tbox = nullptr;  // box of every tile (sized for the smallest tile height)
  int64_t tbox_cap = 0;
  int64_t ntiles = 0;
  int th = 16, hf = 1, occ = 2, grid = 0;
  MsgRec *tab = nullptr;
  MsgHdr *hdr = nullptr;
  int64_t tab_cap = 0;
  unsigned *bar = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t epoch = -1;
  int gth = 0, ghf = 0, ggrid = 0;
  const PlanInst *ginst = nullptr;  // the plan instance the graph was captured with
};

static void drop_graph(Batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

static void free_batches() {
  for (Batch *b : R.batches) {
    if (!b) continue;
    drop_graph(b);
    for (auto &kv : b->pl.insts) free_inst(kv.second);
    for (auto &kv : b->pl.mats) dfree(kv.second.first);
    dfree(b->pl.mem);
    dfree(b->d_wb);
    dfree(b->d_tbox);
    dfree(b->tab);
    dfree(b->hdr);
    dfree(b->bar);
    delete b;
  }
  R.batches.clear();
  R.rec.clear();
  R.recording = false;
}

static void last_table(MsgRec **tab, MsgHdr **hdr) {
  *tab = nullptr;
  *hdr = nullptr;
  if (R.last_batch >= 0 && R.last_batch < (int)R.batches.size()) {
    *tab = R.batches[R.last_batch]->tab;
    *hdr = R.batches[R.last_batch]->hdr;
  } else if (R.last_ptab) {
    *tab = R.last_ptab;
    *hdr = R.last_phdr;
  } else if (R.last_tab >= 0) {
    *tab = R.tab[R.last_tab];
    *hdr = R.hdr[R.last_tab];
  }
}

// Tiles of one box of a batch: one-wave tiles of th rows (hf 0, 1) or
// four waves stacked down 4 * th rows (hf 2; a copy box's one-wave tiles
// four to a workgroup).
static int64_t batch_tiles(const WorkBox &w, int th, int hf) {
  const int esize = R.arrays[w.aout]->esize;
  if (hf != 2) return tiles_for(w.kind, w, esize, th);
  if (w.kind == 2) return (tiles_for(w.kind, w, esize, th) + 3) / 4;
  return tiles_for(w.kind, w, esize, 4 * th);
}

static int batch_config(Batch *b, int th, int hf, int occ) {
  int64_t t0 = 0;
  for (WorkBox &w : b->boxes) {
    w.tile0 = t0;
    t0 += batch_tiles(w, th, hf);
  }
  b->ntiles = t0;
  // one workgroup per tile in the user-kernel launch
  if (t0 > b->tbox_cap || t0 > INT32_MAX) return fail(HD_EINVAL);
  std::vector<int32_t> tb((size_t)t0);
  for (size_t i = 0; i < b->boxes.size(); ++i) {
    const int64_t e = i + 1 < b->boxes.size() ? b->boxes[i + 1].tile0 : t0;
    std::fill(tb.begin() + b->boxes[i].tile0, tb.begin() + e, (int32_t)i);
  }
  HIPCK(hipStreamSynchronize(R.data));
  if (!b->boxes.empty())
    HIPCK(hipMemcpy(b->d_wb, b->boxes.data(), sizeof(WorkBox) * b->boxes.size(), hipMemcpyHostToDevice));
  if (t0 > 0) HIPCK(hipMemcpy(b->d_tbox, tb.data(), sizeof(int32_t) * t0, hipMemcpyHostToDevice));
  b->th = th;
  b->hf = hf;
  b->occ = occ;
  b->grid = batch_max_blocks(occ);
  if (b->grid <= 0) return fail(HD_EHIP);
  return HD_OK;
}

extern "C" int hdarray_batch_begin(void) {
  if (!R.inited) return fail(HD_ESTATE);
  if (R.recording) return fail(HD_ESTATE);
  R.recording = true;
  R.rec.clear();
  return HD_OK;
}

extern "C" int hdarray_batch_end(void) {
  if (!R.inited || !R.recording) return fail(HD_ESTATE);
  R.recording = false;
  std::vector<CallArray> all;
  std::vector<WorkBox> boxes;
  std::vector<int> seen;
  for (RecCall &c : R.rec) {
    for (CallArray &ca : c.cas) {
      if (std::find(seen.begin(), seen.end(), ca.a->id) != seen.end()) {
        R.rec.clear();
        return fail(HD_EINVAL);  // calls of a batch must touch distinct arrays
      }
      seen.push_back(ca.a->id);
    }
  }
  size_t ncas = 0;
  for (RecCall &c : R.rec) ncas += c.cas.size();
  if (ncas > (size_t)kCompactCarr) {
    R.rec.clear();
    return fail(HD_EINVAL);  // more array arguments than one compaction handles
  }
  for (RecCall &c : R.rec) {
    for (CallArray &ca : c.cas) all.push_back(std::move(ca));
    boxes.insert(boxes.end(), c.boxes.begin(), c.boxes.end());
  }
  R.rec.clear();
  Batch *b = new Batch();
  if (build_plan(all, &b->pl) != HD_OK) {
    for (auto &kv : b->pl.insts) free_inst(kv.second);
    for (auto &kv : b->pl.mats) dfree(kv.second.first);
    dfree(b->pl.mem);
    delete b;
    return g_last_error;
  }
  b->boxes = boxes;
  b->tab_cap = R.ws_items;
  b->tab = (MsgRec *)dalloc(sizeof(MsgRec) * b->tab_cap);
  b->hdr = (MsgHdr *)dalloc(sizeof(MsgHdr));
  b->bar = (unsigned *)dalloc(512);  // barrier counter, then 32 phase-clock stamps at byte 256
  b->d_wb = (WorkBox *)dalloc(sizeof(WorkBox) * (boxes.size() + 1));
  // the tile -> box table, sized for the largest tile count of the tile
  // heights the batch may be configured with
  for (int th : {4, 8, 16}) {
    int64_t nt = 0;
    for (const WorkBox &w : boxes) nt += tiles_for(w.kind, w, R.arrays[w.aout]->esize, th);
    b->tbox_cap = std::max(b->tbox_cap, nt);
  }
  b->d_tbox = (int32_t *)dalloc(sizeof(int32_t) * (b->tbox_cap + 1));
  if (!b->tab || !b->hdr || !b->bar || !b->d_wb || !b->d_tbox) return fail(HD_ENOMEM);
  HIPCK(hipMemset(b->hdr, 0, sizeof(MsgHdr)));
  HIPCK(hipMemset(b->bar, 0, 256));
  if (batch_config(b, 16, 1, 2) != HD_OK) return g_last_error;
  R.batches.push_back(b);
  R.stats.plans_built++;
  return (int)R.batches.size() - 1;
}

static int batch_capture(Batch *b) {
  drop_graph(b);
  // the batch may have grown the workspace: its plan was built before
  int dev = 0, rate_khz = 0;
  HIPCK(hipGetDevice(&dev));
  if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || rate_khz <= 0)
    rate_khz = 100000;
  BatchArgs a{};
  a.P = b->pl.P;
  a.L1 = make_level(1, b->pl.P);
  a.L2 = make_level(2, b->pl.P);
  a.W = R.W;
  a.A = R.d_arrs;
  a.tab = b->tab;
  a.hdr = b->hdr;
  a.tab_cap = b->tab_cap;
  a.stg = (uint32_t *)R.staging;
  a.wb = b->d_wb;
  a.tbox = b->d_tbox;
  a.nbox = (int)b->boxes.size();
  a.ntiles = b->ntiles;
  a.bar = b->bar;
  a.spin_limit = (int64_t)rate_khz * 2000;  // two seconds
  a.clk = reinterpret_cast<int64_t *>(reinterpret_cast<char *>(b->bar) + 256);
  a.cs = R.cscratch;
  HIPCK(hipStreamBeginCapture(R.cap, hipStreamCaptureModeRelaxed));
  hipError_t e = launch_batch(a, b->th, b->hf, b->grid, R.cap);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(R.cap, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(HD_EHIP);
  }
  b->graph = g;
  HIPCK(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
  b->epoch = R.ws_epoch;
  b->gth = b->th;
  b->ghf = b->hf;
  b->ggrid = b->grid;
  b->ginst = b->pl.cur;
  return HD_OK;
}

extern "C" int hdarray_batch_run(int id) {
  if (!R.inited || R.recording) return fail(HD_ESTATE);
  if (id < 0 || id >= (int)R.batches.size() || !R.batches[id]) return fail(HD_EINVAL);
  Batch *b = R.batches[id];
  // the instance for the arrays' current bands (its band-list copies go
  // ahead on the metadata stream); the graph holds one instance's records
  if (select_inst(&b->pl) != HD_OK) return g_last_error;
  if (!b->exec || b->epoch != R.ws_epoch || b->gth != b->th || b->ghf != b->hf || b->ggrid != b->grid ||
      b->ginst != b->pl.cur)
    if (batch_capture(b) != HD_OK) return g_last_error;
  // ordered after the metadata work of earlier calls, and before later ones
  HIPCK(hipEventRecord(R.ev_meta, R.meta));
  HIPCK(hipStreamWaitEvent(R.data, R.ev_meta, 0));
  {
    PhaseTimer tm(3, R.data);
    HIPCK(hipGraphLaunch(b->exec, R.data));
  }
  HIPCK(hipEventRecord(R.ev_data, R.data));
  HIPCK(hipStreamWaitEvent(R.meta, R.ev_data, 0));
  advance_hist(&b->pl);
  advance_bands(&b->pl);
  R.last_ptab = nullptr;
  R.last_phdr = nullptr;
  R.last_batch = id;
  R.stats.calls++;
  return HD_OK;
}

extern "C" int hdarray_batch_phase_us(int id, double *us, int max) {
  if (!R.inited || !us || max <= 0) return fail(HD_EINVAL);
  if (id < 0 || id >= (int)R.batches.size() || !R.batches[id] || !R.batches[id]->exec) return fail(HD_EINVAL);
  const Batch *b = R.batches[id];
  HIPCK(hipStreamSynchronize(R.data));
  int64_t clk[32];
  HIPCK(hipMemcpy(clk, reinterpret_cast<const char *>(b->bar) + 256, sizeof(clk), hipMemcpyDeviceToHost));
  int dev = 0, rate_khz = 0;
  HIPCK(hipGetDevice(&dev));
  if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || rate_khz <= 0)
    rate_khz = 100000;
  const int nst = b->pl.P.has3d ? 12 : 8;
  int n = 0;
  for (int k = 1; k < nst && n < max; ++k) us[n++] = (double)(clk[k] - clk[k - 1]) * 1e3 / rate_khz;
  return n;
}

extern "C" int hdarray_batch_autotune(const int *ids, int n, int reps) {
  if (!R.inited || !ids || n <= 0 || reps <= 0) return fail(HD_EINVAL);
  for (int i = 0; i < n; ++i)
    if (ids[i] < 0 || ids[i] >= (int)R.batches.size()) return fail(HD_EINVAL);
  // rows per wave x tile shape (0: one wave, tiles down columns first; 1:
  // one wave, along rows; 2: four waves stacked) x workgroups per CU of
  // the persistent kernel (fewer make cheaper grid barriers, more run the
  // metadata phases wider)
  const int ths[3] = {4, 8, 16}, hfs[3] = {0, 1, 2}, occs[3] = {1, 2, 4};
  hipEvent_t e0, e1;
  HIPCK(hipEventCreate(&e0));
  HIPCK(hipEventCreate(&e1));
  float best = 1e30f;
  int bth = 8, bhf = 0, bocc = 2;
  for (int occ : occs)
  for (int th : ths)
    for (int hf : hfs) {
      if (hf == 2 && th != 4) continue;  // the stacked shape has four rows per wave
      for (int i = 0; i < n; ++i)
        if (batch_config(R.batches[ids[i]], th, hf, occ) != HD_OK) return g_last_error;
      for (int i = 0; i < n; ++i)
        if (hdarray_batch_run(ids[i]) != HD_OK) return g_last_error;
      HIPCK(hipEventRecord(e0, R.data));
      for (int r = 0; r < reps; ++r)
        for (int i = 0; i < n; ++i)
          if (hdarray_batch_run(ids[i]) != HD_OK) return g_last_error;
      HIPCK(hipEventRecord(e1, R.data));
      HIPCK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        bth = th;
        bhf = hf;
        bocc = occ;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (int i = 0; i < n; ++i)
    if (batch_config(R.batches[ids[i]], bth, bhf, bocc) != HD_OK) return g_last_error;
  int rc = hdarray_sync();
  if (rc != HD_OK) return rc;
  return (bocc << 16) | (bth << 8) | bhf;
}

// ---------------------------------------------------------------- adjoint
extern "C" int hdarray_apply_adjoint(const char *kname, int part, hd_array_t *dinh, hd_array_t *douth,
                                     hd_array_t *uh, const float *coef, double *cbar) {
  if (!R.inited) return fail(HD_ESTATE);
  Kernel *k = get_kernel(kname);
  if (!k) return fail(HD_EKERNEL);
  if (k->builtin != 3) return fail(HD_EKERNEL);
  hd_array *din = get_arr(dinh), *dout = get_arr(douth), *u = get_arr(uh);
  if (!din || !dout || !u || !coef || part < 0 || part >= (int)R.parts.size()) return fail(HD_EINVAL);
  if (din == dout || din == u || dout == u) return fail(HD_EINVAL);
  for (hd_array *a : {din, dout, u})
    if (a->type != 0 || a->dim != 3 || memcmp(a->n, u->n, sizeof(u->n))) return fail(HD_EINVAL);
  const Partition &pt = R.parts[part];
  if (pt.dim != 3) return fail(HD_EINVAL);
  for (int d = 0; d < pt.ndev; ++d)
    for (int j = 0; j < 3; ++j)
      if (pt.hi[d][j] > u->n[j]) return fail(HD_EBOUNDS);
  std::vector<int64_t> key = {3, (int64_t)(k - &R.kernels[0]), part, k->version, din->id, dout->id, u->id};
  Plan *pl = nullptr;
  auto it = R.plans.find(key);
  if (it != R.plans.end()) {
    pl = it->second;
  } else {
    std::vector<CallArray> cas(1);
    cas[0].a = din;
    cas[0].argpos = 0;
    cas[0].no_holders = true;
    std::vector<WorkBox> wb;
    for (int d = 0; d < pt.ndev; ++d) {
      if (part_dev_empty(pt, d)) continue;
      // the use region of the forward input, on the cotangent array
      arg_region(*k, part, 1, u, 0, d, pt.lo[d], pt.hi[d], cas[0].use[d]);
      cas[0].def[d].push_back(part_shape(pt, d));
      for (hd_array *a : {din, dout, u})
        if (ensure_full(a, d) != HD_OK) return g_last_error;
      WorkBox w{};
      w.dev = d;
      w.kind = 3;
      for (int q = 0; q < 3; ++q) {
        w.lo[q] = (int32_t)pt.lo[d][q];
        w.hi[q] = (int32_t)pt.hi[d][q];
      }
      w.aout = din->id;
      w.ain = dout->id;
      w.ain2 = u->id;
      wb.push_back(w);
    }
    pl = new Plan();
    if (build_plan(cas, pl) != HD_OK) {
      plan_free(pl);
      return g_last_error;
    }
    int64_t t0 = 0;
    for (WorkBox &w : wb) {
      w.seg = R.s3d_seg;
      w.tile0 = t0;
      t0 += adj_tiles(w, u->n);
    }
    pl->adjoint = true;
    pl->nbox = (int)wb.size();
    pl->ntiles = t0;
    pl->part = (double *)dalloc(sizeof(double) * 8 * (t0 + 1));
    if (!pl->part) return fail(HD_ENOMEM);
    if (!wb.empty()) HIPCK(hipMemcpy(pl->wb, wb.data(), sizeof(WorkBox) * wb.size(), hipMemcpyHostToDevice));
    R.plans[key] = pl;
    R.stats.plans_built++;
  }
  R.adj_cbar = cbar;
  R.stats.calls++;
  return enqueue(pl, coef);
}

// The partition's regions of a as boxes for k_ext_copy (built once per plan).
static int ext_boxes(Plan *pl, int part, hd_array *a) {
  if (pl->xn >= 0) return HD_OK;
  const Partition &pt = R.parts[part];
  std::vector<WorkBox> v;
  int64_t rows = 0;
  for (int d = 0; d < pt.ndev; ++d) {
    if (part_dev_empty(pt, d)) continue;
    WorkBox w{};
    w.dev = d;
    w.aout = w.ain = a->id;
    for (int q = 0; q < 3; ++q) {
      w.lo[q] = (int32_t)pt.lo[d][q];
      w.hi[q] = (int32_t)pt.hi[d][q];
    }
    w.tile0 = rows;
    rows += (int64_t)(w.hi[0] - w.lo[0]) * (w.hi[1] - w.lo[1]);
    v.push_back(w);
  }
  WorkBox *dst = pl->wbj[2];
  if (!v.empty()) HIPCK(hipMemcpy(dst, v.data(), sizeof(WorkBox) * v.size(), hipMemcpyHostToDevice));
  pl->xn = (int)v.size();
  pl->xrows = rows;
  return HD_OK;
}

extern "C" int hdarray_write_device(hd_array_t *ah, const void *dptr, int part) {
  if (!R.inited) return fail(HD_ESTATE);
  hd_array *a = get_arr(ah);
  if (!a || !dptr) return fail(HD_EINVAL);
  Plan *pl = io_plan(3, part, a);
  if (!pl) return g_last_error;
  if (ext_boxes(pl, part, a) != HD_OK) return g_last_error;
  // every device's region in one launch (rows of the regions, in device order)
  HIPCK(launch_ext_copy(pl->wbj[2], pl->xn, pl->xrows, R.d_arrs, a->id, const_cast<void *>(dptr), 0, R.data));
  if (select_inst(pl) != HD_OK) return g_last_error;
  HIPCK(launch_gdef(pl->P, R.d_arrs, R.W, meta_stream()));
  advance_hist(pl);
  advance_bands(pl);
  return HD_OK;
}

extern "C" int hdarray_read_device(hd_array_t *ah, void *dptr, int part) {
  if (!R.inited) return fail(HD_ESTATE);
  hd_array *a = get_arr(ah);
  if (!a || !dptr) return fail(HD_EINVAL);
  Plan *pl = io_plan(1, part, a);
  if (!pl) return g_last_error;
  if (enqueue(pl, nullptr) != HD_OK) return g_last_error;
  if (ext_boxes(pl, part, a) != HD_OK) return g_last_error;
  HIPCK(launch_ext_copy(pl->wbj[2], pl->xn, pl->xrows, R.d_arrs, a->id, dptr, 1, R.data));
  return HD_OK;
}

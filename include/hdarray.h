/*
 * hdarray.h — C ABI of the MI355X HDArray runtime (libhdarray.so).
 *
 * The runtime implements the HDArray interface of Cho, Kwon & Midkiff,
 * "HDArray: Parallel Array Interface for Distributed Heterogeneous Devices"
 * (arXiv 1809.05657).  One GPU holds up to 63 logical devices ("partitions");
 * each (array, device) pair owns a full-extent buffer in HBM, as in the
 * paper's Create (Sec. 3.1).  Every ApplyKernel derives the communication set
 * from the last-definer map (GDEF) and the use sections (LUSE) on the GPU,
 * packs and unpacks the messages, runs the kernel over all partitions in one
 * launch and updates GDEF from the def sections (LDEF) — Sec. 2.2, Eq. 1-4.
 *
 * Conventions used by every call:
 *   - Endpoints: logical devices 0..62; HD_HOST (63) is the host.
 *   - Coordinates: every rectangle is half-open [lo, hi) per dimension (the
 *     partition clause of Sec. 3, Listing 1, shares the cut point between
 *     neighbouring devices).  Trapezoid corners are inclusive element
 *     positions.
 *   - Arrays are row-major, 1 to 3 dimensions, element type "float" (fp32),
 *     "int" (int32) or "double" (fp64).  Built-in kernels compute in fp32.
 *   - Ownership: the library owns every hd_array_t and every device buffer;
 *     hdarray_exit() frees them.  User arrays (uA) stay owned by the caller
 *     and are not retained after a call returns.
 *   - Streams: data movement and kernels are enqueued on the stream given to
 *     hdarray_set_stream() (default: the null stream); communication-set
 *     derivation and GDEF updates run on an internal stream ordered with it
 *     by events.  Only Read, Reduce, hdarray_sync() and the debug dumps wait
 *     for the GPU.
 *   - Errors: functions return 0 (or a non-negative id) on success and a
 *     negative HD_E* code on failure; hdarray_create() returns NULL.  The
 *     paper's void functions keep their semantics through
 *     hdarray_last_error().  Errors raised by device code (capacity of the
 *     per-row GDEF lists) are reported by the next synchronising call.
 *   - Not thread-safe: one host thread drives the runtime (the paper's SPMD
 *     model, Sec. 2.1).
 */
#ifndef HDARRAY_H
#define HDARRAY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HD_HOST 63
#define HD_MAX_DEVICES 63
/* '*' in an offset: the whole array extent in that dimension (Sec. 3, Table 1) */
#define HD_STAR INT32_MIN

/* error codes */
#define HD_OK 0
#define HD_EINVAL (-1)    /* bad argument, unknown id, mismatched shapes */
#define HD_EBOUNDS (-2)   /* a section or region outside the array */
#define HD_ERACE (-3)     /* def sections of two devices overlap in one call */
#define HD_EKERNEL (-4)   /* unknown kernel name or built-in */
#define HD_ENOMEM (-5)    /* device or host allocation failed */
#define HD_EHIP (-6)      /* a HIP runtime call failed */
#define HD_ESTATE (-7)    /* runtime not initialised / already shut down */
#define HD_ECAPACITY (-8) /* a per-row GDEF list or a work pool overflowed */
#define HD_ENOPLAN (-9)   /* no-allocation call without the plan an earlier call built */

typedef struct hd_array hd_array_t;

/* Table 2, PART_T */
typedef enum { HD_ROW = 0, HD_COL = 1, HD_BLOCK = 2 } hd_part_t;
/* Table 2, REDUCE_OP */
typedef enum { HD_SUM = 0, HD_PROD = 1, HD_MAX = 2, HD_MIN = 3 } hd_reduce_t;

/* A kernel argument: an array handle or a scalar. */
typedef enum { HD_ARG_ARRAY = 0, HD_ARG_FLOAT = 1, HD_ARG_INT = 2 } hd_arg_kind_t;
typedef struct {
  int32_t kind; /* hd_arg_kind_t */
  int32_t pad;
  union {
    hd_array_t *array;
    double f;
    int64_t i;
  } v;
} hd_arg_t;

/* ------------------------------------------------------------ Table 2 */

/* HDArrayInit (Sec. 3.1, Table 2).  Attaches to the current HIP device and
 * creates the runtime's internal stream.  kpath names the kernel source in
 * the paper; here kernels are built in (see hdarray_register_kernel), so kpath
 * may be NULL.  dpath (device info file) is unused on one GPU and may be NULL.
 * argv may carry "--hd-row-cap=N" (capacity of a per-row GDEF list,
 * 4..256, default 64; a row needing more intervals raises HD_ECAPACITY) and
 * "--hd-windows=compact" (each device keeps, per 2-D array, only a box of
 * the array around every section it holds or its kernels read, instead of
 * a whole-array buffer; less memory, slower 2-D stencils) or
 * "--hd-windows=full" (the default).
 * Environment, read here: HD_SERIAL=1 runs the communication-set
 * derivation and GDEF update on the data stream instead of overlapping
 * them (a measurement aid); HD_JACOBI_ROWS=4|8|16|32|64, HD_JACOBI_WAVES=1|4
 * and HD_JACOBI_ORDER=0|1 fix the tile shape of the 2-D stencil kernels as
 * hdarray_set_stencil_shape does; HD_S3D_SEG=N sets the number of planes
 * each row of the 3-D stencil kernels marches through (default 32);
 * HD_EVENT_SCOPE=system makes the runtime's inter-stream events use HIP's
 * default system-scope release instead of a device-scope one, and
 * HD_RUNS_WAVE_MAX=N finds the runs of levels with fewer than N use rows
 * with one wave per row instead of one lane per row, and HD_FUSED_META=0
 * derives small plan instances (at most 64 slices and groups) with the
 * general kernel sequence instead of the two-launch form (measurement
 * aids).  Returns the HIP device id (>= 0) or a negative error. */
int hdarray_init(int argc, char **argv, const char *kpath, const char *dpath);

/* HDArrayExit: waits for the GPU, frees every array, plan and buffer. */
void hdarray_exit(void);

/* HDArrayShowDeviceInfo: prints the GPU's name, CU count and memory. */
void hdarray_show_device_info(int dev_id);

/* HDArrayCreate (Sec. 3.1): allocates the host buffer (pinned) and GDEF; the
 * device buffers of a logical device are allocated when that device first
 * touches the array.  type is "float", "int" or "double"; sizes[dim] are the
 * extents.  uA (optional, dense row-major, sizes elements) is copied into the
 * host buffer; GDEF starts with the host as owner and only holder of every
 * element.  Returns NULL on error (see hdarray_last_error). */
hd_array_t *hdarray_create(const char *sym, const char *type, const void *uA, int dim, const int64_t *sizes);

/* Runtime-wide id of an array (creation order, from 0), or -1. */
int hdarray_array_id(const hd_array_t *a);

/* HDArrayPartition (Table 2): even split of the work-item region
 * [region_lo, region_hi) of an index space of extents sizes[dim] over ndev
 * logical devices.  ROW splits dimension 0, COL dimension 1 (dimension 0 for
 * 1-D), BLOCK a balanced grid with non-increasing factors from dimension 0,
 * device ids row-major over the grid.  Along a dimension of length N starting
 * at L, grid slot i of P gets [L + floor(i*N/P), L + floor((i+1)*N/P)).
 * Returns the partition id (>= 0). */
int hdarray_partition(hd_part_t type, int dim, const int64_t *sizes, const int64_t *region_lo,
                      const int64_t *region_hi, int ndev);

/* Partition clause (Sec. 3, Listing 1): device d's work region is
 * [lo[d*dim..], hi[d*dim..]).  Empty regions (lo == hi) are allowed. */
int hdarray_partition_manual(int dim, int ndev, const int64_t *lo, const int64_t *hi);

/* Work region of device dev in normalised (planes, rows, cols) coordinates. */
int hdarray_partition_region(int part, int dev, int64_t *lo3, int64_t *hi3);

/* Kernel table entry (replaces the frontend's file M, Sec. 4.1).  builtin is
 * one of "jacobi2d", "copy", "matmul", "tri2d", "stencil3d7", "conv2d9".
 * Argument order: jacobi2d/tri2d/copy/stencil3d7/conv2d9 (out, in), matmul
 * (A, B, C).  stencil3d7 takes 7 float scalars after the arrays (centre,
 * -i, +i, -j, +j, -k, +k); conv2d9 (the 8-neighbour convolution of
 * Sec. 5.1) takes 9: the 3 x 3 weights row by row, out[i][j] = the
 * first-rounded product w0*in[i-1][j-1] followed by one fused multiply-add
 * per further window cell in the same order, boundary cells copied. */
int hdarray_register_kernel(const char *kname, const char *builtin);

/* use / def offset clauses (Table 1): noff offsets, each given as 3 int32
 * (only the array's dim first entries are read), HD_STAR = whole dimension.
 * use_or_def: 0 = use, 1 = def.  LUSE_d (LDEF_d) is the union of the work
 * region of d shifted by each offset, clipped to the array. */
int hdarray_set_offsets(const char *kname, int arg, int use_or_def, int noff, const int32_t *off);

/* HDArraySetAbsoluteUse / SetAbsoluteDef (Table 2): one more section
 * [lo, hi) (dim entries each) of array a for device dev, kernel kname,
 * partition part.  Sections accumulate per (kernel, partition, array,
 * device); once any exists for (kernel, partition, array), they replace the
 * offsets of that array for that kernel and partition. */
int hdarray_set_absolute_use(const char *kname, int part, hd_array_t *a, int dev, int dim, const int64_t *lo,
                             const int64_t *hi);
int hdarray_set_absolute_def(const char *kname, int part, hd_array_t *a, int dev, int dim, const int64_t *lo,
                             const int64_t *hi);

/* HDArraySetTrapezoidUse / SetTrapezoidDef (Table 2), 2-D arrays only:
 * corners = {UL.row, UL.col, UR.row, UR.col, BL.row, BL.col, BR.row, BR.col},
 * inclusive; UL.row == UR.row and BL.row == BR.row (else HD_EINVAL).  Row r
 * in [r0, r1] spans [UL.col + floor((r-r0)(BL.col-UL.col)/(r1-r0)),
 * UR.col + floor((r-r0)(BR.col-UR.col)/(r1-r0))], clipped to the array. */
int hdarray_set_trapezoid_use(const char *kname, int part, hd_array_t *a, int dev, const int64_t *corners);
int hdarray_set_trapezoid_def(const char *kname, int part, hd_array_t *a, int dev, const int64_t *corners);

/* Drops the absolute / trapezoid sections of (kernel, part, array); dev < 0
 * means every device. */
int hdarray_clear_sections(const char *kname, int part, hd_array_t *a, int dev);

/* HDArrayApplyKernel (Sec. 3.1, Fig. 3 logic): derive LUSE/LDEF, the
 * communication set (Eq. 1-2) on the GPU, pack, unpack, run the kernel on
 * every device of the partition in one launch, update GDEF (Eq. 3-4, a
 * definition by d leaves d the only holder).  Asynchronous. */
int hdarray_apply_kernel(const char *kname, int part, int nargs, const hd_arg_t *args);

/* HDArrayWrite (Table 2): device d receives uA's elements inside its region
 * of partition part; d becomes their owner, d and the host their holders.
 * Overlapping regions give HD_EINVAL.  uA is dense, the array's full extent. */
int hdarray_write(hd_array_t *a, const void *uA, int part);

/* HDArrayRead (Table 2): the host uses the union of the partition's regions;
 * whatever it does not hold comes from the owner; the values are copied into
 * uA (dense, full extent; elements outside the regions are not touched).
 * Synchronises. */
int hdarray_read(hd_array_t *a, void *uA, int part);

/* HDArrayReduce (Table 2): each device uses its region (communication
 * first), reduces it, and the partial results are combined in device order.
 * float/double accumulate in fp64; int SUM/PROD wrap modulo 2^32.  res
 * receives one element of the array's type.  Synchronises. */
int hdarray_reduce(hd_array_t *a, void *res, hd_reduce_t op, int part);

/* Reduce without allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments, result and error behaviour as
 * hdarray_reduce, with two differences: the partial results and the
 * device-side result live in a static device array of the library (64 KiB
 * per GPU, held until the process ends; a partition of n non-empty boxes
 * needs 256 + 768 n bytes, always within it for the 63 devices a partition
 * may have; more would give HD_ECAPACITY), and the communication plan of
 * (a, part) must already exist: an earlier hdarray_reduce on the same array
 * and partition builds it, otherwise HD_ENOPLAN and nothing runs.  No
 * device or host memory is allocated.  Every call on one GPU shares that
 * GPU's array, so calls that overlap on one GPU (other host threads) race.
 * Phase timing (hdarray_profile) is suspended during the call.
 * Synchronises. */
int hdarray_reduce_noalloc(hd_array_t *a, void *res, hd_reduce_t op, int part);

/* ---------------------------------------------------------- extensions */

/* Batched step.  Between hdarray_batch_begin() and hdarray_batch_end(),
 * hdarray_apply_kernel() validates and records its call instead of running
 * it.  The recorded calls must touch pairwise distinct arrays and use the
 * built-ins jacobi2d, tri2d or copy, with at most 1024 array arguments in
 * total (HD_EINVAL otherwise).  hdarray_batch_end() returns a batch id;
 * hdarray_batch_run(id) enqueues one execution of every recorded call —
 * communication sets, packs, unpacks, GDEF updates and kernels — as one
 * HIP graph replay: a persistent kernel for the communication sets, packs,
 * unpacks and GDEF updates (phases separated by grid-wide barriers with a
 * bounded wait), then one launch of the user kernels of every call (one
 * wave per tile).  Results are bit-identical to running the calls one by
 * one.  Within a batch a use row may produce at most 64 runs and a GDEF row
 * update at most 256 interval boundaries (the per-workgroup scratch is kept
 * small so that four workgroups share a CU); beyond that the next
 * synchronising call returns HD_ECAPACITY.  A barrier that times out
 * (workgroups not co-resident) makes the launch exit early; the next
 * synchronising call then returns HD_EHIP.  HD_EINVAL also when the user
 * kernels of a batch have more than 2^31 - 1 tiles. */
int hdarray_batch_begin(void);
int hdarray_batch_end(void);
int hdarray_batch_run(int batch);
/* Chooses the stencil tile shape (one wave per tile of 4, 8 or 16 rows
 * with tiles numbered along rows first (shape 1) or down columns (shape
 * 0), or four waves of 4 rows stacked down a tile, sharing halo rows
 * through LDS (shape 2)) and the workgroups per CU of the persistent kernel
 * (1, 2, 4; capped by its occupancy) of the given batches by timing each of
 * the 21 candidates on `reps` runs of the sequence batches[0..n) after one
 * warm-up run.  These runs are real steps of the program: 21 * (reps + 1)
 * sequences execute.  No candidate changes any result.  Returns the chosen
 * (per_cu << 16 | rows << 8 | shape) or a negative error. */
int hdarray_batch_autotune(const int *batches, int n, int reps);
/* Device time of each phase of the last run of a batch, in microseconds, from
 * clock stamps taken by workgroup 0 at the phase boundaries (a measurement
 * aid; synchronises).  Phases of the persistent kernel up to the message
 * table, for 2-D batches: runs, band flags, band scan, heads, compaction
 * (chunk scans, prefixes, writes: 3 phases) (7); 3-D batches insert the
 * first level's compaction and the second level's band flags, band scan and
 * heads before the three compaction phases (11).  The pack + unpack, GDEF
 * update and user-kernel launch that follow are not stamped.  Writes at
 * most max values to us and returns their number, or a negative error. */
int hdarray_batch_phase_us(int batch, double *us, int max);

/* Adjoint of one ApplyKernel of a "stencil3d7" kernel kname on partition
 * part (reverse mode, for differentiation through time steps):
 *   du_in   cotangent of the step's input (written here),
 *   du_out  cotangent of the step's output (read on each device's work box),
 *   u       the step's input values, holding the halos its forward step
 *           exchanged,
 *   coef    the 7 weights (host pointer),
 *   cbar    device pointer to 7 doubles; the coefficient gradients of this
 *           step, sum over interior outputs y of du_out[y] * u[y + off_e]
 *           accumulated in FP64 in a fixed order, are added to it (may be
 *           NULL).
 * Each device computes the contribution of its own outputs on its use
 * region (work box +- the kernel's use offsets); the contributions on halo
 * cells travel back along the reverse of the use-region messages (derived
 * from du_in's GDEF, in which every element is held by its owner only) and
 * are added to the owners' values in message-table order.  du_in is then
 * defined by the owners of the work boxes.  Asynchronous. */
int hdarray_apply_adjoint(const char *kname, int part, hd_array_t *du_in, hd_array_t *du_out, hd_array_t *u,
                          const float *coef, double *cbar);

/* Write / Read with a device pointer instead of a host array (dense,
 * full extent, device memory of the current GPU).  Write: each device's
 * region is copied from dptr; that device becomes owner and only holder.
 * Read: each device first obtains what it does not hold of its region
 * (communication as for Reduce), then the regions are copied to dptr.
 * Both are asynchronous on the data stream. */
int hdarray_write_device(hd_array_t *a, const void *dptr, int part);
int hdarray_read_device(hd_array_t *a, void *dptr, int part);

/* Stream (hipStream_t) for data movement and kernels. */
int hdarray_set_stream(void *hip_stream);

/* Device memory comes from alloc/free when set (e.g. a framework's caching
 * allocator); otherwise hipMalloc/hipFree. */
typedef void *(*hd_alloc_fn)(size_t bytes, void *ctx);
typedef void (*hd_free_fn)(void *ptr, void *ctx);
int hdarray_set_allocator(hd_alloc_fn alloc, hd_free_fn free_fn, void *ctx);

/* Waits for all enqueued work; returns the first deferred device error. */
int hdarray_sync(void);

/* Error of the last failed call (thread-local) and its text. */
int hdarray_last_error(void);
const char *hdarray_error_string(int code);

/* Per-call and cumulative counters (filled after a sync). */
typedef struct {
  int64_t calls;           /* ApplyKernel calls */
  int64_t last_messages;   /* messages of the last communication */
  int64_t last_bytes;      /* bytes packed (= unpacked) by it */
  int64_t total_messages;
  int64_t total_bytes;
  int64_t plans_built;     /* distinct (kernel, partition, arrays) plans */
  int64_t stencil_rows;    /* tile shape of the last Jacobi / triangular launch: */
  int64_t stencil_waves;   /* rows per tile, waves per workgroup */
  int64_t cache_hits;      /* plan-cache calls that reused a message table */
  int64_t cache_misses;    /* plan-cache calls that derived one */
  int64_t stencil_order;   /* tile order of the last stencil launch (1 along rows, 0 down columns) */
  int64_t allocs;          /* device and pinned host allocations the library has made */
  int64_t stencil_vec;     /* 1: the last stencil launch read every row as float4; 2: also with its boxes passed by value */
  int64_t cache_gdef_hits; /* plan-cache misses whose GDEF comparison on the GPU found the table current */
} hd_stats_t;
int hdarray_get_stats(hd_stats_t *st);

/* Tile shape of the 2-D stencil kernels (jacobi2d, tri2d, conv2d9) for
 * later calls: rows = 4, 8 or 16 rows per wave with waves = 1 (one wave per
 * workgroup, a tile of rows x 256 columns) or 4 (four waves stacked down a
 * tile of 4 x rows x 256 columns, the rows above and below each wave's rows
 * shared through LDS); order = 1: consecutive tiles of an XCD run along a
 * row of tiles, 0: down a column of tiles (one-wave shapes only; stacked
 * tiles always run along rows).  rows = 32 or 64 selects tall strips of that
 * many rows, one wave each, streaming through an 8-row register window
 * (waves and order ignored).  (0, 0, any)
 * restores the default: the runtime times four candidate shapes on the
 * first 32 calls of each work-box geometry (eight calls each, interleaved)
 * and keeps the one with the least median time.  No shape changes
 * a result.  HD_EINVAL for other values, HD_ESTATE before init. */
int hdarray_set_stencil_shape(int rows, int waves, int order);

/* Plan cache (Sec. 4.2; off by default).  With it on, an ApplyKernel call
 * whose arrays all have the GDEF that the call's plan last derived its
 * communication under reuses that plan's message table and runs: the
 * derivation is skipped and only the GDEF update and the data path run.
 * First step, on the host: each array keeps the list of plan updates
 * applied to it since a call that defined all of it without using it, and
 * equal lists give equal GDEF (cache_hits).  Second step, when the lists do
 * not decide (an array with no such call behind it, a list longer than 8,
 * a different list): for plans of at most 64 cells with use sections, the
 * GPU compares the lists the call's derivation would read with those the
 * plan's last derivation read and leaves the derivation out when they are
 * equal (cache_gdef_hits; such calls also count as cache_misses).  Each
 * plan gets its own table, run and snapshot buffers on its first cached
 * call.  Results equal those with the cache off.  HD_ESTATE before
 * hdarray_init. */
int hdarray_set_plan_cache(int on);

/* Per-phase device timing with HIP events recorded on the stream each phase
 * runs on (opt-in; adds an event pair per timed phase and call).  enable is a
 * bit mask over the phases (bit p times phase p, 0 disables).  Phases:
 * 0 communication-set derivation + GDEF update (internal stream), 1 pack
 * (with the unpack in the same pass), 2 unpack (when separate), 3 user
 * kernel, 4 adjoint step (reverse pack, adjoint kernel, scatter-add; data
 * stream).  hdarray_profile_read
 * synchronises, adds up the elapsed times since the last read and resets. */
typedef struct {
  double ms[5];
  int64_t count[5];
} hd_profile_t;
int hdarray_profile(int enable);
int hdarray_profile_read(hd_profile_t *out);

/* Parity dumps (synchronise).  Messages: 12 int64 each, {argument position,
 * array id, src, dst, lo[3], hi[3], pack offset (bytes), bytes}, in the
 * order (argument, lower corner row-major, destination); returns the count. */
int64_t hdarray_debug_messages(int64_t *out, int64_t cap);
/* Pack (staging) buffer of the last communication; returns its size. */
int64_t hdarray_debug_pack(void *out, int64_t cap);
/* GDEF expanded per element: owner (0..62, 63 = host) and holder bits. */
int hdarray_debug_gdef(hd_array_t *a, int8_t *owner, uint64_t *holders);
/* Device dev's buffer at the array's full extent, n0*n1*n2 elements row-major
 * (dev = HD_HOST: the host buffer).  A device keeps only a window of the
 * array (a box around every section it holds or reads); elements outside it
 * read as zero. */
int hdarray_debug_device_buffer(hd_array_t *a, int dev, void *out);
/* Device pointer of (array, device)'s buffer laid out as the whole array,
 * row-major with dense strides: allocates it, or widens the device's window
 * to the whole array, if needed (a widened window stays whole). */
void *hdarray_device_ptr(hd_array_t *a, int dev);

#ifdef __cplusplus
}
#endif
#endif

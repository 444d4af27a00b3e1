/*
 * hdoracle.h — CPU oracle for the HDArray ApplyKernel path (test infrastructure).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links or
 * calls this file; only tests/, the smoke entry and the benchmark's CPU-baseline
 * leg load it.  It shares no code with the HIP path.
 *
 * What it computes (paper: Sec. 2.1 "HDArray Structures", Sec. 2.2 Eq. 1-4,
 * Sec. 3.1 Table 2):
 *   - a per-element last-definer map: owner[x] in {0..62, HOST=63} and a holder
 *     set holders[x] (bit e set <=> endpoint e holds the current value of x).
 *     sGDEF_{p,q} = {x : owner[x]=p, q not in holders[x]} and
 *     rGDEF_{p,q} = {x : owner[x]=q, p not in holders[x]}.
 *   - the communication set of every ApplyKernel call by brute force over the
 *     elements of every device's use region (Eq. 1-2), in a canonical
 *     rectangle decomposition, and the GDEF update of Eq. 3-4 with the
 *     overwrite-kill reading (a definition by d leaves holders = {d}).
 *   - the array values by evaluating each kernel on the whole global array
 *     (FP32 in the stated operation order, plus an FP64 shadow), and a
 *     per-device buffer simulation that checks the coherence invariant.
 *
 * All rectangles are half-open [lo, hi) in normalised 3-D coordinates
 * (planes, rows, cols): a 1-D array of n is (1,1,n), a 2-D array r x c is
 * (1,r,c).  Error codes are negative ints, 0 is success.
 */
#ifndef HDORACLE_H
#define HDORACLE_H
#include <stdint.h>

#define ORC_HOST 63
#define ORC_MAXDEV 63

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EBOUNDS (-2)
#define ORC_ERACE (-3)
#define ORC_EKERNEL (-4)
#define ORC_ENOMEM (-5)
#define ORC_ESTATE (-7)
#define ORC_ECOHERENCE (-9)

enum { ORC_F32 = 0, ORC_I32 = 1, ORC_F64 = 2 };
enum { ORC_ROW = 0, ORC_COL = 1, ORC_BLOCK = 2 };
enum { ORC_SUM = 0, ORC_PROD = 1, ORC_MAX = 2, ORC_MIN = 3 };
enum { ORC_K_JACOBI2D = 1, ORC_K_COPY = 2, ORC_K_MATMUL = 3, ORC_K_TRI2D = 4, ORC_K_STENCIL3D7 = 5, ORC_K_CONV2D9 = 6 };

/* one message record: 12 int64 */
enum { ORC_MSG_ARG = 0, ORC_MSG_ARRAY, ORC_MSG_SRC, ORC_MSG_DST, ORC_MSG_LO0, ORC_MSG_LO1, ORC_MSG_LO2,
       ORC_MSG_HI0, ORC_MSG_HI1, ORC_MSG_HI2, ORC_MSG_OFF, ORC_MSG_BYTES, ORC_MSG_NF };

typedef struct orc_ctx orc_ctx;

orc_ctx *orc_new(void);
void orc_free(orc_ctx *c);
/* simulate_devices: keep per-device buffers and check coherence;
 * eval_kernels: 0 = metadata only (values become stale), 1 = evaluate. */
void orc_set_mode(orc_ctx *c, int simulate_devices, int eval_kernels);
int orc_create(orc_ctx *c, int type, int dim, const int64_t *sizes, const void *uA);
int orc_partition(orc_ctx *c, int type, int dim, const int64_t *sizes, const int64_t *rlo,
                  const int64_t *rhi, int ndev);
int orc_partition_manual(orc_ctx *c, int dim, int ndev, const int64_t *lo, const int64_t *hi);
int orc_part_region(orc_ctx *c, int part, int dev, int64_t *lo3, int64_t *hi3);
int orc_kernel(orc_ctx *c, const char *name, int builtin);
int orc_set_offsets(orc_ctx *c, int k, int arg, int use_or_def, int noff, const int32_t *off);
int orc_set_absolute(orc_ctx *c, int k, int part, int arr, int dev, int use_or_def, const int64_t *lo,
                     const int64_t *hi);
int orc_set_trapezoid(orc_ctx *c, int k, int part, int arr, int dev, int use_or_def,
                      const int64_t *corners);
int orc_clear_sections(orc_ctx *c, int k, int part, int arr, int dev);
int orc_apply(orc_ctx *c, int k, int part, int nargs, const int *arrs, int nscal, const double *scal);
int orc_write(orc_ctx *c, int arr, const void *uA, int part);
int orc_read(orc_ctx *c, int arr, void *uA, int part);
int orc_reduce(orc_ctx *c, int arr, int op, int part, double *res_f, int64_t *res_i);

int64_t orc_last_nmsgs(orc_ctx *c);
int64_t orc_last_messages(orc_ctx *c, int64_t *out, int64_t cap);
int64_t orc_last_pack_bytes(orc_ctx *c);
int64_t orc_last_pack(orc_ctx *c, void *out, int64_t cap);
int orc_gdef(orc_ctx *c, int arr, int8_t *owner, uint64_t *holders);
int orc_truth(orc_ctx *c, int arr, void *out);
int orc_truth64(orc_ctx *c, int arr, double *out);
int orc_device_buffer(orc_ctx *c, int arr, int dev, void *out);
/* number of kernel reads of non-coherent data seen so far (under-declared use) */
int64_t orc_bad_reads(orc_ctx *c);
/* fault injection for the self-check test: drop message #idx of the next call */
void orc_inject_drop(orc_ctx *c, int64_t idx);

/* global FP64 reference computations (no partitioning) */
int orc_threads(void);
void orc_s3d_forward64(const int64_t *n, const double *u0, const double *cf, int T, double *uT);
void orc_s3d_adjoint64(const int64_t *n, const double *u0, const double *cf, int T, const double *w,
                       double *gu0, double *gcf);
#endif

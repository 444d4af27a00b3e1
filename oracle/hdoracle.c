/*
 * hdoracle.c — plain, slow CPU oracle for the HDArray ApplyKernel path.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, the smoke entry and the
 * benchmark's CPU-baseline leg; never by the product library.  Every
 * decision here is made per element, by brute force, so that it can be read
 * against the paper directly.  See hdoracle.h for the conventions.
 *
 * Paper passages followed (section / equation / table of arXiv 1809.05657):
 *   Sec. 2.1            GDEF / LDEF / LUSE sets, sGDEF and rGDEF meaning
 *   Sec. 2.2, Eq. 1-2   communication = GDEF intersected with LUSE, taken
 *                       immediately before the kernel launch
 *   Sec. 2.2, Eq. 3-4   GDEF update: remove what was communicated, add LDEF
 *   Sec. 3, Table 1     use/def offset clauses ('*' = whole dimension),
 *                       absolute sections, partition clause
 *   Sec. 3.1, Table 2   Init/Create/Partition/ApplyKernel/Read/Write/Reduce,
 *                       SetAbsoluteUse/Def, SetTrapezoidUse/Def
 *   Sec. 3.2            GEMM case study (use A (0,*), use B (*,0), def C (0,0))
 *   Sec. 5.1            Jacobi update A = (B[i][j-1]+B[i][j+1]+B[i-1][j]+B[i+1][j])/4
 *   Sec. 4.2            merging adjacent sections (canonical rectangles here)
 */
#include <omp.h>
#include "hdoracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define BIT(e) (1ull << (e))

/* ------------------------------------------------------------------ shapes */
typedef struct {
  int kind; /* 0 = box, 1 = trapezoid (2-D only) */
  int64_t lo[3], hi[3];  /* box, normalised, half-open */
  int64_t c[8];          /* trapezoid corners (row,col) UL, UR, BL, BR (inclusive) */
} shape_t;

typedef struct {
  int n, cap;
  shape_t *s;
} region_t;

static void region_push(region_t *r, const shape_t *s) {
  if (r->n == r->cap) {
    r->cap = r->cap ? 2 * r->cap : 8;
    r->s = (shape_t *)realloc(r->s, sizeof(shape_t) * (size_t)r->cap);
  }
  r->s[r->n++] = *s;
}
static void region_free(region_t *r) {
  free(r->s);
  r->s = NULL;
  r->n = r->cap = 0;
}

static int64_t floordiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) q--;
  return q;
}

/* Row span [left,right] (inclusive) of a trapezoid at row r, before clipping.
 * Edges are straight lines between the corners; the top and bottom edges are
 * horizontal (Table 2: SetTrapezoidUse/Def take four corner positions). */
static int trap_row(const int64_t *c, int64_t r, int64_t *left, int64_t *right) {
  int64_t r0 = c[0], r1 = c[4];
  if (r < r0 || r > r1) return 0;
  if (r1 == r0) {
    *left = c[1];
    *right = c[3];
  } else {
    *left = c[1] + floordiv((r - r0) * (c[5] - c[1]), r1 - r0);
    *right = c[3] + floordiv((r - r0) * (c[7] - c[3]), r1 - r0);
  }
  return *left <= *right;
}

/* Mark every element of the shape inside the window [wlo,whi) of an array
 * with normalised extents n into mask (window-relative, row-major). */
static void shape_mark(const shape_t *s, const int64_t *n, const int64_t *wlo, const int64_t *whi,
                       unsigned char *mask) {
  int64_t W1 = whi[1] - wlo[1], W2 = whi[2] - wlo[2];
  if (s->kind == 0) {
    int64_t lo[3], hi[3];
    for (int k = 0; k < 3; k++) {
      lo[k] = s->lo[k] > wlo[k] ? s->lo[k] : wlo[k];
      hi[k] = s->hi[k] < whi[k] ? s->hi[k] : whi[k];
      if (lo[k] >= hi[k]) return;
    }
    for (int64_t p = lo[0]; p < hi[0]; p++)
      for (int64_t r = lo[1]; r < hi[1]; r++)
        memset(mask + ((p - wlo[0]) * W1 + (r - wlo[1])) * W2 + (lo[2] - wlo[2]), 1,
               (size_t)(hi[2] - lo[2]));
  } else {
    for (int64_t r = s->c[0]; r <= s->c[4]; r++) {
      int64_t l, rt;
      if (r < 0 || r >= n[1] || r < wlo[1] || r >= whi[1]) continue;
      if (!trap_row(s->c, r, &l, &rt)) continue;
      if (l < 0) l = 0;
      if (rt > n[2] - 1) rt = n[2] - 1;
      if (l < wlo[2]) l = wlo[2];
      if (rt > whi[2] - 1) rt = whi[2] - 1;
      if (l > rt) continue;
      memset(mask + (0 * W1 + (r - wlo[1])) * W2 + (l - wlo[2]), 1, (size_t)(rt - l + 1));
    }
  }
}

/* bounding box (clipped to the array) of a region; returns 0 if empty */
static int region_bbox(const region_t *rg, const int64_t *n, int64_t *lo, int64_t *hi) {
  int any = 0;
  for (int k = 0; k < 3; k++) {
    lo[k] = INT64_MAX;
    hi[k] = INT64_MIN;
  }
  for (int i = 0; i < rg->n; i++) {
    const shape_t *s = &rg->s[i];
    int64_t a[3], b[3];
    if (s->kind == 0) {
      for (int k = 0; k < 3; k++) {
        a[k] = s->lo[k] < 0 ? 0 : s->lo[k];
        b[k] = s->hi[k] > n[k] ? n[k] : s->hi[k];
      }
    } else {
      int64_t cmin = s->c[1] < s->c[5] ? s->c[1] : s->c[5];
      int64_t cmax = s->c[3] > s->c[7] ? s->c[3] : s->c[7];
      a[0] = 0;
      b[0] = 1;
      a[1] = s->c[0] < 0 ? 0 : s->c[0];
      b[1] = s->c[4] + 1 > n[1] ? n[1] : s->c[4] + 1;
      a[2] = cmin < 0 ? 0 : cmin;
      b[2] = cmax + 1 > n[2] ? n[2] : cmax + 1;
    }
    if (a[0] >= b[0] || a[1] >= b[1] || a[2] >= b[2]) continue;
    any = 1;
    for (int k = 0; k < 3; k++) {
      if (a[k] < lo[k]) lo[k] = a[k];
      if (b[k] > hi[k]) hi[k] = b[k];
    }
  }
  return any;
}

/* Full-array membership mask (1 byte per element) of a region. */
static unsigned char *region_mask_full(const region_t *rg, const int64_t *n) {
  int64_t N = n[0] * n[1] * n[2];
  unsigned char *m = (unsigned char *)calloc((size_t)N, 1);
  int64_t z[3] = {0, 0, 0};
  for (int i = 0; i < rg->n; i++) shape_mark(&rg->s[i], n, z, n, m);
  return m;
}

/* ------------------------------------------------------------------ state */
typedef struct {
  int live, type, esize, dim;
  int64_t n[3], N;
  unsigned char *truth;  /* coherent global value (FP32 run) */
  double *truth64;       /* FP64 shadow run (float arrays) */
  int8_t *owner;         /* last definer endpoint */
  uint64_t *holders;     /* endpoints holding the current value */
  unsigned char *host;   /* host buffer */
  unsigned char *dev[ORC_MAXDEV];
} arr_t;

typedef struct {
  int dim, ndev;
  int64_t lo[ORC_MAXDEV][3], hi[ORC_MAXDEV][3]; /* normalised */
} part_t;

typedef struct {
  int part, arr, dev, use_or_def;
  region_t rg;
} abs_t;

typedef struct {
  char name[64];
  int builtin;
  int noff[8][2];
  int32_t off[8][2][64][3];
  int nabs, capabs;
  abs_t *abs;
} kern_t;

struct orc_ctx {
  int nar, capar;
  arr_t *ar;
  int npart, cappart;
  part_t *pt;
  int nk, capk;
  kern_t *kn;
  int simulate, evalk;
  /* last communication */
  int64_t nmsg, capmsg;
  int64_t *msg;
  int64_t packbytes, cappack;
  unsigned char *pack;
  int64_t bad_reads;
  int64_t drop_idx;
};

orc_ctx *orc_new(void) {
  orc_ctx *c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
  c->simulate = 1;
  c->evalk = 1;
  c->drop_idx = -1;
  return c;
}

static void arr_release(arr_t *a) {
  free(a->truth);
  free(a->truth64);
  free(a->owner);
  free(a->holders);
  free(a->host);
  for (int d = 0; d < ORC_MAXDEV; d++) free(a->dev[d]);
  memset(a, 0, sizeof(*a));
}

void orc_free(orc_ctx *c) {
  if (!c) return;
  for (int i = 0; i < c->nar; i++) arr_release(&c->ar[i]);
  free(c->ar);
  free(c->pt);
  for (int i = 0; i < c->nk; i++) {
    for (int j = 0; j < c->kn[i].nabs; j++) region_free(&c->kn[i].abs[j].rg);
    free(c->kn[i].abs);
  }
  free(c->kn);
  free(c->msg);
  free(c->pack);
  free(c);
}

void orc_set_mode(orc_ctx *c, int simulate_devices, int eval_kernels) {
  c->simulate = simulate_devices;
  c->evalk = eval_kernels;
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

/* Table 2, HDArrayCreate: host and device buffers plus GDEF.  Before any
 * device writes, the only holder (and the last definer) is the host. */
int orc_create(orc_ctx *c, int type, int dim, const int64_t *sizes, const void *uA) {
  if (dim < 1 || dim > 3) return ORC_EINVAL;
  if (type < ORC_F32 || type > ORC_F64) return ORC_EINVAL;
  int64_t n[3];
  normalise(dim, sizes, 1, n);
  for (int k = 0; k < 3; k++)
    if (n[k] < 1) return ORC_EINVAL;
  if (c->nar == c->capar) {
    c->capar = c->capar ? 2 * c->capar : 8;
    c->ar = (arr_t *)realloc(c->ar, sizeof(arr_t) * (size_t)c->capar);
  }
  arr_t *a = &c->ar[c->nar];
  memset(a, 0, sizeof(*a));
  a->live = 1;
  a->type = type;
  a->esize = type == ORC_F64 ? 8 : 4;
  a->dim = dim;
  memcpy(a->n, n, sizeof(n));
  a->N = n[0] * n[1] * n[2];
  size_t bytes = (size_t)a->N * (size_t)a->esize;
  a->truth = (unsigned char *)malloc(bytes);
  a->host = (unsigned char *)malloc(bytes);
  a->owner = (int8_t *)malloc((size_t)a->N);
  a->holders = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)a->N);
  a->truth64 = (double *)malloc(sizeof(double) * (size_t)a->N);
  if (!a->truth || !a->host || !a->owner || !a->holders || !a->truth64) {
    arr_release(a);
    return ORC_ENOMEM;
  }
  if (uA)
    memcpy(a->truth, uA, bytes);
  else
    memset(a->truth, 0, bytes);
  memcpy(a->host, a->truth, bytes);
  for (int64_t x = 0; x < a->N; x++) {
    a->owner[x] = ORC_HOST;
    a->holders[x] = BIT(ORC_HOST);
    if (type == ORC_F32)
      a->truth64[x] = ((const float *)a->truth)[x];
    else if (type == ORC_F64)
      a->truth64[x] = ((const double *)a->truth)[x];
    else
      a->truth64[x] = ((const int32_t *)a->truth)[x];
  }
  return c->nar++;
}

static arr_t *get_arr(orc_ctx *c, int id) {
  if (id < 0 || id >= c->nar || !c->ar[id].live) return NULL;
  return &c->ar[id];
}

static unsigned char *devbuf(arr_t *a, int d) {
  if (d == ORC_HOST) return a->host;
  if (!a->dev[d]) a->dev[d] = (unsigned char *)calloc((size_t)a->N, (size_t)a->esize);
  return a->dev[d];
}

/* ------------------------------------------------------------- partitions */
/* Balanced factorisation of P into dim factors, non-increasing from the
 * slowest dimension (reading of Table 2's BLOCK type; see the design notes). */
static void block_factors(int P, int dim, int *f) {
  int best[3] = {P, 1, 1}, bestspread = P + 1, bestmax = P + 1;
  if (dim == 1) {
    f[0] = P;
    return;
  }
  for (int a = 1; a <= P; a++) {
    if (P % a) continue;
    if (dim == 2) {
      int b = P / a;
      if (a < b) continue;
      int spread = a - b;
      if (spread < bestspread || (spread == bestspread && a < bestmax)) {
        bestspread = spread;
        bestmax = a;
        best[0] = a;
        best[1] = b;
      }
    } else {
      for (int b = 1; b <= P / a; b++) {
        if ((P / a) % b) continue;
        int cc = P / a / b;
        if (!(a >= b && b >= cc)) continue;
        int spread = a - cc;
        if (spread < bestspread || (spread == bestspread && a < bestmax)) {
          bestspread = spread;
          bestmax = a;
          best[0] = a;
          best[1] = b;
          best[2] = cc;
        }
      }
    }
  }
  for (int k = 0; k < dim; k++) f[k] = best[k];
}

static int add_part(orc_ctx *c, part_t *p) {
  if (c->npart == c->cappart) {
    c->cappart = c->cappart ? 2 * c->cappart : 8;
    c->pt = (part_t *)realloc(c->pt, sizeof(part_t) * (size_t)c->cappart);
  }
  c->pt[c->npart] = *p;
  return c->npart++;
}

/* Table 2, HDArrayPartition: even split of the work-item region.  Device i
 * of P along a dimension of length N starting at L gets
 * [L + floor(i*N/P), L + floor((i+1)*N/P)). */
int orc_partition(orc_ctx *c, int type, int dim, const int64_t *sizes, const int64_t *rlo,
                  const int64_t *rhi, int ndev) {
  if (dim < 1 || dim > 3 || ndev < 1 || ndev > ORC_MAXDEV) return ORC_EINVAL;
  if (type < ORC_ROW || type > ORC_BLOCK) return ORC_EINVAL;
  for (int k = 0; k < dim; k++)
    if (rlo[k] < 0 || rhi[k] > sizes[k] || rlo[k] > rhi[k]) return ORC_EBOUNDS;
  int f[3] = {1, 1, 1};
  if (type == ORC_ROW)
    f[0] = ndev;
  else if (type == ORC_COL) {
    if (dim == 1)
      f[0] = ndev;
    else
      f[1] = ndev;
  } else
    block_factors(ndev, dim, f);
  part_t p;
  memset(&p, 0, sizeof(p));
  p.dim = dim;
  p.ndev = ndev;
  for (int d = 0; d < ndev; d++) {
    int g[3];
    int rem = d;
    for (int k = dim - 1; k >= 0; k--) {
      g[k] = rem % f[k];
      rem /= f[k];
    }
    int64_t lo[3], hi[3];
    for (int k = 0; k < dim; k++) {
      int64_t L = rlo[k], N = rhi[k] - rlo[k];
      lo[k] = L + (int64_t)g[k] * N / f[k];
      hi[k] = L + ((int64_t)g[k] + 1) * N / f[k];
    }
    normalise(dim, lo, 0, p.lo[d]);
    normalise(dim, hi, 1, p.hi[d]);
  }
  return add_part(c, &p);
}

/* Sec. 3, partition clause: the user gives each device's work region. */
int orc_partition_manual(orc_ctx *c, int dim, int ndev, const int64_t *lo, const int64_t *hi) {
  if (dim < 1 || dim > 3 || ndev < 1 || ndev > ORC_MAXDEV) return ORC_EINVAL;
  part_t p;
  memset(&p, 0, sizeof(p));
  p.dim = dim;
  p.ndev = ndev;
  for (int d = 0; d < ndev; d++) {
    for (int k = 0; k < dim; k++)
      if (lo[d * dim + k] < 0 || lo[d * dim + k] > hi[d * dim + k]) return ORC_EBOUNDS;
    normalise(dim, lo + d * dim, 0, p.lo[d]);
    normalise(dim, hi + d * dim, 1, p.hi[d]);
  }
  return add_part(c, &p);
}

int orc_part_region(orc_ctx *c, int part, int dev, int64_t *lo3, int64_t *hi3) {
  if (part < 0 || part >= c->npart) return ORC_EINVAL;
  part_t *p = &c->pt[part];
  if (dev < 0 || dev >= p->ndev) return ORC_EINVAL;
  memcpy(lo3, p->lo[dev], sizeof(int64_t) * 3);
  memcpy(hi3, p->hi[dev], sizeof(int64_t) * 3);
  return ORC_OK;
}

/* ----------------------------------------------------------------- kernels */
int orc_kernel(orc_ctx *c, const char *name, int builtin) {
  if (builtin < ORC_K_JACOBI2D || builtin > ORC_K_CONV2D9) return ORC_EKERNEL;
  for (int i = 0; i < c->nk; i++)
    if (!strcmp(c->kn[i].name, name)) return ORC_EINVAL;
  if (c->nk == c->capk) {
    c->capk = c->capk ? 2 * c->capk : 8;
    c->kn = (kern_t *)realloc(c->kn, sizeof(kern_t) * (size_t)c->capk);
  }
  kern_t *k = &c->kn[c->nk];
  memset(k, 0, sizeof(*k));
  snprintf(k->name, sizeof(k->name), "%s", name);
  k->builtin = builtin;
  return c->nk++;
}

#define ORC_STAR INT32_MIN
/* Table 1 use/def clauses: offsets relative to the work item, '*' = the whole
 * array extent in that dimension. */
int orc_set_offsets(orc_ctx *c, int k, int arg, int use_or_def, int noff, const int32_t *off) {
  if (k < 0 || k >= c->nk || arg < 0 || arg >= 8 || use_or_def < 0 || use_or_def > 1) return ORC_EINVAL;
  if (noff < 0 || noff > 64) return ORC_EINVAL;
  kern_t *kn = &c->kn[k];
  kn->noff[arg][use_or_def] = noff;
  /* offsets are stored per dimension of the array; dimension count is only
   * known at apply time, so keep up to 3 entries and the caller's layout
   * (noff x dim) is re-read there: store raw triples */
  for (int i = 0; i < noff; i++)
    for (int j = 0; j < 3; j++) kn->off[arg][use_or_def][i][j] = off[i * 3 + j];
  return ORC_OK;
}

static abs_t *abs_find(kern_t *kn, int part, int arr, int dev, int uod, int create) {
  for (int i = 0; i < kn->nabs; i++) {
    abs_t *e = &kn->abs[i];
    if (e->part == part && e->arr == arr && e->dev == dev && e->use_or_def == uod) return e;
  }
  if (!create) return NULL;
  if (kn->nabs == kn->capabs) {
    kn->capabs = kn->capabs ? 2 * kn->capabs : 8;
    kn->abs = (abs_t *)realloc(kn->abs, sizeof(abs_t) * (size_t)kn->capabs);
  }
  abs_t *e = &kn->abs[kn->nabs++];
  memset(e, 0, sizeof(*e));
  e->part = part;
  e->arr = arr;
  e->dev = dev;
  e->use_or_def = uod;
  return e;
}

/* Table 2, SetAbsoluteUse/Def: absolute sections accumulate per
 * (kernel, partition, array, device). */
int orc_set_absolute(orc_ctx *c, int k, int part, int arr, int dev, int use_or_def, const int64_t *lo,
                     const int64_t *hi) {
  if (k < 0 || k >= c->nk || part < 0 || part >= c->npart) return ORC_EINVAL;
  arr_t *a = get_arr(c, arr);
  if (!a || dev < 0 || dev >= ORC_MAXDEV || use_or_def < 0 || use_or_def > 1) return ORC_EINVAL;
  shape_t s;
  memset(&s, 0, sizeof(s));
  normalise(a->dim, lo, 0, s.lo);
  normalise(a->dim, hi, 1, s.hi);
  for (int j = 0; j < 3; j++)
    if (s.lo[j] < 0 || s.hi[j] > a->n[j] || s.lo[j] > s.hi[j]) return ORC_EBOUNDS;
  region_push(&abs_find(&c->kn[k], part, arr, dev, use_or_def, 1)->rg, &s);
  return ORC_OK;
}

/* Table 2, SetTrapezoidUse/Def: 2-D shape from four corners, top and bottom
 * edges horizontal.  Parts outside the array are clipped. */
int orc_set_trapezoid(orc_ctx *c, int k, int part, int arr, int dev, int use_or_def,
                      const int64_t *corners) {
  if (k < 0 || k >= c->nk || part < 0 || part >= c->npart) return ORC_EINVAL;
  arr_t *a = get_arr(c, arr);
  if (!a || a->dim != 2 || dev < 0 || dev >= ORC_MAXDEV || use_or_def < 0 || use_or_def > 1)
    return ORC_EINVAL;
  if (corners[0] != corners[2] || corners[4] != corners[6] || corners[0] > corners[4]) return ORC_EINVAL;
  shape_t s;
  memset(&s, 0, sizeof(s));
  s.kind = 1;
  memcpy(s.c, corners, sizeof(s.c));
  region_push(&abs_find(&c->kn[k], part, arr, dev, use_or_def, 1)->rg, &s);
  return ORC_OK;
}

int orc_clear_sections(orc_ctx *c, int k, int part, int arr, int dev) {
  if (k < 0 || k >= c->nk) return ORC_EINVAL;
  kern_t *kn = &c->kn[k];
  for (int i = 0; i < kn->nabs; i++) {
    abs_t *e = &kn->abs[i];
    if (e->part == part && e->arr == arr && (dev < 0 || e->dev == dev)) region_free(&e->rg);
  }
  return ORC_OK;
}

/* -------------------------------------------------------- message records */
static void msg_reset(orc_ctx *c) {
  c->nmsg = 0;
  c->packbytes = 0;
}

static void msg_push(orc_ctx *c, const int64_t *m) {
  if (c->nmsg == c->capmsg) {
    c->capmsg = c->capmsg ? 2 * c->capmsg : 256;
    c->msg = (int64_t *)realloc(c->msg, sizeof(int64_t) * ORC_MSG_NF * (size_t)c->capmsg);
  }
  memcpy(c->msg + c->nmsg * ORC_MSG_NF, m, sizeof(int64_t) * ORC_MSG_NF);
  c->nmsg++;
}

typedef struct {
  int64_t src, dst, lo[3], hi[3];
} box_t;

typedef struct {
  int64_t n, cap;
  box_t *b;
} boxes_t;

static void boxes_push(boxes_t *v, const box_t *b) {
  if (v->n == v->cap) {
    v->cap = v->cap ? 2 * v->cap : 64;
    v->b = (box_t *)realloc(v->b, sizeof(box_t) * (size_t)v->cap);
  }
  v->b[v->n++] = *b;
}

static int box_cmp(const void *pa, const void *pb) {
  const box_t *a = (const box_t *)pa, *b = (const box_t *)pb;
  for (int k = 0; k < 3; k++) {
    if (a->lo[k] != b->lo[k]) return a->lo[k] < b->lo[k] ? -1 : 1;
  }
  if (a->dst != b->dst) return a->dst < b->dst ? -1 : 1;
  return 0;
}

/* Canonical rectangle decomposition of one destination's message elements
 * (the "merging adjacent sections" of Sec. 4.2, made unique):
 *   1. maximal runs along the innermost dimension with one source;
 *   2. runs with identical (src, c0, c1) on consecutive rows of a plane are
 *      stacked into rectangles;
 *   3. rectangles with identical (src, r0, r1, c0, c1) on consecutive planes
 *      are stacked into boxes.
 * srcmap covers the window [wlo, whi) (row-major); -1 = no message. */
typedef struct {
  int64_t src, a0, a1, b0, b1, start;
  int live;
} open_t;

static void rle_dst(const int8_t *srcmap, const int64_t *wlo, const int64_t *whi, int dst, boxes_t *out) {
  int64_t W0 = whi[0] - wlo[0], W1 = whi[1] - wlo[1], W2 = whi[2] - wlo[2];
  open_t *ob = NULL; /* open boxes (level 2), from previous plane */
  int64_t nob = 0, capob = 0;
  for (int64_t p = 0; p < W0; p++) {
    open_t *orr = NULL; /* open rects (level 1), from previous row */
    int64_t nor = 0, capor = 0;
    open_t *pr = NULL; /* closed rects of this plane */
    int64_t npr = 0, cappr = 0;
    for (int64_t r = 0; r <= W1; r++) {
      /* runs of row r (none past the last row) */
      for (int64_t i = 0; i < nor; i++) orr[i].live = 0;
      if (r < W1) {
        const int8_t *row = srcmap + (p * W1 + r) * W2;
        int64_t cidx = 0;
        while (cidx < W2) {
          if (row[cidx] < 0) {
            cidx++;
            continue;
          }
          int64_t s = row[cidx], c0 = cidx;
          while (cidx < W2 && row[cidx] == s) cidx++;
          int found = 0;
          for (int64_t i = 0; i < nor; i++) {
            if (orr[i].src == s && orr[i].a0 == c0 && orr[i].a1 == cidx && orr[i].b1 == r) {
              orr[i].b1 = r + 1;
              orr[i].live = 1;
              found = 1;
              break;
            }
          }
          if (!found) {
            if (nor == capor) {
              capor = capor ? 2 * capor : 16;
              orr = (open_t *)realloc(orr, sizeof(open_t) * (size_t)capor);
            }
            open_t o = {s, c0, cidx, r, r + 1, r, 1};
            orr[nor++] = o;
          }
        }
      }
      /* close the rects that did not continue onto row r */
      int64_t keep = 0;
      for (int64_t i = 0; i < nor; i++) {
        if (orr[i].live) {
          orr[keep++] = orr[i];
        } else {
          if (npr == cappr) {
            cappr = cappr ? 2 * cappr : 16;
            pr = (open_t *)realloc(pr, sizeof(open_t) * (size_t)cappr);
          }
          pr[npr++] = orr[i];
        }
      }
      nor = keep;
    }
    free(orr);
    /* level 2: stack this plane's rects onto the open boxes of plane p-1 */
    for (int64_t i = 0; i < nob; i++) ob[i].live = 0;
    for (int64_t j = 0; j < npr; j++) {
      open_t *q = &pr[j]; /* a0,a1 = cols, b0,b1 = rows */
      int found = 0;
      for (int64_t i = 0; i < nob; i++) {
        if (!ob[i].live && ob[i].src == q->src && ob[i].a0 == q->a0 && ob[i].a1 == q->a1 &&
            ob[i].b0 == q->b0 && ob[i].b1 == q->b1) {
          /* every box still open was extended on plane p-1 */
          ob[i].live = 1;
          found = 1;
          break;
        }
      }
      if (!found) {
        if (nob == capob) {
          capob = capob ? 2 * capob : 16;
          ob = (open_t *)realloc(ob, sizeof(open_t) * (size_t)capob);
        }
        open_t o = {q->src, q->a0, q->a1, q->b0, q->b1, p, 2};
        ob[nob++] = o;
      }
    }
    free(pr);
    /* boxes not extended onto plane p close at plane p; new ones (live==2) stay */
    int64_t keep = 0;
    for (int64_t i = 0; i < nob; i++) {
      if (ob[i].live) {
        ob[i].live = 0;
        ob[keep++] = ob[i];
      } else {
        box_t b;
        b.src = ob[i].src;
        b.dst = dst;
        b.lo[0] = wlo[0] + ob[i].start;
        b.hi[0] = wlo[0] + p;
        b.lo[1] = wlo[1] + ob[i].b0;
        b.hi[1] = wlo[1] + ob[i].b1;
        b.lo[2] = wlo[2] + ob[i].a0;
        b.hi[2] = wlo[2] + ob[i].a1;
        boxes_push(out, &b);
      }
    }
    nob = keep;
  }
  for (int64_t i = 0; i < nob; i++) {
    box_t b;
    b.src = ob[i].src;
    b.dst = dst;
    b.lo[0] = wlo[0] + ob[i].start;
    b.hi[0] = wlo[0] + W0;
    b.lo[1] = wlo[1] + ob[i].b0;
    b.hi[1] = wlo[1] + ob[i].b1;
    b.lo[2] = wlo[2] + ob[i].a0;
    b.hi[2] = wlo[2] + ob[i].a1;
    boxes_push(out, &b);
  }
  free(ob);
}

/* Eq. 1-2 per element: for every endpoint d and every x in LUSE_d that d
 * does not hold, one message element (owner[x] -> d, x).  The sender is the
 * owner: sGDEF only lists what a process wrote (Sec. 2.1). */
static void derive_messages(orc_ctx *c, int argpos, int arrid, arr_t *a, region_t *use /*[64]*/,
                            boxes_t *out) {
  /* every destination on its own (OpenMP over devices), joined in device order */
  boxes_t per[64];
  memset(per, 0, sizeof(per));
#pragma omp parallel for schedule(dynamic, 1)
  for (int d = 0; d < 64; d++) {
    if (use[d].n == 0) continue;
    int64_t lo[3], hi[3];
    if (!region_bbox(&use[d], a->n, lo, hi)) continue;
    int64_t W1 = hi[1] - lo[1], W2 = hi[2] - lo[2];
    int64_t V = (hi[0] - lo[0]) * W1 * W2;
    unsigned char *mask = (unsigned char *)calloc((size_t)V, 1);
    int8_t *srcmap = (int8_t *)malloc((size_t)V);
    for (int i = 0; i < use[d].n; i++) shape_mark(&use[d].s[i], a->n, lo, hi, mask);
    for (int64_t p = lo[0]; p < hi[0]; p++)
      for (int64_t r = lo[1]; r < hi[1]; r++)
        for (int64_t q = lo[2]; q < hi[2]; q++) {
          int64_t w = ((p - lo[0]) * W1 + (r - lo[1])) * W2 + (q - lo[2]);
          int64_t x = (p * a->n[1] + r) * a->n[2] + q;
          srcmap[w] = -1;
          if (mask[w] && !(a->holders[x] & BIT(d))) srcmap[w] = a->owner[x];
        }
    rle_dst(srcmap, lo, hi, d, &per[d]);
    free(mask);
    free(srcmap);
  }
  for (int d = 0; d < 64; d++) {
    for (int64_t i = 0; i < per[d].n; i++) boxes_push(out, &per[d].b[i]);
    free(per[d].b);
  }
  (void)c;
  (void)argpos;
  (void)arrid;
}

static void for_box(const box_t *b, const int64_t *n, void (*fn)(void *, int64_t), void *ctx) {
  for (int64_t p = b->lo[0]; p < b->hi[0]; p++)
    for (int64_t r = b->lo[1]; r < b->hi[1]; r++)
      for (int64_t q = b->lo[2]; q < b->hi[2]; q++) fn(ctx, (p * n[1] + r) * n[2] + q);
}

typedef struct {
  orc_ctx *c;
  arr_t *a;
  unsigned char *dstp, *srcp, *packp;
  uint64_t bit;
} apply_ctx;

static void apply_elem(void *vctx, int64_t x) {
  apply_ctx *t = (apply_ctx *)vctx;
  size_t es = (size_t)t->a->esize;
  if (t->packp) {
    memcpy(t->packp, t->srcp + (size_t)x * es, es);
    t->packp += es;
  }
  if (t->dstp) memcpy(t->dstp + (size_t)x * es, t->srcp + (size_t)x * es, es);
  t->a->holders[x] |= t->bit;
}

/* Record, pack and deliver the messages of one array (canonical order), then
 * the receiver becomes a holder (the subtraction in Eq. 3-4). */
static void comm_array(orc_ctx *c, int argpos, int arrid, region_t *use) {
  arr_t *a = &c->ar[arrid];
  boxes_t bx = {0, 0, NULL};
  derive_messages(c, argpos, arrid, a, use, &bx);
  qsort(bx.b, (size_t)bx.n, sizeof(box_t), box_cmp);
  int64_t first = c->nmsg;
  for (int64_t i = 0; i < bx.n; i++) {
    box_t *b = &bx.b[i];
    int64_t vol = (b->hi[0] - b->lo[0]) * (b->hi[1] - b->lo[1]) * (b->hi[2] - b->lo[2]);
    int64_t off = (c->packbytes + a->esize - 1) / a->esize * a->esize;
    int64_t m[ORC_MSG_NF] = {argpos, arrid, b->src, b->dst, b->lo[0], b->lo[1], b->lo[2],
                             b->hi[0], b->hi[1], b->hi[2], off, vol * a->esize};
    msg_push(c, m);
    c->packbytes = off + vol * a->esize;
  }
  if (c->packbytes > c->cappack) {
    c->cappack = c->packbytes;
    c->pack = (unsigned char *)realloc(c->pack, (size_t)c->cappack);
  }
  {
    int64_t start = first > 0 ? c->msg[(first - 1) * ORC_MSG_NF + ORC_MSG_OFF] + c->msg[(first - 1) * ORC_MSG_NF + ORC_MSG_BYTES] : 0;
    if (c->packbytes > start) memset(c->pack + start, 0, (size_t)(c->packbytes - start));
  }
  for (int64_t i = 0; i < bx.n; i++) {
    box_t *b = &bx.b[i];
    int64_t *m = c->msg + (first + i) * ORC_MSG_NF;
    apply_ctx t;
    t.c = c;
    t.a = a;
    t.bit = BIT(b->dst);
    t.packp = c->pack + m[ORC_MSG_OFF];
    if (c->simulate) {
      t.srcp = devbuf(a, (int)b->src);
      t.dstp = devbuf(a, (int)b->dst);
    } else {
      t.srcp = a->truth;
      t.dstp = NULL;
    }
    if (c->drop_idx == first + i) { /* fault injection: the message is lost */
      t.dstp = NULL;
      t.bit = 0;
    }
    for_box(b, a->n, apply_elem, &t);
  }
  free(bx.b);
}

/* coherence invariant: every endpoint holds the current value of everything
 * it is about to use */
static int64_t check_coherent(orc_ctx *c, arr_t *a, region_t *use) {
  int64_t bad = 0;
  for (int d = 0; d < 64; d++) {
    if (use[d].n == 0) continue;
    unsigned char *m = region_mask_full(&use[d], a->n);
    unsigned char *buf = c->simulate ? devbuf(a, d) : NULL;
    int64_t bd = 0;
#pragma omp parallel for reduction(+ : bd) schedule(static)
    for (int64_t x = 0; x < a->N; x++) {
      if (!m[x]) continue;
      if (!(a->holders[x] & BIT(d))) bd++;
      else if (buf && memcmp(buf + (size_t)x * (size_t)a->esize, a->truth + (size_t)x * (size_t)a->esize,
                             (size_t)a->esize))
        bd++;
    }
    bad += bd;
    free(m);
  }
  return bad;
}

/* ------------------------------------------------------- kernel evaluation */
/* Built-in kernels.  Each writes its work region (TRI2D: the part with col <=
 * row) of the output argument and reads its inputs as stated. */
typedef struct {
  int nargs, out, nin, in[2], dim, nscal;
} kspec_t;

static int kspec(int builtin, kspec_t *s) {
  memset(s, 0, sizeof(*s));
  switch (builtin) {
    case ORC_K_JACOBI2D:
    case ORC_K_TRI2D:
      s->nargs = 2, s->out = 0, s->nin = 1, s->in[0] = 1, s->dim = 2;
      return 1;
    case ORC_K_COPY:
      s->nargs = 2, s->out = 0, s->nin = 1, s->in[0] = 1, s->dim = 0;
      return 1;
    case ORC_K_MATMUL:
      s->nargs = 3, s->out = 2, s->nin = 2, s->in[0] = 0, s->in[1] = 1, s->dim = 2;
      return 1;
    case ORC_K_STENCIL3D7:
      s->nargs = 2, s->out = 0, s->nin = 1, s->in[0] = 1, s->dim = 3, s->nscal = 7;
      return 1;
    case ORC_K_CONV2D9:
      s->nargs = 2, s->out = 0, s->nin = 1, s->in[0] = 1, s->dim = 2, s->nscal = 9;
      return 1;
  }
  return 0;
}

typedef struct {
  const unsigned char *in0, *in1; /* FP32 (or raw) inputs */
  unsigned char *out;
  const double *in0d, *in1d;
  double *outd;
  const uint64_t *h0, *h1; /* holders of the inputs (read validity), or NULL */
  uint64_t bit;
  int64_t bad;
  arr_t *ain0, *ain1, *aout;
  float cf[9];
  double cfd[9];
} keval_t;

#define RD(t, x) ((t)->h0 && !((t)->h0[(x)] & (t)->bit) ? ((t)->bad++, 0) : 0)

static inline float ldf(const unsigned char *b, int64_t x) {
  float v;
  memcpy(&v, b + 4 * x, 4);
  return v;
}
static inline void stf(unsigned char *b, int64_t x, float v) { memcpy(b + 4 * x, &v, 4); }

/* Jacobi (Sec. 5.1): A[i][j] = (B[i][j-1] + B[i][j+1] + B[i-1][j] + B[i+1][j]) / 4,
 * summed left to right; cells on the array boundary are copied. */
static void eval_jacobi_cell(keval_t *t, int64_t i, int64_t j, int tri) {
  int64_t nr = t->aout->n[1], nc = t->aout->n[2];
  int64_t x = i * nc + j;
  int interior = i >= 1 && i <= nr - 2 && j >= 1 && j <= nc - 2;
  if (tri) interior = j >= 1 && j < i && i <= nr - 2;
  if (!interior) {
    RD(t, x);
    if (t->out) memcpy(t->out + 4 * x, t->in0 + 4 * x, 4);
    if (t->outd) t->outd[x] = t->in0d[x];
    return;
  }
  RD(t, x - 1);
  RD(t, x + 1);
  RD(t, x - nc);
  RD(t, x + nc);
  if (t->out) {
    float s = ldf(t->in0, x - 1) + ldf(t->in0, x + 1);
    s = s + ldf(t->in0, x - nc);
    s = s + ldf(t->in0, x + nc);
    stf(t->out, x, s / 4.0f);
  }
  if (t->outd) {
    double s = t->in0d[x - 1] + t->in0d[x + 1];
    s = s + t->in0d[x - nc];
    s = s + t->in0d[x + nc];
    t->outd[x] = s / 4.0;
  }
}

/* 7-point stencil: acc = c0*u; then one fused multiply-add per neighbour in
 * the order -i, +i, -j, +j, -k, +k; boundary cells are copied. */
static void eval_s3d_cell(keval_t *t, int64_t i, int64_t j, int64_t k) {
  const int64_t *n = t->aout->n;
  int64_t x = (i * n[1] + j) * n[2] + k;
  int64_t si = n[1] * n[2], sj = n[2];
  int interior = i >= 1 && i <= n[0] - 2 && j >= 1 && j <= n[1] - 2 && k >= 1 && k <= n[2] - 2;
  if (!interior) {
    RD(t, x);
    if (t->out) memcpy(t->out + 4 * x, t->in0 + 4 * x, 4);
    if (t->outd) t->outd[x] = t->in0d[x];
    return;
  }
  RD(t, x);
  RD(t, x - si);
  RD(t, x + si);
  RD(t, x - sj);
  RD(t, x + sj);
  RD(t, x - 1);
  RD(t, x + 1);
  if (t->out) {
    const unsigned char *u = t->in0;
    float acc = t->cf[0] * ldf(u, x);
    acc = fmaf(t->cf[1], ldf(u, x - si), acc);
    acc = fmaf(t->cf[2], ldf(u, x + si), acc);
    acc = fmaf(t->cf[3], ldf(u, x - sj), acc);
    acc = fmaf(t->cf[4], ldf(u, x + sj), acc);
    acc = fmaf(t->cf[5], ldf(u, x - 1), acc);
    acc = fmaf(t->cf[6], ldf(u, x + 1), acc);
    stf(t->out, x, acc);
  }
  if (t->outd) {
    const double *u = t->in0d;
    double acc = t->cfd[0] * u[x];
    acc += t->cfd[1] * u[x - si];
    acc += t->cfd[2] * u[x + si];
    acc += t->cfd[3] * u[x - sj];
    acc += t->cfd[4] * u[x + sj];
    acc += t->cfd[5] * u[x - 1];
    acc += t->cfd[6] * u[x + 1];
    t->outd[x] = acc;
  }
}

/* 2-D convolution with the eight neighbours of Sec. 5.1 (weights given by
 * the caller): out[i][j] = sum over the 3 x 3 window of w[3(di+1)+(dj+1)] *
 * in[i+di][j+dj], the window taken row by row (di = -1, 0, 1, and inside
 * a row dj = -1, 0, 1): the first product rounded, then one fused
 * multiply-add per further cell.  Cells on the array boundary are copied. */
static void eval_conv_cell(keval_t *t, int64_t i, int64_t j) {
  int64_t nr = t->aout->n[1], nc = t->aout->n[2];
  int64_t x = i * nc + j;
  int interior = i >= 1 && i <= nr - 2 && j >= 1 && j <= nc - 2;
  if (!interior) {
    RD(t, x);
    if (t->out) memcpy(t->out + 4 * x, t->in0 + 4 * x, 4);
    if (t->outd) t->outd[x] = t->in0d[x];
    return;
  }
  for (int di = -1; di <= 1; di++)
    for (int dj = -1; dj <= 1; dj++) RD(t, x + di * nc + dj);
  if (t->out) {
    float acc = 0.0f;
    int w = 0;
    for (int di = -1; di <= 1; di++)
      for (int dj = -1; dj <= 1; dj++, w++) {
        float v = ldf(t->in0, x + di * nc + dj);
        acc = w == 0 ? t->cf[0] * v : fmaf(t->cf[w], v, acc);
      }
    stf(t->out, x, acc);
  }
  if (t->outd) {
    double acc = 0.0;
    int w = 0;
    for (int di = -1; di <= 1; di++)
      for (int dj = -1; dj <= 1; dj++, w++) acc += t->cfd[w] * t->in0d[x + di * nc + dj];
    t->outd[x] = acc;
  }
}

/* GEMM of Sec. 3.2 with alpha = 1, beta = 0: C[i][j] = sum_k A[i][k]*B[k][j],
 * FP32 accumulation in k order. */
static void eval_mm_cell(keval_t *t, int64_t i, int64_t j) {
  int64_t K = t->ain0->n[2], M = t->ain1->n[2];
  if (t->h0)
    for (int64_t k = 0; k < K; k++) {
      if (!(t->h0[i * K + k] & t->bit)) t->bad++;
      if (!(t->h1[k * M + j] & t->bit)) t->bad++;
    }
  if (t->out) {
    float acc = 0.0f;
    for (int64_t k = 0; k < K; k++) {
      float p = ldf(t->in0, i * K + k) * ldf(t->in1, k * M + j);
      acc = acc + p;
    }
    stf(t->out, i * M + j, acc);
  }
  if (t->outd) {
    double acc = 0.0;
    for (int64_t k = 0; k < K; k++) acc += t->in0d[i * K + k] * t->in1d[k * M + j];
    t->outd[i * M + j] = acc;
  }
}

/* Every cell of the box [lo, hi) is evaluated on its own (the inputs are not
 * the output), so the rows are shared out over OpenMP threads; each thread
 * counts its reads of non-coherent data and the counts are summed. */
static void eval_region(keval_t *t, int builtin, const int64_t *lo, const int64_t *hi) {
  int64_t bad = 0;
#pragma omp parallel for collapse(2) reduction(+ : bad) schedule(static)
  for (int64_t p = lo[0]; p < hi[0]; p++)
    for (int64_t r = lo[1]; r < hi[1]; r++) {
      keval_t u = *t;
      u.bad = 0;
      for (int64_t q = lo[2]; q < hi[2]; q++) {
        switch (builtin) {
          case ORC_K_JACOBI2D:
            eval_jacobi_cell(&u, r, q, 0);
            break;
          case ORC_K_TRI2D:
            if (q <= r) eval_jacobi_cell(&u, r, q, 1);
            break;
          case ORC_K_STENCIL3D7:
            eval_s3d_cell(&u, p, r, q);
            break;
          case ORC_K_CONV2D9:
            eval_conv_cell(&u, r, q);
            break;
          case ORC_K_MATMUL:
            eval_mm_cell(&u, r, q);
            break;
          case ORC_K_COPY: {
            int64_t x = (p * u.aout->n[1] + r) * u.aout->n[2] + q;
            size_t es = (size_t)u.aout->esize;
            RD(&u, x);
            if (u.out) memcpy(u.out + es * (size_t)x, u.in0 + es * (size_t)x, es);
            if (u.outd) u.outd[x] = u.in0d[x];
          } break;
        }
      }
      bad += u.bad;
    }
  t->bad += bad;
}

/* --------------------------------------------------------- region builder */
/* LUSE_d / LDEF_d of one argument: absolute sections if any were set for this
 * (kernel, partition, array), else the offsets composed with the device's
 * work region (shift, '*' -> whole extent, clip to the array). */
static void build_region(orc_ctx *c, kern_t *kn, int part, int arg, int arrid, int uod, int d,
                         const int64_t *wlo, const int64_t *whi, region_t *out) {
  arr_t *a = &c->ar[arrid];
  int absmode = 0;
  for (int i = 0; i < kn->nabs; i++) {
    abs_t *e = &kn->abs[i];
    if (e->part == part && e->arr == arrid && e->use_or_def == uod && e->rg.n > 0) absmode = 1;
  }
  if (absmode) {
    abs_t *e = abs_find(kn, part, arrid, d, uod, 0);
    if (e)
      for (int i = 0; i < e->rg.n; i++) region_push(out, &e->rg.s[i]);
    return;
  }
  for (int o = 0; o < kn->noff[arg][uod]; o++) {
    int32_t raw[3];
    int dim = a->dim;
    /* offsets are given in the array's own dimension order */
    for (int j = 0; j < 3; j++) raw[j] = kn->off[arg][uod][o][j];
    int32_t off3[3] = {0, 0, 0};
    int star3[3] = {0, 0, 0};
    for (int j = 0; j < dim; j++) {
      int nj = 3 - dim + j;
      if (raw[j] == ORC_STAR)
        star3[nj] = 1;
      else
        off3[nj] = raw[j];
    }
    shape_t s;
    memset(&s, 0, sizeof(s));
    int empty = 0;
    for (int k = 0; k < 3; k++) {
      if (star3[k]) {
        s.lo[k] = 0;
        s.hi[k] = a->n[k];
      } else {
        s.lo[k] = wlo[k] + off3[k];
        s.hi[k] = whi[k] + off3[k];
        if (s.lo[k] < 0) s.lo[k] = 0;
        if (s.hi[k] > a->n[k]) s.hi[k] = a->n[k];
      }
      if (s.lo[k] >= s.hi[k]) empty = 1;
    }
    if (!empty) region_push(out, &s);
  }
}

/* ------------------------------------------------------------ ApplyKernel */
/* Table 2 HDArrayApplyKernel; the order of Sec. 3.1: derive LUSE, intersect
 * with GDEF (Eq. 1-2), communicate, update GDEF for the receivers, run the
 * kernel, then update LDEF/GDEF for the defined arrays (Eq. 3-4). */
int orc_apply(orc_ctx *c, int k, int part, int nargs, const int *arrs, int nscal, const double *scal) {
  if (k < 0 || k >= c->nk || part < 0 || part >= c->npart) return ORC_EINVAL;
  kern_t *kn = &c->kn[k];
  part_t *pt = &c->pt[part];
  kspec_t ks;
  if (!kspec(kn->builtin, &ks)) return ORC_EKERNEL;
  if (nargs != ks.nargs || nscal < ks.nscal) return ORC_EINVAL;
  arr_t *A[8];
  for (int i = 0; i < nargs; i++) {
    A[i] = get_arr(c, arrs[i]);
    if (!A[i]) return ORC_EINVAL;
  }
  arr_t *ao = A[ks.out];
  for (int i = 0; i < ks.nin; i++)
    if (arrs[ks.in[i]] == arrs[ks.out]) return ORC_EINVAL;
  if (ao->type != ORC_F32 && kn->builtin != ORC_K_COPY) return ORC_EINVAL;
  if (ks.dim && ao->dim != ks.dim) return ORC_EINVAL;
  if (pt->dim != ao->dim) return ORC_EINVAL;
  switch (kn->builtin) {
    case ORC_K_JACOBI2D:
    case ORC_K_COPY:
    case ORC_K_STENCIL3D7:
    case ORC_K_CONV2D9:
      if (memcmp(A[0]->n, A[1]->n, sizeof(A[0]->n)) || A[0]->esize != A[1]->esize) return ORC_EINVAL;
      if (kn->builtin != ORC_K_COPY && A[1]->type != ORC_F32) return ORC_EINVAL;
      break;
    case ORC_K_TRI2D:
      if (memcmp(A[0]->n, A[1]->n, sizeof(A[0]->n)) || A[1]->type != ORC_F32 || A[0]->n[1] != A[0]->n[2])
        return ORC_EINVAL;
      break;
    case ORC_K_MATMUL:
      if (A[0]->type != ORC_F32 || A[1]->type != ORC_F32 || A[0]->dim != 2 || A[1]->dim != 2) return ORC_EINVAL;
      if (A[0]->n[2] != A[1]->n[1] || A[2]->n[1] != A[0]->n[1] || A[2]->n[2] != A[1]->n[2]) return ORC_EINVAL;
      break;
  }
  for (int d = 0; d < pt->ndev; d++)
    for (int j = 0; j < 3; j++)
      if (pt->hi[d][j] > ao->n[j]) return ORC_EBOUNDS;

  /* distinct arrays in argument order, with their use / def regions */
  int dist[8], nd = 0, firstpos[8];
  for (int i = 0; i < nargs; i++) {
    int seen = 0;
    for (int j = 0; j < nd; j++)
      if (dist[j] == arrs[i]) seen = 1;
    if (!seen) {
      firstpos[nd] = i;
      dist[nd++] = arrs[i];
    }
  }
  region_t (*use)[64] = (region_t(*)[64])calloc((size_t)nd, sizeof(region_t[64]));
  region_t (*def)[64] = (region_t(*)[64])calloc((size_t)nd, sizeof(region_t[64]));
  for (int j = 0; j < nd; j++)
    for (int i = 0; i < nargs; i++) {
      if (arrs[i] != dist[j]) continue;
      for (int d = 0; d < pt->ndev; d++) {
        if (pt->lo[d][0] >= pt->hi[d][0] || pt->lo[d][1] >= pt->hi[d][1] || pt->lo[d][2] >= pt->hi[d][2])
          continue; /* device without work */
        build_region(c, kn, part, i, dist[j], 0, d, pt->lo[d], pt->hi[d], &use[j][d]);
        build_region(c, kn, part, i, dist[j], 1, d, pt->lo[d], pt->hi[d], &def[j][d]);
      }
    }
  int rc = ORC_OK;
  /* race-free requirement (Sec. 1): definitions of different devices in one
   * call must not overlap */
  for (int j = 0; j < nd && rc == ORC_OK; j++) {
    arr_t *a = &c->ar[dist[j]];
    int8_t *wr = NULL;
    for (int d = 0; d < pt->ndev && rc == ORC_OK; d++) {
      if (def[j][d].n == 0) continue;
      if (!wr) {
        wr = (int8_t *)malloc((size_t)a->N);
        memset(wr, -1, (size_t)a->N);
      }
      unsigned char *m = region_mask_full(&def[j][d], a->n);
      int race = 0;
#pragma omp parallel for reduction(| : race) schedule(static)
      for (int64_t x = 0; x < a->N; x++)
        if (m[x]) {
          if (wr[x] >= 0 && wr[x] != d) race = 1;
          wr[x] = (int8_t)d;
        }
      if (race) rc = ORC_ERACE;
      free(m);
    }
    free(wr);
  }
  if (rc == ORC_OK) {
    /* Eq. 1-2: all messages come from the state before the call */
    msg_reset(c);
    for (int j = 0; j < nd; j++) comm_array(c, firstpos[j], dist[j], use[j]);
    c->drop_idx = -1;
    for (int j = 0; j < nd; j++)
      if (check_coherent(c, &c->ar[dist[j]], use[j])) rc = ORC_ECOHERENCE;
  }
  if (rc == ORC_OK && c->evalk) {
    keval_t t;
    memset(&t, 0, sizeof(t));
    t.aout = ao;
    t.ain0 = A[ks.in[0]];
    t.ain1 = ks.nin > 1 ? A[ks.in[1]] : NULL;
    for (int i = 0; i < 9 && i < nscal; i++) {
      t.cf[i] = (float)scal[i];
      t.cfd[i] = (double)(float)scal[i];
    }
    /* global evaluation of the FP32 and FP64 runs (inputs are distinct from
     * the output, so the pre-call snapshot is the inputs themselves) */
    size_t obytes = (size_t)ao->N * (size_t)ao->esize;
    unsigned char *newv = (unsigned char *)malloc(obytes);
    double *newd = (double *)malloc(sizeof(double) * (size_t)ao->N);
    memcpy(newv, ao->truth, obytes);
    memcpy(newd, ao->truth64, sizeof(double) * (size_t)ao->N);
    t.in0 = t.ain0->truth;
    t.in1 = t.ain1 ? t.ain1->truth : NULL;
    t.in0d = t.ain0->truth64;
    t.in1d = t.ain1 ? t.ain1->truth64 : NULL;
    t.out = newv;
    t.outd = newd;
    for (int d = 0; d < pt->ndev; d++) eval_region(&t, kn->builtin, pt->lo[d], pt->hi[d]);
    /* per-device runs on each device's own buffer */
    if (c->simulate) {
      for (int d = 0; d < pt->ndev; d++) {
        keval_t u = t;
        u.in0 = devbuf(t.ain0, d);
        u.in1 = t.ain1 ? devbuf(t.ain1, d) : NULL;
        u.h0 = t.ain0->holders;
        u.h1 = t.ain1 ? t.ain1->holders : NULL;
        u.bit = BIT(d);
        u.bad = 0;
        u.out = devbuf(ao, d);
        u.outd = NULL;
        u.in0d = NULL;
        eval_region(&u, kn->builtin, pt->lo[d], pt->hi[d]);
        c->bad_reads += u.bad;
      }
    }
    memcpy(ao->truth, newv, obytes);
    memcpy(ao->truth64, newd, sizeof(double) * (size_t)ao->N);
    free(newv);
    free(newd);
    /* each device's written cells must now equal the global result */
    if (c->simulate && c->bad_reads == 0) {
      for (int d = 0; d < pt->ndev && rc == ORC_OK; d++) {
        unsigned char *b = devbuf(ao, d);
        for (int64_t p = pt->lo[d][0]; p < pt->hi[d][0]; p++)
          for (int64_t r = pt->lo[d][1]; r < pt->hi[d][1]; r++)
            for (int64_t q = pt->lo[d][2]; q < pt->hi[d][2]; q++) {
              if (kn->builtin == ORC_K_TRI2D && q > r) continue;
              int64_t x = (p * ao->n[1] + r) * ao->n[2] + q;
              if (memcmp(b + (size_t)x * (size_t)ao->esize, ao->truth + (size_t)x * (size_t)ao->esize,
                         (size_t)ao->esize))
                rc = ORC_ECOHERENCE;
            }
      }
    }
  }
  if (rc == ORC_OK) {
    /* Eq. 3-4, "union LDEF", with overwrite kill: the definer becomes the
     * owner and the only holder */
    for (int j = 0; j < nd; j++) {
      arr_t *a = &c->ar[dist[j]];
      for (int d = 0; d < pt->ndev; d++) {
        if (def[j][d].n == 0) continue;
        unsigned char *m = region_mask_full(&def[j][d], a->n);
#pragma omp parallel for schedule(static)
        for (int64_t x = 0; x < a->N; x++)
          if (m[x]) {
            a->owner[x] = (int8_t)d;
            a->holders[x] = BIT(d);
          }
        free(m);
      }
    }
  }
  for (int j = 0; j < nd; j++)
    for (int d = 0; d < 64; d++) {
      region_free(&use[j][d]);
      region_free(&def[j][d]);
    }
  free(use);
  free(def);
  return rc;
}

/* ---------------------------------------------------- Write / Read / Reduce */
static int part_regions(orc_ctx *c, int part, arr_t *a, region_t *rg /*[64]*/) {
  part_t *pt = &c->pt[part];
  if (pt->dim != a->dim) return ORC_EINVAL;
  for (int d = 0; d < pt->ndev; d++) {
    shape_t s;
    memset(&s, 0, sizeof(s));
    int empty = 0;
    for (int k = 0; k < 3; k++) {
      s.lo[k] = pt->lo[d][k];
      s.hi[k] = pt->hi[d][k];
      if (s.hi[k] > a->n[k]) return ORC_EBOUNDS;
      if (s.lo[k] >= s.hi[k]) empty = 1;
    }
    if (!empty) region_push(&rg[d], &s);
  }
  /* overlapping device regions make Write/Reduce ambiguous */
  for (int d = 0; d < pt->ndev; d++)
    for (int e = d + 1; e < pt->ndev; e++) {
      if (!rg[d].n || !rg[e].n) continue;
      int ov = 1;
      for (int k = 0; k < 3; k++)
        if (rg[d].s[0].hi[k] <= rg[e].s[0].lo[k] || rg[e].s[0].hi[k] <= rg[d].s[0].lo[k]) ov = 0;
      if (ov) return ORC_EINVAL;
    }
  return ORC_OK;
}

/* Table 2 HDArrayWrite: the partition's section of uA goes to each device;
 * that device (and the host, which got the same values) now hold it. */
int orc_write(orc_ctx *c, int arr, const void *uA, int part) {
  arr_t *a = get_arr(c, arr);
  if (!a || part < 0 || part >= c->npart || !uA) return ORC_EINVAL;
  region_t rg[64];
  memset(rg, 0, sizeof(rg));
  int rc = part_regions(c, part, a, rg);
  if (rc == ORC_OK) {
    msg_reset(c);
    size_t es = (size_t)a->esize;
    for (int d = 0; d < 64; d++) {
      if (!rg[d].n) continue;
      shape_t *s = &rg[d].s[0];
      unsigned char *buf = c->simulate ? devbuf(a, d) : NULL;
      for (int64_t p = s->lo[0]; p < s->hi[0]; p++)
        for (int64_t r = s->lo[1]; r < s->hi[1]; r++)
          for (int64_t q = s->lo[2]; q < s->hi[2]; q++) {
            int64_t x = (p * a->n[1] + r) * a->n[2] + q;
            const unsigned char *v = (const unsigned char *)uA + (size_t)x * es;
            memcpy(a->truth + (size_t)x * es, v, es);
            memcpy(a->host + (size_t)x * es, v, es);
            if (buf) memcpy(buf + (size_t)x * es, v, es);
            if (a->type == ORC_F32)
              a->truth64[x] = ldf(a->truth, x);
            else if (a->type == ORC_F64)
              memcpy(&a->truth64[x], v, 8);
            else {
              int32_t iv;
              memcpy(&iv, v, 4);
              a->truth64[x] = iv;
            }
            a->owner[x] = (int8_t)d;
            a->holders[x] = BIT(d) | BIT(ORC_HOST);
          }
    }
  }
  for (int d = 0; d < 64; d++) region_free(&rg[d]);
  return rc;
}

/* Table 2 HDArrayRead: the host is the user of the partition's sections;
 * whatever it does not hold comes from the owner. */
int orc_read(orc_ctx *c, int arr, void *uA, int part) {
  arr_t *a = get_arr(c, arr);
  if (!a || part < 0 || part >= c->npart || !uA) return ORC_EINVAL;
  region_t rg[64];
  memset(rg, 0, sizeof(rg));
  int rc = part_regions(c, part, a, rg);
  if (rc == ORC_OK) {
    region_t use[64];
    memset(use, 0, sizeof(use));
    for (int d = 0; d < 64; d++)
      for (int i = 0; i < rg[d].n; i++) region_push(&use[ORC_HOST], &rg[d].s[i]);
    msg_reset(c);
    comm_array(c, 0, arr, use);
    c->drop_idx = -1;
    if (check_coherent(c, a, use)) rc = ORC_ECOHERENCE;
    size_t es = (size_t)a->esize;
    unsigned char *m = region_mask_full(&use[ORC_HOST], a->n);
    for (int64_t x = 0; x < a->N; x++)
      if (m[x]) memcpy((unsigned char *)uA + (size_t)x * es, (c->simulate ? a->host : a->truth) + (size_t)x * es, es);
    free(m);
    for (int d = 0; d < 64; d++) region_free(&use[d]);
  }
  for (int d = 0; d < 64; d++) region_free(&rg[d]);
  return rc;
}

/* Table 2 HDArrayReduce: each device's section is that device's use (so the
 * communication happens first), each device reduces its section in row-major
 * order, and the partial results are combined in device order.  Float data
 * is accumulated in FP64; integer SUM/PROD wrap modulo 2^32. */
int orc_reduce(orc_ctx *c, int arr, int op, int part, double *res_f, int64_t *res_i) {
  arr_t *a = get_arr(c, arr);
  if (!a || part < 0 || part >= c->npart || op < ORC_SUM || op > ORC_MIN) return ORC_EINVAL;
  region_t rg[64];
  memset(rg, 0, sizeof(rg));
  int rc = part_regions(c, part, a, rg);
  if (rc == ORC_OK) {
    msg_reset(c);
    comm_array(c, 0, arr, rg);
    c->drop_idx = -1;
    if (check_coherent(c, a, rg)) rc = ORC_ECOHERENCE;
    double fr = op == ORC_SUM ? 0.0 : op == ORC_PROD ? 1.0 : op == ORC_MAX ? -INFINITY : INFINITY;
    uint32_t ir = op == ORC_SUM ? 0u : op == ORC_PROD ? 1u : op == ORC_MAX ? 0x80000000u : 0x7fffffffu;
    for (int d = 0; d < 64; d++) {
      if (!rg[d].n) continue;
      shape_t *s = &rg[d].s[0];
      const unsigned char *b = c->simulate ? devbuf(a, d) : a->truth;
      double fp = op == ORC_SUM ? 0.0 : op == ORC_PROD ? 1.0 : op == ORC_MAX ? -INFINITY : INFINITY;
      uint32_t ip = op == ORC_SUM ? 0u : op == ORC_PROD ? 1u : op == ORC_MAX ? 0x80000000u : 0x7fffffffu;
      for (int64_t p = s->lo[0]; p < s->hi[0]; p++)
        for (int64_t r = s->lo[1]; r < s->hi[1]; r++)
          for (int64_t q = s->lo[2]; q < s->hi[2]; q++) {
            int64_t x = (p * a->n[1] + r) * a->n[2] + q;
            if (a->type == ORC_I32) {
              int32_t v;
              memcpy(&v, b + 4 * x, 4);
              if (op == ORC_SUM) ip += (uint32_t)v;
              if (op == ORC_PROD) ip *= (uint32_t)v;
              if (op == ORC_MAX && v > (int32_t)ip) ip = (uint32_t)v;
              if (op == ORC_MIN && v < (int32_t)ip) ip = (uint32_t)v;
            } else {
              double v;
              if (a->type == ORC_F32)
                v = ldf(b, x);
              else
                memcpy(&v, b + 8 * x, 8);
              if (op == ORC_SUM) fp += v;
              if (op == ORC_PROD) fp *= v;
              if (op == ORC_MAX && v > fp) fp = v;
              if (op == ORC_MIN && v < fp) fp = v;
            }
          }
      if (a->type == ORC_I32) {
        if (op == ORC_SUM) ir += ip;
        if (op == ORC_PROD) ir *= ip;
        if (op == ORC_MAX && (int32_t)ip > (int32_t)ir) ir = ip;
        if (op == ORC_MIN && (int32_t)ip < (int32_t)ir) ir = ip;
      } else {
        if (op == ORC_SUM) fr += fp;
        if (op == ORC_PROD) fr *= fp;
        if (op == ORC_MAX && fp > fr) fr = fp;
        if (op == ORC_MIN && fp < fr) fr = fp;
      }
    }
    if (res_f) *res_f = fr;
    if (res_i) *res_i = (int32_t)ir;
  }
  for (int d = 0; d < 64; d++) region_free(&rg[d]);
  return rc;
}

/* ------------------------------------------------------------------- dumps */
int64_t orc_last_nmsgs(orc_ctx *c) { return c->nmsg; }
int64_t orc_last_messages(orc_ctx *c, int64_t *out, int64_t cap) {
  int64_t n = c->nmsg < cap ? c->nmsg : cap;
  memcpy(out, c->msg, sizeof(int64_t) * ORC_MSG_NF * (size_t)n);
  return c->nmsg;
}
int64_t orc_last_pack_bytes(orc_ctx *c) { return c->packbytes; }
int64_t orc_last_pack(orc_ctx *c, void *out, int64_t cap) {
  int64_t n = c->packbytes < cap ? c->packbytes : cap;
  if (n > 0) memcpy(out, c->pack, (size_t)n);
  return c->packbytes;
}
int orc_gdef(orc_ctx *c, int arr, int8_t *owner, uint64_t *holders) {
  arr_t *a = get_arr(c, arr);
  if (!a) return ORC_EINVAL;
  if (owner) memcpy(owner, a->owner, (size_t)a->N);
  if (holders) memcpy(holders, a->holders, sizeof(uint64_t) * (size_t)a->N);
  return ORC_OK;
}
int orc_truth(orc_ctx *c, int arr, void *out) {
  arr_t *a = get_arr(c, arr);
  if (!a) return ORC_EINVAL;
  memcpy(out, a->truth, (size_t)a->N * (size_t)a->esize);
  return ORC_OK;
}
int orc_truth64(orc_ctx *c, int arr, double *out) {
  arr_t *a = get_arr(c, arr);
  if (!a) return ORC_EINVAL;
  memcpy(out, a->truth64, sizeof(double) * (size_t)a->N);
  return ORC_OK;
}
int orc_device_buffer(orc_ctx *c, int arr, int dev, void *out) {
  arr_t *a = get_arr(c, arr);
  if (!a || dev < 0 || dev > ORC_HOST) return ORC_EINVAL;
  memcpy(out, devbuf(a, dev), (size_t)a->N * (size_t)a->esize);
  return ORC_OK;
}
int64_t orc_bad_reads(orc_ctx *c) { return c->bad_reads; }
void orc_inject_drop(orc_ctx *c, int64_t idx) { c->drop_idx = idx; }

/* ------------------------------------------------- FP64 global references */
/* u_{t+1} = S(u_t), S the 7-point stencil with fixed boundary (see
 * eval_s3d_cell), in FP64 on the whole array. */
static void s3d_step64(const int64_t *n, const double *u, const double *cf, double *v) {
  int64_t si = n[1] * n[2], sj = n[2];
  for (int64_t i = 0; i < n[0]; i++)
    for (int64_t j = 0; j < n[1]; j++)
      for (int64_t k = 0; k < n[2]; k++) {
        int64_t x = i * si + j * sj + k;
        int interior = i >= 1 && i <= n[0] - 2 && j >= 1 && j <= n[1] - 2 && k >= 1 && k <= n[2] - 2;
        if (!interior) {
          v[x] = u[x];
          continue;
        }
        v[x] = cf[0] * u[x] + cf[1] * u[x - si] + cf[2] * u[x + si] + cf[3] * u[x - sj] + cf[4] * u[x + sj] +
               cf[5] * u[x - 1] + cf[6] * u[x + 1];
      }
}

void orc_s3d_forward64(const int64_t *n, const double *u0, const double *cf, int T, double *uT) {
  int64_t N = n[0] * n[1] * n[2];
  double *a = (double *)malloc(sizeof(double) * (size_t)N), *b = (double *)malloc(sizeof(double) * (size_t)N);
  memcpy(a, u0, sizeof(double) * (size_t)N);
  for (int t = 0; t < T; t++) {
    s3d_step64(n, a, cf, b);
    double *tmp = a;
    a = b;
    b = tmp;
  }
  memcpy(uT, a, sizeof(double) * (size_t)N);
  free(a);
  free(b);
}

/* Reverse mode of L = sum(w * u_T) through T steps of S, by the definition
 * of the transpose: for an interior output y, u_{t+1}[y] depends on
 * u_t[y + e] with weight c_e, so gbar_t[y + e] += c_e * gbar_{t+1}[y] and
 * cbar_e += gbar_{t+1}[y] * u_t[y + e]; a boundary output copies its input. */
void orc_s3d_adjoint64(const int64_t *n, const double *u0, const double *cf, int T, const double *w,
                       double *gu0, double *gcf) {
  int64_t N = n[0] * n[1] * n[2];
  int64_t si = n[1] * n[2], sj = n[2];
  double *states = (double *)malloc(sizeof(double) * (size_t)N * (size_t)(T + 1));
  memcpy(states, u0, sizeof(double) * (size_t)N);
  for (int t = 0; t < T; t++) s3d_step64(n, states + (size_t)t * (size_t)N, cf, states + (size_t)(t + 1) * (size_t)N);
  double *g = (double *)malloc(sizeof(double) * (size_t)N), *h = (double *)malloc(sizeof(double) * (size_t)N);
  memcpy(g, w, sizeof(double) * (size_t)N);
  for (int e = 0; e < 7; e++) gcf[e] = 0.0;
  const int64_t offs[7] = {0, -si, si, -sj, sj, -1, 1};
  for (int t = T - 1; t >= 0; t--) {
    const double *u = states + (size_t)t * (size_t)N;
    memset(h, 0, sizeof(double) * (size_t)N);
    for (int64_t i = 0; i < n[0]; i++)
      for (int64_t j = 0; j < n[1]; j++)
        for (int64_t k = 0; k < n[2]; k++) {
          int64_t y = i * si + j * sj + k;
          int interior = i >= 1 && i <= n[0] - 2 && j >= 1 && j <= n[1] - 2 && k >= 1 && k <= n[2] - 2;
          if (!interior) {
            h[y] += g[y];
            continue;
          }
          for (int e = 0; e < 7; e++) {
            h[y + offs[e]] += cf[e] * g[y];
            gcf[e] += g[y] * u[y + offs[e]];
          }
        }
    double *tmp = g;
    g = h;
    h = tmp;
  }
  memcpy(gu0, g, sizeof(double) * (size_t)N);
  free(states);
  free(g);
  free(h);
}

/* Threads the OpenMP loops of the oracle use (timing reports only). */
int orc_threads(void) { return omp_get_max_threads(); }

// hd_internal.hpp — structures shared by the host planner and the gfx950
// kernels of the HDArray runtime.  All are plain data, laid out identically
// on host and device.
//
// GDEF representation (Sec. 2.1 "GDEF", per element exact): every array is
// viewed as G = n0*n1 rows of n2 elements (normalised planes, rows, cols).
// Each row holds a run-length list of intervals [start_i, start_{i+1}) with
// one (owner, holders) state each; adjacent intervals always differ, so the
// list of a row is unique.  The list of row g lives at ivl[g*cap .. g*cap+cnt[g]).
//
// Bands: the host keeps, per array, plane and row breakpoints; the rows of
// a band (planes [pbrk[i], pbrk[i+1]) x rows [rbrk[k], rbrk[k+1])) all have
// the list stored at the band's first row, its representative (the other
// rows' storage is stale unless the array was last used row by row).  A
// call's derivation works on cells (a band of planes x a band of rows on
// which the arrays' bands and the call's use and def sections are uniform):
// one slice per cell with use sections, read from the cell's first row, and
// one GDEF update per cell, written to that row only; a cell that does not
// start a band first gets its band's list copied to its first row.  So the
// work of a call is proportional to its sections, not to rows.
#pragma once
#include <stdint.h>

namespace hd {

constexpr int kHost = 63;
constexpr int kMaxDev = 63;
constexpr int kMaxCap = 256;        // largest per-row interval capacity
constexpr int kMaxRunsRow = 256;    // runs one use row may produce
constexpr int kMaxCallArrays = 8;   // distinct arrays in one ApplyKernel
constexpr int kMaxBoundaries = 1024;// elementary boundaries of one GDEF row update
constexpr int kRunSlot = 16;        // runs stored in a use row's own slot; more spill to a pool
constexpr int kCompactCarr = 1024;  // call-arrays one compaction handles (plain calls: at most 8)

struct Ivl {
  int32_t start;
  int32_t owner;
  uint64_t holders;
};

// Endpoint e's buffer holds a window of the array (every element e ever
// holds or its kernels read lies inside it): element (p, r, c) sits at
// buf[e] + (p * ps[e] + r * rs[e] + c) * esize, buf[e] being the window's
// origin shifted back to global (0, 0, 0).  A window is either the whole
// array with the dense strides (rs = n2, ps = n1 * n2; the default, and
// always for 3-D arrays) or a box whose first column and row stride are
// multiples of 4 elements; either way a float4 at a column that is a
// multiple of 4 is aligned when rs is a multiple of 4.  [63] = the host
// buffer (pinned, device-mapped, full extent).
struct ArrDev {
  int64_t n[3];
  int32_t esize;
  int32_t cap;
  Ivl *ivl;
  int32_t *cnt;
  char *buf[64];
  int64_t rs[64];  // row stride (elements)
  int64_t ps[64];  // plane stride (elements)
};

// Element offset of (p, r, c) in endpoint e's buffer.
#define HD_EOFF(a, e, p, r, c) ((int64_t)(p) * (a).ps[e] + (int64_t)(r) * (a).rs[e] + (int64_t)(c))

// A use segment of one row for destination dst, or a def segment of device
// dst (flags bit 0: the host also holds the value afterwards, for Write).
struct Seg {
  int32_t dst;
  int32_t c0, c1;
  int32_t flags;
};

// One item of a stacking level: a run (level 1: src, dst, [a0,a1) = cols) or
// a rectangle (level 2: cols [a0,a1), rows [b0,b1)); pos0/pos1 carry the
// stacked extent once the item is a head.
struct Item {
  int32_t src, dst, a0, a1, b0, b1, pos0, pos1;
};

// A run found in a use row before sorting: source, destination, columns.
struct Run {
  int32_t src, dst, a0, a1;
};

// One level-1 slice (a cell with use sections, read at its representative
// row) as dev_runs reads it: a single record.
struct SliceRec {
  int32_t arr;   // runtime array id
  int32_t seg0;  // first use segment of the row
  int32_t nseg;
  int32_t pad;
  int64_t grow;  // global row (plane * n1 + row)
};

// One cell of a GDEF update as k_gdef reads it (its representative row):
// a single record.
struct GRowRec {
  int32_t arr;    // runtime array id
  int32_t slice;  // level-1 slice whose runs add holders, or -1
  int32_t dseg0;  // first definition segment of the row
  int32_t ndseg;
  int64_t grow;   // global row (plane * n1 + row)
  int32_t full;   // 1: the definitions tile the row and no holders are added
  int32_t pad;
};

struct MsgRec {
  int32_t aidx, arr, src, dst;
  int32_t lo[3], hi[3];
  int32_t argpos, esize;
  int64_t off, bytes;
};

struct CallArr {
  int32_t arr;      // runtime array id
  int32_t argpos;   // first argument position in the call
  int32_t esize;
  int32_t is3d;
  int64_t n[3];
  int32_t slice0, slice1;  // level-1 slices (use rows) of this array
  int32_t grp0, grp1;      // level-1 groups (planes with use rows)
};

struct MsgHdr {
  int64_t nmsg;
  int64_t bytes;
};

// A band list copied from one row to another of the same array before a
// derivation (src: the band's representative, dst: the first row of a cell
// that splits the band).
struct MatRec {
  int32_t arr;
  int32_t pad;
  int64_t src, dst;
};

// One stacking level: slices with a (group, position) key and an item list.
// A slice covers positions [pos, pend) (rows of a band, or planes of a band
// at level 2); pend null: one position each.
struct Level {
  int32_t nsl;
  const int32_t *grp;  // [nsl]
  const int32_t *pos;  // [nsl]
  const int32_t *pend; // [nsl] or null
  const int32_t *ioff; // [nsl]
  const int32_t *icnt; // [nsl]
  const Item *items;
  // scratch
  uint64_t *bmask;     // [nchunk]
  int32_t *bcnt;       // [nchunk]
  int32_t *bbase;      // [nchunk]
  int32_t *bandslice;  // [nsl+1]
  int32_t *nb;         // [1]
  int32_t *hoff;       // [nsl]
  int32_t *hcnt;       // [nsl]
  int64_t *hbytes;     // [nsl] bytes of the band's heads
  int32_t *bcarr;      // [nsl] call-array of the band
  int32_t *nofs;       // [nsl] compaction: first message of the band
  int64_t *bofs;       // [nsl] compaction: byte prefix of the band (before padding)
  const int32_t *grp_carr;  // group -> call-array (level 1); null when groups are call-arrays (level 2)
  const CallArr *carr;
  Item *heads;         // pool
  int32_t *head_top;   // [1]
  int64_t head_cap;
};

// One device's work box of a user kernel launch.  kind: 1 jacobi2d,
// 2 copy, 3 stencil3d7, 4 matmul, 5 tri2d; arrays by runtime id.
struct WorkBox {
  int32_t dev;
  int32_t kind;
  int32_t lo[3], hi[3];
  int32_t aout, ain, ain2, cidx;  // cidx: coefficient set of the box
  int64_t tile0;  // first tile index of this box in the launch
  int32_t seg;    // 3-D stencil kernels: planes marched by one wave
  int32_t pad;
};

// Up to kArgBoxes work boxes of one 2-D stencil launch passed by value
// (kernel arguments sit in the scalar cache): a workgroup finds its box and
// buffers without a dependent global load before its first data load.
constexpr int kArgBoxes = 16;
struct StackArgs {
  int32_t nbox, N1, N2, pad;
  int32_t lo1[kArgBoxes], lo2[kArgBoxes], hi1[kArgBoxes], hi2[kArgBoxes];
  int64_t tile0[kArgBoxes];
  const float *in[kArgBoxes];
  float *out[kArgBoxes];
  int64_t rsi[kArgBoxes], rso[kArgBoxes];  // row strides of the input and output buffers
};

// Per-call constant data uploaded once per plan.
struct PlanDev {
  int32_t ncarr;
  int32_t has3d;
  const CallArr *carr;
  // level 1
  int32_t nsl1;
  const int32_t *grp1;
  const int32_t *pos1;
  const int32_t *pend1;  // end row (exclusive) of each slice's band
  const int64_t *grow1;  // global row of each slice
  const int32_t *seg0;
  const int32_t *nseg;
  const Seg *useg;
  const SliceRec *srec;  // [nsl1]
  int32_t ngrp;
  const int32_t *grp_aidx;   // [ngrp]
  const int32_t *grp_plane;  // [ngrp]
  // level 2 (3-D arrays): slices = groups
  const int32_t *grp2;  // [ngrp] = aidx
  const int32_t *pos2;  // [ngrp] = first plane of the group's band
  const int32_t *pend2; // [ngrp] end plane (exclusive)
  // GDEF update rows: the ngfull rows the definitions tile come first
  int32_t ngrow;
  int32_t ngfull;
  int32_t gdef_lane;  // 1: update the other GDEF rows one per lane first (k_gdef), 0: one wave per row
  const GRowRec *grec;  // [ngrow]
  const Seg *dseg;
};

struct Work {
  int32_t *roff;   // [nsl1] run pool offset of each use row
  int32_t *rcnt;   // [nsl1]
  Item *runs;      // [nsl1 * kRunSlot] row slots, then the spill pool
  int32_t *run_top;  // spill pool top (relative to the pool start)
  int64_t run_cap;
  int32_t *ovf_cnt;   // GDEF rows left to the large-row path ([1]: workgroups done)
  int32_t *ovf_list;
  int32_t *ovf_list2;  // rows with more than 64 boundaries (LDS update)
  int32_t *goff;   // [ngrp] level-1 output offset per group
  int32_t *gcnt;   // [ngrp]
  Item *l1out;     // level-1 output (3-D)
  int64_t l1_cap;
  int32_t *err;    // device error word (first error wins)
  // plan cache, second step: when non-null and *skip is set, the small-form
  // derivation (runs and message table) is left out; the GDEF update runs
  const int32_t *skip;
};

// Arguments of the persistent batched step.
struct BatchArgs {
  PlanDev P;
  Level L1, L2;
  Work W;
  ArrDev *A;
  MsgRec *tab;
  MsgHdr *hdr;
  int64_t tab_cap;
  uint32_t *stg;
  const WorkBox *wb;
  const int32_t *tbox;  // box index of every tile
  int nbox;
  int64_t ntiles;
  unsigned *bar;
  int64_t spin_limit;  // device-clock ticks
  int64_t *clk;        // device-clock stamps taken by workgroup 0 at each phase boundary
  int64_t *cs;         // compaction scratch, 6 * kCompactCarr
};

}  // namespace hd

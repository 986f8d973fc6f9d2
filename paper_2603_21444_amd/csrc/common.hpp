// Device-side definitions shared by the SpGEMM kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spgemm.h"

namespace spg {

constexpr int kWave = 64;
constexpr int kEmpty = -1;          // empty hash slot (column indices are >= 0)
constexpr int kNB = SPG_NBINS;      // row bins
constexpr int kHeavyBin = 12;       // rows beyond every LDS table
constexpr int kMaxLdsBin = 11;      // largest LDS bin index
constexpr int kTail = 32;           // slots after a table: a probe walks at most kTail past it
constexpr int kLdsBitmapCols = 1 << 20;  // columns a heavy row can mark in LDS (128 KiB)
constexpr int kMclMaxCols = 1 << 24;     // MCL keys hold the column in 24 bits

// Status bits raised by kernels in the workspace header.
constexpr int kStatOverflow = 1;
constexpr int kStatCapacity = 2;
constexpr int kStatInvalid = 4;

// Upper edge of bin b (b >= 1): rows whose key (products or nnz) lies in
// (edge(b-1), edge(b)] land in bin b; bin 0 holds rows with key 0.
__host__ __device__ inline int64_t bin_edge(int b) { return b <= 0 ? 0 : (int64_t)8 << b; }

__host__ __device__ inline int bin_of(int64_t key, int maxbin) {
  if (key <= 0) return 0;
  int b = 1;
  while (b <= maxbin && key > bin_edge(b)) ++b;
  return b > maxbin ? kHeavyBin : b;
}

// Upper keys of the row bins as used by a binning pass: up[b] <= bin_edge(b)
// (a row in bin b still fits the tables sized for bin_edge(b)), non-
// decreasing, up[maxbin] = bin_edge(maxbin).  A lower up[b] sends the rows
// with keys in (up[b], bin_edge(b)] to bin b + 1, whose tables are twice as
// large: the bin threshold doubles as the table load factor of those rows.
struct BinEdges {
  int32_t up[kNB];
};

__host__ __device__ inline int bin_of(int64_t key, int maxbin, const BinEdges &E) {
  if (key <= 0) return 0;
  int b = 1;
  while (b <= maxbin && key > E.up[b]) ++b;
  return b > maxbin ? kHeavyBin : b;
}

// Hash table slots of an LDS bin: twice the bin's upper edge (load <= 1/2).
__host__ __device__ inline int bin_slots(int b) { return (int)(2 * bin_edge(b)); }

// One block product A_k B_k of the batched form, or one merge operand
// (a_identity: row i of A_k is the single entry (i, 1)).
struct Part {
  const int32_t *arp, *acol;
  const void *aval;
  const int32_t *brp, *bcol;
  const void *bval;
  int32_t a_identity;
  int32_t kdim;
};

struct Problem {
  int32_t K, m, n;
  Part part[SPG_MAX_PARTS];
};

// Workspace header (first 4 KiB of the caller's workspace).
struct WsHeader {
  int32_t status;
  int32_t pad0;
  int64_t nnz_total;
  int64_t products_total;
  int32_t bin_count[kNB];
  int32_t bin_start[kNB + 1];
  int32_t fallback_count;
  int32_t long_count;  // rows the row-key kernel leaves to k_rowkey_long: one block per row
  int32_t mid_count;   // ... one wave per row
  int32_t queue[kNB + 2];  // work-queue cursors: per bin, fallback rows, heavy rows
};
static_assert(sizeof(WsHeader) <= 256, "the operand descriptors follow at byte 256");

// Heavy rows shared by many blocks.  The symbolic pass describes each such
// row by ranges of 2^kSplitLog2W consecutive columns (products and distinct
// columns per range) and cuts the ranges into segments: a range with more
// than half of kSplitSeg products stands alone, the others are grouped so
// that a segment holds at most kSplitSeg products.  The numeric pass first
// scatters the row's products into per-range runs of a staging area, many
// blocks per row (items of about kSplitItem products), then merges every
// segment in LDS on its own, writing its part of the output row.
constexpr int kSplitLog2W = 13;         // columns per range: 8192
constexpr int kSplitMaxRanges = 1024;   // ranges per row: n <= 2^23
constexpr int kSplitSeg = 4096;         // products of a sorted segment at most
constexpr int kSplitItem = 2048;        // products per scatter item (target)

// Counters of the split path: staging entries, segments and items reserved
// by the symbolic pass (cleared with the header's counters), work-queue
// cursors of the numeric pass (cleared at every pass).
struct SplitCtl {
  unsigned long long stage;
  int32_t segs, items;
  int32_t q_scatter, q_accum;
  int32_t nuns;  // numeric pass: heavy rows left to the one-block kernels
};
// One split row (index h in the row list from the first split bin): first
// staging entry (-1: the row is not split), scatter items, products, and
// the row of C.
struct SplitRow {
  int32_t base, items, products, row;
};
// A segment of split row h (-1: unused): columns [c0, c1), products at
// staging entries stage .. stage + pcount, distinct columns dstart ..
// dstart + dcount of the row; out = row_ptr[row] + dstart, filled in by the
// numeric pass (-1: the row_ptr does not match).
struct SplitSeg {
  int32_t h, c0, c1, stage, pcount, dstart, dcount, out;
};
// Scatter item of split row h (-1: unused), row i of C: the products of
// the row's A entries [e0, e1) (all parts in order, numbered from 0).
struct SplitItem {
  int32_t h, i, e0, e1;
};
// Device view of the split region of a workspace.  F == 0: no split rows
// (the symbolic pass only counts).
struct SplitArgs {
  SplitCtl *ctl;
  SplitRow *rows;
  int32_t *fo;   // per row: F + 1 exclusive prefix sums of the products per range
  int32_t *cur;  // per row: F cursors of the scatter
  SplitSeg *segs;
  SplitItem *items;
  int32_t *scol;  // staging: columns, then values (pcap entries each)
  void *sval;
  int32_t F, hmax, segcap, itemcap;
  int64_t pcap;
  int32_t bin;  // first bin of the split rows
};

constexpr int kQueueFallback = kNB;
constexpr int kQueueHeavy = kNB + 1;

// Device work queue of a persistent launch: its blocks take the rows (items)
// of their list one at a time from a cursor in the workspace header, so a
// block that drew short rows takes more of them (the rows of one list can
// differ in work by orders of magnitude: power-law hubs sit next to short
// rows).  Thread 0 takes the item and the block reads it from LDS; the first
// barrier keeps thread 0 from overwriting the previous item too early.
__device__ __forceinline__ int block_next(int *cursor, int *item) {
  __syncthreads();
  if (threadIdx.x == 0) *item = atomicAdd(cursor, 1);
  __syncthreads();
  return *item;
}

// Operand arrays are read through global-address-space pointers: the
// pointers come from memory (the device copy of the Problem), and without
// the cast the compiler would emit flat loads, which also hold up every LDS
// wait and cannot be reordered around LDS atomics.
#define SPG_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const SPG_GLOBAL T *gp(const T *p) {
  return (const SPG_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ SPG_GLOBAL T *gpw(T *p) {
  return (SPG_GLOBAL T *)p;
}

__device__ inline int lane_id() { return __lane_id(); }

// Number of set bits of `mask` strictly below this lane.
__device__ inline int mbcnt(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

// Order-preserving home slot: floor(col * T / n) computed as the high half of
// col * floor(T * 2^32 / n); `mul` == 0 means T >= n and the slot is col.
__device__ inline uint32_t mono_slot(uint32_t col, uint32_t mul) { return __umulhi(col, mul); }

// Multiplier of the order-preserving home slot floor(col * T / n).  With
// T >= n it is 2^32 - 1, giving max(col - 1, 0): still non-decreasing in col
// and below T, and the slot computation needs no branch.
__host__ inline uint32_t mono_mul(int64_t T, int64_t n) {
  if (T >= n) return 0xffffffffu;
  return (uint32_t)(((uint64_t)T << 32) / (uint64_t)n);
}

// Fibonacci hashing for tables that need no order.
__device__ inline uint32_t scramble_slot(uint32_t col, int log2T) {
  return (col * 2654435769u) >> (32 - log2T);
}

template <typename T>
__device__ inline void lds_add(T *p, T v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// LDS float add by compare-and-swap: on this chip cheaper than the LDS
// float atomic when lanes rarely hit the same word.  FP64 keeps the atomic.
__device__ __forceinline__ void lds_add_cas(float *p, float v) {
  uint32_t *u = reinterpret_cast<uint32_t *>(p);
  uint32_t old = *u, seen;
  do {
    seen = old;
    old = atomicCAS(u, seen, __float_as_uint(__uint_as_float(seen) + v));
  } while (old != seen);
}
__device__ __forceinline__ void lds_add_cas(double *p, double v) { lds_add(p, v); }

template <typename T>
__device__ inline void global_add(T *p, T v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ inline T ld_val(const void *p, int64_t i) {
  return static_cast<const T *>(p)[i];
}

// Entries of row i of A_k: [start, end) into acol/aval (identity: one entry).
__device__ inline void a_row(const Part &P, int i, int &s, int &e) {
  if (P.a_identity) { s = 0; e = 1; }
  else { s = gp(P.arp)[i]; e = gp(P.arp)[i + 1]; }
}

template <typename VT>
__device__ inline void a_entry(const Part &P, int i, int p, int &brow, VT &a) {
  if (P.a_identity) { brow = i; a = VT(1); }
  else { brow = gp(P.acol)[p]; a = gp(static_cast<const VT *>(P.aval))[p]; }
}

__device__ inline int a_entry_row(const Part &P, int i, int p) {
  return P.a_identity ? i : gp(P.acol)[p];
}

}  // namespace spg

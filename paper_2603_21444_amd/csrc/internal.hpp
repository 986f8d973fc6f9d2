// Host-side internals shared by the launchers and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.hpp"

namespace spg {

struct DevInfo {
  int device = -1;
  int cus = 256;
  size_t lds_per_block = 65536;
  size_t lds_per_cu = 163840;
  int sym_maxbin = kMaxLdsBin;   // largest LDS bin of the symbolic pass
  int num_maxbin_f32 = 10;       // largest LDS bin of the FP32 numeric pass
  int num_maxbin_f64 = 9;        // largest LDS bin of the FP64 numeric pass
  int mcl_maxbin = 10;           // largest LDS bin of the MCL iteration
  int split_bin = 10;            // first bin of the rows split over many blocks
};

const DevInfo &dev_info();

// Byte offsets of the workspace regions.
struct WsLayout {
  size_t problem, binid, rows, fbrows, blockhist, scanpart, heavyacc, heavymap, total;
  int heavy_slots;
  // split heavy rows (staging in the heavy accumulator region); split_F == 0: off
  size_t split_ctl = 0, split_rows = 0, split_fo = 0, split_cur = 0, split_segs = 0,
         split_items = 0;
  int split_F = 0, split_hmax = 0, split_segcap = 0, split_itemcap = 0;
  int64_t split_pcap = 0;
  size_t mcl_rabs = 0, mcl_slots = 0;  // MCL only: row sums of |x|, heavy-row slots
};

// MCL heavy rows: per-slot scratch (candidate list, and cursor, end and value
// of the entries of rows too long for LDS: 20 B per column) and the number of
// slots (concurrent heavy rows, at most 512, at most 4 GiB of scratch).
inline size_t mcl_slot_bytes(int64_t n) {
  return ((size_t)20 * (size_t)(n > 0 ? n : 1) + 255) & ~(size_t)255;
}
inline int mcl_heavy_slots(int64_t n) {
  const int64_t s = ((int64_t)4 << 30) / (int64_t)mcl_slot_bytes(n);
  return (int)(s < 1 ? 1 : (s > 512 ? 512 : s));
}

WsLayout ws_layout(int64_t m, int64_t n, int heavy_slots);
int default_heavy_slots(int64_t n);

// What a pass needs to know about the bins: counts when read back (eager),
// lanes per row and lanes per A entry, per bin.
struct BinPlan {
  bool known = false;
  int count[kNB] = {0};
  int lanes[kNB] = {0};
  int sub[kNB] = {0};       // lanes sharing one A entry's B row, per bin
  int maxbin = kMaxLdsBin;  // last LDS bin; bins above go to the heavy kernel
  int heavy_slots = 1;
  int m = 0;  // rows
  int n = 0;
  int maxwin = 32;
};

hipError_t launch_setup(const Problem &pr, Problem *dst, WsHeader *hdr, bool reset,
                        bool clear_status, hipStream_t st, SplitCtl *sc = nullptr);
hipError_t launch_clear_status(WsHeader *hdr, hipStream_t st);
hipError_t launch_validate(const int32_t *rp, const int32_t *col, int rows, int ncols,
                           int64_t nnz, WsHeader *hdr, hipStream_t st);
// Default edges: up[b] = bin_edge(b).
BinEdges default_edges();
hipError_t launch_binning(const Problem *dpr, int m, int maxbin, const BinEdges &edges,
                          const WsLayout &L, char *ws,
                          int32_t *cnt_zero, hipStream_t st);
hipError_t launch_scan(int32_t *rp, int m, int64_t capacity, const WsLayout &L, char *ws,
                       hipStream_t st);
hipError_t launch_symbolic_bins(const Problem *dpr, const BinPlan &bp, const WsLayout &L,
                                char *ws, int32_t *cnt, hipStream_t st);
hipError_t launch_numeric(const Problem *dpr, const BinPlan &bp, const WsLayout &L, char *ws,
                          const int32_t *crp, int32_t *ccol, void *cval, int dtype,
                          hipStream_t st);
hipError_t configure_lds_limits(size_t lds_max);

// detws: NULL (dB by float atomics) or det_workspace_bytes(nnzB) bytes for
// the deterministic dB.
hipError_t launch_backward(const Problem *dpr, const BinPlan &bp, const WsLayout &L, char *ws,
                           const int32_t *crp, const int32_t *ccol, const void *w, int64_t nnzC,
                           const void *aval, void *dA, int64_t nnzA, void *dB, int64_t nnzB,
                           void *detws, int dtype, hipStream_t st);
size_t det_workspace_bytes(int64_t nnzB);
hipError_t configure_backward_lds(size_t lds_max);

// rpre: exponent before the normalisation; rpost: 0 = renormalise after the
// prune and top-k, else the exponent applied to the kept entries instead.
hipError_t launch_mcl(const Problem *dpr, const BinPlan &bp, const WsLayout &L, char *ws,
                      int rpre, int rpost, float prune, int topk, int cap, int32_t *pcol,
                      float *pval, int32_t *ycnt, hipStream_t st);
hipError_t launch_mcl_compact(int n, int cap, const int32_t *yrp, const int32_t *pcol,
                              const float *pval, int32_t *ycol, float *yval, const WsHeader *hdr,
                              hipStream_t st);
hipError_t configure_mcl_lds(size_t lds_max);
size_t mcl_lds_bytes(int b, int G);
int num_table_slots(int b, int G);

// One-row-per-wave pipelined kernels (bins whose rows use 64 lanes).
size_t sym_wave_lds_bytes(int b);
size_t num_wave_lds_bytes(int b, size_t vbytes, bool pack);
void launch_sym_wave(const Problem *dpr, const int32_t *rows, const WsHeader *hdr, int bin,
                     int lS, int count, int32_t *cnt, hipStream_t st);
void launch_num_wave(const Problem *dpr, const int32_t *rows, WsHeader *hdr, int bin, int lS,
                     int count, uint32_t mul, int maxwin, bool pack, const int32_t *crp,
                     int32_t *ccol, void *cval, bool f64, int32_t *fb, hipStream_t st);
hipError_t configure_wave_lds(size_t lds_max);

// Permutation B[prow[i], pcol[j]] = A[i, j] (either array may be NULL:
// identity).  Workspace regions from perm_workspace_bytes.
size_t perm_workspace_bytes(int64_t m, int64_t n, size_t *rinv_off, size_t *cinv_off,
                            size_t *long_off, size_t *scan_off);
hipError_t launch_permute(const spg_csr &A, const int32_t *prow, const int32_t *pcol, int dtype,
                          int32_t *brp, int32_t *bcol, void *bval, char *ws, hipStream_t st);

// One thread per row for bin 1 (at most 16 products per row): tuning lanes
// value 1 selects these kernels.
void launch_sym_tiny(const Problem *dpr, const int32_t *rows, const WsHeader *hdr, int bin,
                     int count, bool known, int32_t *cnt, hipStream_t st);
void launch_num_tiny(const Problem *dpr, const int32_t *rows, WsHeader *hdr, int bin, int count,
                     bool known, const int32_t *crp, int32_t *ccol, void *cval, bool f64,
                     hipStream_t st);

// Rows split over many blocks: the symbolic kernel of the rows from bin blo
// on (counts, and the split description when sa.F > 0), and the numeric
// pass of the split rows from bin blo on (rows handled by the LDS kernels
// of the pass's dtype sit below blo).
SplitArgs split_args(const WsLayout &L, char *ws, int bin);
SplitCtl *split_ctl(const WsLayout &L, char *ws);  // NULL when the layout has no split region
size_t split_sym_static_lds();
hipError_t launch_sym_split(const Problem *dpr, const int32_t *rows, WsHeader *hdr, int blo,
                            int lS, bool lds_map, uint32_t *gbitmap, int grid, size_t lds,
                            int32_t *cnt, const SplitArgs &sa, hipStream_t st);
hipError_t launch_num_split(const Problem *dpr, const int32_t *rows, WsHeader *hdr, int blo,
                            int lS, const SplitArgs &sa, int32_t *ulist, const int32_t *crp,
                            int32_t *ccol, void *cval, bool f64, hipStream_t st);
hipError_t configure_split_lds(size_t lds_max);

// LDS bytes of one block of the symbolic / numeric kernel of bin b with G
// lanes per row.
size_t sym_lds_bytes(int b, int G);
size_t num_lds_bytes(int b, int G, size_t vbytes, bool pack);

}  // namespace spg

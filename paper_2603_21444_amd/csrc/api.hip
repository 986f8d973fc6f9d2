// C ABI of the local SpGEMM library (declared in include/spgemm.h).
//
// Host code only: argument checks, workspace layout, plan bookkeeping and
// the launch sequence of each call.  All arithmetic runs in the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "internal.hpp"

using namespace spg;

struct spg_plan_s {
  uint32_t flags = 0;
  spg_tuning tun{};
  bool tun_set = false;
  // state of the last symbolic (or merge count) call
  bool sym_done = false;
  bool merge_mode = false;
  bool counts_known = false;
  int K = 0, m = 0, n = 0;
  int kdim[SPG_MAX_PARTS] = {0};
  int64_t annz[SPG_MAX_PARTS] = {0}, bnnz[SPG_MAX_PARTS] = {0};
  int num_count[kNB] = {0};
  int sym_count[kNB] = {0};
  int64_t nnz = -1, products = -1;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  WsLayout L{};
  int32_t *crp = nullptr;
  hipStream_t stream = nullptr;
  WsHeader *host_hdr = nullptr;  // pinned readback buffer
  // workspace whose status word this plan has cleared at least once: a
  // capture-safe call clears it only on first use of a workspace, so an
  // error raised by one call of a captured sequence reaches the end of it
  const void *status_ws = nullptr;
  // lanes per A entry never exceed the mean B row length rounded up to a
  // power of two: with short B rows (an aggregation operator has one entry
  // per row) wider groups would leave lanes idle
  int sub_cap = 64;
};

namespace spg {

static std::mutex g_dev_mu;
constexpr int kMaxDevices = 64;
static DevInfo g_dev[kMaxDevices];  // fixed table: no allocation on any call
static int g_ndev = 0;

// Largest bin whose table fits one block (one row per block, 1024 lanes).
static int maxbin_for(size_t lds, int pass, size_t vbytes) {
  int b = kMaxLdsBin;
  auto bytes = [&](int bb) {
    if (pass == 0) return sym_lds_bytes(bb, 1024);
    if (pass == 1) return num_lds_bytes(bb, 1024, vbytes, false);
    return mcl_lds_bytes(bb, 1024);
  };
  while (b > 1 && bytes(b) > lds) --b;
  return b;
}

const DevInfo &dev_info() {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> g(g_dev_mu);
  for (int t = 0; t < g_ndev; ++t)
    if (g_dev[t].device == dev) return g_dev[t];
  DevInfo d;
  d.device = dev;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
    d.cus = v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
      v > 0)
    d.lds_per_block = (size_t)v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
          hipSuccess &&
      v > 0)
    d.lds_per_cu = (size_t)v;
  if (d.lds_per_cu < d.lds_per_block) d.lds_per_cu = d.lds_per_block;
  // the largest table of each pass that fits one block's LDS
  d.sym_maxbin = maxbin_for(d.lds_per_block, 0, 0);
  d.num_maxbin_f32 = maxbin_for(d.lds_per_block, 1, 4);
  d.num_maxbin_f64 = maxbin_for(d.lds_per_block, 1, 8);
  d.mcl_maxbin = maxbin_for(d.lds_per_block, 2, 4);
  d.split_bin = std::min(std::min(d.num_maxbin_f32, d.num_maxbin_f64) + 1, d.sym_maxbin + 1);
  (void)configure_lds_limits(d.lds_per_block);
  (void)configure_backward_lds(d.lds_per_block);
  (void)configure_mcl_lds(d.lds_per_block);
  (void)configure_split_lds(d.lds_per_block);
  (void)configure_wave_lds(d.lds_per_block);
  (void)hipGetLastError();
  if (g_ndev == kMaxDevices) {  // more devices than the table: reuse the last entry
    g_dev[kMaxDevices - 1] = d;
    return g_dev[kMaxDevices - 1];
  }
  g_dev[g_ndev] = d;
  return g_dev[g_ndev++];
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int default_heavy_slots(int64_t n) {
  const int64_t budget = (int64_t)2 << 30;  // dense accumulators of concurrent heavy rows
  int64_t s = budget / (std::max<int64_t>(n, 1) * 8);
  return (int)std::max<int64_t>(1, std::min<int64_t>(256, s));
}

WsLayout ws_layout(int64_t m, int64_t n, int heavy_slots) {
  WsLayout L{};
  const int64_t nblk = m == 0 ? 1 : (m + 255) / 256;
  const int64_t nparts = m == 0 ? 1 : (m + 2047) / 2048;
  size_t o = 0;
  o = align256(sizeof(WsHeader));
  L.problem = o;
  o = align256(o + sizeof(Problem));
  o = std::max<size_t>(o, 4096);
  L.binid = o;
  o = align256(o + (size_t)std::max<int64_t>(m, 1));
  L.rows = o;
  o = align256(o + 4 * (size_t)std::max<int64_t>(m, 1));
  L.fbrows = o;
  o = align256(o + 4 * (size_t)std::max<int64_t>(m, 1));
  L.blockhist = o;
  o = align256(o + 4 * (size_t)(nblk * kNB));
  L.scanpart = o;
  o = align256(o + 8 * (size_t)nparts);
  L.heavy_slots = heavy_slots;
  L.heavyacc = o;
  o = align256(o + (size_t)heavy_slots * (size_t)(std::max<int64_t>(n, 1) + 4) * 8);
  L.heavymap = o;  // used when a heavy row's bitmap does not fit in LDS
  o = align256(o + (size_t)heavy_slots * (size_t)((std::max<int64_t>(n, 1) + 31) / 32) * 4);
  // Split heavy rows: the products are staged in the heavy accumulator
  // region (a column and an FP64 value each, whatever the pass's dtype);
  // every split row has more than 4096 products, which bounds the rows, and
  // a row takes at most 3 segments and 1 item per 2048 products, plus one.
  const size_t acc_bytes = (size_t)heavy_slots * (size_t)(std::max<int64_t>(n, 1) + 4) * 8;
  const int64_t pcap = std::min<int64_t>((int64_t)(acc_bytes > 512 ? (acc_bytes - 512) / 12 : 0),
                                         (int64_t)INT32_MAX - 1);
  if (pcap >= 8192 && m > 0 && n > 0 && n <= ((int64_t)kSplitMaxRanges << kSplitLog2W)) {
    const int64_t hmax = std::min<int64_t>(m, pcap / 4096 + 1);
    L.split_F = (int)((n + (1 << kSplitLog2W) - 1) >> kSplitLog2W);
    L.split_pcap = pcap;
    L.split_hmax = (int)hmax;
    L.split_segcap = (int)std::min<int64_t>(INT32_MAX / 2, 3 * pcap / 2048 + hmax);
    L.split_itemcap = (int)std::min<int64_t>(INT32_MAX / 2, pcap / kSplitItem + hmax);
    L.split_ctl = o;
    o = align256(o + sizeof(SplitCtl));
    L.split_rows = o;
    o = align256(o + (size_t)hmax * sizeof(SplitRow));
    L.split_fo = o;
    o = align256(o + (size_t)hmax * (size_t)(L.split_F + 1) * 4);
    L.split_cur = o;
    o = align256(o + (size_t)hmax * (size_t)L.split_F * 4);
    L.split_segs = o;
    o = align256(o + (size_t)L.split_segcap * sizeof(SplitSeg));
    L.split_items = o;
    o = align256(o + (size_t)L.split_itemcap * sizeof(SplitItem));
  }
  L.total = o;
  return L;
}

SplitCtl *split_ctl(const WsLayout &L, char *ws) {
  return L.split_F > 0 ? reinterpret_cast<SplitCtl *>(ws + L.split_ctl) : nullptr;
}

SplitArgs split_args(const WsLayout &L, char *ws, int bin) {
  SplitArgs a{};
  a.bin = bin;
  if (L.split_F <= 0) return a;
  a.ctl = reinterpret_cast<SplitCtl *>(ws + L.split_ctl);
  a.rows = reinterpret_cast<SplitRow *>(ws + L.split_rows);
  a.fo = reinterpret_cast<int32_t *>(ws + L.split_fo);
  a.cur = reinterpret_cast<int32_t *>(ws + L.split_cur);
  a.segs = reinterpret_cast<SplitSeg *>(ws + L.split_segs);
  a.items = reinterpret_cast<SplitItem *>(ws + L.split_items);
  a.scol = reinterpret_cast<int32_t *>(ws + L.heavyacc);
  a.sval = ws + L.heavyacc + (((size_t)L.split_pcap * 4 + 255) & ~(size_t)255);
  a.F = L.split_F;
  a.hmax = L.split_hmax;
  a.segcap = L.split_segcap;
  a.itemcap = L.split_itemcap;
  a.pcap = L.split_pcap;
  return a;
}

}  // namespace spg

namespace {

spg_tuning default_tuning() {
  spg_tuning t{};
  // lanes per row for bins of at most 16, 32, ..., 16384 products or entries
  const int lanes[kNB] = {0, 8, 16, 16, 32, 64, 128, 256, 256, 512, 1024, 1024, 1024, 1024, 1024, 1024};
  for (int b = 0; b < kNB; ++b) {
    t.lanes[b] = lanes[b];
    // lanes per A entry: 16, but 32 for bin 9 (rows of 2049..4096 products,
    // 512-lane groups) and for the heavy rows (their B rows are the long
    // ones of power-law inputs), and 4 for the count's one-wave kernel (bin
    // 5), which gains from more A entries in flight
    t.sub[b] = b == 9 || b == kHeavyBin ? 32 : 16;
    t.sym_sub[b] = b == 5 ? 4 : b == 9 || b == kHeavyBin ? 32 : 16;
  }
  t.heavy_slots = 0;
  t.max_window = kTail;
  for (int b = 0; b < kNB; ++b) t.bin_edge[b] = 0;  // 0: the table capacity 8 * 2^b
  return t;
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int check_tuning(const spg_tuning &t) {
  for (int b = 1; b < kNB; ++b) {
    const bool one_per_row = b == 1 && t.lanes[b] == 1;  // bin 1 only
    if (!one_per_row && (!pow2(t.lanes[b]) || t.lanes[b] < 8 || t.lanes[b] > 1024))
      return SPG_ERR_ARG;
    if (!pow2(t.sub[b]) || t.sub[b] > 64) return SPG_ERR_ARG;
    if (!pow2(t.sym_sub[b]) || t.sym_sub[b] > 64) return SPG_ERR_ARG;
  }
  if (t.heavy_slots < 0 || t.max_window < 1 || t.max_window > kTail) return SPG_ERR_ARG;
  for (int b = 1; b < kNB; ++b)
    if (t.bin_edge[b] < 0 || t.bin_edge[b] > bin_edge(b)) return SPG_ERR_ARG;
  return SPG_OK;
}

// Upper keys of the product bins from the tuning: the tuned edge of each
// LDS bin (at most its table capacity), non-decreasing, and the last LDS bin
// always up to its capacity (rows above it are heavy rows either way).
BinEdges tuned_edges(const spg_tuning &t, int maxbin) {
  BinEdges E = default_edges();
  for (int b = 1; b < maxbin && b < kNB; ++b) {
    int32_t u = t.bin_edge[b] > 0 ? t.bin_edge[b] : (int32_t)bin_edge(b);
    if (u < E.up[b - 1]) u = E.up[b - 1];
    E.up[b] = u;
  }
  return E;
}

int hip_status(hipError_t e) { return e == hipSuccess ? SPG_OK : SPG_ERR_HIP; }

int read_header(spg_plan p, hipStream_t st) {
  if (!p->host_hdr) {
    if (hipHostMalloc(reinterpret_cast<void **>(&p->host_hdr), sizeof(WsHeader)) != hipSuccess) {
      p->host_hdr = nullptr;
      return SPG_ERR_HIP;
    }
  }
  if (hipMemcpyAsync(p->host_hdr, p->ws, sizeof(WsHeader), hipMemcpyDeviceToHost, st) !=
      hipSuccess)
    return SPG_ERR_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return SPG_ERR_HIP;
  return SPG_OK;
}

int status_from_bits(int bits) {
  if (bits & kStatInvalid) return SPG_ERR_INVALID;
  if (bits & kStatOverflow) return SPG_ERR_OVERFLOW;
  if (bits & kStatCapacity) return SPG_ERR_CAPACITY;
  return SPG_OK;
}

// Mean B row length (the products of one A entry), rounded up to a power of
// two, at most 64.
int sub_cap_for(int K, const spg_csr *B) {
  int64_t nz = 0, rows = 0;
  for (int k = 0; k < K; ++k) {
    nz += B[k].nnz;
    rows += B[k].nrows;
  }
  const int64_t mean = rows > 0 ? (nz + rows - 1) / rows : 1;
  int c = 1;
  while (c < mean && c < 64) c <<= 1;
  return c;
}

BinPlan make_binplan(spg_plan p, int maxbin, bool counts_known, const int *counts,
                     bool symbolic = false) {
  BinPlan bp;
  bp.known = counts_known;
  if (counts_known)
    for (int b = 0; b < kNB; ++b) bp.count[b] = counts[b];
  for (int b = 0; b < kNB; ++b) {
    bp.lanes[b] = p->tun.lanes[b];
    bp.sub[b] = symbolic ? p->tun.sym_sub[b] : p->tun.sub[b];
    if (bp.sub[b] > p->sub_cap) bp.sub[b] = p->sub_cap;
  }
  bp.maxbin = maxbin;
  bp.heavy_slots = p->L.heavy_slots;
  bp.m = p->m;
  bp.n = p->n;
  bp.maxwin = p->tun.max_window;
  return bp;
}

// Shared symbolic sequence for products (identity == false) and merges.
int run_symbolic(spg_plan p, const Problem &pr, const spg_csr *A, const spg_csr *B,
                 int32_t *C_row_ptr, int64_t *C_nnz_host, int64_t capacity, void *workspace,
                 size_t ws_bytes, hipStream_t st, int heavy_override = 0) {
  const int m = pr.m, n = pr.n;
  const int heavy = heavy_override > 0         ? heavy_override
                    : p->tun.heavy_slots > 0 ? p->tun.heavy_slots
                                             : default_heavy_slots(n);
  const WsLayout L = ws_layout(m, n, heavy);
  if (!workspace || ws_bytes < L.total) return SPG_ERR_WORKSPACE;
  if (!C_nnz_host && capacity < 0) return SPG_ERR_ARG;
  const bool eager = C_nnz_host != nullptr;
  const bool clear = eager || p->status_ws != workspace;
  p->sym_done = false;
  p->counts_known = false;
  p->ws = static_cast<char *>(workspace);
  p->ws_bytes = ws_bytes;
  p->status_ws = workspace;
  p->sub_cap = sub_cap_for(pr.K, B);
  p->L = L;
  p->crp = C_row_ptr;
  p->stream = st;
  p->K = pr.K;
  p->m = m;
  p->n = n;
  p->nnz = -1;
  p->products = -1;
  const DevInfo &D = dev_info();
  char *ws = p->ws;
  WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
  Problem *dpr = reinterpret_cast<Problem *>(ws + L.problem);
  hipError_t e = launch_setup(pr, dpr, hdr, true, clear, st, split_ctl(L, ws));
  if (e != hipSuccess) return SPG_ERR_HIP;
  if (p->flags & SPG_FLAG_VALIDATE) {
    // every later kernel exits once the status word is raised, so invalid
    // operands are never dereferenced; eagerly the call returns right here
    for (int k = 0; k < pr.K; ++k) {
      if (A) e = launch_validate(A[k].row_ptr, A[k].col_idx, A[k].nrows, A[k].ncols, A[k].nnz, hdr, st);
      if (e != hipSuccess) return SPG_ERR_HIP;
      e = launch_validate(B[k].row_ptr, B[k].col_idx, B[k].nrows, B[k].ncols, B[k].nnz, hdr, st);
      if (e != hipSuccess) return SPG_ERR_HIP;
    }
    if (eager) {
      int rc = read_header(p, st);
      if (rc) return rc;
      rc = status_from_bits(p->host_hdr->status);
      if (rc) return rc;
    }
  }
  // a1 + a2: products per row and bins by products
  e = launch_binning(dpr, m, D.sym_maxbin, tuned_edges(p->tun, D.sym_maxbin), L, ws, C_row_ptr,
                     st);
  if (e != hipSuccess) return SPG_ERR_HIP;
  BinPlan sbp;
  if (eager) {
    int rc = read_header(p, st);
    if (rc) return rc;
    rc = status_from_bits(p->host_hdr->status);
    if (rc) return rc;
    sbp = make_binplan(p, D.sym_maxbin, true, p->host_hdr->bin_count, true);
    for (int b = 0; b < kNB; ++b) p->sym_count[b] = p->host_hdr->bin_count[b];
  } else {
    sbp = make_binplan(p, D.sym_maxbin, false, nullptr, true);
  }
  // a3: exact row counts, then the scan into row_ptr
  e = launch_symbolic_bins(dpr, sbp, L, ws, C_row_ptr, st);
  if (e != hipSuccess) return SPG_ERR_HIP;
  e = launch_scan(C_row_ptr, m, eager ? -1 : capacity, L, ws, st);
  if (e != hipSuccess) return SPG_ERR_HIP;
  // The numeric pass keeps the bins by products: a row's products bound its
  // distinct columns, so every numeric table or staging area sized by them
  // holds the row, and no second binning pass is needed.
  if (eager) {
    int rc = read_header(p, st);
    if (rc) return rc;
    rc = status_from_bits(p->host_hdr->status);
    if (rc) return rc;
    p->nnz = p->host_hdr->nnz_total;
    p->products = p->host_hdr->products_total;
    for (int b = 0; b < kNB; ++b) p->num_count[b] = p->sym_count[b];
    p->counts_known = true;
    *C_nnz_host = p->nnz;
  }
  p->sym_done = true;
  return SPG_OK;
}

int fill_parts(Problem &pr, int K, const spg_csr *A, const spg_csr *B, bool identity) {
  if (K < 1 || K > SPG_MAX_PARTS) return SPG_ERR_ARG;
  if (!B || (!identity && !A)) return SPG_ERR_ARG;
  std::memset(&pr, 0, sizeof(pr));
  pr.K = K;
  pr.m = identity ? B[0].nrows : A[0].nrows;
  pr.n = B[0].ncols;
  if (pr.m < 0 || pr.n < 0) return SPG_ERR_SHAPE;
  for (int k = 0; k < K; ++k) {
    Part &P = pr.part[k];
    if (identity) {
      if (B[k].nrows != pr.m || B[k].ncols != pr.n) return SPG_ERR_SHAPE;
      P.a_identity = 1;
      P.kdim = pr.m;
    } else {
      if (A[k].nrows != pr.m || B[k].ncols != pr.n || A[k].ncols != B[k].nrows)
        return SPG_ERR_SHAPE;
      if (A[k].nnz < 0 || A[k].nnz > 0x7fffffffLL) return SPG_ERR_ARG;
      if (!A[k].row_ptr || (A[k].nnz > 0 && !A[k].col_idx)) return SPG_ERR_ARG;
      P.arp = A[k].row_ptr;
      P.acol = A[k].col_idx;
      P.aval = A[k].vals;
      P.kdim = A[k].ncols;
    }
    if (B[k].nnz < 0 || B[k].nnz > 0x7fffffffLL) return SPG_ERR_ARG;
    if (!B[k].row_ptr || (B[k].nnz > 0 && !B[k].col_idx)) return SPG_ERR_ARG;
    P.brp = B[k].row_ptr;
    P.bcol = B[k].col_idx;
    P.bval = B[k].vals;
  }
  return SPG_OK;
}

int check_values(int K, const spg_csr *A, const spg_csr *B, bool identity) {
  for (int k = 0; k < K; ++k) {
    if (!identity && A[k].nnz > 0 && !A[k].vals) return SPG_ERR_ARG;
    if (B[k].nnz > 0 && !B[k].vals) return SPG_ERR_ARG;
  }
  return SPG_OK;
}

void remember_operands(spg_plan p, int K, const spg_csr *A, const spg_csr *B) {
  for (int k = 0; k < K; ++k) {
    p->kdim[k] = A ? A[k].ncols : p->m;
    p->annz[k] = A ? A[k].nnz : -1;
    p->bnnz[k] = B[k].nnz;
  }
}

bool same_operands(spg_plan p, int K, const spg_csr *A, const spg_csr *B) {
  if (K != p->K) return false;
  for (int k = 0; k < K; ++k) {
    if ((A ? A[k].ncols : p->m) != p->kdim[k]) return false;
    if ((A ? A[k].nnz : -1) != p->annz[k] || B[k].nnz != p->bnnz[k]) return false;
    if (B[k].ncols != p->n || (A ? A[k].nrows : B[k].nrows) != p->m) return false;
  }
  return true;
}

int run_numeric(spg_plan p, const Problem &pr, spg_dtype dtype, int32_t *C_col_idx,
                void *C_vals, hipStream_t st) {
  if (dtype != SPG_F32 && dtype != SPG_F64) return SPG_ERR_ARG;
  if (p->counts_known && p->nnz > 0 && (!C_col_idx || !C_vals)) return SPG_ERR_ARG;
  const DevInfo &D = dev_info();
  char *ws = p->ws;
  WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
  Problem *dpr = reinterpret_cast<Problem *>(ws + p->L.problem);
  hipError_t e = launch_setup(pr, dpr, hdr, false, false, st, split_ctl(p->L, ws));
  if (e != hipSuccess) return SPG_ERR_HIP;
  const int maxbin = dtype == SPG_F64 ? D.num_maxbin_f64 : D.num_maxbin_f32;
  BinPlan bp = make_binplan(p, maxbin, p->counts_known, p->num_count);
  e = launch_numeric(dpr, bp, p->L, ws, p->crp, C_col_idx, C_vals, (int)dtype, st);
  p->stream = st;
  return hip_status(e);
}

int run_backward(spg_plan plan, const spg_csr *A, const spg_csr *B, const spg_csr *dC,
                 spg_dtype dtype, void *dA_vals, void *dB_vals, void *detws, size_t det_bytes,
                 void *stream) {
  (void)det_bytes;
  if (!plan || !A || !B || !dC) return SPG_ERR_ARG;
  if (!plan->sym_done || plan->merge_mode || plan->K != 1) return SPG_ERR_ARG;
  if (dtype != SPG_F32 && dtype != SPG_F64) return SPG_ERR_ARG;
  Problem pr;
  int rc = fill_parts(pr, 1, A, B, false);
  if (rc) return rc;
  if (!same_operands(plan, 1, A, B)) return SPG_ERR_SHAPE;
  rc = check_values(1, A, B, false);
  if (rc) return rc;
  if (dC->nrows != plan->m || dC->ncols != plan->n) return SPG_ERR_SHAPE;
  if (plan->nnz >= 0 && dC->nnz != plan->nnz) return SPG_ERR_SHAPE;
  if (!dC->row_ptr || (dC->nnz > 0 && (!dC->col_idx || !dC->vals))) return SPG_ERR_ARG;
  if (!dA_vals && !dB_vals) return SPG_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const DevInfo &D = dev_info();
  char *ws = plan->ws;
  WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
  Problem *dpr = reinterpret_cast<Problem *>(ws + plan->L.problem);
  hipError_t e = launch_setup(pr, dpr, hdr, false, false, st);
  if (e != hipSuccess) return SPG_ERR_HIP;
  const int maxbin = dtype == SPG_F64 ? D.num_maxbin_f64 : D.num_maxbin_f32;
  BinPlan bp = make_binplan(plan, maxbin, plan->counts_known, plan->num_count);
  e = launch_backward(dpr, bp, plan->L, ws, dC->row_ptr, dC->col_idx, dC->vals, dC->nnz, A->vals,
                      dA_vals, A->nnz, dB_vals, B->nnz, dB_vals ? detws : nullptr, (int)dtype, st);
  plan->stream = st;
  return hip_status(e);
}

}  // namespace

extern "C" {

int spgemm_plan_create(uint32_t flags, spg_plan *plan_out) {
  if (!plan_out) return SPG_ERR_ARG;
  *plan_out = nullptr;
  spg_plan p = new (std::nothrow) spg_plan_s();
  if (!p) return SPG_ERR_ARG;
  p->flags = flags;
  p->tun = default_tuning();
  *plan_out = p;
  return SPG_OK;
}

void spgemm_plan_destroy(spg_plan plan) {
  if (!plan) return;
  if (plan->host_hdr) (void)hipHostFree(plan->host_hdr);
  delete plan;
}

int spgemm_workspace_size(int32_t m, int32_t n, int32_t kmax, size_t *bytes) {
  if (!bytes || m < 0 || n < 0 || kmax < 0) return SPG_ERR_ARG;
  *bytes = ws_layout(m, n, default_heavy_slots(n)).total;
  return SPG_OK;
}

int spgemm_plan_status(spg_plan plan, int32_t *device_status_host) {
  if (!plan || !device_status_host) return SPG_ERR_ARG;
  if (!plan->ws) {
    *device_status_host = SPG_OK;
    return SPG_OK;
  }
  int rc = read_header(plan, plan->stream);
  if (rc) return rc;
  *device_status_host = status_from_bits(plan->host_hdr->status);
  plan->nnz = plan->host_hdr->nnz_total;
  plan->products = plan->host_hdr->products_total;
  return SPG_OK;
}

int spgemm_plan_clear_status(spg_plan plan, void *stream) {
  if (!plan) return SPG_ERR_ARG;
  if (!plan->ws) return SPG_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = launch_clear_status(reinterpret_cast<WsHeader *>(plan->ws), st);
  return hip_status(e);
}

int spgemm_plan_info(spg_plan plan, int64_t *nnz, int64_t *products) {
  if (!plan) return SPG_ERR_ARG;
  if (nnz) *nnz = plan->nnz;
  if (products) *products = plan->products;
  return SPG_OK;
}

const char *spgemm_status_string(int status) {
  switch (status) {
    case SPG_OK: return "ok";
    case SPG_ERR_INVALID: return "invalid CSR input";
    case SPG_ERR_SHAPE: return "operand shapes do not match";
    case SPG_ERR_OVERFLOW: return "output nnz exceeds 2^31-1";
    case SPG_ERR_CAPACITY: return "output larger than the given capacity";
    case SPG_ERR_WORKSPACE: return "workspace missing or too small";
    case SPG_ERR_HIP: return "HIP runtime error";
    case SPG_ERR_UNSUPPORTED: return "unsupported argument combination";
    case SPG_ERR_ARG: return "bad argument";
    case SPG_ERR_SCRATCH: return "problem too large for the library's static scratch buffer";
    default: return "unknown status";
  }
}

int spgemm_plan_bins(spg_plan plan, int32_t *sym_counts, int32_t *num_counts) {
  if (!plan || !plan->counts_known) return SPG_ERR_ARG;
  for (int b = 0; b < kNB; ++b) {
    if (sym_counts) sym_counts[b] = plan->sym_count[b];
    if (num_counts) num_counts[b] = plan->num_count[b];
  }
  return SPG_OK;
}

int spgemm_default_tuning(spg_tuning *t) {
  if (!t) return SPG_ERR_ARG;
  *t = default_tuning();
  return SPG_OK;
}

int spgemm_plan_set_tuning(spg_plan plan, const spg_tuning *t) {
  if (!plan || !t) return SPG_ERR_ARG;
  int rc = check_tuning(*t);
  if (rc) return rc;
  plan->tun = *t;
  plan->tun_set = true;
  return SPG_OK;
}

int spgemm_symbolic(spg_plan plan, int32_t K, const spg_csr *A, const spg_csr *B,
                    int32_t *C_row_ptr, int64_t *C_nnz_host, int64_t capacity, void *workspace,
                    size_t ws_bytes, void *stream) {
  if (!plan || !C_row_ptr) return SPG_ERR_ARG;
  Problem pr;
  int rc = fill_parts(pr, K, A, B, false);
  if (rc) return rc;
  plan->merge_mode = false;
  rc = run_symbolic(plan, pr, A, B, C_row_ptr, C_nnz_host, capacity, workspace, ws_bytes,
                    static_cast<hipStream_t>(stream));
  if (rc == SPG_OK) remember_operands(plan, K, A, B);
  return rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Static scratch for spgemm_symbolic_noalloc: one array per device, held by
// the device until the process ends.  In host code `scratch` names a host
// stand-in, never the device memory: host code only ever uses the address
// that hipGetSymbolAddress returns for the current device (g_scratch_ptr).
namespace {

__device__ __align__(256) char scratch[SPG_SCRATCH_BYTES];

std::mutex g_scratch_mu;
int g_scratch_dev[kMaxDevices];
char *g_scratch_ptr[kMaxDevices];
int g_nscratch = 0;

// Device address of this device's scratch (looked up once per device, with
// the device current); nullptr if the lookup fails.
char *scratch_for_current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  for (int t = 0; t < g_nscratch; ++t)
    if (g_scratch_dev[t] == dev) return g_scratch_ptr[t];
  if (g_nscratch == kMaxDevices) return nullptr;
  void *ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return nullptr;
  }
  g_scratch_dev[g_nscratch] = dev;
  g_scratch_ptr[g_nscratch] = static_cast<char *>(ptr);
  return g_scratch_ptr[g_nscratch++];
}

}  // namespace

extern "C" {

int spgemm_symbolic_noalloc(spg_plan plan, int32_t K, const spg_csr *A, const spg_csr *B,
                            int32_t *C_row_ptr, int64_t capacity, void *stream) {
  if (!plan || !C_row_ptr || capacity < 0) return SPG_ERR_ARG;
  Problem pr;
  int rc = fill_parts(pr, K, A, B, false);
  if (rc) return rc;
  // as many concurrent heavy rows as the scratch holds, at most the usual
  // number (at least one)
  const int want = plan->tun.heavy_slots > 0 ? plan->tun.heavy_slots : default_heavy_slots(pr.n);
  int heavy = want;
  while (heavy > 1 && ws_layout(pr.m, pr.n, heavy).total > (size_t)SPG_SCRATCH_BYTES) heavy /= 2;
  if (ws_layout(pr.m, pr.n, heavy).total > (size_t)SPG_SCRATCH_BYTES) return SPG_ERR_SCRATCH;
  (void)dev_info();  // per-device set-up (kernel attributes) before the first launch
  char *ws = scratch_for_current_device();
  if (!ws) return SPG_ERR_HIP;
  plan->merge_mode = false;
  rc = run_symbolic(plan, pr, A, B, C_row_ptr, nullptr, capacity, ws,
                    (size_t)SPG_SCRATCH_BYTES, static_cast<hipStream_t>(stream), heavy);
  if (rc == SPG_OK) remember_operands(plan, K, A, B);
  return rc;
}

int spgemm_numeric(spg_plan plan, int32_t K, const spg_csr *A, const spg_csr *B,
                   spg_dtype dtype, int32_t *C_col_idx, void *C_vals, void *stream) {
  if (!plan) return SPG_ERR_ARG;
  if (!plan->sym_done || plan->merge_mode) return SPG_ERR_ARG;
  Problem pr;
  int rc = fill_parts(pr, K, A, B, false);
  if (rc) return rc;
  if (!same_operands(plan, K, A, B)) return SPG_ERR_SHAPE;
  rc = check_values(K, A, B, false);
  if (rc) return rc;
  return run_numeric(plan, pr, dtype, C_col_idx, C_vals, static_cast<hipStream_t>(stream));
}

int spgemm_merge(spg_plan plan, int32_t K, const spg_csr *P, spg_dtype dtype,
                 int32_t *C_row_ptr, int64_t *C_nnz_host, int64_t capacity, int32_t *C_col_idx,
                 void *C_vals, void *workspace, size_t ws_bytes, void *stream) {
  if (!plan) return SPG_ERR_ARG;
  Problem pr;
  int rc = fill_parts(pr, K, nullptr, P, true);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!C_col_idx && !C_vals) {
    if (!C_row_ptr) return SPG_ERR_ARG;
    plan->merge_mode = true;
    rc = run_symbolic(plan, pr, nullptr, P, C_row_ptr, C_nnz_host, capacity, workspace,
                      ws_bytes, st);
    if (rc == SPG_OK) remember_operands(plan, K, nullptr, P);
    return rc;
  }
  if (!plan->sym_done || !plan->merge_mode) return SPG_ERR_ARG;
  if (!same_operands(plan, K, nullptr, P)) return SPG_ERR_SHAPE;
  rc = check_values(K, nullptr, P, true);
  if (rc) return rc;
  return run_numeric(plan, pr, dtype, C_col_idx, C_vals, st);
}

int spgemm_backward(spg_plan plan, const spg_csr *A, const spg_csr *B, const spg_csr *dC,
                    spg_dtype dtype, void *dA_vals, void *dB_vals, void *stream) {
  return run_backward(plan, A, B, dC, dtype, dA_vals, dB_vals, nullptr, 0, stream);
}

int spgemm_backward_deterministic_workspace_size(int64_t nnzB, size_t *bytes) {
  if (!bytes || nnzB < 0) return SPG_ERR_ARG;
  *bytes = det_workspace_bytes(nnzB);
  return SPG_OK;
}

int spgemm_backward_deterministic(spg_plan plan, const spg_csr *A, const spg_csr *B,
                                  const spg_csr *dC, spg_dtype dtype, void *dA_vals,
                                  void *dB_vals, void *workspace, size_t ws_bytes, void *stream) {
  if (!B) return SPG_ERR_ARG;
  if (dB_vals) {
    if (!workspace || ws_bytes < det_workspace_bytes(B->nnz)) return SPG_ERR_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(workspace) % 8) return SPG_ERR_ARG;
  }
  return run_backward(plan, A, B, dC, dtype, dA_vals, dB_vals, workspace, ws_bytes, stream);
}

int spgemm_permute_workspace_size(int32_t m, int32_t n, size_t *bytes) {
  if (!bytes || m < 0 || n < 0) return SPG_ERR_ARG;
  size_t a, b, c, d;
  *bytes = perm_workspace_bytes(m, n, &a, &b, &c, &d);
  return SPG_OK;
}

int spgemm_permute(spg_plan plan, const spg_csr *A, const int32_t *row_perm,
                   const int32_t *col_perm, spg_dtype dtype, int32_t *B_row_ptr,
                   int32_t *B_col_idx, void *B_vals, void *workspace, size_t ws_bytes,
                   void *stream) {
  if (!plan || !A || !B_row_ptr) return SPG_ERR_ARG;
  if (dtype != SPG_F32 && dtype != SPG_F64) return SPG_ERR_ARG;
  if (A->nrows < 0 || A->ncols < 0 || A->nnz < 0 || A->nnz > 0x7fffffffLL) return SPG_ERR_ARG;
  if (!A->row_ptr || (A->nnz > 0 && (!A->col_idx || !B_col_idx))) return SPG_ERR_ARG;
  if (B_vals && A->nnz > 0 && !A->vals) return SPG_ERR_ARG;
  size_t r0, c0, l0, s0;
  const size_t need = perm_workspace_bytes(A->nrows, A->ncols, &r0, &c0, &l0, &s0);
  if (!workspace || ws_bytes < need) return SPG_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool clear = plan->status_ws != workspace;
  plan->status_ws = workspace;
  plan->ws = static_cast<char *>(workspace);
  plan->ws_bytes = ws_bytes;
  plan->stream = st;
  plan->sym_done = false;
  plan->counts_known = false;
  plan->nnz = A->nnz;
  plan->products = -1;
  WsHeader *hdr = reinterpret_cast<WsHeader *>(workspace);
  Problem pr;
  std::memset(&pr, 0, sizeof(pr));
  hipError_t e = launch_setup(pr, reinterpret_cast<Problem *>(plan->ws + 256), hdr, true, clear, st);
  if (e != hipSuccess) return SPG_ERR_HIP;
  e = launch_permute(*A, row_perm, col_perm, (int)dtype, B_row_ptr, B_col_idx, B_vals,
                     plan->ws, st);
  return hip_status(e);
}

static void mcl_layout(int32_t n, int32_t topk, WsLayout &L, size_t &pcol, size_t &pval,
                       size_t &total, int &cap) {
  L = ws_layout(n, n, 0);
  cap = topk < n ? topk : n;
  if (cap < 1) cap = 1;
  const size_t pad = (size_t)std::max(n, 1) * (size_t)cap;
  pcol = (L.total + 255) & ~(size_t)255;
  pval = (pcol + 4 * pad + 255) & ~(size_t)255;
  L.mcl_rabs = (pval + 4 * pad + 255) & ~(size_t)255;
  L.mcl_slots = (L.mcl_rabs + 8 * (size_t)std::max(n, 1) + 255) & ~(size_t)255;
  total = L.mcl_slots + (size_t)mcl_heavy_slots(n) * mcl_slot_bytes(n);
}

int spgemm_mcl_workspace_size(int32_t n, int32_t topk, size_t *bytes) {
  if (!bytes || n < 0 || topk < 1) return SPG_ERR_ARG;
  WsLayout L;
  size_t pc, pv, tot;
  int cap;
  mcl_layout(n, topk, L, pc, pv, tot, cap);
  *bytes = tot;
  return SPG_OK;
}

int spgemm_mcl_iteration(spg_plan plan, const spg_csr *X, int32_t r, float prune, int32_t topk,
                         int32_t *Y_row_ptr, int32_t *Y_col_idx, float *Y_vals, int64_t capacity,
                         int64_t *Y_nnz_host, void *workspace, size_t ws_bytes, void *stream) {
  return spgemm_mcl_iteration_order(plan, X, SPG_MCL_INFLATE_FIRST, r, prune, topk, Y_row_ptr,
                                    Y_col_idx, Y_vals, capacity, Y_nnz_host, workspace, ws_bytes,
                                    stream);
}

int spgemm_mcl_iteration_order(spg_plan plan, const spg_csr *X, int32_t order, int32_t r,
                               float prune, int32_t topk, int32_t *Y_row_ptr, int32_t *Y_col_idx,
                               float *Y_vals, int64_t capacity, int64_t *Y_nnz_host,
                               void *workspace, size_t ws_bytes, void *stream) {
  if (!plan || !X || !Y_row_ptr) return SPG_ERR_ARG;
  if (order != SPG_MCL_INFLATE_FIRST && order != SPG_MCL_PAPER) return SPG_ERR_ARG;
  if (X->nrows != X->ncols) return SPG_ERR_SHAPE;
  if (r < 1 || r > 8 || topk < 1 || !(prune >= 0.f) || !(prune < 1e30f)) return SPG_ERR_ARG;
  if (X->ncols > kMclMaxCols) return SPG_ERR_UNSUPPORTED;  // 24-bit columns in the LDS tables
  if (!Y_nnz_host && capacity < 0) return SPG_ERR_ARG;
  if (X->nnz > 0 && (!X->col_idx || !X->vals)) return SPG_ERR_ARG;
  const int n = X->nrows;
  WsLayout L;
  size_t pcol_off, pval_off, total;
  int cap;
  mcl_layout(n, topk, L, pcol_off, pval_off, total, cap);
  if (!workspace || ws_bytes < total) return SPG_ERR_WORKSPACE;
  Problem pr;
  int rc = fill_parts(pr, 1, X, X, false);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool eager = Y_nnz_host != nullptr;
  const bool clear = eager || plan->status_ws != workspace;
  plan->sym_done = false;
  plan->counts_known = false;
  plan->ws = static_cast<char *>(workspace);
  plan->ws_bytes = ws_bytes;
  plan->status_ws = workspace;
  plan->sub_cap = sub_cap_for(1, X);
  plan->L = L;
  plan->stream = st;
  plan->m = plan->n = n;
  plan->nnz = -1;
  const DevInfo &D = dev_info();
  char *ws = plan->ws;
  WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
  Problem *dpr = reinterpret_cast<Problem *>(ws + L.problem);
  int32_t *pcol = reinterpret_cast<int32_t *>(ws + pcol_off);
  float *pval = reinterpret_cast<float *>(ws + pval_off);
  hipError_t e = launch_setup(pr, dpr, hdr, true, clear, st);
  if (e != hipSuccess) return SPG_ERR_HIP;
  if (plan->flags & SPG_FLAG_VALIDATE) {
    e = launch_validate(X->row_ptr, X->col_idx, n, n, X->nnz, hdr, st);
    if (e != hipSuccess) return SPG_ERR_HIP;
    if (eager) {
      rc = read_header(plan, st);
      if (rc) return rc;
      rc = status_from_bits(plan->host_hdr->status);
      if (rc) return rc;
    }
  }
  // one bin past the largest LDS table: MCL rows repeat columns a lot, so
  // most rows of that bin still fit the largest table; those whose probes
  // overflow go to the panel kernel with the heavier bins
  const int mcl_bins = D.mcl_maxbin + 1 < kHeavyBin ? D.mcl_maxbin + 1 : D.mcl_maxbin;
  e = launch_binning(dpr, n, mcl_bins, default_edges(), L, ws, Y_row_ptr, st);
  if (e != hipSuccess) return SPG_ERR_HIP;
  BinPlan bp;
  if (eager) {
    rc = read_header(plan, st);
    if (rc) return rc;
    rc = status_from_bits(plan->host_hdr->status);
    if (rc) return rc;
    bp = make_binplan(plan, mcl_bins, true, plan->host_hdr->bin_count);
  } else {
    bp = make_binplan(plan, mcl_bins, false, nullptr);
  }
  // the exponent before the normalisation, and after the prune (0: renormalise)
  const int rpre = order == SPG_MCL_PAPER ? 1 : r;
  const int rpost = order == SPG_MCL_PAPER ? r : 0;
  e = launch_mcl(dpr, bp, L, ws, rpre, rpost, prune, topk, cap, pcol, pval, Y_row_ptr, st);
  if (e != hipSuccess) return SPG_ERR_HIP;
  e = launch_scan(Y_row_ptr, n, capacity, L, ws, st);  // capacity < 0: unchecked
  if (e != hipSuccess) return SPG_ERR_HIP;
  if (eager) {
    rc = read_header(plan, st);
    if (rc) return rc;
    rc = status_from_bits(plan->host_hdr->status);
    if (rc) return rc;
    plan->nnz = plan->host_hdr->nnz_total;
    plan->products = plan->host_hdr->products_total;
    *Y_nnz_host = plan->nnz;
    if (plan->nnz > 0 && (!Y_col_idx || !Y_vals)) return SPG_ERR_ARG;
  }
  e = launch_mcl_compact(n, cap, Y_row_ptr, pcol, pval, Y_col_idx, Y_vals, hdr, st);
  return hip_status(e);
}

}  // extern "C"

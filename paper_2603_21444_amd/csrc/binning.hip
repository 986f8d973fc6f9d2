// Kernels around the row kernels of the local product C = sum_k A_k B_k
// (K = 1: C = A B, paper §2) on gfx950: problem setup, optional operand
// validation, products per row and row binning, and the scan of row counts
// into the CSR row pointer of C.
//
// Every kernel reads the operand descriptors from a device copy of the
// Problem (scalar loads; the copy is made by k_setup in the same stream) and
// the row lists and bin counts from the workspace header, so the same
// launches work eagerly and inside a captured graph.  Kernels with row lists
// loop over them grid-stride style, so any grid size is correct.
#include "common.hpp"
#include "internal.hpp"

namespace spg {

// ---------------------------------------------------------------------------
// Setup: copy the problem into the workspace, clear the header's counters
// (reset) and the status word (clear_status).  A status word that is not
// cleared stays raised, so every later kernel of a captured sequence exits.
// The split rows' reservations are cleared with the counters, their queue
// cursors at every call.
__global__ void k_setup(Problem pr, Problem *dst, WsHeader *hdr, int reset, int clear_status,
                        SplitCtl *sc) {
  if (threadIdx.x == 0) *dst = pr;
  if (reset && threadIdx.x < kNB) {
    hdr->bin_count[threadIdx.x] = 0;
    hdr->bin_start[threadIdx.x] = 0;
  }
  if (clear_status && threadIdx.x == 0) hdr->status = 0;
  if (reset && threadIdx.x == 0) {
    hdr->nnz_total = 0;
    hdr->products_total = 0;
    hdr->bin_start[kNB] = 0;
  }
  if (threadIdx.x == 0) {
    hdr->fallback_count = 0;
    hdr->long_count = 0;
    hdr->mid_count = 0;
  }
  if (threadIdx.x < kNB + 2) hdr->queue[threadIdx.x] = 0;
  if (sc && threadIdx.x == 0) {
    if (reset) {
      sc->stage = 0;
      sc->segs = 0;
      sc->items = 0;
    }
    sc->q_scatter = 0;
    sc->q_accum = 0;
    sc->nuns = 0;
  }
}

// Optional validation of one CSR operand: row_ptr[0] == 0, non-decreasing,
// row_ptr[rows] == nnz, columns in range.
__global__ void k_validate(const int32_t *rp, const int32_t *col, int rows, int ncols,
                           int64_t nnz, WsHeader *hdr) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  if (t == 0) bad = bad || rp[0] != 0 || (int64_t)rp[rows] != nnz;
  for (int64_t i = t; i < rows; i += stride) bad = bad || rp[i + 1] < rp[i];
  for (int64_t p = t; p < nnz; p += stride) bad = bad || col[p] < 0 || col[p] >= ncols;
  if (bad) atomicOr(&hdr->status, kStatInvalid);
}

// ---------------------------------------------------------------------------
// a1/a2: row key (products per row) and bin id; per-block bin histogram and
// the product total.  One thread per row, 256 rows per block.  A thread
// reads its row's A columns four at a time (16-byte loads) and the bounds of
// each selected B row with one 8-byte load: the rows of a wave's lanes lie
// far apart, so every load instruction touches up to 64 cache lines and the
// number of instructions is what costs.  Rows of more than kKeyWave A
// entries (over all block products) are deferred to k_rowkey_long: a group
// of kKeyGroup lanes per row for up to kKeyLong entries, one block per row
// beyond.  Power-law
// hubs sit next to each other (R-MAT puts them at the low row indices), so a
// wave that summed its own long rows would take dozens of them one after
// another while the rest of the grid idles; the deferred lists spread them
// over all waves instead.
constexpr int kBinBlock = 256;
constexpr int kKeyWave = 256;
constexpr int kKeyGroup = 16;  // lanes per deferred row of at most kKeyLong entries
constexpr int kKeyLong = 2048;
constexpr int kKeyLongBlock = 256;  // threads of k_rowkey_long
constexpr uint8_t kBinDeferred = 0xff;

__device__ __forceinline__ int brow_len(const SPG_GLOBAL int32_t *brp, int r) {
  int2 b;
  __builtin_memcpy(&b, brp + r, sizeof(b));  // brp[r], brp[r + 1] in one load
  return b.y - b.x;
}

__global__ __launch_bounds__(kBinBlock) void k_rowkey(const Problem *__restrict__ pr,
                                                      int maxbin, BinEdges edges, uint8_t *binid,
                                                      int32_t *blockhist, int32_t *cnt_zero,
                                                      int32_t *longrows, WsHeader *hdr) {
  __shared__ int hist[kNB];
  __shared__ long long psum[kBinBlock / kWave];
  if (hdr->status) return;  // invalid operands or overflow: touch nothing
  if (threadIdx.x < kNB) hist[threadIdx.x] = 0;
  __syncthreads();
  const int m = pr->m;
  const int i = blockIdx.x * kBinBlock + threadIdx.x;
  int64_t key = 0;
  bool deferred = false, longrow = false;
  if (i < m) {
    const int K = pr->K;
    int len = 0;
    for (int k = 0; k < K; ++k) {
      int as, ae;
      a_row(pr->part[k], i, as, ae);
      len += ae - as;
    }
    deferred = len > kKeyWave;  // counted by k_rowkey_long
    longrow = len > kKeyLong;
    for (int k = 0; k < K && !deferred; ++k) {
      const Part &P = pr->part[k];
      int as, ae;
      a_row(P, i, as, ae);
      const SPG_GLOBAL int32_t *brp = gp(P.brp);
      if (P.a_identity) {  // A = I: the row's products are B row i
        key += brow_len(brp, i);
        continue;
      }
      const SPG_GLOBAL int32_t *acol = gp(P.acol);
      int p = as;
      for (; p + 8 <= ae; p += 8) {  // eight entries, eight gathers in flight
        int r[8];
        __builtin_memcpy(&r[0], acol + p, 4 * sizeof(int));
        __builtin_memcpy(&r[4], acol + p + 4, 4 * sizeof(int));
#pragma unroll
        for (int u = 0; u < 8; ++u) key += brow_len(brp, r[u]);
      }
      for (; p < ae; ++p) key += brow_len(brp, acol[p]);
    }
  }
  // deferred rows: long ones to the front of the list, the others to the
  // back, one atomic per wave and list
  {
    const uint64_t lm = __ballot(deferred && longrow), mm = __ballot(deferred && !longrow);
    const uint64_t lt = lane_id() == 0 ? 0ull : (~0ull >> (kWave - lane_id()));
    int lb = 0, mb = 0;
    if (lane_id() == 0) {
      if (lm) lb = atomicAdd(&hdr->long_count, __popcll(lm));
      if (mm) mb = atomicAdd(&hdr->mid_count, __popcll(mm));
    }
    lb = __shfl(lb, 0);
    mb = __shfl(mb, 0);
    if (deferred && longrow) longrows[lb + __popcll(lm & lt)] = i;
    if (deferred && !longrow) longrows[m - 1 - (mb + __popcll(mm & lt))] = i;
  }
  if (i < m && deferred) {
    binid[i] = kBinDeferred;
  } else if (i < m) {
    if (key == 0) cnt_zero[i] = 0;
    int b = bin_of(key, maxbin, edges);
    binid[i] = (uint8_t)b;
    atomicAdd(&hist[b], 1);
  }
  // block sum of products -> header (int64)
  long long v = key;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (lane_id() == 0) psum[threadIdx.x / kWave] = v;
  __syncthreads();
  // bin-major: blockhist[b * nblk + block]
  if (threadIdx.x < kNB) blockhist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = hist[threadIdx.x];
  if (threadIdx.x == 0) {
    long long s = 0;
    for (int w = 0; w < kBinBlock / kWave; ++w) s += psum[w];
    atomicAdd((unsigned long long *)&hdr->products_total, (unsigned long long)s);
  }
}

// The products of row i summed by NT threads (t = thread index among them),
// part by part, four gathers in flight per thread; every thread holds a
// partial sum.
template <int NT>
__device__ __forceinline__ long long row_products(const Problem *__restrict__ pr, int i, int t) {
  long long part = 0;
  for (int k = 0; k < pr->K; ++k) {
    const Part &P = pr->part[k];
    int as, ae;
    a_row(P, i, as, ae);
    const SPG_GLOBAL int32_t *brp = gp(P.brp);
    int p = as + t;
    for (; p + 3 * NT < ae; p += 4 * NT) {
      int r[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) r[u] = a_entry_row(P, i, p + u * NT);
#pragma unroll
      for (int u = 0; u < 4; ++u) part += brow_len(brp, r[u]);
    }
    for (; p < ae; p += NT) part += brow_len(brp, a_entry_row(P, i, p));
  }
  return part;
}

// The deferred row of key `key`: its bin, its place in its block's
// histogram (the histogram k_rowkey wrote), and the empty-row mark.
__device__ __forceinline__ void place_row(int i, long long key, int maxbin, const BinEdges &edges,
                                          uint8_t *binid, int32_t *blockhist, int nblk,
                                          int32_t *cnt_zero) {
  if (key == 0) cnt_zero[i] = 0;
  const int b = bin_of(key, maxbin, edges);
  binid[i] = (uint8_t)b;
  atomicAdd(&blockhist[(int64_t)b * nblk + i / kBinBlock], 1);
}

// Row keys of the rows k_rowkey deferred: rows of more than kKeyLong A
// entries one block per row, then the others one group of kKeyGroup lanes
// per row.
__global__ __launch_bounds__(kKeyLongBlock) void k_rowkey_long(const Problem *__restrict__ pr, int maxbin,
                                                      BinEdges edges, uint8_t *binid,
                                                      int32_t *blockhist, int nblk,
                                                      int32_t *cnt_zero,
                                                      const int32_t *__restrict__ longrows,
                                                      WsHeader *hdr) {
  __shared__ long long wsum[kKeyLongBlock / kWave];
  if (hdr->status) return;
  const int count = hdr->long_count;
  const int tid = threadIdx.x;
  long long mine = 0;  // this lane's share of the product total
  for (int li = blockIdx.x; li < count; li += gridDim.x) {
    const int i = longrows[li];
    long long part = row_products<kKeyLongBlock>(pr, i, tid);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) part += __shfl_xor(part, off);
    if (lane_id() == 0) wsum[tid / kWave] = part;
    __syncthreads();
    if (tid == 0) {
      long long key = 0;
      for (int w = 0; w < kKeyLongBlock / kWave; ++w) key += wsum[w];
      place_row(i, key, maxbin, edges, binid, blockhist, nblk, cnt_zero);
      mine += key;
    }
    __syncthreads();
  }
  const int m = pr->m;
  const int mcount = hdr->mid_count;
  constexpr int kGpb = kKeyLongBlock / kKeyGroup;
  const int g = tid / kKeyGroup, gl = tid % kKeyGroup;
  // the loop bound is the same for the whole wave (its groups share the
  // shuffles below), rows past the list end count nothing
  const int first = blockIdx.x * kGpb + (tid / kWave) * (kWave / kKeyGroup);
  for (int l0 = first; l0 < mcount; l0 += gridDim.x * kGpb) {
    const int li = l0 + g % (kWave / kKeyGroup);
    const int i = li < mcount ? longrows[m - 1 - li] : -1;
    long long part = i >= 0 ? row_products<kKeyGroup>(pr, i, gl) : 0;
#pragma unroll
    for (int off = kKeyGroup / 2; off > 0; off >>= 1) part += __shfl_xor(part, off, kKeyGroup);
    if (gl == 0 && i >= 0) {
      place_row(i, part, maxbin, edges, binid, blockhist, nblk, cnt_zero);
      mine += part;
    }
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) mine += __shfl_xor(mine, off);
  if (lane_id() == 0 && mine) atomicAdd((unsigned long long *)&hdr->products_total, (unsigned long long)mine);
}

// Exclusive scan of one bin's per-block counts (block b of kNB; the counts
// of a bin are contiguous), in place and relative to the bin's start; the
// bin's total goes to the header.  Each thread takes four consecutive
// counts of a 4096-count chunk: one load round trip and one block scan per
// chunk.
__global__ __launch_bounds__(1024) void k_binscan(int32_t *blockhist, int nblk, WsHeader *hdr) {
  __shared__ int wsum[1024 / kWave];
  const int b = blockIdx.x, t = threadIdx.x, lane = lane_id(), w = t / kWave;
  int32_t *h = blockhist + (int64_t)b * nblk;
  int carry = 0;
  for (int c0 = 0; c0 < nblk; c0 += 4 * 1024) {
    int v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = c0 + 4 * t + u;
      v[u] = idx < nblk ? h[idx] : 0;
    }
    const int s = v[0] + v[1] + v[2] + v[3];
    int x = s;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const int y = __shfl_up(x, off);
      if (lane >= off) x += y;
    }
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    int pre = 0, tot = 0;
#pragma unroll
    for (int ww = 0; ww < 1024 / kWave; ++ww) {
      const int c = wsum[ww];
      pre += ww < w ? c : 0;
      tot += c;
    }
    __syncthreads();  // wsum is rewritten by the next chunk
    int run = carry + pre + x - s;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = c0 + 4 * t + u;
      if (idx < nblk) h[idx] = run;
      run += v[u];
    }
    carry += tot;
  }
  if (t == 0) hdr->bin_count[b] = carry;
}

// Stable scatter of row ids into the per-bin lists: bin start (prefix of
// the bin totals) + the block's offset within the bin + rank in the block.
// Block 0 publishes the bin starts.
__global__ __launch_bounds__(kBinBlock) void k_binscatter(const uint8_t *binid, int m,
                                                          const int32_t *blockoff,
                                                          int32_t *rows, WsHeader *hdr) {
  __shared__ int wcnt[kBinBlock / kWave][kNB];
  __shared__ int binbase[kNB + 1];
  if (threadIdx.x <= kNB) {
    int s = 0;
    for (int bb = 0; bb < (int)threadIdx.x; ++bb) s += hdr->bin_count[bb];
    binbase[threadIdx.x] = s;
    if (blockIdx.x == 0) hdr->bin_start[threadIdx.x] = s;
  }
  if (hdr->status) return;
  const int i = blockIdx.x * kBinBlock + threadIdx.x;
  const int w = threadIdx.x / kWave;
  const int b = i < m ? binid[i] : -1;
  int myrank = 0;
  for (int bb = 0; bb < kNB; ++bb) {
    uint64_t mask = __ballot(b == bb);
    if (b == bb) myrank = mbcnt(mask);
    if (lane_id() == 0) wcnt[w][bb] = __popcll(mask);
  }
  __syncthreads();
  if (i < m) {
    int off = binbase[b] + blockoff[(int64_t)b * gridDim.x + blockIdx.x];
    for (int ww = 0; ww < w; ++ww) off += wcnt[ww][b];
    rows[off + myrank] = i;
  }
}

// ---------------------------------------------------------------------------
// a3 scan: in-place exclusive scan of per-row counts into row_ptr[0..m]
// (int64 running total; > 2^31-1 raises the overflow status).
constexpr int kScanTile = 2048;  // 256 threads x 8

__global__ __launch_bounds__(256) void k_scan_reduce(const int32_t *cnt, int m, int64_t *part,
                                                    const WsHeader *hdr) {
  __shared__ long long ws[4];
  if (hdr->status) return;  // the counts were never written
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  long long s = 0;
  for (int j = 0; j < 8; ++j) {
    const int64_t i = base + j * 256 + threadIdx.x;
    if (i < m) s += cnt[i];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane_id() == 0) ws[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ __launch_bounds__(1024) void k_scan_mid(int64_t *part, int nparts, int64_t capacity,
                                                   WsHeader *hdr) {
  __shared__ long long wsum[16];
  __shared__ long long carry;
  if (hdr->status) return;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int c0 = 0; c0 < nparts; c0 += 1024) {
    const int idx = c0 + threadIdx.x;
    const long long v = idx < nparts ? part[idx] : 0;
    long long x = v;
    for (int off = 1; off < kWave; off <<= 1) {
      long long y = __shfl_up(x, off);
      if (lane_id() >= off) x += y;
    }
    if (lane_id() == kWave - 1) wsum[threadIdx.x / kWave] = x;
    __syncthreads();
    long long wpre = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
      if (w < (int)threadIdx.x / kWave) wpre += wsum[w];
      tot += wsum[w];
    }
    if (idx < nparts) part[idx] = carry + wpre + x - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    hdr->nnz_total = carry;
    int st = 0;
    if (carry > 0x7fffffffLL) st |= kStatOverflow;
    if (capacity >= 0 && carry > capacity) st |= kStatCapacity;
    if (st) atomicOr(&hdr->status, st);
  }
}

__global__ __launch_bounds__(256) void k_scan_apply(int32_t *rp, int m, const int64_t *part,
                                                    const WsHeader *hdr) {
  __shared__ long long wsum[4];
  if (hdr->status) return;  // failed earlier or the total overflowed: row_ptr stays as it is
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  // each thread owns 8 consecutive entries
  const int64_t i0 = base + threadIdx.x * 8;
  int v[8];
  long long s = 0;
  for (int j = 0; j < 8; ++j) {
    v[j] = (i0 + j < m) ? rp[i0 + j] : 0;
    s += v[j];
  }
  long long x = s;
  for (int off = 1; off < kWave; off <<= 1) {
    long long y = __shfl_up(x, off);
    if (lane_id() >= off) x += y;
  }
  if (lane_id() == kWave - 1) wsum[threadIdx.x / kWave] = x;
  __syncthreads();
  long long wpre = 0;
  for (int w = 0; w < (int)threadIdx.x / kWave; ++w) wpre += wsum[w];
  int64_t run = part[blockIdx.x] + wpre + x - s;
  for (int j = 0; j < 8; ++j) {
    if (i0 + j < m) rp[i0 + j] = (int32_t)run;
    run += v[j];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) rp[m] = (int32_t)hdr->nnz_total;
}

// Host launchers.

BinEdges default_edges() {
  BinEdges E{};
  for (int b = 0; b < kNB; ++b) E.up[b] = (int32_t)bin_edge(b);
  return E;
}

hipError_t launch_setup(const Problem &pr, Problem *dst, WsHeader *hdr, bool reset,
                        bool clear_status, hipStream_t st, SplitCtl *sc) {
  hipLaunchKernelGGL(k_setup, dim3(1), dim3(64), 0, st, pr, dst, hdr, reset ? 1 : 0,
                     clear_status ? 1 : 0, sc);
  return hipGetLastError();
}

__global__ void k_clear_status(WsHeader *hdr) {
  if (threadIdx.x == 0) hdr->status = 0;
}

hipError_t launch_clear_status(WsHeader *hdr, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, st, hdr);
  return hipGetLastError();
}

hipError_t launch_validate(const int32_t *rp, const int32_t *col, int rows, int ncols,
                           int64_t nnz, WsHeader *hdr, hipStream_t st) {
  hipLaunchKernelGGL(k_validate, dim3(256), dim3(256), 0, st, rp, col, rows, ncols, nnz, hdr);
  return hipGetLastError();
}

hipError_t launch_binning(const Problem *dpr, int m, int maxbin, const BinEdges &edges,
                          const WsLayout &L, char *ws, int32_t *cnt_zero, hipStream_t st) {
  WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
  const int nblk = m == 0 ? 1 : (m + kBinBlock - 1) / kBinBlock;
  uint8_t *binid = reinterpret_cast<uint8_t *>(ws + L.binid);
  int32_t *bh = reinterpret_cast<int32_t *>(ws + L.blockhist);
  int32_t *rows = reinterpret_cast<int32_t *>(ws + L.rows);
  int32_t *longrows = reinterpret_cast<int32_t *>(ws + L.fbrows);  // free until the row kernels
  hipLaunchKernelGGL(k_rowkey, dim3(nblk), dim3(kBinBlock), 0, st, dpr, maxbin, edges,
                     binid, bh, cnt_zero, longrows, hdr);
  hipLaunchKernelGGL(k_rowkey_long, dim3(dev_info().cus * 8), dim3(kKeyLongBlock), 0, st, dpr,
                     maxbin, edges,
                     binid, bh, nblk, cnt_zero, longrows, hdr);
  hipLaunchKernelGGL(k_binscan, dim3(kNB), dim3(1024), 0, st, bh, nblk, hdr);
  hipLaunchKernelGGL(k_binscatter, dim3(nblk), dim3(kBinBlock), 0, st, binid, m, bh, rows, hdr);
  return hipGetLastError();
}

hipError_t launch_scan(int32_t *rp, int m, int64_t capacity, const WsLayout &L, char *ws,
                       hipStream_t st) {
  WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
  int64_t *part = reinterpret_cast<int64_t *>(ws + L.scanpart);
  const int nparts = m == 0 ? 1 : (m + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_reduce, dim3(nparts), dim3(256), 0, st, rp, m, part, hdr);
  hipLaunchKernelGGL(k_scan_mid, dim3(1), dim3(1024), 0, st, part, nparts, capacity, hdr);
  hipLaunchKernelGGL(k_scan_apply, dim3(nparts), dim3(256), 0, st, rp, m, part, hdr);
  return hipGetLastError();
}

}  // namespace spg

// Kernels of the local product C = sum_k A_k B_k (K = 1: C = A B, paper §2)
// on gfx950: row keys and binning, symbolic count, scan, numeric pass.
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
// Setup: copy the problem into the workspace, clear the header.
__global__ void k_setup(Problem pr, Problem *dst, WsHeader *hdr, int reset) {
  if (threadIdx.x == 0) *dst = pr;
  if (reset && threadIdx.x < kNB) {
    hdr->bin_count[threadIdx.x] = 0;
    hdr->bin_start[threadIdx.x] = 0;
  }
  if (reset && threadIdx.x == 0) {
    hdr->status = 0;
    hdr->nnz_total = 0;
    hdr->products_total = 0;
    hdr->bin_start[kNB] = 0;
  }
  if (threadIdx.x == 0) {
    hdr->fallback_count = 0;
    hdr->heavy_cursor = 0;
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
// a1/a2: row key (products per row, or nnz of a C row) and bin id; per-block
// bin histogram.  One thread per row, 256 rows per block.
constexpr int kBinBlock = 256;

__global__ __launch_bounds__(kBinBlock) void k_rowkey(const Problem *__restrict__ pr,
                                                      const int32_t *__restrict__ crp,
                                                      int mode, int maxbin, uint8_t *binid,
                                                      int32_t *blockhist, int32_t *cnt_zero,
                                                      WsHeader *hdr) {
  __shared__ int hist[kNB];
  __shared__ long long psum[kBinBlock / kWave];
  if (hdr->status) return;  // invalid operands or overflow: touch nothing
  if (threadIdx.x < kNB) hist[threadIdx.x] = 0;
  __syncthreads();
  const int m = pr->m;
  const int i = blockIdx.x * kBinBlock + threadIdx.x;
  int64_t key = 0;
  if (i < m) {
    if (mode == 0) {
      const int K = pr->K;
      for (int k = 0; k < K; ++k) {
        const Part &P = pr->part[k];
        int as, ae;
        a_row(P, i, as, ae);
        for (int p = as; p < ae; ++p) {
          int r = a_entry_row(P, i, p);
          key += P.brp[r + 1] - P.brp[r];
        }
      }
      if (key == 0) cnt_zero[i] = 0;
    } else {
      key = crp[i + 1] - crp[i];
    }
    int b = bin_of(key, maxbin);
    binid[i] = (uint8_t)b;
    atomicAdd(&hist[b], 1);
  }
  if (mode == 0) {
    // block sum of products -> header (int64)
    long long v = key;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane_id() == 0) psum[threadIdx.x / kWave] = v;
  }
  __syncthreads();
  if (threadIdx.x < kNB) blockhist[(int64_t)blockIdx.x * kNB + threadIdx.x] = hist[threadIdx.x];
  if (mode == 0 && threadIdx.x == 0) {
    long long s = 0;
    for (int w = 0; w < kBinBlock / kWave; ++w) s += psum[w];
    atomicAdd((unsigned long long *)&hdr->products_total, (unsigned long long)s);
  }
}

// Exclusive scan of the per-block histograms in bin-major order (one block).
__global__ __launch_bounds__(1024) void k_binscan(int32_t *blockhist, int nblk, WsHeader *hdr) {
  __shared__ int wsum[16];
  __shared__ int carry;
  const int tid = threadIdx.x;
  int base_all = 0;
  for (int b = 0; b < kNB; ++b) {
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int c0 = 0; c0 < nblk; c0 += 1024) {
      int idx = c0 + tid;
      int v = idx < nblk ? blockhist[(int64_t)idx * kNB + b] : 0;
      // inclusive wave scan
      int x = v;
      for (int off = 1; off < kWave; off <<= 1) {
        int y = __shfl_up(x, off);
        if (lane_id() >= off) x += y;
      }
      if (lane_id() == kWave - 1) wsum[tid / kWave] = x;
      __syncthreads();
      int wpre = 0, tot = 0;
      for (int w = 0; w < 16; ++w) {
        if (w < tid / kWave) wpre += wsum[w];
        tot += wsum[w];
      }
      int excl = carry + wpre + x - v;
      if (idx < nblk) blockhist[(int64_t)idx * kNB + b] = base_all + excl;
      __syncthreads();
      if (tid == 0) carry += tot;
      __syncthreads();
    }
    if (tid == 0) {
      hdr->bin_count[b] = carry;
      hdr->bin_start[b] = base_all;
    }
    base_all += carry;
    __syncthreads();
  }
  if (tid == 0) hdr->bin_start[kNB] = base_all;
}

// Stable scatter of row ids into the per-bin lists.
__global__ __launch_bounds__(kBinBlock) void k_binscatter(const uint8_t *binid, int m,
                                                          const int32_t *blockoff,
                                                          int32_t *rows, const WsHeader *hdr) {
  __shared__ int wcnt[kBinBlock / kWave][kNB];
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
    int off = blockoff[(int64_t)blockIdx.x * kNB + b];
    for (int ww = 0; ww < w; ++ww) off += wcnt[ww][b];
    rows[off + myrank] = i;
  }
}

// ---------------------------------------------------------------------------
// a3: symbolic count with an LDS hash set per row.  G lanes per row, S lanes
// share one B row, T slots (power of 2, >= 2x the bin's product bound).
template <int WG>
__global__ __launch_bounds__(WG) void k_sym_hash(const Problem *__restrict__ pr,
                                                 const int32_t *__restrict__ rows,
                                                 const WsHeader *__restrict__ hdr, int bin,
                                                 int G, int S, int log2T,
                                                 int32_t *__restrict__ cnt) {
  extern __shared__ int smem[];
  const int T = 1 << log2T;
  const int R = WG / G;
  const int grp = threadIdx.x / G, l = threadIdx.x % G;
  int *tab = smem + grp * T;
  int *rowcnt = smem + R * T;
  if (hdr->status) return;
  const int count = hdr->bin_count[bin];
  const int start = hdr->bin_start[bin];
  const int K = pr->K;
  const int ES = G / S;
  for (int base = blockIdx.x * R; base < count; base += gridDim.x * R) {
    const int ri = base + grp;
    const bool active = ri < count;
    const int i = active ? rows[start + ri] : 0;
    for (int s = l; s < T; s += G) tab[s] = kEmpty;
    if (l == 0) rowcnt[grp] = 0;
    __syncthreads();
    int mine = 0;
    if (active) {
      for (int k = 0; k < K; ++k) {
        const Part &P = pr->part[k];
        int as, ae;
        a_row(P, i, as, ae);
        for (int p = as + l / S; p < ae; p += ES) {
          const int r = a_entry_row(P, i, p);
          const int bs = P.brp[r], be = P.brp[r + 1];
          for (int q = bs + l % S; q < be; q += S) {
            const int col = P.bcol[q];
            uint32_t h = scramble_slot((uint32_t)col, log2T);
            while (true) {
              const int old = atomicCAS(&tab[h], kEmpty, col);
              if (old == kEmpty) { ++mine; break; }
              if (old == col) break;
              h = (h + 1) & (T - 1);
            }
          }
        }
      }
      if (mine) atomicAdd(&rowcnt[grp], mine);
    }
    __syncthreads();
    if (active && l == 0) cnt[i] = rowcnt[grp];
    __syncthreads();
  }
}

// Symbolic count of heavy rows: a column bitmap (LDS when it fits, else the
// slot's global bitmap), one block per row.
template <bool LDSMAP>
__global__ __launch_bounds__(1024) void k_sym_heavy(const Problem *__restrict__ pr,
                                                    const int32_t *__restrict__ rows,
                                                    const WsHeader *__restrict__ hdr, int blo,
                                                    int S, uint32_t *gbitmap, int32_t *cnt) {
  extern __shared__ uint32_t lmap[];
  __shared__ int total;
  const int n = pr->n;
  const int nw = (n + 31) >> 5;
  uint32_t *map = LDSMAP ? lmap : gbitmap + (size_t)blockIdx.x * nw;
  if (hdr->status) return;
  const int start = hdr->bin_start[blo];
  const int count = hdr->bin_start[kHeavyBin + 1] - start;
  const int K = pr->K;
  const int tid = threadIdx.x;
  const int ES = 1024 / S;
  for (int ri = blockIdx.x; ri < count; ri += gridDim.x) {
    const int i = rows[start + ri];
    for (int w = tid; w < nw; w += 1024) map[w] = 0u;
    if (tid == 0) total = 0;
    if (!LDSMAP) __threadfence();
    __syncthreads();
    int mine = 0;
    for (int k = 0; k < K; ++k) {
      const Part &P = pr->part[k];
      int as, ae;
      a_row(P, i, as, ae);
      for (int p = as + tid / S; p < ae; p += ES) {
        const int r = a_entry_row(P, i, p);
        const int bs = P.brp[r], be = P.brp[r + 1];
        for (int q = bs + tid % S; q < be; q += S) {
          const uint32_t col = (uint32_t)P.bcol[q];
          const uint32_t bit = 1u << (col & 31);
          const uint32_t old = atomicOr(&map[col >> 5], bit);
          mine += (old & bit) ? 0 : 1;
        }
      }
    }
    if (mine) atomicAdd(&total, mine);
    __syncthreads();
    if (tid == 0) cnt[i] = total;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// a3 scan: in-place exclusive scan of per-row counts into row_ptr[0..m]
// (int64 running total; > 2^31-1 raises the overflow status).
constexpr int kScanTile = 2048;  // 256 threads x 8

__global__ __launch_bounds__(256) void k_scan_reduce(const int32_t *cnt, int m, int64_t *part) {
  __shared__ long long ws[4];
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

// ---------------------------------------------------------------------------
// a5: numeric pass, LDS hash with an order-preserving home slot.
//
// The home slot floor(col * T / n) is monotone in col and linear probing
// walks forward only (T + kTail slots, no wrap), so two keys are out of
// order in the table only when the larger one sits in the same run of
// occupied slots before the smaller one.  The rank of a key is therefore
// (occupied slots before it) + (smaller keys after it in its run) -
// (larger keys before it in its run), and each lane writes its entries
// straight to their final position.  A run longer than `maxwin`, or a probe
// past the tail, sends the row to the sort-based fallback kernel.
template <int WG, typename VT>
__global__ __launch_bounds__(WG) void k_num_hash(const Problem *__restrict__ pr,
                                                 const int32_t *__restrict__ rows,
                                                 WsHeader *__restrict__ hdr, int bin, int G,
                                                 int S, int T, uint32_t mul, int maxwin,
                                                 const int32_t *__restrict__ crp,
                                                 int32_t *__restrict__ ccol,
                                                 VT *__restrict__ cval,
                                                 int32_t *__restrict__ fb_rows) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int TT = T + kTail;
  const int R = WG / G;
  VT *vals = reinterpret_cast<VT *>(smem_raw);
  int *keys = reinterpret_cast<int *>(vals + (size_t)R * TT);
  int *rowflag = keys + (size_t)R * TT;
  int *wtot = rowflag + R;  // per-wave totals (G > 64)
  if (hdr->status) return;
  const int grp = threadIdx.x / G, l = threadIdx.x % G;
  int *key = keys + (size_t)grp * TT;
  VT *val = vals + (size_t)grp * TT;
  const int count = hdr->bin_count[bin];
  const int start = hdr->bin_start[bin];
  const int K = pr->K;
  const int ES = G / S;
  const int lane = lane_id();
  const int g0 = (G < kWave) ? (lane / G) * G : 0;
  const uint64_t gmask = (G >= kWave) ? ~0ull : (((1ull << G) - 1ull) << g0);
  const uint64_t ltmask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  for (int base = blockIdx.x * R; base < count; base += gridDim.x * R) {
    const int ri = base + grp;
    const bool active = ri < count;
    const int i = active ? rows[start + ri] : 0;
    for (int s = l; s < TT; s += G) {
      key[s] = kEmpty;
      val[s] = VT(0);
    }
    if (l == 0) rowflag[grp] = 0;
    __syncthreads();
    if (active) {
      for (int k = 0; k < K; ++k) {
        const Part &P = pr->part[k];
        int as, ae;
        a_row(P, i, as, ae);
        for (int p = as + l / S; p < ae; p += ES) {
          int r;
          VT a;
          a_entry<VT>(P, i, p, r, a);
          const int bs = P.brp[r], be = P.brp[r + 1];
          const VT *bv = static_cast<const VT *>(P.bval);
          for (int q = bs + l % S; q < be; q += S) {
            const int col = P.bcol[q];
            const VT prod = a * bv[q];
            int h = (int)mono_slot((uint32_t)col, mul);
            while (true) {
              const int old = atomicCAS(&key[h], kEmpty, col);
              if (old == kEmpty || old == col) {
                lds_add(&val[h], prod);
                break;
              }
              if (++h == TT) {  // table tail exhausted: fallback row
                rowflag[grp] = 1;
                break;
              }
            }
          }
        }
      }
    }
    __syncthreads();
    const bool ok = active && rowflag[grp] == 0;
    const int rs = active ? crp[i] : 0;
    const int nnz = active ? crp[i + 1] - rs : 0;
    int pre = 0;
    bool longrun = false;
    for (int s0 = 0; s0 < TT; s0 += G) {
      const int s = s0 + l;
      const int x = (s < TT) ? key[s] : kEmpty;
      const bool occ = x != kEmpty;
      const uint64_t mask = __ballot(occ);
      int pos;
      if (G <= kWave) {
        const uint64_t gm = mask & gmask;
        pos = pre + __popcll(gm & ltmask);
        pre += __popcll(gm);
      } else {
        const int wg = threadIdx.x / kWave, nwv = G / kWave, w0 = grp * nwv;
        if (lane == 0) wtot[wg] = __popcll(mask);
        __syncthreads();
        int wp = 0, tot = 0;
        for (int ww = w0; ww < w0 + nwv; ++ww) {
          const int c = wtot[ww];
          wp += (ww < wg) ? c : 0;
          tot += c;
        }
        pos = pre + wp + __popcll(mask & ltmask);
        pre += tot;
        __syncthreads();
      }
      if (ok && occ) {
        int r = pos;
        int c = 0;
        for (int t = s - 1; t >= 0; --t) {
          const int y = key[t];
          if (y == kEmpty) break;
          if (++c > maxwin) { longrun = true; break; }
          r -= (y > x);
        }
        c = 0;
        for (int t = s + 1; t < TT; ++t) {
          const int y = key[t];
          if (y == kEmpty) break;
          if (++c > maxwin) { longrun = true; break; }
          r += (y < x);
        }
        r = r < 0 ? 0 : (r >= nnz ? nnz - 1 : r);
        if (nnz > 0) {
          ccol[rs + r] = x;
          cval[rs + r] = val[s];
        }
      }
    }
    if (longrun) rowflag[grp] = 2;
    if (ok && l == 0 && pre != nnz) atomicOr(&hdr->status, kStatInvalid);
    __syncthreads();
    if (active && l == 0 && rowflag[grp] != 0) {
      const int slot = atomicAdd(&hdr->fallback_count, 1);
      fb_rows[slot] = i;
    }
    __syncthreads();
  }
}

// Block-wide exclusive prefix of a 0/1 flag over 1024 threads; returns the
// position and the block total.
__device__ inline int block_flag_prefix(bool f, int *wtot, int &total) {
  const uint64_t mask = __ballot(f);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) wtot[w] = __popcll(mask);
  __syncthreads();
  int wp = 0, tot = 0;
  for (int ww = 0; ww < 1024 / kWave; ++ww) {
    const int c = wtot[ww];
    wp += (ww < w) ? c : 0;
    tot += c;
  }
  __syncthreads();
  total = tot;
  const uint64_t lt = (lane_id() == 0) ? 0ull : (~0ull >> (kWave - lane_id()));
  return wp + __popcll(mask & lt);
}

// Fallback numeric pass: scrambled LDS hash, in-place compaction, bitonic
// sort of (column, value) pairs, coalesced write.  One row per block.
template <typename VT>
__global__ __launch_bounds__(1024) void k_num_fallback(const Problem *__restrict__ pr,
                                                       const int32_t *__restrict__ fb_rows,
                                                       WsHeader *__restrict__ hdr, int TF,
                                                       const int32_t *__restrict__ crp,
                                                       int32_t *__restrict__ ccol,
                                                       VT *__restrict__ cval) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int wtot[16];
  VT *val = reinterpret_cast<VT *>(smem_raw);
  int *key = reinterpret_cast<int *>(val + TF);
  if (hdr->status) return;
  const int count = hdr->fallback_count;
  const int K = pr->K;
  const int tid = threadIdx.x;
  for (int ri = blockIdx.x; ri < count; ri += gridDim.x) {
    const int i = fb_rows[ri];
    const int rs = crp[i];
    const int nnz = crp[i + 1] - rs;
    int P2 = 1;
    while (P2 < nnz) P2 <<= 1;
    int T = 2 * P2;
    if (T > TF) T = TF;
    int log2T = 0;
    while ((1 << log2T) < T) ++log2T;
    for (int s = tid; s < T; s += 1024) {
      key[s] = kEmpty;
      val[s] = VT(0);
    }
    __syncthreads();
    for (int k = 0; k < K; ++k) {
      const Part &P = pr->part[k];
      int as, ae;
      a_row(P, i, as, ae);
      for (int p = as + tid / 16; p < ae; p += 1024 / 16) {
        int r;
        VT a;
        a_entry<VT>(P, i, p, r, a);
        const int bs = P.brp[r], be = P.brp[r + 1];
        const VT *bv = static_cast<const VT *>(P.bval);
        for (int q = bs + tid % 16; q < be; q += 16) {
          const int col = P.bcol[q];
          const VT prod = a * bv[q];
          uint32_t h = scramble_slot((uint32_t)col, log2T);
          for (int probes = 0;; ++probes) {
            const int old = atomicCAS(&key[h], kEmpty, col);
            if (old == kEmpty || old == col) {
              lds_add(&val[h], prod);
              break;
            }
            if (probes >= T) {  // more distinct columns than the symbolic pass counted
              atomicOr(&hdr->status, kStatInvalid);
              break;
            }
            h = (h + 1) & (T - 1);
          }
        }
      }
    }
    __syncthreads();
    // in-place compaction in slot order (reads of a round precede its writes)
    int pre = 0;
    for (int s0 = 0; s0 < T; s0 += 1024) {
      const int s = s0 + tid;
      const int x = s < T ? key[s] : kEmpty;
      const VT v = s < T ? val[s] : VT(0);
      int tot;
      const int pos = pre + block_flag_prefix(x != kEmpty, wtot, tot);
      if (x != kEmpty) {
        key[pos] = x;
        val[pos] = v;
      }
      pre += tot;
      __syncthreads();
    }
    if (tid == 0 && pre != nnz) atomicOr(&hdr->status, kStatInvalid);
    for (int s = nnz + tid; s < P2; s += 1024) key[s] = 0x7fffffff;
    __syncthreads();
    // bitonic sort of P2 pairs by key
    for (int kk = 2; kk <= P2; kk <<= 1) {
      for (int j = kk >> 1; j > 0; j >>= 1) {
        for (int t = tid; t < P2 / 2; t += 1024) {
          const int a = 2 * j * (t / j) + (t % j);
          const int b = a + j;
          const bool up = (a & kk) == 0;
          const int ka = key[a], kb = key[b];
          if ((ka > kb) == up) {
            key[a] = kb;
            key[b] = ka;
            const VT va = val[a];
            val[a] = val[b];
            val[b] = va;
          }
        }
        __syncthreads();
      }
    }
    for (int t = tid; t < nnz; t += 1024) {
      ccol[rs + t] = key[t];
      cval[rs + t] = val[t];
    }
    __syncthreads();
  }
}

// Numeric pass of heavy rows: a column bitmap (LDS when it fits, else the
// slot's global bitmap) and the slot's dense accumulator in global memory.
// Pass 1 marks columns and zeroes the accumulator entries it marks first,
// pass 2 adds the products, pass 3 walks the bitmap in column order, so the
// output row comes out sorted.  One block per row; block b owns slot b.
template <bool LDSMAP, typename VT>
__global__ __launch_bounds__(1024) void k_num_heavy(const Problem *__restrict__ pr,
                                                    const int32_t *__restrict__ rows,
                                                    WsHeader *__restrict__ hdr, int blo, int S,
                                                    uint32_t *gbitmap, VT *gacc,
                                                    const int32_t *__restrict__ crp,
                                                    int32_t *__restrict__ ccol,
                                                    VT *__restrict__ cval) {
  extern __shared__ uint32_t lmap[];
  __shared__ int wtot[16];
  if (hdr->status) return;
  const int n = pr->n;
  const int nw = (n + 31) >> 5;
  uint32_t *map = LDSMAP ? lmap : gbitmap + (size_t)blockIdx.x * nw;
  VT *acc = gacc + (size_t)blockIdx.x * n;
  const int start = hdr->bin_start[blo];
  const int count = hdr->bin_start[kHeavyBin + 1] - start;
  const int K = pr->K;
  const int tid = threadIdx.x;
  const int ES = 1024 / S;
  for (int ri = blockIdx.x; ri < count; ri += gridDim.x) {
    const int i = rows[start + ri];
    for (int w = tid; w < nw; w += 1024) map[w] = 0u;
    __threadfence();
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      for (int k = 0; k < K; ++k) {
        const Part &P = pr->part[k];
        int as, ae;
        a_row(P, i, as, ae);
        for (int p = as + tid / S; p < ae; p += ES) {
          int r;
          VT a;
          a_entry<VT>(P, i, p, r, a);
          const int bs = P.brp[r], be = P.brp[r + 1];
          const VT *bv = static_cast<const VT *>(P.bval);
          for (int q = bs + tid % S; q < be; q += S) {
            const uint32_t col = (uint32_t)P.bcol[q];
            if (pass == 0) {
              const uint32_t bit = 1u << (col & 31);
              const uint32_t old = atomicOr(&map[col >> 5], bit);
              if (!(old & bit)) acc[col] = VT(0);
            } else {
              global_add(&acc[col], a * bv[q]);
            }
          }
        }
      }
      // the accumulator lives in global memory: complete the stores/atomics
      // of this pass at device scope and drop stale L1 lines before reading
      __threadfence();
      __syncthreads();
    }
    const int rs = crp[i];
    const int re = crp[i + 1];
    int pre = 0;
    for (int w0 = 0; w0 < nw; w0 += 1024) {
      const int w = w0 + tid;
      const uint32_t bits = w < nw ? map[w] : 0u;
      const int c = __popc(bits);
      // block exclusive scan of c
      int x = c;
      for (int off = 1; off < kWave; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane_id() >= off) x += y;
      }
      if (lane_id() == kWave - 1) wtot[tid / kWave] = x;
      __syncthreads();
      int wp = 0, tot = 0;
      for (int ww = 0; ww < 16; ++ww) {
        const int cc = wtot[ww];
        wp += (ww < tid / kWave) ? cc : 0;
        tot += cc;
      }
      int o = rs + pre + wp + x - c;
      uint32_t b = bits;
      while (b) {
        const int j = __ffs(b) - 1;
        b &= b - 1;
        const int col = (w << 5) + j;
        if (o < re) {  // the symbolic count bounds the row (a changed pattern is flagged)
          ccol[o] = col;
          cval[o] = acc[col];
        }
        ++o;
      }
      pre += tot;
      __syncthreads();
    }
    if (tid == 0 && pre != re - rs) atomicOr(&hdr->status, kStatInvalid);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Host launchers.

static int blocks_per_cu(size_t lds, int wg, size_t lds_limit_cu) {
  int by_lds = lds ? (int)(lds_limit_cu / lds) : 64;
  int by_thr = 2048 / wg;
  int b = by_lds < by_thr ? by_lds : by_thr;
  return b < 1 ? 1 : b;
}

// A heavy row's column bitmap lives in LDS when it fits one block.
static bool lds_bitmap_fits(int n) {
  return n <= kLdsBitmapCols && (size_t)((n + 31) >> 5) * 4 + 1024 <= dev_info().lds_per_block;
}

static int wg_for(int G) { return G <= 256 ? 256 : (G <= 512 ? 512 : 1024); }

static int log2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

hipError_t launch_setup(const Problem &pr, Problem *dst, WsHeader *hdr, bool reset,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_setup, dim3(1), dim3(64), 0, st, pr, dst, hdr, reset ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_validate(const int32_t *rp, const int32_t *col, int rows, int ncols,
                           int64_t nnz, WsHeader *hdr, hipStream_t st) {
  hipLaunchKernelGGL(k_validate, dim3(256), dim3(256), 0, st, rp, col, rows, ncols, nnz, hdr);
  return hipGetLastError();
}

hipError_t launch_binning(const Problem *dpr, const int32_t *crp, int mode, int m, int maxbin,
                          const WsLayout &L, char *ws, int32_t *cnt_zero, hipStream_t st) {
  WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
  const int nblk = m == 0 ? 1 : (m + kBinBlock - 1) / kBinBlock;
  uint8_t *binid = reinterpret_cast<uint8_t *>(ws + L.binid);
  int32_t *bh = reinterpret_cast<int32_t *>(ws + L.blockhist);
  int32_t *rows = reinterpret_cast<int32_t *>(ws + L.rows);
  hipLaunchKernelGGL(k_rowkey, dim3(nblk), dim3(kBinBlock), 0, st, dpr, crp, mode, maxbin,
                     binid, bh, cnt_zero, hdr);
  hipLaunchKernelGGL(k_binscan, dim3(1), dim3(1024), 0, st, bh, nblk, hdr);
  hipLaunchKernelGGL(k_binscatter, dim3(nblk), dim3(kBinBlock), 0, st, binid, m, bh, rows, hdr);
  return hipGetLastError();
}

hipError_t launch_scan(int32_t *rp, int m, int64_t capacity, const WsLayout &L, char *ws,
                       hipStream_t st) {
  WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
  int64_t *part = reinterpret_cast<int64_t *>(ws + L.scanpart);
  const int nparts = m == 0 ? 1 : (m + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_reduce, dim3(nparts), dim3(256), 0, st, rp, m, part);
  hipLaunchKernelGGL(k_scan_mid, dim3(1), dim3(1024), 0, st, part, nparts, capacity, hdr);
  hipLaunchKernelGGL(k_scan_apply, dim3(nparts), dim3(256), 0, st, rp, m, part, hdr);
  return hipGetLastError();
}

// rows in bins [lo, hi]: known count (eager) or -1
static int bins_count(const BinPlan &bp, int lo, int hi) {
  if (!bp.known) return -1;
  int c = 0;
  for (int b = lo; b <= hi; ++b) c += bp.count[b];
  return c;
}

static int grid_for(int count, int rows_per_block, int cap) {
  if (count < 0) return cap;
  const int need = (count + rows_per_block - 1) / rows_per_block;
  return need < cap ? need : cap;
}

template <int WG>
static void sym_launch(const Problem *dpr, const int32_t *rows, const WsHeader *hdr, int bin,
                       int G, int S, int log2T, int32_t *cnt, int grid, size_t lds,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_sym_hash<WG>, dim3(grid), dim3(WG), lds, st, dpr, rows, hdr, bin, G, S,
                     log2T, cnt);
}

hipError_t launch_symbolic_bins(const Problem *dpr, const BinPlan &bp, const WsLayout &L,
                                char *ws, int32_t *cnt, hipStream_t st) {
  WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
  const int32_t *rows = reinterpret_cast<const int32_t *>(ws + L.rows);
  const DevInfo &D = dev_info();
  for (int b = 1; b <= bp.maxbin; ++b) {
    if (bp.known && bp.count[b] == 0) continue;
    const int G = bp.lanes[b];
    const int WG = wg_for(G);
    const int S = bp.sub < G ? bp.sub : G;
    const int T = bin_slots(b);
    const int R = WG / G;
    const size_t lds = (size_t)R * T * 4 + (size_t)R * 4;
    const int grid = grid_for(bins_count(bp, b, b), R, D.cus * blocks_per_cu(lds, WG, D.lds_per_cu));
    if (WG == 256)
      sym_launch<256>(dpr, rows, hdr, b, G, S, log2i(T), cnt, grid, lds, st);
    else if (WG == 512)
      sym_launch<512>(dpr, rows, hdr, b, G, S, log2i(T), cnt, grid, lds, st);
    else
      sym_launch<1024>(dpr, rows, hdr, b, G, S, log2i(T), cnt, grid, lds, st);
  }
  const int hc = bins_count(bp, bp.maxbin + 1, kHeavyBin);
  if (hc != 0) {
    const int grid = grid_for(hc, 1, bp.heavy_slots);
    if (lds_bitmap_fits(bp.n)) {
      const size_t lds = (size_t)((bp.n + 31) >> 5) * 4;
      hipLaunchKernelGGL(k_sym_heavy<true>, dim3(grid), dim3(1024), lds, st, dpr, rows, hdr,
                         bp.maxbin + 1, bp.sub, (uint32_t *)nullptr, cnt);
    } else {
      hipLaunchKernelGGL(k_sym_heavy<false>, dim3(grid), dim3(1024), 0, st, dpr, rows, hdr,
                         bp.maxbin + 1, bp.sub, reinterpret_cast<uint32_t *>(ws + L.heavymap),
                         cnt);
    }
  }
  return hipGetLastError();
}

template <int WG, typename VT>
static void num_launch(const Problem *dpr, const int32_t *rows, WsHeader *hdr, int bin, int G,
                       int S, int T, uint32_t mul, int maxwin, const int32_t *crp,
                       int32_t *ccol, VT *cval, int32_t *fb, int grid, size_t lds,
                       hipStream_t st) {
  hipLaunchKernelGGL((k_num_hash<WG, VT>), dim3(grid), dim3(WG), lds, st, dpr, rows, hdr, bin, G,
                     S, T, mul, maxwin, crp, ccol, cval, fb);
}

template <typename VT>
static hipError_t numeric_impl(const Problem *dpr, const BinPlan &bp, const WsLayout &L,
                               char *ws, const int32_t *crp, int32_t *ccol, VT *cval,
                               hipStream_t st) {
  WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
  const int32_t *rows = reinterpret_cast<const int32_t *>(ws + L.rows);
  int32_t *fb = reinterpret_cast<int32_t *>(ws + L.fbrows);
  const DevInfo &D = dev_info();
  for (int b = 1; b <= bp.maxbin; ++b) {
    if (bp.known && bp.count[b] == 0) continue;
    const int G = bp.lanes[b];
    const int WG = wg_for(G);
    const int S = bp.sub < G ? bp.sub : G;
    const int T = bin_slots(b);
    const int R = WG / G;
    const size_t lds = (size_t)R * (T + kTail) * (sizeof(VT) + 4) + (size_t)R * 4 + 64;
    const int grid = grid_for(bins_count(bp, b, b), R, D.cus * blocks_per_cu(lds, WG, D.lds_per_cu));
    const uint32_t mul = mono_mul(T, bp.n);
    if (WG == 256)
      num_launch<256, VT>(dpr, rows, hdr, b, G, S, T, mul, bp.maxwin, crp, ccol, cval, fb, grid,
                          lds, st);
    else if (WG == 512)
      num_launch<512, VT>(dpr, rows, hdr, b, G, S, T, mul, bp.maxwin, crp, ccol, cval, fb, grid,
                          lds, st);
    else
      num_launch<1024, VT>(dpr, rows, hdr, b, G, S, T, mul, bp.maxwin, crp, ccol, cval, fb, grid,
                           lds, st);
  }
  if (bins_count(bp, 1, bp.maxbin) != 0) {
    // rows the LDS kernels hand over (long runs, exhausted table tail)
    const int TF = bin_slots(bp.maxbin);
    const size_t lds = (size_t)TF * (sizeof(VT) + 4);
    hipLaunchKernelGGL(k_num_fallback<VT>, dim3(D.cus), dim3(1024), lds, st, dpr, fb, hdr, TF,
                       crp, ccol, cval);
  }
  const int hc = bins_count(bp, bp.maxbin + 1, kHeavyBin);
  if (hc != 0) {
    const int grid = grid_for(hc, 1, bp.heavy_slots);
    VT *acc = reinterpret_cast<VT *>(ws + L.heavyacc);
    if (lds_bitmap_fits(bp.n)) {
      const size_t lds = (size_t)((bp.n + 31) >> 5) * 4;
      hipLaunchKernelGGL((k_num_heavy<true, VT>), dim3(grid), dim3(1024), lds, st, dpr, rows,
                         hdr, bp.maxbin + 1, bp.sub, (uint32_t *)nullptr, acc, crp, ccol, cval);
    } else {
      hipLaunchKernelGGL((k_num_heavy<false, VT>), dim3(grid), dim3(1024), 0, st, dpr, rows, hdr,
                         bp.maxbin + 1, bp.sub, reinterpret_cast<uint32_t *>(ws + L.heavymap),
                         acc, crp, ccol, cval);
    }
  }
  return hipGetLastError();
}

hipError_t launch_numeric(const Problem *dpr, const BinPlan &bp, const WsLayout &L, char *ws,
                          const int32_t *crp, int32_t *ccol, void *cval, int dtype,
                          hipStream_t st) {
  if (dtype == SPG_F64)
    return numeric_impl<double>(dpr, bp, L, ws, crp, ccol, static_cast<double *>(cval), st);
  return numeric_impl<float>(dpr, bp, L, ws, crp, ccol, static_cast<float *>(cval), st);
}

// Kernels that may use more than 64 KiB of dynamic LDS are opted in once.
hipError_t configure_lds_limits(size_t lds_max) {
  const void *ks[] = {
      reinterpret_cast<const void *>(&k_sym_hash<256>),
      reinterpret_cast<const void *>(&k_sym_hash<512>),
      reinterpret_cast<const void *>(&k_sym_hash<1024>),
      reinterpret_cast<const void *>(&k_sym_heavy<true>),
      reinterpret_cast<const void *>(&k_num_hash<256, float>),
      reinterpret_cast<const void *>(&k_num_hash<512, float>),
      reinterpret_cast<const void *>(&k_num_hash<1024, float>),
      reinterpret_cast<const void *>(&k_num_hash<256, double>),
      reinterpret_cast<const void *>(&k_num_hash<512, double>),
      reinterpret_cast<const void *>(&k_num_hash<1024, double>),
      reinterpret_cast<const void *>(&k_num_fallback<float>),
      reinterpret_cast<const void *>(&k_num_fallback<double>),
      reinterpret_cast<const void *>(&k_num_heavy<true, float>),
      reinterpret_cast<const void *>(&k_num_heavy<true, double>),
  };
  for (const void *k : ks) {
    hipError_t e =
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace spg

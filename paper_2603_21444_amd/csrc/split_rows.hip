// Heavy rows shared by many blocks: the symbolic description of a split
// row, the scatter of its products into column ranges, and the merge of
// each segment of ranges (paper §4.4: the level of the row-wise product's
// multi-level accumulator beyond shared memory; here no row is left to a
// single compute unit).
//
// A row of C = sum_k A_k B_k with many products (a power-law hub) used to
// be one block's work from its first product to its last output, so the
// largest row set the length of the whole pass.  Here:
//  - the symbolic kernel (one block per row, column bitmap in LDS) also
//    counts products and distinct columns per range of 8192 columns, cuts
//    the ranges into segments and reserves the row's staging entries;
//  - the scatter kernel takes items of about kSplitItem products of any
//    split row (a window of the row's A entries) and drops each product
//    into its range's run of the row's staging area;
//  - the merge kernel takes one segment at a time: at most kSplitSeg
//    products, placed into order-preserving buckets over the segment's
//    columns in LDS, sorted, summed by column and written at the segment's
//    output offset; or a single range with more products, summed in a
//    dense LDS panel of 8192 columns.
// A row the workspace cannot describe or stage stays with the one-block
// heavy kernels, which take the list of such rows.
#include "internal.hpp"
#include "rowops.hpp"

namespace spg {

constexpr int kSplitSymUnroll = 4;
constexpr int kSplitUnroll = 2;
constexpr int kScatterNT = 256;         // threads of a scatter block
constexpr int kSplitBuf = 3072;         // products an item keeps in LDS
constexpr int kAccumNT = 512;           // threads of a merge block
constexpr int kRangeWords = (1 << kSplitLog2W) >> 5;  // bitmap words per range
static_assert(kSplitSeg % kAccumNT == 0, "whole products per thread");

// ---------------------------------------------------------------------------
// Symbolic: distinct columns of every row from bin blo on (heavy rows, one
// block per row, column bitmap in LDS or in the slot's global bitmap), and
// for rows h < hmax (sa.F > 0) the split description.

template <bool LDSMAP>
__global__ __launch_bounds__(1024) void k_sym_split(const Problem *__restrict__ pr,
                                                    const int32_t *__restrict__ rows,
                                                    WsHeader *__restrict__ hdr, int blo, int lS,
                                                    uint32_t *gbitmap, int32_t *cnt,
                                                    SplitArgs sa) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int sb[1024], sl[1024];
  __shared__ int pe[kSplitMaxRanges + 1], de[kSplitMaxRanges + 1];
  __shared__ int sstart[kSplitMaxRanges];
  __shared__ int wtot[16];
  __shared__ int total, item, okflag, segbase, itembase, stagebase, nentries;
  __shared__ unsigned long long prod64;  // the row's products (the range counters are 32-bit)
  const int n = pr->n;
  const int nw = (n + 31) >> 5;
  uint32_t *map = LDSMAP ? reinterpret_cast<uint32_t *>(smem_raw) : gbitmap + (size_t)blockIdx.x * nw;
  if (hdr->status) return;
  const int start = hdr->bin_start[blo];
  const int count = hdr->bin_start[kHeavyBin + 1] - start;
  const int tid = threadIdx.x;
  const int F = sa.F;
  Stage<float> st{sb, sl, nullptr};
  for (int ri = block_next(&hdr->queue[kQueueHeavy], &item); ri < count;
       ri = block_next(&hdr->queue[kQueueHeavy], &item)) {
    const int i = rows[start + ri];
    const bool rec = F > 0 && ri < sa.hmax;  // the same in every thread
    for (int w = tid; w < nw; w += 1024) map[w] = 0u;
    if (rec)
      for (int c = tid; c <= F; c += 1024) {
        pe[c] = 0;
        de[c] = 0;
      }
    if (tid == 0) {
      total = 0;
      prod64 = 0;
    }
    if (!LDSMAP) __threadfence();
    __syncthreads();
    int mine = 0;  // described rows: products; others: new distinct columns
    auto fmark = each_product([&](int col, float) {
      const uint32_t bit = 1u << (col & 31);
      if (rec) {  // distinct columns come from the popcounts below
        atomicOr(&map[col >> 5], bit);
        atomicAdd(&pe[col >> kSplitLog2W], 1);
        ++mine;
      } else {
        const uint32_t old = atomicOr(&map[col >> 5], bit);
        mine += (old & bit) ? 0 : 1;
      }
    });
    for_each_product<true, false, 1024, kSplitSymUnroll, float>(pr, i, true, tid, lS, st, fmark);
    if (mine) {
      if (rec) atomicAdd(&prod64, (unsigned long long)mine);
      else atomicAdd(&total, mine);
    }
    if (!LDSMAP) __threadfence();
    __syncthreads();
    if (!rec) {
      if (tid == 0) cnt[i] = total;
      continue;
    }
    // distinct columns per range: the 64 words a wave reads lie in one range
    for (int w0 = 0; w0 < nw; w0 += 1024) {
      const int w = w0 + tid;
      int pop = w < nw ? __popc(map[w]) : 0;
#pragma unroll
      for (int off = kWave / 2; off > 0; off >>= 1) pop += __shfl_xor(pop, off);
      if (lane_id() == 0 && pop) atomicAdd(&de[w / kRangeWords], pop);
    }
    __syncthreads();
    const int pc = tid < F ? pe[tid] : 0;
    const int dc = tid < F ? de[tid] : 0;
    int P, D;
    const int pex = group_excl_scan<true, 1024>(pc, tid, wtot, P);
    const int dex = group_excl_scan<true, 1024>(dc, tid, wtot, D);
    if (tid < F) {
      pe[tid] = pex;
      de[tid] = dex;
    }
    if (tid == 0) {
      pe[F] = P;
      de[F] = D;
    }
    __syncthreads();
    // segment starts: a range holding more than half a segment stands
    // alone; the others group while their product prefix stays in the same
    // multiple of half a segment (so a group holds fewer than kSplitSeg)
    constexpr int H = kSplitSeg / 2;
    int flag = 0;
    if (tid < F) {
      const int a = pe[tid];
      if (tid == 0) {
        flag = 1;
      } else {
        const int ap = pe[tid - 1];
        const bool big = pe[tid + 1] - a > H, bigp = a - ap > H;
        flag = (big || bigp || a / H != ap / H) ? 1 : 0;
      }
    }
    int nseg;
    const int sidx = group_excl_scan<true, 1024>(flag, tid, wtot, nseg);
    if (flag) sstart[sidx] = tid;
    const int J = (P + kSplitItem - 1) / kSplitItem;
    if (tid == 0) {
      int E = 0;  // A entries of the row over all parts
      for (int k = 0; k < pr->K; ++k) {
        int as, ae;
        a_row(pr->part[k], i, as, ae);
        E += ae - as;
      }
      nentries = E;
      // a row of more products than the staging area holds (then its
      // 32-bit range counters may also have wrapped) is not described
      int ok = prod64 > 0 && prod64 <= (unsigned long long)sa.pcap && nseg > 0;
      long long b = -1;
      int sg = -1, ib = -1;
      if (ok) {
        b = (long long)atomicAdd(&sa.ctl->stage, (unsigned long long)P);
        ok = b + P <= sa.pcap;
      }
      if (ok) {
        sg = atomicAdd(&sa.ctl->segs, nseg);
        ib = atomicAdd(&sa.ctl->items, J);
        ok = sg <= sa.segcap - nseg && ib <= sa.itemcap - J;
      }
      okflag = ok;
      stagebase = ok ? (int)b : -1;
      segbase = sg;
      itembase = ib;
      cnt[i] = D;
      sa.rows[ri] = SplitRow{ok ? (int32_t)b : -1, J, P, i};
    }
    __syncthreads();
    if (okflag) {
      int32_t *fo = sa.fo + (size_t)ri * (F + 1);
      for (int c = tid; c <= F; c += 1024) fo[c] = pe[c];
      for (int s = tid; s < nseg; s += 1024) {
        const int f0 = sstart[s], f1 = s + 1 < nseg ? sstart[s + 1] : F;
        sa.segs[segbase + s] =
            SplitSeg{ri, f0 << kSplitLog2W, min(n, f1 << kSplitLog2W), stagebase + pe[f0],
                     pe[f1] - pe[f0], de[f0], de[f1] - de[f0], -1};
      }
      const int E = nentries;
      for (int j = tid; j < J; j += 1024)
        sa.items[itembase + j] =
            SplitItem{ri, i, (int)((int64_t)j * E / J), (int)((int64_t)(j + 1) * E / J)};
    } else if (segbase >= 0) {
      // reserved but unusable entries are marked unused
      for (int s = tid; s < nseg && segbase + s < sa.segcap; s += 1024) sa.segs[segbase + s].h = -1;
      for (int j = tid; j < J && itembase + j < sa.itemcap; j += 1024) sa.items[itembase + j].h = -1;
    }
  }
}

// ---------------------------------------------------------------------------
// Numeric, step 0: the scatter cursors of the split rows start at zero, and
// the heavy rows from bin blo on that are not split are listed for the
// one-block kernels.

__global__ void k_split_prepare(const int32_t *__restrict__ rows, WsHeader *__restrict__ hdr,
                                int blo, SplitArgs sa, const int32_t *__restrict__ crp,
                                int32_t *__restrict__ ulist) {
  if (hdr->status) return;
  const int sbin = hdr->bin_start[sa.bin];
  const int nsplit = min(hdr->bin_start[kHeavyBin + 1] - sbin, sa.hmax);
  const int64_t total = (int64_t)nsplit * sa.F;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = t0; t < total; t += step)
    if (sa.rows[t / sa.F].base >= 0) sa.cur[t] = 0;
  const int start = hdr->bin_start[blo];
  const int count = hdr->bin_start[kHeavyBin + 1] - start;
  for (int64_t t = t0; t < count; t += step) {
    const int h = start + (int)t - sbin;
    if (!(h >= 0 && h < sa.hmax && sa.rows[h].base >= 0))
      ulist[atomicAdd(&sa.ctl->nuns, 1)] = rows[start + t];
  }
  // output positions of the segments
  const int nseg = min(sa.ctl->segs, sa.segcap);
  for (int64_t t = t0; t < nseg; t += step) {
    const SplitSeg sg = sa.segs[t];
    if (sg.h < 0) continue;
    const int i = sa.rows[sg.h].row;
    int out = crp[i] + sg.dstart;
    if (out + sg.dcount > crp[i + 1]) {  // the row_ptr does not match the description
      atomicOr(&hdr->status, kStatInvalid);
      out = -1;
    }
    sa.segs[t].out = out;
  }
}

// Products of the item's window [e0, e1) of the row's A entries (all parts
// in order), every lane of the block taking part.
template <bool VALUES, typename VT, typename Fn>
__device__ __forceinline__ void window_products(const Problem *__restrict__ pr, int i, int e0,
                                                int e1, int tid, int lS, Stage<VT> st, Fn &f) {
  int off = 0;
  for (int k = 0; k < pr->K; ++k) {
    const Part &P = pr->part[k];
    int as, ae;
    a_row(P, i, as, ae);
    const int nk = ae - as;
    const int lo = max(e0 - off, 0), hi = min(e1 - off, nk);
    if (lo < hi)
      part_products<true, VALUES, kScatterNT, kSplitUnroll, VT>(P, i, true, tid, lS, st, f, 0, 1,
                                                                 lo, hi);
    off += nk;
  }
}

// Pass 1 of an item: products per range (LDS counters), and the products
// themselves in the LDS buffer while it has room (slots taken per wave).
template <typename VT>
struct ScatterCount {
  int *lc;
  int *nb;
  int32_t *bcol;
  VT *bval;
  template <int N>
  __device__ __forceinline__ void batch(const int (&col)[N], const VT (&v)[N]) {
    uint64_t m[N];
    int tot = 0;
#pragma unroll
    for (int u = 0; u < N; ++u) {
      if (col[u] >= 0) atomicAdd(&lc[col[u] >> kSplitLog2W], 1);
      m[u] = __ballot(col[u] >= 0);
      tot += __popcll(m[u]);
    }
    const uint64_t act = __ballot(true);
    const int leader = __ffsll((unsigned long long)act) - 1;
    int p0 = 0;
    if (tot > 0 && lane_id() == leader) p0 = atomicAdd(nb, tot);
    p0 = __shfl(p0, leader);
    const uint64_t below = lanes_below();
#pragma unroll
    for (int u = 0; u < N; ++u) {
      const int p = p0 + __popcll(m[u] & below);
      p0 += __popcll(m[u]);
      if (col[u] >= 0 && p < kSplitBuf) {
        bcol[p] = col[u];
        bval[p] = v[u];
      }
    }
  }
};

// The staging area of the split rows: FP32 products as one 8-byte word
// (column in the low half, value bits in the high half: one store in the
// scatter, one load in the merge); FP64 products as a column array and a
// value array.  Global-address-space pointers: global, not flat, memory
// instructions.
template <typename VT>
struct Staging {
  SPG_GLOBAL int32_t *col;
  SPG_GLOBAL VT *val;
  __device__ __forceinline__ void put(int p, int c, VT v) const {
    col[p] = c;
    val[p] = v;
  }
  __device__ __forceinline__ void get(int p, int &c, VT &v) const {
    c = col[p];
    v = val[p];
  }
};
template <>
struct Staging<float> {
  SPG_GLOBAL int32_t *col;  // the area's base, 256-byte aligned: 8-byte words
  SPG_GLOBAL float *val;    // unused
  __device__ __forceinline__ void put(int p, int c, float v) const {
    reinterpret_cast<SPG_GLOBAL unsigned long long *>(col)[p] =
        (unsigned long long)(uint32_t)c | ((unsigned long long)__float_as_uint(v) << 32);
  }
  __device__ __forceinline__ void get(int p, int &c, float &v) const {
    const unsigned long long w = reinterpret_cast<const SPG_GLOBAL unsigned long long *>(col)[p];
    c = (int)(uint32_t)w;
    v = __uint_as_float((uint32_t)(w >> 32));
  }
};

// Pass 2 of an item whose products overflowed the buffer: every product
// straight to its range's next staging entry.
template <typename VT>
struct ScatterPlace {
  int *lc;
  Staging<VT> sg;
  template <int N>
  __device__ __forceinline__ void batch(const int (&col)[N], const VT (&v)[N]) {
#pragma unroll
    for (int u = 0; u < N; ++u) {
      if (col[u] >= 0) {
        const int p = atomicAdd(&lc[col[u] >> kSplitLog2W], 1);
        if (p >= 0) sg.put(p, col[u], v[u]);
      }
    }
  }
};

// Numeric, step 1: items of the split rows from bin blo on.  The item's
// products are counted per range; one atomic per (item, range) on the
// row's range cursor reserves the item's run inside the range; then each
// product goes to the next entry of its run.
template <typename VT>
__global__ __launch_bounds__(kScatterNT) void k_split_scatter(const Problem *__restrict__ pr,
                                                              WsHeader *__restrict__ hdr, int blo,
                                                              int lS, SplitArgs sa) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int32_t *bcol = reinterpret_cast<int32_t *>(smem_raw);
  VT *bval = reinterpret_cast<VT *>(bcol + kSplitBuf);
  __shared__ int lc[kSplitMaxRanges];
  __shared__ int sb[kScatterNT], sl[kScatterNT];
  __shared__ VT sav[kScatterNT];
  __shared__ int nb, item;
  if (hdr->status) return;
  const int sbin = hdr->bin_start[sa.bin];
  const int hlo = hdr->bin_start[blo] - sbin;
  const int nitems = min(sa.ctl->items, sa.itemcap);
  const int tid = threadIdx.x;
  const int F = sa.F;
  const Staging<VT> stg{gpw(sa.scol), gpw(static_cast<VT *>(sa.sval))};
  Stage<VT> st{sb, sl, sav};
  for (int t = block_next(&sa.ctl->q_scatter, &item); t < nitems;
       t = block_next(&sa.ctl->q_scatter, &item)) {
    const SplitItem it = sa.items[t];
    // unused, or a row of an LDS bin of this pass
    if (it.h < hlo || it.h >= sa.hmax) continue;
    const int base = sa.rows[it.h].base;
    if (base < 0) continue;
    const int i = it.i, e0 = it.e0, e1 = it.e1;
    for (int c = tid; c < F; c += kScatterNT) lc[c] = 0;
    if (tid == 0) nb = 0;
    __syncthreads();
    ScatterCount<VT> fc{lc, &nb, bcol, bval};
    window_products<true, VT>(pr, i, e0, e1, tid, lS, st, fc);
    __syncthreads();
    // the item's run in each range it touches
    const int32_t *fo = sa.fo + (size_t)it.h * (F + 1);
    int32_t *cur = sa.cur + (size_t)it.h * F;
    for (int c = tid; c < F; c += kScatterNT) {
      const int k = lc[c];
      if (k) {
        const int p = atomicAdd(&cur[c], k);
        const int lim = fo[c + 1] - fo[c];
        if (p > lim - k) {  // more products than the symbolic pass saw
          atomicOr(&hdr->status, kStatInvalid);
          lc[c] = INT32_MIN / 2;
        } else {
          lc[c] = base + fo[c] + p;
        }
      }
    }
    __syncthreads();
    const int nbuf = nb;
    if (nbuf <= kSplitBuf) {
      for (int s = tid; s < nbuf; s += kScatterNT) {
        const int col = bcol[s];
        const int p = atomicAdd(&lc[col >> kSplitLog2W], 1);
        if (p >= 0) stg.put(p, col, bval[s]);
      }
    } else {
      ScatterPlace<VT> fp{lc, stg};
      window_products<true, VT>(pr, i, e0, e1, tid, lS, st, fp);
    }
  }
}

// ---------------------------------------------------------------------------
// Numeric, step 2: one segment at a time.

// A single range with more products than a sorted segment holds: sums in a
// dense LDS panel of the range's columns, a presence bitmap walked in
// column order.  Returns the distinct columns written.
template <typename VT>
__device__ int merge_dense(const Staging<VT> &stg, int P,
                           int c0, int D, VT *panel, uint32_t *bm, int *wtot,
                           SPG_GLOBAL int32_t *cb, SPG_GLOBAL VT *vb, WsHeader *hdr) {
  constexpr int W = 1 << kSplitLog2W;
  const int tid = threadIdx.x;
  for (int c = tid; c < W; c += kAccumNT) panel[c] = VT(0);
  for (int w = tid; w < kRangeWords; w += kAccumNT) bm[w] = 0u;
  __syncthreads();
  bool bad = false;
  constexpr int U = 4;
  for (int p0 = tid; p0 < P; p0 += U * kAccumNT) {
    int c[U];
    VT v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = p0 + u * kAccumNT;
      c[u] = -1;
      v[u] = VT(0);
      if (p < P) {
        stg.get(p, c[u], v[u]);
        c[u] -= c0;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (p0 + u * kAccumNT < P) {
        if ((unsigned)c[u] < (unsigned)W) {
          lds_add_cas(&panel[c[u]], v[u]);
          atomicOr(&bm[c[u] >> 5], 1u << (c[u] & 31));
        } else {
          bad = true;
        }
      }
    }
  }
  if (bad) atomicOr(&hdr->status, kStatInvalid);
  __syncthreads();
  uint32_t wd = tid < kRangeWords ? bm[tid] : 0u;
  int tot;
  int o = group_excl_scan<true, kAccumNT>(__popc(wd), tid, wtot, tot);
  while (wd) {
    const int c = (tid << 5) + __ffs(wd) - 1;
    wd &= wd - 1;
    if (o < D) {
      cb[o] = c0 + c;
      vb[o] = panel[c];
    }
    ++o;
  }
  return tot;
}

// Start of bucket b: the counters hold two 16-bit values per word.
__device__ __forceinline__ int seg_bucket(const uint32_t *cnt, uint32_t b) {
  return (int)((cnt[b >> 1] >> ((b & 1u) << 4)) & 0xffffu);
}

// At most kSplitSeg products over the columns [c0, c0 + span): placed into
// T order-preserving buckets (bucket of column c: floor(c T / span), two
// 16-bit counters per word), buckets sorted (or the whole segment when a
// bucket is large), runs of equal columns summed.  Returns the distinct
// columns written.
template <typename VT>
__device__ int merge_buckets(const Staging<VT> &stg, int P,
                             int c0, int span, int D, uint32_t *cnt, uint32_t *ikey, VT *ival,
                             int *wtot, int *bigmax, SPG_GLOBAL int32_t *cb, SPG_GLOBAL VT *vb,
                             WsHeader *hdr) {
  constexpr int J = kSplitSeg / kAccumNT;
  const int tid = threadIdx.x;
  int T = 64;
  while (T < P) T <<= 1;
  const int TW = T >> 1;
  const uint32_t mul = T >= span ? 0xffffffffu : (uint32_t)(((uint64_t)T << 32) / (uint64_t)span);
  for (int w = tid; w < TW; w += kAccumNT) cnt[w] = 0u;
  if (tid == 0) *bigmax = 0;
  __syncthreads();
  uint32_t kc[J], kbt[J];  // column; bucket | ticket << 16 (both below 2^16)
  VT kv[J];
  bool bad = false;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int p = tid + j * kAccumNT;
    kc[j] = 0u;
    kv[j] = VT(0);
    if (p < P) {
      int c;
      stg.get(p, c, kv[j]);
      kc[j] = (uint32_t)(c - c0);
    }
  }
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (tid + j * kAccumNT < P) {
      if (kc[j] >= (uint32_t)span) {  // outside the segment: a changed pattern
        bad = true;
        kc[j] = (uint32_t)span - 1;
      }
      const uint32_t b = mono_slot(kc[j], mul);
      const uint32_t sh = (b & 1u) << 4;
      kbt[j] = b | (atomicAdd(&cnt[b >> 1], 1u << sh) >> sh) << 16;
    }
  }
  if (bad) atomicOr(&hdr->status, kStatInvalid);
  __syncthreads();
  // bucket starts: exclusive scan, each thread a contiguous chunk of words
  {
    const int per = (TW + kAccumNT - 1) / kAccumNT;
    const int w0 = tid * per;
    int loc = 0, mx = 0;
    for (int q = 0; q < per; ++q)
      if (w0 + q < TW) {
        const uint32_t v = cnt[w0 + q];
        loc += (int)(v & 0xffffu) + (int)(v >> 16);
        mx = max(mx, (int)max(v & 0xffffu, v >> 16));
      }
    if (mx > kBigBucket) atomicMax(bigmax, mx);
    int tot;
    int run = group_excl_scan<true, kAccumNT>(loc, tid, wtot, tot);
    for (int q = 0; q < per; ++q)
      if (w0 + q < TW) {
        const uint32_t v = cnt[w0 + q];
        const uint32_t lo = (uint32_t)run;
        run += (int)(v & 0xffffu);
        cnt[w0 + q] = lo | ((uint32_t)run << 16);
        run += (int)(v >> 16);
      }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (tid + j * kAccumNT < P) {
      const int pos = seg_bucket(cnt, kbt[j] & 0xffffu) + (int)(kbt[j] >> 16);
      ikey[pos] = kc[j];
      ival[pos] = kv[j];
    }
  }
  __syncthreads();
  const bool big = *bigmax > kBigBucket;
  if (P == D && !big) {
    // no repeated column: bucket start + smaller columns in the bucket
    for (int p = tid; p < P; p += kAccumNT) {
      const uint32_t c = ikey[p];
      const uint32_t b = mono_slot(c, mul);
      const int s0 = seg_bucket(cnt, b);
      const int s1 = (int)b + 1 < T ? seg_bucket(cnt, b + 1) : P;
      int r = s0;
      for (int q = s0; q < s1; ++q) r += ikey[q] < c ? 1 : 0;
      cb[r] = c0 + (int)c;
      vb[r] = ival[p];
    }
    return P;
  }
  if (big) {
    lds_sort_pairs<true, kAccumNT, VT>(ikey, ival, P, tid);
  } else {
    for (int b = tid; b < T; b += kAccumNT) {
      const int s0 = seg_bucket(cnt, (uint32_t)b);
      const int s1 = b + 1 < T ? seg_bucket(cnt, (uint32_t)b + 1) : P;
      for (int q = s0 + 1; q < s1; ++q) {
        const uint32_t kq = ikey[q];
        const VT vq = ival[q];
        int r = q - 1;
        while (r >= s0 && ikey[r] > kq) {
          ikey[r + 1] = ikey[r];
          ival[r + 1] = ival[r];
          --r;
        }
        ikey[r + 1] = kq;
        ival[r + 1] = vq;
      }
    }
    __syncthreads();
  }
  // runs of equal columns: each thread a contiguous range of positions
  const int per = (P + kAccumNT - 1) / kAccumNT;
  const int p0 = tid * per, p1 = min(P, p0 + per);
  int firsts = 0;
  for (int p = p0; p < p1; ++p) firsts += (p == 0 || ikey[p] != ikey[p - 1]) ? 1 : 0;
  int tot;
  int d = group_excl_scan<true, kAccumNT>(firsts, tid, wtot, tot);
  for (int p = p0; p < p1; ++p) {
    const uint32_t c = ikey[p];
    if (p == 0 || c != ikey[p - 1]) {
      VT sum = ival[p];
      for (int q = p + 1; q < P && ikey[q] == c; ++q) sum += ival[q];
      if (d < D) {
        cb[d] = c0 + (int)c;
        vb[d] = sum;
      }
      ++d;
    }
  }
  return tot;
}

template <typename VT>
__global__ __launch_bounds__(kAccumNT, sizeof(VT) == 4 ? 8 : 4) void k_split_merge(WsHeader *__restrict__ hdr, int blo,
                                                          SplitArgs sa,
                                                          int32_t *__restrict__ ccol,
                                                          VT *__restrict__ cval) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // bucket merge: counters (two per word) | keys | values; dense merge:
  // panel | bitmap
  uint32_t *cnt = reinterpret_cast<uint32_t *>(smem_raw);
  uint32_t *ikey = cnt + kSplitSeg / 2;
  VT *ival = reinterpret_cast<VT *>(ikey + kSplitSeg);
  VT *panel = reinterpret_cast<VT *>(smem_raw);
  uint32_t *bm = reinterpret_cast<uint32_t *>(panel + (1 << kSplitLog2W));
  __shared__ int wtot[kAccumNT / kWave];
  __shared__ int item, bigmax;
  if (hdr->status) return;
  const int sbin = hdr->bin_start[sa.bin];
  const int hlo = hdr->bin_start[blo] - sbin;
  const int nseg = min(sa.ctl->segs, sa.segcap);
  const int tid = threadIdx.x;
  for (int t = block_next(&sa.ctl->q_accum, &item); t < nseg;
       t = block_next(&sa.ctl->q_accum, &item)) {
    const SplitSeg sg = sa.segs[t];
    // unused, a row of an LDS bin of this pass, or a row_ptr mismatch
    if (sg.h < hlo || sg.out < 0) continue;
    if (sg.pcount == 0) {
      if (tid == 0 && sg.dcount != 0) atomicOr(&hdr->status, kStatInvalid);
      continue;
    }
    // the segment's part of the staging area (FP32: 8-byte words)
    const Staging<VT> stg{gpw(sa.scol + (sizeof(VT) == 4 ? 2 : 1) * (size_t)sg.stage),
                          gpw(static_cast<VT *>(sa.sval) + sg.stage)};
    SPG_GLOBAL int32_t *cb = gpw(ccol) + sg.out;
    SPG_GLOBAL VT *vb = gpw(cval) + sg.out;
    const int got = sg.pcount > kSplitSeg
                        ? merge_dense<VT>(stg, sg.pcount, sg.c0, sg.dcount, panel, bm,
                                          wtot, cb, vb, hdr)
                        : merge_buckets<VT>(stg, sg.pcount, sg.c0, sg.c1 - sg.c0,
                                            sg.dcount, cnt, ikey, ival, wtot, &bigmax, cb, vb,
                                            hdr);
    if (tid == 0 && got != sg.dcount) atomicOr(&hdr->status, kStatInvalid);
  }
}

// ---------------------------------------------------------------------------
// Launchers.

size_t split_sym_static_lds() {
  return (size_t)2 * 1024 * 4 + (size_t)2 * (kSplitMaxRanges + 1) * 4 +
         (size_t)kSplitMaxRanges * 4 + 16 * 4 + 64;
}

template <typename VT>
static size_t scatter_lds() {
  return (size_t)kSplitBuf * (4 + sizeof(VT));
}

template <typename VT>
static size_t merge_lds() {
  const size_t buckets = (size_t)kSplitSeg * (6 + sizeof(VT));
  const size_t dense = ((size_t)sizeof(VT) << kSplitLog2W) + (size_t)kRangeWords * 4;
  return buckets > dense ? buckets : dense;
}

static int per_cu(size_t lds, size_t stat, int threads) {
  const DevInfo &D = dev_info();
  int b = (int)(D.lds_per_cu / (lds + stat));
  const int bt = 2048 / threads;
  b = b < bt ? b : bt;
  return b < 1 ? 1 : b;
}

hipError_t launch_sym_split(const Problem *dpr, const int32_t *rows, WsHeader *hdr, int blo,
                            int lS, bool lds_map, uint32_t *gbitmap, int grid, size_t lds,
                            int32_t *cnt, const SplitArgs &sa, hipStream_t st) {
  if (lds_map)
    hipLaunchKernelGGL(k_sym_split<true>, dim3(grid), dim3(1024), lds, st, dpr, rows, hdr, blo,
                       lS, (uint32_t *)nullptr, cnt, sa);
  else
    hipLaunchKernelGGL(k_sym_split<false>, dim3(grid), dim3(1024), 0, st, dpr, rows, hdr, blo,
                       lS, gbitmap, cnt, sa);
  return hipGetLastError();
}

template <typename VT>
static void num_split(const Problem *dpr, const int32_t *rows, WsHeader *hdr, int blo, int lS,
                      const SplitArgs &sa, int32_t *ulist, const int32_t *crp, int32_t *ccol,
                      VT *cval, hipStream_t st) {
  const DevInfo &D = dev_info();
  hipLaunchKernelGGL(k_split_prepare, dim3(D.cus * 4), dim3(256), 0, st, rows, hdr, blo, sa,
                     crp, ulist);
  const size_t sl = scatter_lds<VT>();
  const int sg = D.cus * per_cu(sl, (size_t)kSplitMaxRanges * 4 + (size_t)kScatterNT * (8 + sizeof(VT)),
                                kScatterNT);
  hipLaunchKernelGGL(k_split_scatter<VT>, dim3(sg), dim3(kScatterNT), sl, st, dpr, hdr, blo, lS,
                     sa);
  const size_t ml = merge_lds<VT>();
  const int mg = D.cus * per_cu(ml, 256, kAccumNT);
  hipLaunchKernelGGL(k_split_merge<VT>, dim3(mg), dim3(kAccumNT), ml, st, hdr, blo, sa, ccol,
                     cval);
}

hipError_t launch_num_split(const Problem *dpr, const int32_t *rows, WsHeader *hdr, int blo,
                            int lS, const SplitArgs &sa, int32_t *ulist, const int32_t *crp,
                            int32_t *ccol, void *cval, bool f64, hipStream_t st) {
  if (sa.F <= 0) return hipSuccess;
  if (f64)
    num_split<double>(dpr, rows, hdr, blo, lS, sa, ulist, crp, ccol, static_cast<double *>(cval), st);
  else
    num_split<float>(dpr, rows, hdr, blo, lS, sa, ulist, crp, ccol, static_cast<float *>(cval), st);
  return hipGetLastError();
}

hipError_t configure_split_lds(size_t lds_max) {
  const void *ks[] = {
      reinterpret_cast<const void *>(&k_sym_split<true>),
      reinterpret_cast<const void *>(&k_split_scatter<float>),
      reinterpret_cast<const void *>(&k_split_scatter<double>),
      reinterpret_cast<const void *>(&k_split_merge<float>),
      reinterpret_cast<const void *>(&k_split_merge<double>),
  };
  for (const void *k : ks) {
    hipError_t e =
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace spg

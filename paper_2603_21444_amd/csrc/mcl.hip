// One Markov-clustering iteration (a8; paper §5.7) on X = M^T in CSR, FP32,
// in one of two step orders:
//   rpost == 0 (the synthetic workload's order):
//     E = X X;  e <- e^r;  row /= row sum;  drop e < prune;  keep the topk
//     largest (ties to the smaller column);  an emptied row keeps its
//     largest entry;  row /= new row sum.
//   rpost >= 1 (the order the paper describes for its runs):
//     E = X X;  row /= row sum;  drop e < prune;  top-k and emptied rows as
//     above;  e <- e^rpost;  no second normalisation.
// Both are the same kernels with the exponent before the normalisation
// (rpre = r, or 1) and the final step (renormalise, or the power) as
// parameters.
// The unpruned product is never stored.  Row c of Y is written at its final
// column rank into a padded buffer (cap = min(topk, n) slots per row) with
// its length in cnt[c]; a scan of cnt and a compaction copy produce CSR.
//
// Rows whose products fit an LDS table use the numeric kernel's
// order-preserving hash (rank = occupied slots before + inversion counter)
// and run the whole epilogue in LDS; kept entries are flagged by clearing
// the sign of their value slot.  Rows beyond the tables are swept in column
// panels (k_mcl_panel below).
#include <vector>

#include "internal.hpp"
#include "rowops.hpp"

namespace spg {

constexpr int kMclUnroll = 4;

__device__ __forceinline__ float ipow(float e, int r) {
  float p = e;
  for (int q = 1; q < r; ++q) p *= e;
  return p;
}

// (value, column) -> orderable key: larger value first, then smaller column
// (values are >= 0, so their bit patterns order like the values).
__device__ __forceinline__ unsigned long long vc_key(float v, int col) {
  return ((unsigned long long)__float_as_uint(v) << 32) | (uint32_t)(~(uint32_t)col);
}

template <int G>
struct MGeom {
  static constexpr bool BLOCK = G > kWave;
  static constexpr int WG = BLOCK ? G : 256;
  static constexpr int R = WG / G;
};

// Batched insert of the expansion products (first probes of all N issued
// together).  Wave groups store the value of a column's first insert and add
// repeats after a wave fence (LDS float atomics are slow), so their value
// table needs no clearing; block groups add atomically into a cleared table.
template <bool PLAIN>
struct MclInsert {
  int *key;
  float *val;
  int *flag;
  uint32_t mul;
  int maxwin;
  template <int N>
  __device__ __forceinline__ void batch(const int (&col)[N], const float (&v)[N]) {
    int h[N], old[N];
    bool ok[N];
#pragma unroll
    for (int u = 0; u < N; ++u) {
      h[u] = (int)mono_slot((uint32_t)col[u], mul);
      old[u] = col[u] >= 0 ? atomicCAS(&key[h[u]], kEmpty, (int)((uint32_t)col[u] | 0x80000000u))
                           : kEmpty;
    }
#pragma unroll
    for (int u = 0; u < N; ++u) {
      ok[u] = col[u] >= 0;
      int d = 0;
      while (ok[u] && old[u] != kEmpty && (int)((uint32_t)old[u] & 0xffffffu) != col[u]) {
        if (d == maxwin) {  // the heavy kernel redoes this row
          *flag = 1;
          ok[u] = false;
          break;
        }
        ++d;
        ++h[u];
        old[u] = atomicCAS(&key[h[u]], kEmpty, (int)((uint32_t)col[u] | 0x80000000u));
      }
    }
    if (PLAIN) {
#pragma unroll
      for (int u = 0; u < N; ++u)
        if (ok[u] && old[u] == kEmpty) val[h[u]] = v[u];
      group_sync<false>();
#pragma unroll
      for (int u = 0; u < N; ++u)
        if (ok[u] && old[u] != kEmpty) lds_add_cas(&val[h[u]], v[u]);
    } else {
#pragma unroll
      for (int u = 0; u < N; ++u)
        if (ok[u]) lds_add_cas(&val[h[u]], v[u]);
    }
  }
};

// LDS rows.  Key words pack (col | (128 + counter) << 24), n <= 2^24.
template <int G>
__global__ __launch_bounds__(MGeom<G>::WG) void k_mcl_rows(
    const Problem *__restrict__ pr, const int32_t *__restrict__ rows, WsHeader *__restrict__ hdr,
    int bin, int lS, int TT, uint32_t mul, int maxwin, int r, int rpost, float prune, int topk,
    int cap,
    int32_t *__restrict__ ycol, float *__restrict__ yval, int32_t *__restrict__ ycnt,
    int32_t *__restrict__ fb_rows) {
  using GM = MGeom<G>;
  constexpr bool BLOCK = GM::BLOCK;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ float redf[16];
  __shared__ int redi[16];
  __shared__ unsigned long long redu[16];
  const int rslot = threadIdx.x / G, l = threadIdx.x % G;
  float *vals_all = reinterpret_cast<float *>(smem_raw);
  float *sa_all = vals_all + (size_t)GM::R * TT;
  int *keys_all = reinterpret_cast<int *>(sa_all + (size_t)GM::R * G);
  int *sb_all = keys_all + (size_t)GM::R * TT;
  int *sl_all = sb_all + (size_t)GM::R * G;
  int *rowflag = sl_all + (size_t)GM::R * G;
  float *val = vals_all + (size_t)rslot * TT;
  int *key = keys_all + (size_t)rslot * TT;
  Stage<float> st{sb_all + rslot * G, sl_all + rslot * G, sa_all + rslot * G};
  if (hdr->status) return;
  const int count = hdr->bin_count[bin];
  const int start = hdr->bin_start[bin];
  const int c = TT / G;
  const int s0 = l * c;
  for (int ri = blockIdx.x * GM::R + rslot; ri < count; ri += gridDim.x * GM::R) {
    int i = rows[start + ri];
    if (G >= kWave) i = __builtin_amdgcn_readfirstlane(i);
    int4 *k4 = reinterpret_cast<int4 *>(key);
    for (int s = l; s < TT / 4; s += G) k4[s] = make_int4(kEmpty, kEmpty, kEmpty, kEmpty);
    if (BLOCK)
      for (int s = l; s < TT; s += G) val[s] = 0.f;
    if (l == 0) rowflag[rslot] = 0;
    group_sync<BLOCK>();
    // 1. expansion E = X X (accumulate row i)
    MclInsert<!BLOCK> fins{key, val, rowflag + rslot, mul, maxwin};
    for_each_product<BLOCK, true, G, kMclUnroll, float>(pr, i, true, l, lS, st, fins);
    group_sync<BLOCK>();
    if (rowflag[rslot]) {  // redone by the heavy kernel
      if (l == 0) fb_rows[atomicAdd(&hdr->fallback_count, 1)] = i;
      group_sync<BLOCK>();
      continue;
    }
    // 2. inflation and row sum
    float part = 0.f;
    for (int j = 0; j < c; ++j) {
      if (key[s0 + j] != kEmpty) {
        const float p = ipow(val[s0 + j], r);
        val[s0 + j] = p;
        part += p;
      }
    }
    const float S = group_sum<BLOCK, G>(part, redf);
    // 3./4. normalise and prune; kept entries have a clear sign bit
    int kept = 0;
    unsigned long long best = 0;
    for (int j = 0; j < c; ++j) {
      const int w = key[s0 + j];
      if (w != kEmpty) {
        const float v = val[s0 + j] / S;
        const unsigned long long kk = vc_key(v, (int)((uint32_t)w & 0xffffffu));
        best = kk > best ? kk : best;
        if (v < prune) {
          val[s0 + j] = -v - 1.f;  // dropped (keeps v recoverable)
        } else {
          val[s0 + j] = v;
          ++kept;
        }
      }
    }
    const int nkept = group_sum<BLOCK, G>(kept, redi);
    if (nkept > topk) {
      // 5. threshold: the largest bit pattern tau with #{kept v >= tau} >= topk
      uint32_t lo = 0, hi = 0x7f800000u;
      while (lo < hi) {
        const uint32_t mid = lo + (hi - lo + 1) / 2;
        int cc = 0;
        for (int j = 0; j < c; ++j) {
          const float v = val[s0 + j];
          cc += (key[s0 + j] != kEmpty && v >= 0.f && __float_as_uint(v) >= mid) ? 1 : 0;
        }
        if (group_sum<BLOCK, G>(cc, redi) >= topk) lo = mid;
        else hi = mid - 1;
      }
      int gt = 0;
      for (int j = 0; j < c; ++j) {
        const float v = val[s0 + j];
        gt += (key[s0 + j] != kEmpty && v >= 0.f && __float_as_uint(v) > lo) ? 1 : 0;
      }
      const int need = topk - group_sum<BLOCK, G>(gt, redi);
      // ties at tau: keep the `need` smallest columns
      for (int j = 0; j < c; ++j) {
        const int w = key[s0 + j];
        const float v = val[s0 + j];
        if (w == kEmpty || v < 0.f) continue;
        const uint32_t b = __float_as_uint(v);
        bool keep = b > lo;
        if (b == lo) {
          const int col = (int)((uint32_t)w & 0xffffffu);
          int before = 0;
          for (int t = 0; t < TT; ++t) {
            const int w2 = key[t];
            const float v2 = val[t];
            if (w2 != kEmpty && v2 >= 0.f && __float_as_uint(v2) == lo &&
                (int)((uint32_t)w2 & 0xffffffu) < col)
              ++before;
          }
          keep = before < need;
        }
        if (!keep) val[s0 + j] = -v - 1.f;
      }
    }
    group_sync<BLOCK>();
    // 6. never empty: keep the largest entry of step 3
    if (nkept == 0) {
      const unsigned long long bb = group_max_u64<BLOCK, G>(best, redu);
      const int bcol = (int)~(uint32_t)(bb & 0xffffffffu);
      for (int j = 0; j < c; ++j) {
        const int w = key[s0 + j];
        if (w != kEmpty && (int)((uint32_t)w & 0xffffffu) == bcol) val[s0 + j] = -val[s0 + j] - 1.f;
      }
    }
    group_sync<BLOCK>();
    // 7. new row sum; counters of the kept entries' order
    float part2 = 0.f;
    for (int j = 0; j < c; ++j) {
      const int w = key[s0 + j];
      if (w != kEmpty) {
        key[s0 + j] = (int)(((uint32_t)w & 0xffffffu) | 0x80000000u);  // counter := 0
        if (val[s0 + j] >= 0.f) part2 += val[s0 + j];
      }
    }
    const float S2 = group_sum<BLOCK, G>(part2, redf);
    group_sync<BLOCK>();
    for (int j = 0; j < c; ++j) {
      const int s = s0 + j;
      const int w = key[s];
      if (w == kEmpty || val[s] < 0.f) continue;
      const int col = (int)((uint32_t)w & 0xffffffu);
      const int home = (int)mono_slot((uint32_t)col, mul);
      int larger = 0;
      for (int t = home; t < s; ++t) {
        const int w2 = key[t];
        if (val[t] >= 0.f && (int)((uint32_t)w2 & 0xffffffu) > col) {
          atomicAdd(&key[t], 1 << 24);
          ++larger;
        }
      }
      if (larger) atomicSub(&key[s], larger << 24);
    }
    group_sync<BLOCK>();
    int mine = 0;
    for (int j = 0; j < c; ++j) mine += (key[s0 + j] != kEmpty && val[s0 + j] >= 0.f) ? 1 : 0;
    int total;
    int rk = group_excl_scan<BLOCK, G>(mine, l, redi, total);
    SPG_GLOBAL int32_t *cb = gpw(ycol) + (size_t)i * cap;
    SPG_GLOBAL float *vb = gpw(yval) + (size_t)i * cap;
    for (int j = 0; j < c; ++j) {
      const int w = key[s0 + j];
      const float v = val[s0 + j];
      if (w != kEmpty && v >= 0.f) {
        int rr = rk + (int)((uint32_t)w >> 24) - 128;
        rr = rr < 0 ? 0 : (rr >= cap ? cap - 1 : rr);
        cb[rr] = (int)((uint32_t)w & 0xffffffu);
        vb[rr] = rpost == 0 ? v / S2 : ipow(v, rpost);
        ++rk;
      }
    }
    if (l == 0) ycnt[i] = total < cap ? total : cap;
    group_sync<BLOCK>();
  }
}

// ---------------------------------------------------------------------------
// Heavy rows: column panels with fixed-point accumulators in LDS.
//
// A heavy row (more products than an LDS table holds, or handed over by the
// LDS kernel) is swept in panels of kPanel consecutive columns.  Every entry
// a_ik of X row i keeps a cursor into B row k (sorted, as X is canonical).
// In a panel, S lanes of a wave read S consecutive elements of one entry's B
// row (coalesced), a wave serves several entries at once so that several loads
// are in flight, and a ballot over the S lanes tells how far the entry got
// (elements are ascending, so those inside the panel are a prefix).  S is
// chosen per row from the mean number of elements an entry has per panel.
// A product a_ik * b_kj (exact in FP64) is scaled
// by 2^s and rounded to an int64 that is added into the panel's LDS slot with
// an integer atomic: integer LDS atomics are far cheaper than float ones on
// this chip, and the sum no longer depends on the order of the adds.  The
// scale is chosen per row from sum_k |a_ik| * sum_j |b_kj| (row_abs below) so
// that no partial sum can overflow; the rounding error of an entry is at most
// (terms) * 2^-62 of that bound, far below the FP32 rounding of the result.
//
// After a panel, its present columns are inflated (p = v^r) and p is summed
// into the row's running sum.  A column can only survive the prune if
// p >= prune * (final sum) >= prune * (sum of the panels before), so only
// such candidates are appended, in column order, to the row's list in the
// slot scratch (capacity n).  At the end the list is filtered with the exact
// test on p / sum, the top-k threshold is found by bisection on the float
// bit patterns, ties go to the smaller columns (list order), and the result is
// renormalised and written in column order.
constexpr int kPanel = 16384;  // columns per panel: 128 KiB of int64 in LDS
constexpr int kPT = 1024;      // threads of a heavy block
constexpr int kCPT = kPanel / kPT;  // panel columns per thread in the epilogue
// Entry groups a wave serves at once: six for rows whose entries have 32 or
// more elements per panel (32 or 64 lanes per entry), four otherwise; more
// groups spill past the 128 registers a 1024-thread block allows.
constexpr int kPUDense = 6, kPUSparse = 4;
constexpr int kPE = 1024;     // entries whose cursors stay in LDS
static_assert(kCPT == 16, "the epilogue reads one 16-bit half of a bitmap word per thread");

struct PanelRed {
  double s;
  int total, excl, mn;
  unsigned long long best;
};

// Block-wide sum (double), inclusive/exclusive count scan, min and max in one
// barrier.  The caller synchronises before the shared arrays are reused.
__device__ __forceinline__ PanelRed panel_reduce(double s, int c, int mn, unsigned long long best,
                                                 double *rs, int *rc, int *rm,
                                                 unsigned long long *rb) {
  const int lane = lane_id(), w = threadIdx.x / kWave;
  int x = c;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    s += __shfl_xor(s, off);
    const int m2 = __shfl_xor(mn, off);
    mn = m2 < mn ? m2 : mn;
    const unsigned long long b2 = __shfl_xor(best, off);
    best = b2 > best ? b2 : best;
  }
  if (lane == kWave - 1) rc[w] = x;
  if (lane == 0) {
    rs[w] = s;
    rm[w] = mn;
    rb[w] = best;
  }
  __syncthreads();
  // lane l (mod 16) picks up wave l's partials; a butterfly over 16 lanes
  // gives every lane the same totals (IEEE addition is commutative).
  constexpr int NW = kPT / kWave;
  static_assert(NW == 16, "one partial per lane of a 16-lane segment");
  const int l16 = lane & (NW - 1);
  double ts = rs[l16];
  int tt = rc[l16];
  int tp = l16 < w ? tt : 0;
  int tm = rm[l16];
  unsigned long long tb = rb[l16];
#pragma unroll
  for (int off = NW / 2; off > 0; off >>= 1) {
    ts += __shfl_xor(ts, off, NW);
    tt += __shfl_xor(tt, off, NW);
    tp += __shfl_xor(tp, off, NW);
    const int m2 = __shfl_xor(tm, off, NW);
    tm = m2 < tm ? m2 : tm;
    const unsigned long long b2 = __shfl_xor(tb, off, NW);
    tb = b2 > tb ? b2 : tb;
  }
  return PanelRed{ts, tt, tp + x - c, tm, tb};
}

// Adds the products of entries [0, nA) that fall in [plo, plo + width) and
// advances their cursors; returns this lane's smallest next column.
template <int kPU, typename CurT>
__device__ __forceinline__ int panel_accumulate(const SPG_GLOBAL int32_t *bcol,
                                                const SPG_GLOBAL float *bval, CurT *ecur,
                                                const CurT *eend, const float *eval, int nA,
                                                int lS, double sigma, int plo, uint32_t width,
                                                unsigned long long *pacc, uint32_t *pbm) {
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const int S = 1 << lS, EPW = kWave >> lS;
  const int sub = lane >> lS, q = lane & (S - 1), base = sub << lS;
  const int phi = plo + kPanel;
  int tmn = INT32_MAX;
  for (int e0 = w * EPW * kPU; e0 < nA; e0 += (kPT / kWave) * EPW * kPU) {
    int c[kPU], en[kPU];
    float a[kPU];
    bool act[kPU];
    // Every read below uses an in-range index for every lane (entry 0; B
    // element 0, which exists since a heavy row has products), so the reads
    // of all kPU groups are issued before the first wait.
#pragma unroll
    for (int u = 0; u < kPU; ++u) {
      const int e = e0 + u * EPW + sub;
      act[u] = e < nA;
      const int es = act[u] ? e : 0;
      c[u] = (int)ecur[es];
      en[u] = (int)eend[es];
      a[u] = eval[es];
    }
    bool more = true;
    while (more) {
      int col[kPU];
      float v[kPU];
#pragma unroll
      for (int u = 0; u < kPU; ++u) {
        const int idx = c[u] + q;
        const bool ld = act[u] && idx < en[u];
        const int li = ld ? idx : 0;
        col[u] = bcol[li];
        v[u] = bval[li];
        col[u] = ld ? col[u] : INT32_MAX;
      }
      more = false;
#pragma unroll
      for (int u = 0; u < kPU; ++u) {
        const bool in = col[u] < phi;
        const uint32_t cl = (uint32_t)(col[u] - plo);
        if (in && cl < width) {  // columns outside [0, n) are skipped
          const long long qv = __double2ll_rn((double)a[u] * (double)v[u] * sigma);
          atomicAdd(&pacc[cl], (unsigned long long)qv);
          atomicOr(&pbm[cl >> 5], 1u << (cl & 31));
        }
        const uint64_t m = __ballot(in);
        const int k = __popcll((m >> base) & (S == kWave ? ~0ull : ((1ull << S) - 1)));
        // the group's lane k holds the entry's first column past the panel
        // (INT32_MAX once its row ended, or for an inactive group); the
        // block-wide minimum comes later, so that lane keeps it
        if (q == k) tmn = min(tmn, col[u]);
        if (act[u]) {
          c[u] += k;
          if (k < S) act[u] = false;  // the entry left the panel (or its row ended)
        }
        more = more || act[u];
      }
      more = __any(more);
    }
#pragma unroll
    for (int u = 0; u < kPU; ++u) {
      const int e = e0 + u * EPW + sub;
      if (e < nA && q == 0) ecur[e] = (CurT)c[u];
    }
  }
  return tmn;
}

__global__ __launch_bounds__(kPT) void k_mcl_panel(
    const Problem *__restrict__ pr, const int32_t *__restrict__ rows, WsHeader *__restrict__ hdr,
    int blo, int r, int rpost, float prune, int topk, int cap, const double *__restrict__ rabs,
    char *__restrict__ scratch, size_t slot_bytes, const int32_t *__restrict__ fb_rows,
    int32_t *__restrict__ ycol, float *__restrict__ yval, int32_t *__restrict__ ycnt) {
  extern __shared__ __align__(16) unsigned long long pacc[];
  uint32_t *pbm = reinterpret_cast<uint32_t *>(pacc + kPanel);
  __shared__ double rs[kPT / kWave];
  __shared__ int rc[kPT / kWave], rm[kPT / kWave];
  __shared__ unsigned long long rb[kPT / kWave];
  __shared__ int s_cur[kPE], s_end[kPE];
  __shared__ float s_val[kPE];
  const int n = pr->n;
  const int tid = threadIdx.x;
  char *sp = scratch + (size_t)blockIdx.x * slot_bytes;
  int32_t *lcol = reinterpret_cast<int32_t *>(sp);
  float *lval = reinterpret_cast<float *>(sp + (size_t)4 * n);
  int32_t *ecur = reinterpret_cast<int32_t *>(sp + (size_t)8 * n);
  int32_t *eend = reinterpret_cast<int32_t *>(sp + (size_t)12 * n);
  float *evalg = reinterpret_cast<float *>(sp + (size_t)16 * n);
  __shared__ int stat0;
  if (tid == 0) stat0 = hdr->status;
  __syncthreads();
  if (stat0) return;
  const Part &P = pr->part[0];
  const SPG_GLOBAL int32_t *bcol = gp(P.bcol);
  const SPG_GLOBAL float *bval = gp(static_cast<const float *>(P.bval));
  const int start = hdr->bin_start[blo];
  const int nheavy = hdr->bin_start[kHeavyBin + 1] - start;
  const int count = nheavy + hdr->fallback_count;
  for (int s = tid; s < kPanel; s += kPT) pacc[s] = 0ull;
  for (int s = tid; s < kPanel / 32; s += kPT) pbm[s] = 0u;
  __syncthreads();
  const bool even = (r & 1) == 0;
  __shared__ int item;
  for (int ri = block_next(&hdr->queue[kQueueHeavy], &item); ri < count;
       ri = block_next(&hdr->queue[kQueueHeavy], &item)) {
    const int i = ri < nheavy ? rows[start + ri] : fb_rows[ri - nheavy];
    int as, ae;
    a_row(P, i, as, ae);
    const int nA = ae - as;
    if (nA > n) {  // more entries than columns: a repeated column index
      if (tid == 0) atomicOr(&hdr->status, kStatInvalid);
      break;
    }
    // entries: cursor, end and value, in LDS for rows of at most kPE
    // entries, else in the slot scratch
    const bool lds_state = nA <= kPE;
    int *ccur = lds_state ? s_cur : ecur;
    int *cend = lds_state ? s_end : eend;
    float *cval = lds_state ? s_val : evalg;
    double sb = 0.0;
    int mn = INT32_MAX, plen = 0;
    for (int e = tid; e < nA; e += kPT) {
      const int k = gp(P.acol)[as + e];
      const float av = gp(static_cast<const float *>(P.aval))[as + e];
      const int b0 = gp(P.brp)[k], b1 = gp(P.brp)[k + 1];
      sb += fabs((double)av) * rabs[k];
      ccur[e] = b0;
      cend[e] = b1;
      cval[e] = av;
      plen += b1 - b0;
      if (b0 < b1) mn = min(mn, bcol[b0]);
    }
    PanelRed R = panel_reduce(sb, plen, mn, 0ull, rs, rc, rm, rb);
    __syncthreads();
    // scale 2^s with 2^(62-s) > the row's bound on sum |a b|
    double sigma = 1.0;
    {
      const double bound = R.s * (1.0 + 1.0 / 1048576.0);
      if (bound > 0.0 && bound < 1e300) {
        int ex = 0;
        (void)frexp(bound, &ex);  // bound < 2^ex
        ex = ex < -960 ? -960 : ex;
        sigma = ldexp(1.0, 62 - ex);
      }
    }
    const double inv_sigma = 1.0 / sigma;  // exact: sigma is a power of two
    // lanes per entry: about the mean number of an entry's elements per panel
    int lS = 2;
    {
      const double per = (double)R.total / (double)(nA > 0 ? nA : 1) /
                         (double)((n + kPanel - 1) / kPanel);
      while (lS < 6 && (double)(1 << lS) < per) ++lS;
    }
    int mnext = R.mn;
    double scum = 0.0;
    int nc = 0;
    unsigned long long best = 0ull;
    while (mnext < n) {
      const int plo = mnext & ~(kPanel - 1);
      const uint32_t width = plo < 0 ? 0u : (uint32_t)min(kPanel, n - plo);
      const int tmn =
          lS >= 5 ? panel_accumulate<kPUDense>(bcol, bval, ccur, cend, cval, nA, lS, sigma, plo,
                                               width, pacc, pbm)
                  : panel_accumulate<kPUSparse>(bcol, bval, ccur, cend, cval, nA, lS, sigma, plo,
                                                width, pacc, pbm);
      __syncthreads();
      // epilogue of the panel: thread tid owns columns plo + 16 tid .. + 15
      const double thr = even ? (double)prune * scum * (1.0 - 1.0 / 1024.0) : -HUGE_VAL;
      const uint32_t bits = (pbm[tid >> 1] >> ((tid & 1) * 16)) & 0xffffu;
      double ps = 0.0;
      int cnt = 0;
      for (uint32_t b = bits; b; b &= b - 1) {
        const int cl = tid * kCPT + __ffs(b) - 1;
        const float pw = ipow((float)((double)(long long)pacc[cl] * inv_sigma), r);
        ps += (double)pw;
        const unsigned long long key = vc_key(pw, plo + cl);
        best = key > best ? key : best;
        cnt += (double)pw >= thr ? 1 : 0;
      }
      R = panel_reduce(ps, cnt, tmn, 0ull, rs, rc, rm, rb);
      int o = nc + R.excl;
      for (uint32_t b = bits; b; b &= b - 1) {
        const int cl = tid * kCPT + __ffs(b) - 1;
        const float pw = ipow((float)((double)(long long)pacc[cl] * inv_sigma), r);
        pacc[cl] = 0ull;
        if ((double)pw >= thr) {
          lcol[o] = plo + cl;
          lval[o] = pw;
          ++o;
        }
      }
      if ((tid & 1) == 0) pbm[tid >> 1] = 0u;
      scum += R.s;
      nc += R.total;
      mnext = R.mn;
      __syncthreads();
    }
    // exact prune test on p / sum, compacting the list in place
    const float S = (float)scum;
    int nk = 0;
    for (int c0 = 0; c0 < nc; c0 += kPT) {
      const int idx = c0 + tid;
      int col = 0;
      float q = 0.f;
      bool keep = false;
      if (idx < nc) {
        col = lcol[idx];
        q = lval[idx] / S;
        keep = !(q < prune);
      }
      R = panel_reduce(0.0, keep ? 1 : 0, INT32_MAX, best, rs, rc, rm, rb);
      if (keep) {
        lcol[nk + R.excl] = col;
        lval[nk + R.excl] = q + 0.f;
      }
      nk += R.total;
      __syncthreads();
    }
    R = panel_reduce(0.0, 0, INT32_MAX, best, rs, rc, rm, rb);
    const unsigned long long rowbest = R.best;
    __syncthreads();
    // top-k: largest threshold tau with at least topk kept values >= tau
    uint32_t tau = 0u;
    int need = nk;
    if (nk > topk) {
      uint32_t lo = 0u, hi = 0x7f800000u;
      while (lo < hi) {
        const uint32_t mid = lo + (hi - lo + 1) / 2;
        int cc = 0;
        for (int idx = tid; idx < nk; idx += kPT) cc += __float_as_uint(lval[idx]) >= mid ? 1 : 0;
        R = panel_reduce(0.0, cc, INT32_MAX, 0ull, rs, rc, rm, rb);
        __syncthreads();
        if (R.total >= topk) lo = mid;
        else hi = mid - 1;
      }
      tau = lo;
      int gt = 0;
      for (int idx = tid; idx < nk; idx += kPT) gt += __float_as_uint(lval[idx]) > tau ? 1 : 0;
      R = panel_reduce(0.0, gt, INT32_MAX, 0ull, rs, rc, rm, rb);
      __syncthreads();
      need = topk - R.total;  // ties at tau to keep, in column order
    }
    // renormalising sum of the selected entries, then the ordered write
    const bool select_all = nk <= topk;
    double s2 = 0.0;
    {
      int seen = 0;
      for (int c0 = 0; c0 < nk; c0 += kPT) {
        const int idx = c0 + tid;
        float q = 0.f;
        int tie = 0;
        if (idx < nk) {
          q = lval[idx];
          tie = (!select_all && __float_as_uint(q) == tau) ? 1 : 0;
        }
        R = panel_reduce(0.0, tie, INT32_MAX, 0ull, rs, rc, rm, rb);
        bool sel = false;
        if (idx < nk)
          sel = select_all || __float_as_uint(q) > tau || (tie && seen + R.excl < need);
        seen += R.total;
        if (idx < nk && !sel) lval[idx] = -1.f;  // dropped by the top-k
        s2 += sel ? (double)q : 0.0;
        __syncthreads();
      }
    }
    R = panel_reduce(s2, 0, INT32_MAX, 0ull, rs, rc, rm, rb);
    const float S2 = (float)R.s;
    __syncthreads();
    SPG_GLOBAL int32_t *cb = gpw(ycol) + (size_t)i * cap;
    SPG_GLOBAL float *vb = gpw(yval) + (size_t)i * cap;
    int outn = 0;
    if (nk == 0) {
      if (rowbest != 0ull) {  // emptied row: keep its largest entry
        if (tid == 0) {
          const float q = __uint_as_float((uint32_t)(rowbest >> 32)) / S;
          cb[0] = (int)~(uint32_t)(rowbest & 0xffffffffu);
          vb[0] = rpost == 0 ? q / q : ipow(q, rpost);
        }
        outn = 1;
      }
    } else {
      for (int c0 = 0; c0 < nk; c0 += kPT) {
        const int idx = c0 + tid;
        const bool sel = idx < nk && !(lval[idx] < 0.f);
        R = panel_reduce(0.0, sel ? 1 : 0, INT32_MAX, 0ull, rs, rc, rm, rb);
        const int o = outn + R.excl;
        if (sel && o < cap) {
          cb[o] = lcol[idx];
          vb[o] = rpost == 0 ? lval[idx] / S2 : ipow(lval[idx], rpost);
        }
        outn += R.total;
        __syncthreads();
      }
    }
    if (tid == 0) ycnt[i] = outn < cap ? outn : cap;
    __syncthreads();
  }
}

// Row sums of |x| in FP64 (the heavy kernel's fixed-point scale bound).
__global__ __launch_bounds__(256) void k_row_abs(const Problem *__restrict__ pr,
                                                 const WsHeader *__restrict__ hdr,
                                                 double *__restrict__ rabs) {
  if (hdr->status) return;
  const Part &P = pr->part[0];
  const int n = P.kdim;
  const int lane = lane_id();
  const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwv = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const SPG_GLOBAL float *bval = gp(static_cast<const float *>(P.bval));
  for (int64_t k = wv; k < n; k += nwv) {
    const int s = gp(P.brp)[k], e = gp(P.brp)[k + 1];
    double t = 0.0;
    for (int j = s + lane; j < e; j += kWave) t += fabs((double)bval[j]);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if (lane == 0) rabs[k] = t;
  }
}

// Compaction of the padded rows into CSR (row_ptr from the scan of cnt).
__global__ __launch_bounds__(256) void k_mcl_compact(int n, int cap, const int32_t *__restrict__ yrp,
                                                     const int32_t *__restrict__ pcol,
                                                     const float *__restrict__ pval,
                                                     int32_t *__restrict__ ycol,
                                                     float *__restrict__ yval,
                                                     const WsHeader *__restrict__ hdr) {
  if (hdr->status) return;
  const int lane = threadIdx.x & 63;
  const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwv = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wv; i < n; i += nwv) {
    const int o = yrp[i], len = yrp[i + 1] - o;
    for (int t = lane; t < len; t += 64) {
      ycol[o + t] = pcol[i * cap + t];
      yval[o + t] = pval[i * cap + t];
    }
  }
}

// ---------------------------------------------------------------------------

template <int G>
static void mcl_launch(const Problem *dpr, const int32_t *rows, WsHeader *hdr, int bin, int lS,
                       int TT, uint32_t mul, int maxwin, int r, int rpost, float prune, int topk,
                       int cap,
                       int32_t *ycol, float *yval, int32_t *ycnt, int32_t *fb, int grid,
                       size_t lds, hipStream_t st) {
  hipLaunchKernelGGL(k_mcl_rows<G>, dim3(grid), dim3(MGeom<G>::WG), lds, st, dpr, rows, hdr, bin,
                     lS, TT, mul, maxwin, r, rpost, prune, topk, cap, ycol, yval, ycnt, fb);
}

size_t mcl_lds_bytes(int b, int G) {
  const int WG = G <= kWave ? 256 : G, R = WG / G;
  const size_t TT = (size_t)num_table_slots(b, G);
  return (size_t)R * TT * 8 + (size_t)R * G * 12 + (size_t)R * 4 + 64;
}

hipError_t launch_mcl(const Problem *dpr, const BinPlan &bp, const WsLayout &L, char *ws,
                      int r, int rpost, float prune, int topk, int cap, int32_t *pcol, float *pval,
                      int32_t *ycnt, hipStream_t st) {
  WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
  const int32_t *rows = reinterpret_cast<const int32_t *>(ws + L.rows);
  int32_t *fb = reinterpret_cast<int32_t *>(ws + L.fbrows);
  const DevInfo &D = dev_info();
  const int maxwin = bp.maxwin < kTail ? bp.maxwin : kTail;
  for (int b = 1; b <= bp.maxbin; ++b) {
    if (bp.known && bp.count[b] == 0) continue;
    int G = bp.lanes[b] < 8 ? 8 : bp.lanes[b];  // no one-thread-per-row MCL kernel
    while (G < 1024 && mcl_lds_bytes(b, G) > D.lds_per_block) G *= 2;
    // a bin past the largest table that fits takes that table (rows whose
    // distinct columns overflow it are handed to the panel kernel)
    int tb = b;
    while (tb > 1 && mcl_lds_bytes(tb, G) > D.lds_per_block) --tb;
    const int WG = G <= kWave ? 256 : G;
    const int R = WG / G;
    const size_t lds = mcl_lds_bytes(tb, G);
    int cap_grid = D.cus * (int)std::max<size_t>(1, std::min<size_t>(D.lds_per_cu / lds, 2048 / WG));
    int grid = cap_grid;
    if (bp.known) grid = std::min(cap_grid, (bp.count[b] + R - 1) / R);
    const int TT = num_table_slots(tb, G);
    const uint32_t mul = mono_mul(bin_slots(tb), bp.n);
    int S = bp.sub[b] > 0 ? bp.sub[b] : 16;
    if (S > G) S = G;
    int lS = 0;
    while ((1 << lS) < S) ++lS;
    switch (G) {
#define SPG_MCL_CASE(g) \
  case g: mcl_launch<g>(dpr, rows, hdr, b, lS, TT, mul, maxwin, r, rpost, prune, topk, cap, pcol, pval, ycnt, fb, grid, lds, st); break;
      SPG_MCL_CASE(8)
      SPG_MCL_CASE(16)
      SPG_MCL_CASE(32)
      SPG_MCL_CASE(64)
      SPG_MCL_CASE(128)
      SPG_MCL_CASE(256)
      SPG_MCL_CASE(512)
      default: mcl_launch<1024>(dpr, rows, hdr, b, lS, TT, mul, maxwin, r, rpost, prune, topk, cap, pcol, pval, ycnt, fb, grid, lds, st);
#undef SPG_MCL_CASE
    }
  }
  {
    // heavy bins plus rows handed over by the LDS kernels
    // one 1024-thread block per CU (its register use allows no second one)
    const int grid = std::min(mcl_heavy_slots(bp.n), D.cus);
    double *rabs = reinterpret_cast<double *>(ws + L.mcl_rabs);
    hipLaunchKernelGGL(k_row_abs, dim3(D.cus * 8), dim3(256), 0, st, dpr, hdr, rabs);
    const size_t lds = (size_t)kPanel * 8 + (size_t)kPanel / 8;
    hipLaunchKernelGGL(k_mcl_panel, dim3(grid), dim3(kPT), lds, st, dpr, rows, hdr, bp.maxbin + 1,
                       r, rpost, prune, topk, cap, rabs, ws + L.mcl_slots, mcl_slot_bytes(bp.n), fb,
                       pcol, pval, ycnt);
  }
  return hipGetLastError();
}

hipError_t launch_mcl_compact(int n, int cap, const int32_t *yrp, const int32_t *pcol,
                              const float *pval, int32_t *ycol, float *yval, const WsHeader *hdr,
                              hipStream_t st) {
  const DevInfo &D = dev_info();
  hipLaunchKernelGGL(k_mcl_compact, dim3(D.cus * 8), dim3(256), 0, st, n, cap, yrp, pcol, pval,
                     ycol, yval, hdr);
  return hipGetLastError();
}

hipError_t configure_mcl_lds(size_t lds_max) {
  const void *ks[] = {
      reinterpret_cast<const void *>(&k_mcl_rows<8>),   reinterpret_cast<const void *>(&k_mcl_rows<16>),
      reinterpret_cast<const void *>(&k_mcl_rows<32>),  reinterpret_cast<const void *>(&k_mcl_rows<64>),
      reinterpret_cast<const void *>(&k_mcl_rows<128>), reinterpret_cast<const void *>(&k_mcl_rows<256>),
      reinterpret_cast<const void *>(&k_mcl_rows<512>), reinterpret_cast<const void *>(&k_mcl_rows<1024>),
      reinterpret_cast<const void *>(&k_mcl_panel),
  };
  for (const void *k : ks) {
    hipError_t e =
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace spg

// One Markov-clustering iteration (a8; paper §5.7) on X = M^T in CSR, FP32:
//   E = X X;  e <- e^r;  row /= row sum;  drop e < prune;  keep the topk
//   largest (ties to the smaller column);  an emptied row keeps its largest
//   entry;  row /= new row sum.
// The unpruned product is never stored.  Row c of Y is written at its final
// column rank into a padded buffer (cap = min(topk, n) slots per row) with
// its length in cnt[c]; a scan of cnt and a compaction copy produce CSR.
//
// Rows whose products fit an LDS table use the numeric kernel's
// order-preserving hash (rank = occupied slots before + inversion counter)
// and run the whole epilogue in LDS; rows beyond the tables use a column
// bitmap and the heavy slot's dense accumulator, whose bitmap walk is in
// column order.  Kept entries are flagged by clearing the sign of their
// value slot (LDS rows) or by clearing their bitmap bit (heavy rows).
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
        if (ok[u] && old[u] != kEmpty) lds_add(&val[h[u]], v[u]);
    } else {
#pragma unroll
      for (int u = 0; u < N; ++u)
        if (ok[u]) lds_add(&val[h[u]], v[u]);
    }
  }
};

// LDS rows.  Key words pack (col | (128 + counter) << 24), n <= 2^24.
template <int G>
__global__ __launch_bounds__(MGeom<G>::WG) void k_mcl_rows(
    const Problem *__restrict__ pr, const int32_t *__restrict__ rows, WsHeader *__restrict__ hdr,
    int bin, int lS, int TT, uint32_t mul, int maxwin, int r, float prune, int topk, int cap,
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
        vb[rr] = v / S2;
        ++rk;
      }
    }
    if (l == 0) ycnt[i] = total < cap ? total : cap;
    group_sync<BLOCK>();
  }
}

// Heavy rows: bitmap (LDS, n <= 2^20) + the slot's dense accumulator.  The
// rows come from the bins above the LDS tables and from the LDS kernel's
// hand-over list (probe longer than the window).
__global__ __launch_bounds__(1024) void k_mcl_heavy(
    const Problem *__restrict__ pr, const int32_t *__restrict__ rows, WsHeader *__restrict__ hdr,
    int blo, int lS, int r, float prune, int topk, int cap, float *gacc,
    const int32_t *__restrict__ fb_rows, int32_t *__restrict__ ycol, float *__restrict__ yval,
    int32_t *__restrict__ ycnt) {
  extern __shared__ __align__(16) uint32_t map[];
  __shared__ int sb[1024], sl[1024];
  __shared__ float sa[1024];
  __shared__ float redf[16];
  __shared__ int redi[16];
  __shared__ unsigned long long redu[16];
  const int n = pr->n;
  const int nw = (n + 31) >> 5;
  float *acc = gacc + (size_t)blockIdx.x * n;
  if (hdr->status) return;
  const int start = hdr->bin_start[blo];
  const int nheavy = hdr->bin_start[kHeavyBin + 1] - start;
  const int count = nheavy + hdr->fallback_count;
  const int tid = threadIdx.x;
  Stage<float> st{sb, sl, sa};
  for (int ri = blockIdx.x; ri < count; ri += gridDim.x) {
    const int i = ri < nheavy ? rows[start + ri] : fb_rows[ri - nheavy];
    for (int w = tid; w < nw; w += 1024) map[w] = 0u;
    __syncthreads();
    auto fmark = each_product([&](int col, float) {
      const uint32_t bit = 1u << (col & 31);
      if (!(atomicOr(&map[col >> 5], bit) & bit)) acc[col] = 0.f;
    });
    for_each_product<true, false, 1024, kMclUnroll, float>(pr, i, true, tid, lS, st, fmark);
    __threadfence();
    __syncthreads();
    auto fadd = each_product([&](int col, float v) { global_add(&acc[col], v); });
    for_each_product<true, true, 1024, kMclUnroll, float>(pr, i, true, tid, lS, st, fadd);
    __threadfence();
    __syncthreads();
    // inflation + sum
    float part = 0.f;
    for (int w = tid; w < nw; w += 1024) {
      uint32_t b = map[w];
      while (b) {
        const int col = (w << 5) + __ffs(b) - 1;
        b &= b - 1;
        const float p = ipow(acc[col], r);
        acc[col] = p;
        part += p;
      }
    }
    const float S = group_sum<true, 1024>(part, redf);
    // normalise, prune (clear the bit of a dropped entry), largest entry
    int kept = 0;
    unsigned long long best = 0;
    for (int w = tid; w < nw; w += 1024) {
      uint32_t b = map[w], keepbits = map[w];
      while (b) {
        const int j = __ffs(b) - 1;
        const int col = (w << 5) + j;
        b &= b - 1;
        const float v = acc[col] / S;
        acc[col] = v;
        const unsigned long long kk = vc_key(v, col);
        best = kk > best ? kk : best;
        if (v < prune) keepbits &= ~(1u << j);
        else ++kept;
      }
      map[w] = keepbits;
    }
    const int nkept = group_sum<true, 1024>(kept, redi);
    if (nkept > topk) {
      uint32_t lo = 0, hi = 0x7f800000u;
      while (lo < hi) {
        const uint32_t mid = lo + (hi - lo + 1) / 2;
        int cc = 0;
        for (int w = tid; w < nw; w += 1024) {
          uint32_t b = map[w];
          while (b) {
            const int col = (w << 5) + __ffs(b) - 1;
            b &= b - 1;
            cc += __float_as_uint(acc[col]) >= mid ? 1 : 0;
          }
        }
        if (group_sum<true, 1024>(cc, redi) >= topk) lo = mid;
        else hi = mid - 1;
      }
      int gt = 0;
      for (int w = tid; w < nw; w += 1024) {
        uint32_t b = map[w];
        while (b) {
          const int col = (w << 5) + __ffs(b) - 1;
          b &= b - 1;
          gt += __float_as_uint(acc[col]) > lo ? 1 : 0;
        }
      }
      const int need = topk - group_sum<true, 1024>(gt, redi);
      // ties at tau keep the smallest columns: prefix count in column order
      int done = 0;
      for (int w0 = 0; w0 < nw; w0 += 1024) {
        const int w = w0 + tid;
        uint32_t bits = w < nw ? map[w] : 0u;
        int eq = 0;
        uint32_t b = bits;
        while (b) {
          const int col = (w << 5) + __ffs(b) - 1;
          b &= b - 1;
          eq += __float_as_uint(acc[col]) == lo ? 1 : 0;
        }
        int tot;
        int before = done + group_excl_scan<true, 1024>(eq, tid, redi, tot);
        b = bits;
        uint32_t keepbits = bits;
        while (b) {
          const int j = __ffs(b) - 1;
          const int col = (w << 5) + j;
          b &= b - 1;
          const uint32_t vb = __float_as_uint(acc[col]);
          bool keep = vb > lo;
          if (vb == lo) keep = (before++ < need);
          if (!keep) keepbits &= ~(1u << j);
        }
        if (w < nw) map[w] = keepbits;
        done += tot;
      }
    }
    __syncthreads();
    if (nkept == 0) {
      const unsigned long long bb = group_max_u64<true, 1024>(best, redu);
      if (bb != 0 || true) {
        const int bcol = (int)~(uint32_t)(bb & 0xffffffffu);
        if (tid == 0 && bcol >= 0 && bcol < n) map[bcol >> 5] |= 1u << (bcol & 31);
      }
    }
    __syncthreads();
    float part2 = 0.f;
    for (int w = tid; w < nw; w += 1024) {
      uint32_t b = map[w];
      while (b) {
        const int col = (w << 5) + __ffs(b) - 1;
        b &= b - 1;
        part2 += acc[col];
      }
    }
    const float S2 = group_sum<true, 1024>(part2, redf);
    // write in column order
    int pre = 0;
    SPG_GLOBAL int32_t *cb = gpw(ycol) + (size_t)i * cap;
    SPG_GLOBAL float *vb2 = gpw(yval) + (size_t)i * cap;
    for (int w0 = 0; w0 < nw; w0 += 1024) {
      const int w = w0 + tid;
      const uint32_t bits = w < nw ? map[w] : 0u;
      int tot;
      int o = pre + group_excl_scan<true, 1024>(__popc(bits), tid, redi, tot);
      uint32_t b = bits;
      while (b) {
        const int col = (w << 5) + __ffs(b) - 1;
        b &= b - 1;
        if (o < cap) {
          cb[o] = col;
          vb2[o] = acc[col] / S2;
        }
        ++o;
      }
      pre += tot;
    }
    if (tid == 0) ycnt[i] = pre < cap ? pre : cap;
    __threadfence();
    __syncthreads();
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
                       int TT, uint32_t mul, int maxwin, int r, float prune, int topk, int cap,
                       int32_t *ycol, float *yval, int32_t *ycnt, int32_t *fb, int grid,
                       size_t lds, hipStream_t st) {
  hipLaunchKernelGGL(k_mcl_rows<G>, dim3(grid), dim3(MGeom<G>::WG), lds, st, dpr, rows, hdr, bin,
                     lS, TT, mul, maxwin, r, prune, topk, cap, ycol, yval, ycnt, fb);
}

size_t mcl_lds_bytes(int b, int G) {
  const int WG = G <= kWave ? 256 : G, R = WG / G;
  const size_t TT = (size_t)num_table_slots(b, G);
  return (size_t)R * TT * 8 + (size_t)R * G * 12 + (size_t)R * 4 + 64;
}

hipError_t launch_mcl(const Problem *dpr, const BinPlan &bp, const WsLayout &L, char *ws,
                      int r, float prune, int topk, int cap, int32_t *pcol, float *pval,
                      int32_t *ycnt, hipStream_t st) {
  WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
  const int32_t *rows = reinterpret_cast<const int32_t *>(ws + L.rows);
  int32_t *fb = reinterpret_cast<int32_t *>(ws + L.fbrows);
  const DevInfo &D = dev_info();
  const int maxwin = bp.maxwin < kTail ? bp.maxwin : kTail;
  for (int b = 1; b <= bp.maxbin; ++b) {
    if (bp.known && bp.count[b] == 0) continue;
    int G = bp.lanes[b];
    while (G < 1024 && mcl_lds_bytes(b, G) > D.lds_per_block) G *= 2;
    const int WG = G <= kWave ? 256 : G;
    const int R = WG / G;
    const size_t lds = mcl_lds_bytes(b, G);
    int cap_grid = D.cus * (int)std::max<size_t>(1, std::min<size_t>(D.lds_per_cu / lds, 2048 / WG));
    int grid = cap_grid;
    if (bp.known) grid = std::min(cap_grid, (bp.count[b] + R - 1) / R);
    const int TT = num_table_slots(b, G);
    const uint32_t mul = mono_mul(bin_slots(b), bp.n);
    int S = bp.sub[b] > 0 ? bp.sub[b] : 16;
    if (S > G) S = G;
    int lS = 0;
    while ((1 << lS) < S) ++lS;
    switch (G) {
#define SPG_MCL_CASE(g) \
  case g: mcl_launch<g>(dpr, rows, hdr, b, lS, TT, mul, maxwin, r, prune, topk, cap, pcol, pval, ycnt, fb, grid, lds, st); break;
      SPG_MCL_CASE(8)
      SPG_MCL_CASE(16)
      SPG_MCL_CASE(32)
      SPG_MCL_CASE(64)
      SPG_MCL_CASE(128)
      SPG_MCL_CASE(256)
      SPG_MCL_CASE(512)
      default: mcl_launch<1024>(dpr, rows, hdr, b, lS, TT, mul, maxwin, r, prune, topk, cap, pcol, pval, ycnt, fb, grid, lds, st);
#undef SPG_MCL_CASE
    }
  }
  {
    // heavy bins plus rows handed over by the LDS kernels
    const int grid = bp.heavy_slots;
    int S = bp.sub[kHeavyBin] > 0 ? bp.sub[kHeavyBin] : 16;
    int lS = 0;
    while ((1 << lS) < S) ++lS;
    const size_t lds = (size_t)((bp.n + 31) >> 5) * 4;
    hipLaunchKernelGGL(k_mcl_heavy, dim3(grid), dim3(1024), lds, st, dpr, rows, hdr, bp.maxbin + 1,
                       lS, r, prune, topk, cap, reinterpret_cast<float *>(ws + L.heavyacc), fb, pcol,
                       pval, ycnt);
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
      reinterpret_cast<const void *>(&k_mcl_heavy),
  };
  for (const void *k : ks) {
    hipError_t e =
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace spg

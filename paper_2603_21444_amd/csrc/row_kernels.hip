// Row kernels of the local product C = sum_k A_k B_k (K = 1: C = A B, paper
// §2): symbolic count (a3) and numeric pass (a5) per row bin, the sort-based
// fallback and the heavy-row kernels, with their launchers.
//
// Rows of one bin are processed by groups of G lanes; groups of at most 64
// lanes share a block of 256 threads (several rows per block), larger
// groups are a block of their own.  Every kernel loops over its row list
// grid-stride style and reads the list length from the workspace header,
// so the same launch is valid eagerly (exact grid) and inside a graph
// (persistent grid).
#include <vector>

#include "internal.hpp"
#include "rowops.hpp"

namespace spg {

// Products per lane handed to one batched insert, and the occupancy the
// row kernels are compiled for (waves per SIMD; bounds the registers).
#ifndef SPG_SYM_UNROLL
#define SPG_SYM_UNROLL 4
#endif
#ifndef SPG_NUM_UNROLL
#define SPG_NUM_UNROLL 2
#endif
#ifndef SPG_NUM_WAVES
#define SPG_NUM_WAVES 8
#endif
constexpr int kUnroll = SPG_NUM_UNROLL;
constexpr int kSymUnroll = SPG_SYM_UNROLL;

// Geometry of a row group of G lanes: groups of at most 64 lanes share a
// 256-thread block (R rows per block, each wave's groups independent);
// larger groups are the block.
template <int G>
struct Geom {
  static constexpr bool BLOCK = G > kWave;
  static constexpr int WG = BLOCK ? G : 256;
  static constexpr int R = WG / G;
};

// Row index held by a group; for groups of a whole wave or more it is
// wave-uniform and is moved to a scalar register.
template <int G>
__device__ __forceinline__ int uniform_if_wave(int v) {
  return G >= kWave ? __builtin_amdgcn_readfirstlane(v) : v;
}

// ---------------------------------------------------------------------------
// a3: exact distinct-column count of each row with an LDS hash set.
//
// Inserts take the products of a lane N at a time: the first probe of all N
// is issued before any result is examined, so a wave keeps N LDS atomics in
// flight instead of waiting on each one (the inserts are latency-bound, not
// throughput-bound).
struct SymInsert {
  int *tab;
  int T, log2T;
  int fresh;
  template <int N, typename VT>
  __device__ __forceinline__ void batch(const int (&col)[N], const VT (&)[N]) {
    uint32_t h[N];
    int old[N];
#pragma unroll
    for (int u = 0; u < N; ++u) {
      h[u] = scramble_slot((uint32_t)col[u], log2T);
      old[u] = col[u] >= 0 ? atomicCAS(&tab[h[u]], kEmpty, col[u]) : col[u];
    }
#pragma unroll
    for (int u = 0; u < N; ++u) {
      if (col[u] < 0) continue;
      int o = old[u];
      uint32_t hh = h[u];
      while (o != kEmpty && o != col[u]) {
        hh = (hh + 1) & (T - 1);
        o = atomicCAS(&tab[hh], kEmpty, col[u]);
      }
      fresh += (o == kEmpty) ? 1 : 0;
    }
  }
};
template <int G>
__global__ __launch_bounds__(Geom<G>::WG) void k_sym_rows(const Problem *__restrict__ pr,
                                                          const int32_t *__restrict__ rows,
                                                          const WsHeader *__restrict__ hdr,
                                                          int bin, int lS, int log2T,
                                                          int32_t *__restrict__ cnt) {
  using GM = Geom<G>;
  extern __shared__ __align__(16) int smem[];
  const int T = 1 << log2T;
  const int rslot = threadIdx.x / G, l = threadIdx.x % G;
  int *tab = smem + rslot * T;
  int *sb = smem + GM::R * T + rslot * G;
  int *sl = smem + GM::R * T + GM::R * G + rslot * G;
  int *rowcnt = smem + GM::R * T + 2 * GM::R * G + rslot;
  if (hdr->status) return;
  const int count = hdr->bin_count[bin];
  const int start = hdr->bin_start[bin];
  Stage<float> st{sb, sl, nullptr};
  for (int ri = blockIdx.x * GM::R + rslot; ri < count; ri += gridDim.x * GM::R) {
    const int i = uniform_if_wave<G>(rows[start + ri]);
    int4 *t4 = reinterpret_cast<int4 *>(tab);
    for (int s = l; s < T / 4; s += G) t4[s] = make_int4(kEmpty, kEmpty, kEmpty, kEmpty);
    if (l == 0) *rowcnt = 0;
    group_sync<GM::BLOCK>();
    SymInsert ins{tab, T, log2T, 0};
    for_each_product<GM::BLOCK, false, G, kSymUnroll, float>(pr, i, true, l, lS, st, ins);
    if (ins.fresh) atomicAdd(rowcnt, ins.fresh);
    group_sync<GM::BLOCK>();
    if (l == 0) cnt[i] = *rowcnt;
  }
}

// ---------------------------------------------------------------------------
// a5: numeric pass with an order-preserving home slot.
//
// The home slot floor(col * T / n) never decreases with col and linear
// probing only walks forward, so a key x that ends up after a larger key y
// always has y inside its own probe path [home(x), slot(x)): those are the
// only out-of-order pairs, and every slot on that path was filled before x
// arrived.  So when x is inserted fresh at displacement d > 0 it walks its
// path once, adds one to the counter of each larger key it passed and
// subtracts their number from its own: the final rank of a key is
// (occupied slots before it) + (its counter).  The output pass gives each
// lane a contiguous, odd-length chunk of slots (no LDS bank conflicts), one
// group scan turns its occupied count into a base rank, and the lane writes
// its entries straight to their place in the output row.  A probe longer
// than `maxwin` hands the row to the sort-based fallback kernel.
//
// PACK (n <= 2^24): the counter lives in the top byte of the key word
// (biased by 128; it stays within [-2*kTail, 2*kTail]), so the table is one
// int array plus the values.

template <typename VT, bool PACK, bool PLAIN>
struct NumInsert {
  using KC = KeyCode<PACK>;
  int *key;
  VT *val;
  int *adj;
  int *flag;
  uint32_t mul;
  int maxwin;
  template <int N>
  __device__ __forceinline__ void batch(const int (&col)[N], const VT (&v)[N]) {
    int h[N], old[N];
#pragma unroll
    for (int u = 0; u < N; ++u) {
      h[u] = (int)mono_slot((uint32_t)col[u], mul);
      old[u] = col[u] >= 0 ? atomicCAS(&key[h[u]], kEmpty, KC::make(col[u])) : kEmpty;
    }
    int d[N];
#pragma unroll
    for (int u = 0; u < N; ++u) {
      d[u] = 0;
      if (col[u] < 0) continue;
      while (old[u] != kEmpty && KC::col(old[u]) != col[u]) {
        if (d[u] == maxwin) {  // long probe: the fallback redoes this row
          *flag = 1;
          d[u] = -1;
          break;
        }
        ++d[u];
        ++h[u];  // h <= home + maxwin < TT
        old[u] = atomicCAS(&key[h[u]], kEmpty, KC::make(col[u]));
      }
    }
    if (PLAIN) {
      // wave group: the first insert of a column stores its value, repeats
      // add after the fence (all of this batch's stores precede them)
#pragma unroll
      for (int u = 0; u < N; ++u)
        if (col[u] >= 0 && d[u] >= 0 && old[u] == kEmpty) val[h[u]] = v[u];
      group_sync<false>();
#pragma unroll
      for (int u = 0; u < N; ++u)
        if (col[u] >= 0 && d[u] >= 0 && old[u] != kEmpty) lds_add(&val[h[u]], v[u]);
    } else {
#pragma unroll
      for (int u = 0; u < N; ++u)
        if (col[u] >= 0 && d[u] >= 0) lds_add(&val[h[u]], v[u]);
    }
#pragma unroll
    for (int u = 0; u < N; ++u) {
      if (col[u] < 0 || d[u] <= 0 || old[u] != kEmpty) continue;
      int larger = 0;
      for (int t = h[u] - d[u]; t < h[u]; ++t) {
        if (KC::col(key[t]) > col[u]) {
          if (PACK) atomicAdd(&key[t], 1 << 24);
          else atomicAdd(&adj[t], 1);
          ++larger;
        }
      }
      if (larger) {
        if (PACK) atomicSub(&key[h[u]], larger << 24);
        else atomicSub(&adj[h[u]], larger);
      }
    }
  }
};

// FP32 inserts (slot table, see slot_insert).
template <bool PACK>
struct NumInsertF {
  unsigned long long *slot;
  int *adj;
  int *flag;
  uint32_t mul;
  int maxwin;
  template <int N>
  __device__ __forceinline__ void batch(const int (&col)[N], const float (&v)[N]) {
    slot_insert<PACK, N>(slot, adj, flag, mul, maxwin, col, v);
  }
};

// Waves per SIMD the numeric kernel is compiled for (bounds its registers):
// block groups hold larger tables, which leave room for fewer blocks per CU.
template <int G>
constexpr int num_waves() { return G >= 512 ? 4 : (G >= 128 ? 6 : SPG_NUM_WAVES); }

template <int G, typename VT, bool PACK>
__global__ __launch_bounds__(Geom<G>::WG, num_waves<G>()) void k_num_rows(const Problem *__restrict__ pr,
                                                          const int32_t *__restrict__ rows,
                                                          WsHeader *__restrict__ hdr, int bin,
                                                          int lS, int TT, uint32_t mul,
                                                          int maxwin,
                                                          const int32_t *__restrict__ crp,
                                                          int32_t *__restrict__ ccol,
                                                          VT *__restrict__ cval,
                                                          int32_t *__restrict__ fb_rows) {
  using GM = Geom<G>;
  using KC = KeyCode<PACK>;
  constexpr bool F32 = sizeof(VT) == 4;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int rslot = threadIdx.x / G, l = threadIdx.x % G;
  // F32: slots u64[R*TT] | sa | adj | sb | sl | rowflag | wtot
  // F64: vals VT[R*TT] | sa | keys int[R*TT] | adj | sb | sl | rowflag | wtot
  unsigned long long *slots_all = reinterpret_cast<unsigned long long *>(smem_raw);
  VT *vals_all = reinterpret_cast<VT *>(smem_raw);
  VT *sa_all = F32 ? reinterpret_cast<VT *>(slots_all + (size_t)GM::R * TT)
                   : vals_all + (size_t)GM::R * TT;
  int *keys_all = reinterpret_cast<int *>(sa_all + (size_t)GM::R * G);
  int *adj_all = F32 ? keys_all : keys_all + (size_t)GM::R * TT;
  int *sb_all = adj_all + (PACK ? 0 : (size_t)GM::R * TT);
  int *sl_all = sb_all + (size_t)GM::R * G;
  int *rowflag = sl_all + (size_t)GM::R * G;
  int *wtot = rowflag + GM::R;
  unsigned long long *slot = slots_all + (size_t)rslot * TT;
  VT *val = vals_all + (size_t)rslot * TT;
  int *key = keys_all + (size_t)rslot * TT;
  int *adj = adj_all + (size_t)rslot * TT;
  Stage<VT> st{sb_all + rslot * G, sl_all + rslot * G, sa_all + rslot * G};
  if (hdr->status) return;
  const int count = hdr->bin_count[bin];
  const int start = hdr->bin_start[bin];
  auto key_at = [&](int s) { return F32 ? slot_key(slot[s]) : key[s]; };
  for (int ri = blockIdx.x * GM::R + rslot; ri < count; ri += gridDim.x * GM::R) {
    const int i = uniform_if_wave<G>(rows[start + ri]);
    if (F32) {
      int4 *s4 = reinterpret_cast<int4 *>(slot);
      for (int s = l; s < TT / 2; s += G) s4[s] = make_int4(kEmpty, 0, kEmpty, 0);
    } else {
      int4 *k4 = reinterpret_cast<int4 *>(key);
      for (int s = l; s < TT / 4; s += G) k4[s] = make_int4(kEmpty, kEmpty, kEmpty, kEmpty);
      if (GM::BLOCK)
        for (int s = l; s < TT; s += G) val[s] = VT(0);
    }
    if (!PACK) {
      int4 *a4 = reinterpret_cast<int4 *>(adj);
      for (int s = l; s < TT / 4; s += G) a4[s] = make_int4(0, 0, 0, 0);
    }
    if (l == 0) rowflag[rslot] = 0;
    group_sync<GM::BLOCK>();
    if constexpr (F32) {
      NumInsertF<PACK> ins{slot, adj, rowflag + rslot, mul, maxwin};
      for_each_product<GM::BLOCK, true, G, kUnroll, VT>(pr, i, true, l, lS, st, ins);
    } else {
      NumInsert<VT, PACK, !GM::BLOCK> ins{key, val, adj, rowflag + rslot, mul, maxwin};
      for_each_product<GM::BLOCK, true, G, kUnroll, VT>(pr, i, true, l, lS, st, ins);
    }
    group_sync<GM::BLOCK>();
    const bool ok = rowflag[rslot] == 0;
    const int rs = crp[i];
    const int nnz = crp[i + 1] - rs;
    SPG_GLOBAL int32_t *cb = gpw(ccol) + rs;
    SPG_GLOBAL VT *vb = gpw(cval) + rs;
    // Output: rounds of 64 (or G) consecutive slots; one ballot gives every
    // lane the rank of its key among the round's, so the writes of a round
    // are contiguous.  Block groups first count each wave's slot range and
    // scan the counts across the waves.
    const int gsz = GM::BLOCK ? kWave : G;
    const int g0 = (lane_id() / gsz) * gsz;
    const uint64_t gm = (gsz >= kWave) ? ~0ull : (((1ull << gsz) - 1ull) << g0);
    const uint64_t below = lanes_below();
    const int wl = GM::BLOCK ? l % kWave : l;
    int lo = 0, hi = TT, base = 0, total = 0;
    if (GM::BLOCK) {
      constexpr int NW = GM::BLOCK ? G / kWave : 1;
      const int w = l / kWave;
      const int per = ((TT + kWave - 1) / kWave + NW - 1) / NW * kWave;
      lo = min(TT, w * per);
      hi = min(TT, lo + per);
      int cw = 0;
      for (int s0 = lo; s0 < hi; s0 += kWave) {
        const int s = s0 + wl;
        cw += __popcll(__ballot(s < hi && key_at(s) != kEmpty));
      }
      if (wl == 0) wtot[w] = cw;
      __syncthreads();
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) {
        const int c = wtot[ww];
        base += ww < w ? c : 0;
        total += c;
      }
      __syncthreads();
    }
    for (int s0 = lo; s0 < hi; s0 += gsz) {
      const int s = s0 + wl;
      int w = kEmpty;
      VT v = VT(0);
      if (s < hi) {
        if constexpr (F32) {
          const unsigned long long sv = slot[s];
          w = slot_key(sv);
          v = slot_val(sv);
        } else {
          w = key[s];
          v = val[s];
        }
      }
      const uint64_t m = __ballot(w != kEmpty) & gm;
      if (ok && w != kEmpty && nnz > 0) {
        int rr = base + __popcll(m & below) + (PACK ? KC::adj(w) : adj[s]);
        rr = rr < 0 ? 0 : (rr >= nnz ? nnz - 1 : rr);  // in bounds even for a changed pattern
        cb[(uint32_t)rr] = KC::col(w);
        vb[(uint32_t)rr] = v;
      }
      base += __popcll(m);
    }
    if (!GM::BLOCK) total = base;
    if (ok && l == 0 && total != nnz) atomicOr(&hdr->status, kStatInvalid);
    if (l == 0 && !ok) {
      const int slot_i = atomicAdd(&hdr->fallback_count, 1);
      fb_rows[slot_i] = i;
    }
    group_sync<GM::BLOCK>();
  }
}

// Numeric pass of a block-group bin by bucketing (one row per block of G
// lanes, n <= 2^24): the bucket scheme of the one-row-per-wave kernel
// (tickets in the bucket of the order-preserving home slot, scan,
// placement), here with T = edge buckets and 1.125 edge staged products so
// that three rows of the 2^12-column bin fit one CU's LDS (the hash table
// needs 16 bytes per column, this 11).  Rows with few repeated columns
// rank each product inside its bucket (less the repeats of smaller columns,
// listed first); other rows sort the buckets and give each thread a
// contiguous range of positions, whose run starts one block scan turns into
// output ranks.  Overflowing rows go to the fallback kernel.
constexpr int kBktJ = 12;  // staged products per thread at most
// Rows with at most this many repeated products (products less distinct
// columns) are ranked inside their buckets; rows with more sort them.
constexpr int kDupList = 32;

template <typename VT>
struct BucketInsertB {
  uint32_t *cnt;   // T/2 words: two 16-bit bucket counters per word
  uint32_t *ikey;  // [cap] col | ticket << 24
  VT *ival;        // [cap]
  int *wcount;     // products staged so far (LDS, per block)
  uint32_t mul;
  int cap;
  bool over;
  // LDS flag, raised once a bucket holds more than kBigBucket products: the
  // row's columns cluster and it will be sorted as a whole, so the waves
  // that see the flag stop taking bucket tickets (on which the lanes of a
  // clustered row would contend for a few LDS words).  A stale read only
  // means a few more tickets.
  int *bigflag;
  template <int N>
  __device__ __forceinline__ void batch(const int (&col)[N], const VT (&v)[N]) {
    uint32_t old[N], sh[N];
    const bool skip = *bigflag != 0;
#pragma unroll
    for (int u = 0; u < N; ++u) {
      const uint32_t b = mono_slot((uint32_t)col[u], mul);
      sh[u] = (b & 1u) << 4;
      old[u] = (col[u] >= 0 && !skip) ? atomicAdd(&cnt[b >> 1], 1u << sh[u]) : 0u;
    }
    if (!skip) {
      bool hi = false;
#pragma unroll
      for (int u = 0; u < N; ++u) hi = hi || ((old[u] >> sh[u]) & 0xffffu) > (uint32_t)kBigBucket;
      if (hi) *bigflag = 1;
    }
    uint64_t m[N];
    int tot = 0;
#pragma unroll
    for (int u = 0; u < N; ++u) {
      m[u] = __ballot(col[u] >= 0);
      tot += __popcll(m[u]);
    }
    const uint64_t act = __ballot(true);
    const int leader = __ffsll((unsigned long long)act) - 1;
    int p0 = 0;
    if (tot > 0 && lane_id() == leader) p0 = atomicAdd(wcount, tot);
    p0 = __shfl(p0, leader);
    const uint64_t below = lanes_below();
#pragma unroll
    for (int u = 0; u < N; ++u) {
      const int p = p0 + __popcll(m[u] & below);
      p0 += __popcll(m[u]);
      const uint32_t t = (old[u] >> sh[u]) & 0xffffu;
      if (col[u] >= 0) {
        if (p < cap && t < 256u) {
          ikey[p] = (uint32_t)col[u] | (t << 24);
          ival[p] = v[u];
        } else {
          over = true;
        }
      }
    }
  }
};

__device__ __forceinline__ int bkt_start(const uint32_t *cnt, uint32_t b) {
  return (int)((cnt[b >> 1] >> ((b & 1u) << 4)) & 0xffffu);
}

template <int G, typename VT>
__global__ __launch_bounds__(G) void k_num_bucket_blk(
    const Problem *__restrict__ pr, const int32_t *__restrict__ rows, WsHeader *__restrict__ hdr,
    int bin, int lS, int T, int cap, uint32_t mul, const int32_t *__restrict__ crp,
    int32_t *__restrict__ ccol, VT *__restrict__ cval, int32_t *__restrict__ fb_rows) {
  static_assert(G >= 128 && G <= 1024, "block groups only");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int wcount, overflow, bigmax, bigflag, ndl;
  __shared__ int wtot[G / kWave];
  __shared__ uint32_t dlist[kDupList];
  const int tid = threadIdx.x;
  const int TW = T / 2;
  uint32_t *cnt = reinterpret_cast<uint32_t *>(smem_raw);
  uint32_t *ikey = cnt + TW;
  VT *ival = reinterpret_cast<VT *>(ikey + cap);
  int *sb = reinterpret_cast<int *>(ival + cap);
  int *sl = sb + G;
  VT *sa = reinterpret_cast<VT *>(sl + G);
  Stage<VT> st{sb, sl, sa};
  if (hdr->status) return;
  const int count = hdr->bin_count[bin];
  const int start = hdr->bin_start[bin];
  const int wpt = (TW + G - 1) / G;  // counter words per thread
  __shared__ int item;
  for (int ri = block_next(&hdr->queue[bin], &item); ri < count;
       ri = block_next(&hdr->queue[bin], &item)) {
    const int i = __builtin_amdgcn_readfirstlane(rows[start + ri]);
    const int rs = crp[i];
    const int nnz = crp[i + 1] - rs;
    for (int s = tid; s < TW; s += G) cnt[s] = 0u;
    if (tid == 0) {
      wcount = 0;
      overflow = 0;
      bigmax = 0;
      bigflag = 0;
      ndl = 0;
    }
    __syncthreads();
    BucketInsertB<VT> ins{cnt, ikey, ival, &wcount, mul, cap, false, &bigflag};
    for_each_product<true, true, G, kUnroll, VT>(pr, i, true, tid, lS, st, ins);
    if (ins.over) overflow = 1;
    __syncthreads();
    const int P = wcount;
    if (overflow || P > cap) {  // the fallback redoes this row
      if (tid == 0) fb_rows[atomicAdd(&hdr->fallback_count, 1)] = i;
      __syncthreads();
      continue;
    }
    SPG_GLOBAL int32_t *cb = gpw(ccol) + rs;
    SPG_GLOBAL VT *vb = gpw(cval) + rs;
    if (bigflag) {
      // clustered columns: sort the staged products as a whole (tickets
      // dropped), then the runs pass below
      for (int p = tid; p < P; p += G) ikey[p] &= 0xffffffu;
      __syncthreads();
      lds_sort_pairs<true, G, VT>(ikey, ival, P, tid);
    } else {
      // 1. bucket starts: exclusive scan of the 16-bit counters, in place
      {
        const int w0 = tid * wpt;
        int loc = 0, mx = 0;
        for (int j = 0; j < wpt; ++j) {
          if (w0 + j < TW) {
            const uint32_t wv = cnt[w0 + j];
            loc += (int)(wv & 0xffffu) + (int)(wv >> 16);
            mx = max(mx, (int)max(wv & 0xffffu, wv >> 16));
          }
        }
        if (mx > kBigBucket) atomicMax(&bigmax, mx);
        int total;
        int run = group_excl_scan<true, G>(loc, tid, wtot, total);
        for (int j = 0; j < wpt; ++j) {
          if (w0 + j < TW) {
            const uint32_t wv = cnt[w0 + j];
            const uint32_t lo = (uint32_t)run;
            run += (int)(wv & 0xffffu);
            const uint32_t hi = (uint32_t)run;
            run += (int)(wv >> 16);
            cnt[w0 + j] = lo | (hi << 16);
          }
        }
      }
      __syncthreads();
      // 2. every product to start[bucket] + ticket
      {
        uint32_t kk[kBktJ];
        VT vv[kBktJ];
  #pragma unroll
        for (int j = 0; j < kBktJ; ++j) {
          const int p = tid + j * G;
          kk[j] = p < P ? ikey[p] : 0u;
          vv[j] = p < P ? ival[p] : VT(0);
        }
        __syncthreads();
  #pragma unroll
        for (int j = 0; j < kBktJ; ++j) {
          if (tid + j * G < P) {
            const uint32_t c = kk[j] & 0xffffffu;
            const int pos = bkt_start(cnt, mono_slot(c, mul)) + (int)(kk[j] >> 24);
            ikey[pos] = c;
            ival[pos] = vv[j];
          }
        }
      }
      __syncthreads();
      const bool big = bigmax > kBigBucket;
      const int ndup = P - nnz;  // repeated products, by the symbolic count
      if (!big && ndup >= 0 && ndup <= kDupList) {
        // few repeated columns: a product's output rank is its bucket's
        // start plus the smaller columns in its bucket, less the repeats of
        // smaller columns, which a first pass lists; the first product of a
        // column in its bucket sums the column's products and writes them
        if (ndup > 0) {
          for (int p = tid; p < P; p += G) {
            const uint32_t c = ikey[p];
            for (int q = bkt_start(cnt, mono_slot(c, mul)); q < p; ++q) {
              if (ikey[q] == c) {
                const int e = atomicAdd(&ndl, 1);
                if (e < kDupList) dlist[e] = c;
                break;
              }
            }
          }
          __syncthreads();
        }
        const int nd = min(ndl, kDupList);
        bool bad = ndl != ndup;  // a changed pattern
        for (int p = tid; p < P; p += G) {
          const uint32_t c = ikey[p];
          const uint32_t b = mono_slot(c, mul);
          const int s0 = bkt_start(cnt, b);
          const int s1 = b + 1 < (uint32_t)T ? bkt_start(cnt, b + 1) : P;
          int r = s0;
          bool first = true;
          VT sum = ival[p];
          for (int q = s0; q < s1; ++q) {
            const uint32_t k = ikey[q];
            r += k < c ? 1 : 0;
            if (k == c && q != p) {
              if (q < p) first = false;
              else sum += ival[q];
            }
          }
          if (first) {
            for (int e = 0; e < nd; ++e) r -= dlist[e] < c ? 1 : 0;
            if (r < nnz) {
              cb[r] = (int)c;
              vb[r] = sum;
            } else {
              bad = true;
            }
          } else if (ndup == 0) {
            bad = true;
          }
        }
        if (bad) atomicOr(&hdr->status, kStatInvalid);
        __syncthreads();
        continue;
      }
      // 3. sort every bucket of two or more products by column, or the whole
      //    row when a bucket is large
      if (big) lds_sort_pairs<true, G, VT>(ikey, ival, P, tid);
      for (int b = big ? T : tid; b < T; b += G) {
        const int s0 = bkt_start(cnt, (uint32_t)b);
        const int s1 = b + 1 < T ? bkt_start(cnt, (uint32_t)b + 1) : P;
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
    // 4. each thread a contiguous range of positions: its run starts, one
    //    block scan, then the first of each run sums the run and writes it
    {
      const int per = (P + G - 1) / G;
      const int p0 = tid * per, p1 = min(P, p0 + per);
      int firsts = 0;
      for (int p = p0; p < p1; ++p) firsts += (p == 0 || ikey[p] != ikey[p - 1]) ? 1 : 0;
      int total;
      int d = group_excl_scan<true, G>(firsts, tid, wtot, total);
      for (int p = p0; p < p1; ++p) {
        const uint32_t c = ikey[p];
        if (p == 0 || c != ikey[p - 1]) {
          VT sum = ival[p];
          for (int q = p + 1; q < P && ikey[q] == c; ++q) sum += ival[q];
          if (d < nnz) {  // the symbolic count bounds the row (a changed pattern is flagged)
            cb[d] = (int)c;
            vb[d] = sum;
          }
          ++d;
        }
      }
      if (tid == 0 && total != nnz) atomicOr(&hdr->status, kStatInvalid);
    }
    __syncthreads();
  }
}

// Bins the block bucket kernel serves: n <= 2^24 and edge(b) * 9/8 staged
// products within kBktJ per thread.
int bucket_blk_cap(int b) { return (8 << b) + (1 << b); }
bool bucket_blk_ok(int b, int G) { return G >= 128 && bucket_blk_cap(b) <= kBktJ * G; }
size_t bucket_blk_lds(int b, int G, size_t vbytes) {
  const size_t T = (size_t)(8 << b);
  return T * 2 + (size_t)bucket_blk_cap(b) * (4 + vbytes) + (size_t)G * (8 + vbytes);
}

// Fallback numeric pass: scrambled LDS hash, in-place compaction, bitonic
// sort of (column, value) pairs, coalesced write.  One row per block.
template <typename VT>
__global__ __launch_bounds__(1024) void k_num_fallback(const Problem *__restrict__ pr,
                                                       const int32_t *__restrict__ fb_rows,
                                                       WsHeader *__restrict__ hdr, int TF,
                                                       int lS, const int32_t *__restrict__ crp,
                                                       int32_t *__restrict__ ccol,
                                                       VT *__restrict__ cval) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int wtot[16];
  VT *val = reinterpret_cast<VT *>(smem_raw);
  VT *sa = val + TF;
  int *key = reinterpret_cast<int *>(sa + 1024);
  int *sb = key + TF;
  int *sl = sb + 1024;
  if (hdr->status) return;
  const int count = hdr->fallback_count;
  const int tid = threadIdx.x;
  Stage<VT> st{sb, sl, sa};
  __shared__ int item;
  for (int ri = block_next(&hdr->queue[kQueueFallback], &item); ri < count;
       ri = block_next(&hdr->queue[kQueueFallback], &item)) {
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
    auto fins = each_product([&](int col, VT v) {
      uint32_t h = scramble_slot((uint32_t)col, log2T);
      for (int probes = 0;; ++probes) {
        const int old = atomicCAS(&key[h], kEmpty, col);
        if (old == kEmpty || old == col) {
          lds_add(&val[h], v);
          break;
        }
        if (probes >= T) {  // more distinct columns than the symbolic pass counted
          atomicOr(&hdr->status, kStatInvalid);
          break;
        }
        h = (h + 1) & (T - 1);
      }
    });
    for_each_product<true, true, 1024, kUnroll, VT>(pr, i, true, tid, lS, st, fins);
    __syncthreads();
    // in-place compaction in slot order (a round's reads precede its writes)
    int pre = 0;
    for (int s0 = 0; s0 < T; s0 += 1024) {
      const int s = s0 + tid;
      const int x = s < T ? key[s] : kEmpty;
      const VT v = s < T ? val[s] : VT(0);
      int tot;
      const int pos = pre + group_excl_scan<true, 1024>(x != kEmpty ? 1 : 0, tid, wtot, tot);
      if (x != kEmpty) {
        key[pos] = x;
        val[pos] = v;
      }
      pre += tot;
      __syncthreads();
    }
    if (tid == 0 && pre != nnz) atomicOr(&hdr->status, kStatInvalid);
    __syncthreads();
    // columns are >= 0, so their bit patterns sort like the values
    lds_sort_pairs<true, 1024, VT>(reinterpret_cast<uint32_t *>(key), val, nnz, tid);
    for (int t = tid; t < nnz; t += 1024) {
      ccol[rs + t] = key[t];
      cval[rs + t] = val[t];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Heavy rows (beyond every LDS table) that are not split over many blocks:
// one block of 1024 threads per row; block b owns slot b of the heavy
// scratch.  The symbolic count of every heavy row is k_sym_split's.

// With split rows, the rows left to these kernels are listed (ulist, count
// at *ucount) by the split pass; otherwise they are the row list's rows of
// bins blo and above.
__device__ __forceinline__ const int32_t *heavy_list(const int32_t *rows, const WsHeader *hdr,
                                                     int blo, const int32_t *ulist,
                                                     const int32_t *ucount, int &count) {
  if (ulist) {
    count = *ucount;
    return ulist;
  }
  count = hdr->bin_start[kHeavyBin + 1] - hdr->bin_start[blo];
  return rows + hdr->bin_start[blo];
}

// Numeric pass of heavy rows with the slot's dense accumulator in global
// memory.  One pass over the products marks each column in the bitmap and
// adds the product into the accumulator; then the bitmap is walked in column
// order (so the output row comes out sorted), and each accumulator entry read
// is reset to zero for the slot's next row.
template <bool LDSMAP, typename VT>
__global__ __launch_bounds__(1024) void k_num_heavy(const Problem *__restrict__ pr,
                                                    const int32_t *__restrict__ rows,
                                                    WsHeader *__restrict__ hdr, int blo, int lS,
                                                    uint32_t *gbitmap, VT *gacc,
                                                    const int32_t *__restrict__ crp,
                                                    int32_t *__restrict__ ccol,
                                                    VT *__restrict__ cval,
                                                    const int32_t *ulist, const int32_t *ucount) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int wtot[16];
  __shared__ int sb[1024], sl[1024];
  __shared__ VT sa[1024];
  const int n = pr->n;
  const int nw = (n + 31) >> 5;
  uint32_t *map = LDSMAP ? reinterpret_cast<uint32_t *>(smem_raw) : gbitmap + (size_t)blockIdx.x * nw;
  constexpr int VPV = 16 / sizeof(VT);  // values per 16-byte store
  const size_t astride = (size_t)(n + VPV - 1) / VPV * VPV;  // 16-byte aligned slots
  VT *acc = gacc + (size_t)blockIdx.x * astride;
  if (hdr->status) return;
  int count;
  const int32_t *list = heavy_list(rows, hdr, blo, ulist, ucount, count);
  const int tid = threadIdx.x;
  Stage<VT> st{sb, sl, sa};
  if ((int)blockIdx.x >= count) return;
  // The slot's dense accumulator is cleared once per launch; the output walk
  // resets every entry it reads, so it is all zero again for the next row.
  {
    int4 *a4 = reinterpret_cast<int4 *>(acc);
    const int n4 = (int)(astride / VPV);
    for (int s = tid; s < n4; s += 1024) a4[s] = make_int4(0, 0, 0, 0);
  }
  __shared__ int item;
  for (int ri = block_next(&hdr->queue[kQueueHeavy], &item); ri < count;
       ri = block_next(&hdr->queue[kQueueHeavy], &item)) {
    const int i = list[ri];
    for (int w = tid; w < nw; w += 1024) map[w] = 0u;
    // zeroed accumulator entries visible at device scope before the adds
    __threadfence();
    __syncthreads();
    // one pass: mark the column, add the value
    auto fadd = each_product([&](int col, VT v) {
      const uint32_t bit = 1u << (col & 31);
      if (!(map[col >> 5] & bit)) atomicOr(&map[col >> 5], bit);
      global_add(&acc[col], v);
    });
    for_each_product<true, true, 1024, kUnroll, VT>(pr, i, true, tid, lS, st, fadd);
    // the adds complete at device scope; stale L1 lines are dropped
    __threadfence();
    __syncthreads();
    const int rs = crp[i];
    const int re = crp[i + 1];
    int pre = 0;
    // the bitmap in chunks of 8 words per thread (8192 words per round)
    for (int w0 = 0; w0 < nw; w0 += 8 * 1024) {
      const int wb = w0 + 8 * tid;
      uint32_t wd[8];
      if (LDSMAP && wb + 8 <= nw) {  // two 16-byte LDS reads (the LDS bitmap is 16-byte aligned)
        const uint4 x = reinterpret_cast<const uint4 *>(map + wb)[0];
        const uint4 y = reinterpret_cast<const uint4 *>(map + wb)[1];
        wd[0] = x.x; wd[1] = x.y; wd[2] = x.z; wd[3] = x.w;
        wd[4] = y.x; wd[5] = y.y; wd[6] = y.z; wd[7] = y.w;
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) wd[j] = wb + j < nw ? map[wb + j] : 0u;
      }
      int cnt = 0;
#pragma unroll
      for (int j = 0; j < 8; ++j) cnt += __popc(wd[j]);
      int tot;
      int o = rs + pre + group_excl_scan<true, 1024>(cnt, tid, wtot, tot);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        uint32_t bb = wd[j];
        while (bb) {
          const int col = ((wb + j) << 5) + __ffs(bb) - 1;
          bb &= bb - 1;
          const VT v = acc[col];
          acc[col] = VT(0);
          if (o < re) {  // the symbolic count bounds the row (a changed pattern is flagged)
            ccol[o] = col;
            cval[o] = v;
          }
          ++o;
        }
      }
      pre += tot;
    }
    if (tid == 0 && pre != re - rs) atomicOr(&hdr->status, kStatInvalid);
    __syncthreads();
  }
}

// Numeric pass of heavy rows by column ranges.  The row's products are
// counted per range of W = 2^log2W consecutive columns (LDS counters), a
// block scan gives each range its segment of the slot's staging area, and a
// second enumeration drops every product (column, value) into its range's
// segment.  The ranges are then taken in column order: a range's products
// are added into an LDS panel of W values (a presence bitmap marks the
// columns) and the panel is walked in column order, so the output row comes
// out sorted, with one block scan per non-empty range.  Every atomic stays
// in LDS; the dense global accumulator of k_num_heavy spread the adds of
// all blocks over one accumulator of n values each, far more than L2 holds.
// A row with more products than the staging area holds takes that dense
// path (the slot's memory as accumulator, the panel as bitmap when n fits).
constexpr int kRngMax = 1024;  // column ranges a row may span
constexpr int kRngBuf = 64;    // at most this many ranges get an LDS staging buffer

template <typename VT>
__device__ void heavy_dense_row(const Problem *__restrict__ pr, int i, int lS, Stage<VT> st,
                                uint32_t *map, VT *acc, int n, int *wtot, int rs, int re,
                                int32_t *__restrict__ ccol, VT *__restrict__ cval,
                                WsHeader *__restrict__ hdr) {
  const int tid = threadIdx.x;
  const int nw = (n + 31) >> 5;
  for (int w = tid; w < nw; w += 1024) map[w] = 0u;
  for (int c = tid; c < n; c += 1024) acc[c] = VT(0);
  __threadfence();
  __syncthreads();
  auto fadd = each_product([&](int col, VT v) {
    const uint32_t bit = 1u << (col & 31);
    if (!(map[col >> 5] & bit)) atomicOr(&map[col >> 5], bit);
    global_add(&acc[col], v);
  });
  for_each_product<true, true, 1024, kUnroll, VT>(pr, i, true, tid, lS, st, fadd);
  __threadfence();
  __syncthreads();
  int pre = 0;
  for (int w0 = 0; w0 < nw; w0 += 1024) {
    const int wb = w0 + tid;
    uint32_t wd = wb < nw ? map[wb] : 0u;
    int tot;
    int o = rs + pre + group_excl_scan<true, 1024>(__popc(wd), tid, wtot, tot);
    if (wb < nw) map[wb] = 0u;  // leaves the bitmap (possibly the LDS panel) clear
    while (wd) {
      const int col = (wb << 5) + __ffs(wd) - 1;
      wd &= wd - 1;
      if (o < re) {
        ccol[o] = col;
        cval[o] = acc[col];
      }
      ++o;
    }
    pre += tot;
  }
  if (tid == 0 && pre != re - rs) atomicOr(&hdr->status, kStatInvalid);
  __syncthreads();
}

template <typename VT>
__global__ __launch_bounds__(1024) void k_num_heavy_rng(
    const Problem *__restrict__ pr, const int32_t *__restrict__ rows, WsHeader *__restrict__ hdr,
    int blo, int lS, int log2W, uint32_t *gbitmap, char *slots, size_t slot_bytes,
    const int32_t *__restrict__ crp, int32_t *__restrict__ ccol, VT *__restrict__ cval,
    const int32_t *ulist, const int32_t *ucount) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int W = 1 << log2W;
  VT *panel = reinterpret_cast<VT *>(smem_raw);                 // W values
  uint32_t *pmap = reinterpret_cast<uint32_t *>(panel + W);     // W / 32 words
  __shared__ int rstart[kRngMax + 1];  // range segment starts (exclusive scan of the counts)
  __shared__ int rpos[kRngMax];        // counts, then the next free position of each segment
  __shared__ int bcnt[kRngBuf];        // products in each range's LDS buffer
  __shared__ int wtot[16];
  __shared__ int sb[1024], sl[1024];
  __shared__ VT sa[1024];
  if (hdr->status) return;
  const int n = pr->n;
  int count;
  const int32_t *list = heavy_list(rows, hdr, blo, ulist, ucount, count);
  const int tid = threadIdx.x;
  if ((int)blockIdx.x >= count) return;
  char *slot = slots + (size_t)blockIdx.x * slot_bytes;
  const size_t capz = slot_bytes / (4 + sizeof(VT)) & ~(size_t)1;  // even: values 8-byte aligned
  const int cap = capz < (size_t)INT32_MAX ? (int)capz : INT32_MAX - 1;
  int32_t *scol = reinterpret_cast<int32_t *>(slot);
  VT *sval = reinterpret_cast<VT *>(slot + (size_t)cap * 4);
  const int R = (int)(((int64_t)n + W - 1) >> log2W);  // <= kRngMax (launcher)
  const int nwords = W >> 5;
  Stage<VT> st{sb, sl, sa};
  for (int c = tid; c < W; c += 1024) panel[c] = VT(0);
  for (int w = tid; w < nwords; w += 1024) pmap[w] = 0u;
  __shared__ int item;
  for (int ri = block_next(&hdr->queue[kQueueHeavy], &item); ri < count;
       ri = block_next(&hdr->queue[kQueueHeavy], &item)) {
    const int i = list[ri];
    const int rs = crp[i], re = crp[i + 1];
    // 1. products per range
    for (int r = tid; r < R; r += 1024) rpos[r] = 0;
    __syncthreads();
    auto fcount = each_product([&](int col, VT) { atomicAdd(&rpos[col >> log2W], 1); });
    for_each_product<true, false, 1024, kUnroll, VT>(pr, i, true, tid, lS, st, fcount);
    __syncthreads();
    // 2. segment starts (R <= 1024: one range per thread)
    int P;
    {
      const int c = tid < R ? rpos[tid] : 0;
      int tot;
      const int off = group_excl_scan<true, 1024>(c, tid, wtot, tot);
      if (tid < R) {
        rstart[tid] = off;
        rpos[tid] = off;
      }
      if (tid == 0) rstart[R] = tot;
      P = tot;
      __syncthreads();
    }
    if (P > cap) {  // more products than the staging area holds
      uint32_t *map = n <= W * (int)sizeof(VT) * 8 ? reinterpret_cast<uint32_t *>(panel)
                                                   : gbitmap + (size_t)blockIdx.x * ((n + 31) >> 5);
      heavy_dense_row<VT>(pr, i, lS, st, map, reinterpret_cast<VT *>(slot), n, wtot, rs, re, ccol,
                          cval, hdr);
      continue;
    }
    // 3. every product into its range's segment.  With few ranges the idle
    // panel holds a buffer per range, flushed to the segment with coalesced
    // stores; products past a full buffer go to the segment directly.
    if (R <= kRngBuf)
      for (int r = tid; r < R; r += 1024) bcnt[r] = 0;
    __syncthreads();
    const int bcap = R <= kRngBuf ? (int)(((size_t)W * sizeof(VT) / (4 + sizeof(VT)) / R) & ~1) : 0;
    int32_t *bufc = reinterpret_cast<int32_t *>(panel);
    VT *bufv = reinterpret_cast<VT *>(bufc + (size_t)R * bcap);
    auto fput = each_product([&](int col, VT v) {
      const int r = col >> log2W;
      const int b = bcap > 0 ? atomicAdd(&bcnt[r], 1) : 0;
      if (b < bcap) {
        bufc[r * bcap + b] = col;
        bufv[r * bcap + b] = v;
      } else {
        const int p = atomicAdd(&rpos[r], 1);
        scol[p] = col;
        sval[p] = v;
      }
    });
    for_each_product<true, true, 1024, kUnroll, VT>(pr, i, true, tid, lS, st, fput);
    __syncthreads();
    if (bcap > 0) {
      for (int r = 0; r < R; ++r) {  // buffered products after the direct ones
        const int nb = min(bcnt[r], bcap), base = rpos[r];
        for (int t = tid; t < nb; t += 1024) {
          scol[base + t] = bufc[r * bcap + t];
          sval[base + t] = bufv[r * bcap + t];
        }
      }
      __syncthreads();
      for (int c = tid; c < W; c += 1024) panel[c] = VT(0);  // the panel starts clear
    }
    __threadfence();  // the staged pairs are read back by other threads of the block
    __syncthreads();
    // 4. the ranges in column order
    int o = rs;
    for (int r = 0; r < R; ++r) {
      const int s0 = rstart[r], s1 = rstart[r + 1];
      if (s0 == s1) continue;  // same value in every thread
      const int base = r << log2W;
      for (int p = s0 + tid; p < s1; p += 1024) {
        const int cl = scol[p] - base;
        lds_add_cas(&panel[cl], sval[p]);
        atomicOr(&pmap[cl >> 5], 1u << (cl & 31));
      }
      __syncthreads();
      uint32_t wd = tid < nwords ? pmap[tid] : 0u;
      int tot;
      int off = o + group_excl_scan<true, 1024>(__popc(wd), tid, wtot, tot);
      if (tid < nwords) pmap[tid] = 0u;
      while (wd) {
        const int cl = (tid << 5) + __ffs(wd) - 1;
        wd &= wd - 1;
        const VT v = panel[cl];
        panel[cl] = VT(0);
        if (off < re) {  // the symbolic count bounds the row (a changed pattern is flagged)
          ccol[off] = base + cl;
          cval[off] = v;
        }
        ++off;
      }
      o += tot;
      __syncthreads();
    }
    if (tid == 0 && o != re) atomicOr(&hdr->status, kStatInvalid);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Launchers.

static int blocks_per_cu(size_t lds, int wg, size_t lds_limit_cu) {
  int by_lds = lds ? (int)(lds_limit_cu / lds) : 64;
  int by_thr = 2048 / wg;
  int b = by_lds < by_thr ? by_lds : by_thr;
  return b < 1 ? 1 : b;
}

static int wg_for(int G) { return G <= kWave ? 256 : G; }

static int log2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Bytes of one heavy slot in the workspace's heavy region.
static size_t heavy_slot_bytes(int n) { return ((size_t)(n > 1 ? n : 1) + 4) * 8; }

// Static LDS of k_num_heavy_rng (range starts and cursors, scan partials,
// staged entries).
template <typename VT>
static size_t heavy_rng_static_lds() {
  return (size_t)(kRngMax + 1) * 4 + (size_t)kRngMax * 4 + (size_t)kRngBuf * 4 + 16 * 4 +
         (size_t)1024 * (8 + sizeof(VT)) + 256;  // alignment padding
}

// A heavy row's column bitmap lives in LDS when it fits one block.
static bool lds_bitmap_fits(int n, size_t extra) {
  return n <= kLdsBitmapCols &&
         (size_t)((n + 31) >> 5) * 4 + extra + 1024 <= dev_info().lds_per_block;
}

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

// B-row lanes per entry, never more than the group.
static int sub_log2(const BinPlan &bp, int b, int G) {
  int S = bp.sub[b] > 0 ? bp.sub[b] : 16;
  if (S > G) S = G;
  return log2i(S);
}

size_t sym_lds_bytes(int b, int G) {
  const int WG = wg_for(G), R = WG / G;
  return (size_t)R * bin_slots(b) * 4 + (size_t)2 * R * G * 4 + (size_t)R * 4 + 64;
}

// Table slots of a numeric row: T + at least kTail, a multiple of G (block
// groups: G times an odd chunk length, read without LDS bank conflicts).
int num_table_slots(int b, int G) {
  int c = (bin_slots(b) + kTail + G - 1) / G;
  if (G > kWave && !(c & 1)) ++c;  // block groups read chunks of c slots
  return c * G;
}

// Table slots of the numeric kernel: T plus the probe tail, a multiple of 64
// (its output reads rounds of 64 slots; block groups split them by wave).
int num_rows_slots(int b) { return (bin_slots(b) + kTail + kWave - 1) / kWave * kWave; }

size_t num_lds_bytes(int b, int G, size_t vbytes, bool pack) {
  const int WG = wg_for(G), R = WG / G;
  const size_t TT = (size_t)num_rows_slots(b);
  return (size_t)R * TT * (vbytes + (pack ? 4 : 8)) + (size_t)R * G * (vbytes + 8) +
         (size_t)R * 4 + 64;
}

template <int G>
static void sym_launch(const Problem *dpr, const int32_t *rows, const WsHeader *hdr, int bin,
                       int lS, int log2T, int32_t *cnt, int grid, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL(k_sym_rows<G>, dim3(grid), dim3(Geom<G>::WG), lds, st, dpr, rows, hdr, bin,
                     lS, log2T, cnt);
}

hipError_t launch_symbolic_bins(const Problem *dpr, const BinPlan &bp, const WsLayout &L,
                                char *ws, int32_t *cnt, hipStream_t st) {
  WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
  const int32_t *rows = reinterpret_cast<const int32_t *>(ws + L.rows);
  const DevInfo &D = dev_info();
  // rows from the split bin on are counted (and described) by the split
  // kernel; without a split region only the rows beyond every LDS bin are
  const bool split = L.split_F > 0 && D.split_bin <= bp.maxbin + 1;
  const int sbin = split ? D.split_bin : bp.maxbin + 1;
  for (int b = 1; b < sbin; ++b) {
    if (bp.known && bp.count[b] == 0) continue;
    int G = bp.lanes[b];
    if (G == 1 && b == 1) {  // one thread per row
      launch_sym_tiny(dpr, rows, hdr, b, bins_count(bp, b, b), bp.known, cnt, st);
      continue;
    }
    if (G < 8) G = 8;
    if (G == kWave && sym_wave_lds_bytes(b) <= D.lds_per_block) {
      launch_sym_wave(dpr, rows, hdr, b, sub_log2(bp, b, G), bins_count(bp, b, b), cnt, st);
      continue;
    }
    while (G < 1024 && sym_lds_bytes(b, G) > D.lds_per_block) G *= 2;  // fewer rows per block
    const int WG = wg_for(G);
    const int R = WG / G;
    const size_t lds = sym_lds_bytes(b, G);
    const int grid = grid_for(bins_count(bp, b, b), R, D.cus * blocks_per_cu(lds, WG, D.lds_per_cu));
    const int lt = log2i(bin_slots(b));
    const int lS = sub_log2(bp, b, G);
    switch (G) {
      case 8: sym_launch<8>(dpr, rows, hdr, b, lS, lt, cnt, grid, lds, st); break;
      case 16: sym_launch<16>(dpr, rows, hdr, b, lS, lt, cnt, grid, lds, st); break;
      case 32: sym_launch<32>(dpr, rows, hdr, b, lS, lt, cnt, grid, lds, st); break;
      case 64: sym_launch<64>(dpr, rows, hdr, b, lS, lt, cnt, grid, lds, st); break;
      case 128: sym_launch<128>(dpr, rows, hdr, b, lS, lt, cnt, grid, lds, st); break;
      case 256: sym_launch<256>(dpr, rows, hdr, b, lS, lt, cnt, grid, lds, st); break;
      case 512: sym_launch<512>(dpr, rows, hdr, b, lS, lt, cnt, grid, lds, st); break;
      default: sym_launch<1024>(dpr, rows, hdr, b, lS, lt, cnt, grid, lds, st); break;
    }
  }
  const int hc = bins_count(bp, sbin, kHeavyBin);
  if (hc != 0) {
    const int grid = grid_for(hc, 1, bp.heavy_slots);
    const int lS = sub_log2(bp, kHeavyBin, 1024);
    SplitArgs sa = split_args(L, ws, sbin);
    if (!split) sa.F = 0;
    const bool ldsmap = lds_bitmap_fits(bp.n, split_sym_static_lds());
    return launch_sym_split(dpr, rows, hdr, sbin, lS, ldsmap,
                            reinterpret_cast<uint32_t *>(ws + L.heavymap), grid,
                            ldsmap ? (size_t)((bp.n + 31) >> 5) * 4 : 0, cnt, sa, st);
  }
  return hipGetLastError();
}

template <int G, typename VT, bool PACK>
static void num_launch(const Problem *dpr, const int32_t *rows, WsHeader *hdr, int bin, int lS,
                       int TT, uint32_t mul, int maxwin, const int32_t *crp, int32_t *ccol,
                       VT *cval, int32_t *fb, int grid, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL((k_num_rows<G, VT, PACK>), dim3(grid), dim3(Geom<G>::WG), lds, st, dpr,
                     rows, hdr, bin, lS, TT, mul, maxwin, crp, ccol, cval, fb);
}

template <typename VT, bool PACK>
static void num_launch_g(int G, const Problem *dpr, const int32_t *rows, WsHeader *hdr, int bin,
                         int lS, int TT, uint32_t mul, int maxwin, const int32_t *crp,
                         int32_t *ccol, VT *cval, int32_t *fb, int grid, size_t lds,
                         hipStream_t st) {
  switch (G) {
#define SPG_NUM_CASE(g) \
  case g: num_launch<g, VT, PACK>(dpr, rows, hdr, bin, lS, TT, mul, maxwin, crp, ccol, cval, fb, grid, lds, st); break;
    SPG_NUM_CASE(8)
    SPG_NUM_CASE(16)
    SPG_NUM_CASE(32)
    SPG_NUM_CASE(64)
    SPG_NUM_CASE(128)
    SPG_NUM_CASE(256)
    SPG_NUM_CASE(512)
    default: num_launch<1024, VT, PACK>(dpr, rows, hdr, bin, lS, TT, mul, maxwin, crp, ccol, cval, fb, grid, lds, st);
#undef SPG_NUM_CASE
  }
}

template <typename VT>
static hipError_t numeric_impl(const Problem *dpr, const BinPlan &bp, const WsLayout &L,
                               char *ws, const int32_t *crp, int32_t *ccol, VT *cval,
                               hipStream_t st) {
  WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
  const int32_t *rows = reinterpret_cast<const int32_t *>(ws + L.rows);
  int32_t *fb = reinterpret_cast<int32_t *>(ws + L.fbrows);
  const DevInfo &D = dev_info();
  const int maxwin = bp.maxwin < kTail ? bp.maxwin : kTail;
  const bool pack = bp.n <= (1 << 24);
  for (int b = 1; b <= bp.maxbin; ++b) {
    if (bp.known && bp.count[b] == 0) continue;
    int G = bp.lanes[b];
    if (G == 1 && b == 1) {  // one thread per row
      launch_num_tiny(dpr, rows, hdr, b, bins_count(bp, b, b), bp.known, crp, ccol, cval,
                      sizeof(VT) == 8, st);
      continue;
    }
    if (G < 8) G = 8;
    if (G == kWave && num_wave_lds_bytes(b, sizeof(VT), pack) <= D.lds_per_block) {
      launch_num_wave(dpr, rows, hdr, b, sub_log2(bp, b, G), bins_count(bp, b, b),
                      mono_mul(bin_slots(b), bp.n), maxwin, pack, crp, ccol, cval,
                      sizeof(VT) == 8, fb, st);
      continue;
    }
    if (pack && G > kWave && bucket_blk_ok(b, G) &&
        bucket_blk_lds(b, G, sizeof(VT)) <= D.lds_per_block) {
      const size_t lds = bucket_blk_lds(b, G, sizeof(VT));
      const int grid = grid_for(bins_count(bp, b, b), 1, D.cus * blocks_per_cu(lds, G, D.lds_per_cu));
      const int T = 8 << b;
      const uint32_t mul = mono_mul(T, bp.n);
      const int lS = sub_log2(bp, b, G);
      const int cap = bucket_blk_cap(b);
      switch (G) {
#define SPG_BKT_CASE(g)                                                                        \
  case g:                                                                                      \
    hipLaunchKernelGGL((k_num_bucket_blk<g, VT>), dim3(grid), dim3(g), lds, st, dpr, rows, hdr, \
                       b, lS, T, cap, mul, crp, ccol, cval, fb);                               \
    break;
        SPG_BKT_CASE(128)
        SPG_BKT_CASE(256)
        SPG_BKT_CASE(512)
        default:
          hipLaunchKernelGGL((k_num_bucket_blk<1024, VT>), dim3(grid), dim3(1024), lds, st, dpr,
                             rows, hdr, b, lS, T, cap, mul, crp, ccol, cval, fb);
#undef SPG_BKT_CASE
      }
      continue;
    }
    while (G < 1024 && num_lds_bytes(b, G, sizeof(VT), pack) > D.lds_per_block) G *= 2;
    const int WG = wg_for(G);
    const int R = WG / G;
    const int T = bin_slots(b);
    const int TT = num_rows_slots(b);
    const size_t lds = num_lds_bytes(b, G, sizeof(VT), pack);
    const int grid = grid_for(bins_count(bp, b, b), R, D.cus * blocks_per_cu(lds, WG, D.lds_per_cu));
    const uint32_t mul = mono_mul(T, bp.n);
    const int lS = sub_log2(bp, b, G);
    if (pack)
      num_launch_g<VT, true>(G, dpr, rows, hdr, b, lS, TT, mul, maxwin, crp, ccol, cval, fb, grid, lds, st);
    else
      num_launch_g<VT, false>(G, dpr, rows, hdr, b, lS, TT, mul, maxwin, crp, ccol, cval, fb, grid, lds, st);
  }
  if (bins_count(bp, 1, bp.maxbin) != 0) {
    // rows the LDS kernels hand over (probe longer than the window)
    const int TF = bin_slots(bp.maxbin);
    const size_t lds = (size_t)TF * (sizeof(VT) + 4) + (size_t)1024 * (sizeof(VT) + 8);
    hipLaunchKernelGGL(k_num_fallback<VT>, dim3(D.cus), dim3(1024), lds, st, dpr, fb, hdr, TF,
                       sub_log2(bp, bp.maxbin, 1024), crp, ccol, cval);
  }
  const int hc = bins_count(bp, bp.maxbin + 1, kHeavyBin);
  if (hc != 0) {
    const int grid = grid_for(hc, 1, bp.heavy_slots);
    VT *acc = reinterpret_cast<VT *>(ws + L.heavyacc);
    const int lS = sub_log2(bp, kHeavyBin, 1024);
    // rows split over many blocks first (their staging shares the heavy
    // region with the one-block kernels below, which skip them)
    const int32_t *ulist = nullptr, *ucount = nullptr;
    if (L.split_F > 0 && D.split_bin <= bp.maxbin + 1) {
      const SplitArgs sa = split_args(L, ws, D.split_bin);
      // the rows left over are listed where the fallback rows were (the
      // fallback kernel above has finished with them)
      hipError_t e = launch_num_split(dpr, rows, hdr, bp.maxbin + 1,
                                      sub_log2(bp, kHeavyBin, kWave * 4), sa, fb, crp, ccol,
                                      cval, sizeof(VT) == 8, st);
      if (e != hipSuccess) return e;
      ulist = fb;
      ucount = &sa.ctl->nuns;
    }
    const int log2W = sizeof(VT) == 4 ? 15 : 14;  // a 128 KiB panel
    const size_t rlds = ((size_t)sizeof(VT) << log2W) + ((size_t)4 << (log2W - 5));
    if ((int64_t)bp.n <= ((int64_t)kRngMax << log2W) &&
        rlds + heavy_rng_static_lds<VT>() <= D.lds_per_block) {
      hipLaunchKernelGGL((k_num_heavy_rng<VT>), dim3(grid), dim3(1024), rlds, st, dpr, rows, hdr,
                         bp.maxbin + 1, lS, log2W, reinterpret_cast<uint32_t *>(ws + L.heavymap),
                         ws + L.heavyacc, heavy_slot_bytes(bp.n), crp, ccol, cval, ulist, ucount);
    } else if (lds_bitmap_fits(bp.n, 8 * 1024 + 1024 * sizeof(VT))) {
      const size_t lds = (size_t)((bp.n + 31) >> 5) * 4;
      hipLaunchKernelGGL((k_num_heavy<true, VT>), dim3(grid), dim3(1024), lds, st, dpr, rows,
                         hdr, bp.maxbin + 1, lS, (uint32_t *)nullptr, acc, crp, ccol, cval, ulist,
                         ucount);
    } else {
      hipLaunchKernelGGL((k_num_heavy<false, VT>), dim3(grid), dim3(1024), 0, st, dpr, rows, hdr,
                         bp.maxbin + 1, lS, reinterpret_cast<uint32_t *>(ws + L.heavymap), acc,
                         crp, ccol, cval, ulist, ucount);
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
template <typename VT, bool PACK>
static void num_kernels(std::vector<const void *> &ks) {
  ks.push_back(reinterpret_cast<const void *>(&k_num_rows<8, VT, PACK>));
  ks.push_back(reinterpret_cast<const void *>(&k_num_rows<16, VT, PACK>));
  ks.push_back(reinterpret_cast<const void *>(&k_num_rows<32, VT, PACK>));
  ks.push_back(reinterpret_cast<const void *>(&k_num_rows<64, VT, PACK>));
  ks.push_back(reinterpret_cast<const void *>(&k_num_rows<128, VT, PACK>));
  ks.push_back(reinterpret_cast<const void *>(&k_num_rows<256, VT, PACK>));
  ks.push_back(reinterpret_cast<const void *>(&k_num_rows<512, VT, PACK>));
  ks.push_back(reinterpret_cast<const void *>(&k_num_rows<1024, VT, PACK>));
  if (PACK) {
    ks.push_back(reinterpret_cast<const void *>(&k_num_bucket_blk<128, VT>));
    ks.push_back(reinterpret_cast<const void *>(&k_num_bucket_blk<256, VT>));
    ks.push_back(reinterpret_cast<const void *>(&k_num_bucket_blk<512, VT>));
    ks.push_back(reinterpret_cast<const void *>(&k_num_bucket_blk<1024, VT>));
  }
}

hipError_t configure_lds_limits(size_t lds_max) {
  std::vector<const void *> ks = {
      reinterpret_cast<const void *>(&k_sym_rows<8>),
      reinterpret_cast<const void *>(&k_sym_rows<16>),
      reinterpret_cast<const void *>(&k_sym_rows<32>),
      reinterpret_cast<const void *>(&k_sym_rows<64>),
      reinterpret_cast<const void *>(&k_sym_rows<128>),
      reinterpret_cast<const void *>(&k_sym_rows<256>),
      reinterpret_cast<const void *>(&k_sym_rows<512>),
      reinterpret_cast<const void *>(&k_sym_rows<1024>),
      reinterpret_cast<const void *>(&k_num_fallback<float>),
      reinterpret_cast<const void *>(&k_num_fallback<double>),
      reinterpret_cast<const void *>(&k_num_heavy<true, float>),
      reinterpret_cast<const void *>(&k_num_heavy<true, double>),
      reinterpret_cast<const void *>(&k_num_heavy_rng<float>),
      reinterpret_cast<const void *>(&k_num_heavy_rng<double>),
  };
  num_kernels<float, true>(ks);
  num_kernels<float, false>(ks);
  num_kernels<double, true>(ks);
  num_kernels<double, false>(ks);
  for (const void *k : ks) {
    hipError_t e =
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace spg

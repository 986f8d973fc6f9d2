// Row-level building blocks shared by the row kernels: group
// synchronisation and scans, and the enumeration of every scalar product
// a_ik * b_kj that lands in row i of C = sum_k A_k B_k.
#pragma once

#include "common.hpp"

namespace spg {

// A "group" is the set of lanes working on one row.  Groups of at most 64
// lanes sit inside one wave (lanes [g0, g0+G)) and run independently of the
// wave's other groups; larger groups are a whole block.  group_sync orders
// the group's LDS accesses.
template <bool BLOCK>
__device__ __forceinline__ void group_sync() {
  if (BLOCK) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

__device__ __forceinline__ uint64_t lanes_below() {
  const int lane = lane_id();
  return lane == 0 ? 0ull : (~0ull >> (kWave - lane));
}

// Exclusive prefix sum of v over the group's lanes (l = lane in group);
// `total` gets the group sum.  BLOCK groups use wtot[blockDim/64] in LDS.
template <bool BLOCK, int G>
__device__ __forceinline__ int group_excl_scan(int v, int l, int *wtot, int &total) {
  int x = v;
  if (!BLOCK) {
#pragma unroll
    for (int off = 1; off < G; off <<= 1) {
      const int y = __shfl_up(x, off, G);
      if (l >= off) x += y;
    }
    total = __shfl(x, G - 1, G);
    return x - v;
  }
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int y = __shfl_up(x, off);
    if (lane_id() >= off) x += y;
  }
  const int w = threadIdx.x / kWave;
  if (lane_id() == kWave - 1) wtot[w] = x;
  __syncthreads();
  int pre = 0, tot = 0;
#pragma unroll
  for (int ww = 0; ww < G / kWave; ++ww) {
    const int c = wtot[ww];
    pre += (ww < w) ? c : 0;
    tot += c;
  }
  __syncthreads();
  total = tot;
  return pre + x - v;
}

// Group-wide sum / max.  BLOCK groups reduce through red[blockDim/64].
template <bool BLOCK, int G, typename T>
__device__ __forceinline__ T group_sum(T v, T *red) {
  if (!BLOCK) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
    return v;
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (lane_id() == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  T t = T(0);
#pragma unroll
  for (int w = 0; w < G / kWave; ++w) t += red[w];
  __syncthreads();
  return t;
}

template <bool BLOCK, int G>
__device__ __forceinline__ unsigned long long group_max_u64(unsigned long long v,
                                                           unsigned long long *red) {
  if (!BLOCK) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
      const unsigned long long o = __shfl_xor(v, off, G);
      v = o > v ? o : v;
    }
    return v;
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  if (lane_id() == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  unsigned long long t = 0;
#pragma unroll
  for (int w = 0; w < G / kWave; ++w) t = red[w] > t ? red[w] : t;
  __syncthreads();
  return t;
}

// Sorts key[0..P) ascending, carrying val, in LDS.  A bitonic network in
// the form whose every compare-exchange moves the smaller key to the lower
// position (each merge starts by comparing mirrored positions of its
// block), so the positions past P behave as +infinity and are never
// touched: no padding, any P.  The NT lanes t = 0..NT-1 of the group share
// the pairs of each step; group_sync separates the steps.
template <bool BLOCK, int NT, typename VT>
__device__ void lds_sort_pairs(uint32_t *key, VT *val, int P, int t) {
  int ln = 0;
  while ((1 << ln) < P) ++ln;
  const int half = (1 << ln) >> 1;
  // block sizes and distances are powers of two: shifts and masks, no division
  for (int lk = 1; lk <= ln; ++lk) {
    const int k = 1 << lk;
    for (int lj = lk - 1; lj >= 0; --lj) {
      const int j = 1 << lj;
      for (int q = t; q < half; q += NT) {
        int a, b;
        if (lj == lk - 1) {  // mirrored positions of a block of k
          const int base = (q >> lj) << lk, off = q & (j - 1);
          a = base + off;
          b = base + k - 1 - off;
        } else {  // half-cleaner at distance j
          a = ((q >> lj) << (lj + 1)) + (q & (j - 1));
          b = a + j;
        }
        if (b < P) {
          const uint32_t ka = key[a], kb = key[b];
          if (ka > kb) {
            key[a] = kb;
            key[b] = ka;
            const VT va = val[a];
            val[a] = val[b];
            val[b] = va;
          }
        }
      }
      group_sync<BLOCK>();
    }
  }
}

// Buckets larger than this are not sorted one bucket per lane: the bucket
// kernels sort the whole row instead (columns that cluster in a few
// buckets, as in banded matrices).
constexpr int kBigBucket = 16;

// Key word of the numeric tables.  PACK (n <= 2^24): the column in the low
// 24 bits and a rank counter biased by 128 in the top byte.
template <bool PACK>
struct KeyCode {
  __device__ static int make(int col) { return PACK ? (int)((uint32_t)col | 0x80000000u) : col; }
  __device__ static int col(int w) { return PACK ? (int)((uint32_t)w & 0xffffffu) : w; }
  __device__ static int adj(int w) { return PACK ? (int)((uint32_t)w >> 24) - 128 : 0; }
};

// FP32 numeric tables keep a key word and its value in one 64-bit slot (key
// in the low half, value bits in the high half).  A column's first insert
// writes both with one 64-bit compare-and-swap, so no lane can see the key
// before the value; a repeat adds its value with a compare-and-swap loop on
// the slot.  LDS float atomics are slow on this chip, and repeats are rare
// for most rows, so nearly every product costs one LDS atomic and no fence.
// The rank counters of PACK keys are updated with 64-bit adds on the slot:
// the counter byte stays within [128 - 2*kTail, 128 + 2*kTail], so no carry
// or borrow reaches the value half.
constexpr unsigned long long kEmptySlot = 0xffffffffull;  // key kEmpty, value 0

__device__ __forceinline__ unsigned long long slot_make(int kw, float v) {
  return ((unsigned long long)__float_as_uint(v) << 32) | (uint32_t)kw;
}
__device__ __forceinline__ int slot_key(unsigned long long s) { return (int)(uint32_t)s; }
__device__ __forceinline__ float slot_val(unsigned long long s) {
  return __uint_as_float((uint32_t)(s >> 32));
}

// Inserts N products per lane (col < 0: none) into an order-preserving FP32
// slot table with forward probing of at most maxwin slots (*flag = 1 when a
// probe is longer: the row is redone elsewhere), then lets every displaced
// first insert count the larger keys on its probe path (rank counters).  The
// first probes of all N products are issued before any result is examined.
template <bool PACK, int N>
__device__ __forceinline__ void slot_insert(unsigned long long *slot, int *adj, int *flag,
                                            uint32_t mul, int maxwin, const int (&col)[N],
                                            const float (&v)[N]) {
  using KC = KeyCode<PACK>;
  int h[N], d[N];
  unsigned long long old[N];
#pragma unroll
  for (int u = 0; u < N; ++u) {
    h[u] = (int)mono_slot((uint32_t)col[u], mul);
    old[u] = col[u] >= 0 ? atomicCAS(&slot[h[u]], kEmptySlot, slot_make(KC::make(col[u]), v[u]))
                         : kEmptySlot;
  }
#pragma unroll
  for (int u = 0; u < N; ++u) {
    d[u] = 0;
    if (col[u] < 0) continue;
    while (old[u] != kEmptySlot) {
      if (KC::col(slot_key(old[u])) == col[u]) {  // repeat: add into the slot
        unsigned long long cur = old[u];
        while (true) {
          const unsigned long long nw =
              (cur & 0xffffffffull) |
              ((unsigned long long)__float_as_uint(slot_val(cur) + v[u]) << 32);
          const unsigned long long got = atomicCAS(&slot[h[u]], cur, nw);
          if (got == cur) break;
          cur = got;
        }
        d[u] = -1;
        break;
      }
      if (d[u] == maxwin) {  // long probe: the row is redone elsewhere
        *flag = 1;
        d[u] = -1;
        break;
      }
      ++d[u];
      ++h[u];  // h <= home + maxwin < table size
      old[u] = atomicCAS(&slot[h[u]], kEmptySlot, slot_make(KC::make(col[u]), v[u]));
    }
  }
#pragma unroll
  for (int u = 0; u < N; ++u) {
    if (col[u] < 0 || d[u] <= 0) continue;  // displaced first inserts only
    int larger = 0;
    for (int t = h[u] - d[u]; t < h[u]; ++t) {
      if (KC::col(slot_key(slot[t])) > col[u]) {
        if (PACK) atomicAdd(&slot[t], 1ull << 24);
        else atomicAdd(&adj[t], 1);
        ++larger;
      }
    }
    if (larger) {
      if (PACK) atomicAdd(&slot[h[u]], 0ull - ((unsigned long long)larger << 24));
      else atomicSub(&adj[h[u]], larger);
    }
  }
}

// Staging area of one group in LDS: one A entry per lane of a chunk.
template <typename VT>
struct Stage {
  int *b0;   // start of the B row in bcol/bval
  int *len;  // length of the B row
  VT *a;     // value a_ik
};

// Hands every product (col, a_ik * b_kj) of row i of A_k B_k (one part) to
// f.batch<N>(cols, vals) (N products per lane at once, col < 0 = no
// product), so that f can issue the LDS operations of N products before
// waiting on any of them.  The entries of the A row are taken in chunks of
// G: lane l stages entry c0+l in LDS (one coalesced read of A, one gather of
// B row bounds).  Then S = 2^lS lanes share each entry (S grows while the
// chunk's entries leave lanes idle: few entries with long B rows): lane l
// reads position (l mod S) of the B rows of entries l/S, l/S + G/S, ..., U
// entries at a time so that U loads are in flight together, and consecutive
// lanes read consecutive B entries.  Positions beyond S (B rows longer than
// S) follow in a second loop.  [elo, ehi) restricts the row to a window of
// its entries (a row shared by several blocks).
template <bool BLOCK, bool VALUES, int G, int U, typename VT, typename F>
__device__ __forceinline__ void part_products(const Part &P, int i, bool active, int l, int lS,
                                              Stage<VT> st, F &f, int cfirst = 0,
                                              int cstep = 1, int elo = 0,
                                              int ehi = 0x7fffffff) {
  const SPG_GLOBAL int32_t *brp = gp(P.brp);
  const SPG_GLOBAL int32_t *bcol = gp(P.bcol);
  const SPG_GLOBAL VT *bval = gp(static_cast<const VT *>(P.bval));
  int as = 0, ae = 0;
  if (active) a_row(P, i, as, ae);
  if (ehi < ae - as) ae = as + ehi;
  as += elo;
  const int nA = ae > as ? ae - as : 0;
  for (int c0 = cfirst * G; c0 < nA; c0 += cstep * G) {
    const int e = c0 + l;
    if (e < nA) {
      int r;
      VT a = VT(1);
      if (P.a_identity) {
        r = i;
      } else {
        r = gp(P.acol)[as + e];
        if (VALUES) a = gp(static_cast<const VT *>(P.aval))[as + e];
      }
      const int b0 = brp[r];
      st.b0[l] = b0;
      st.len[l] = brp[r + 1] - b0;
      if (VALUES) st.a[l] = a;
    }
    const int nE = min(G, nA - c0);
    int lSr = lS;
    while (lSr < 6 && (nE << (lSr + 1)) <= G) ++lSr;
    const int S = 1 << lSr;
    const int ES = G >> lSr;
    const int sg = l >> lSr;
    const int q0 = l & (S - 1);
    group_sync<BLOCK>();
    for (int t0 = sg; t0 < nE; t0 += ES * U) {
      // all LDS reads first, then all global loads, then the products: no
      // consumer sits between the U loads, so they are in flight together
      int col[U], b0[U], len[U];
      VT v[U], a[U], bv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int ee = t0 + ES * u;
        const int ec = ee < nE ? ee : 0;
        b0[u] = st.b0[ec];
        len[u] = ee < nE ? st.len[ec] : 0;
        if (VALUES) a[u] = st.a[ec];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        col[u] = -1;
        bv[u] = VT(0);
        if (q0 < len[u]) {
          col[u] = bcol[b0[u] + q0];
          if (VALUES) bv[u] = bval[b0[u] + q0];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = VALUES ? a[u] * bv[u] : VT(0);
      f.template batch<U>(col, v);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        for (int q = q0 + S; q < len[u]; q += S) {
          const int idx = b0[u] + q;
          int c1[1] = {bcol[idx]};
          VT v1[1] = {VALUES ? a[u] * bval[idx] : VT(0)};
          f.template batch<1>(c1, v1);
        }
      }
    }
    group_sync<BLOCK>();
  }
}

// All products of row i of C = sum_k A_k B_k.  A row handled by a whole
// block with K > 1 parts lets its waves run independently on different
// parts, so the parts' chains of dependent loads overlap instead of
// following each other: wave w takes parts w, w + waves, ...  A 1024-lane
// block with fewer parts than waves instead splits the parts' entries into
// chunks of 64 and deals the (part, chunk) items out to the waves, so that
// none idles.  The waves share the block's table and meet at one barrier at
// the end.
template <bool BLOCK, bool VALUES, int G, int U, typename VT, typename F>
__device__ __forceinline__ void for_each_product(const Problem *__restrict__ pr, int i,
                                                 bool active, int l, int lS, Stage<VT> st,
                                                 F &f) {
  const int K = pr->K;
  if (BLOCK && K > 1) {
    constexpr int NWV = G / kWave;
    const int w = l / kWave, lw = l % kWave;
    Stage<VT> sw{st.b0 + w * kWave, st.len + w * kWave, VALUES ? st.a + w * kWave : st.a};
    // every wave has a part of its own (or the block is small): wave w takes
    // parts w, w + NWV, ...  Only the 1024-lane kernels carry the split
    // below; it costs the smaller ones more in code than it saves.
    if (G < 1024 || K >= NWV) {
      for (int k = w; k < K; k += NWV)
        part_products<false, VALUES, kWave, U, VT>(pr->part[k], i, active, lw, lS, sw, f);
      group_sync<true>();
      return;
    }
    if constexpr (G >= 1024) {
      // wave w takes items w, w + NWV, ...: item j is chunk c of part k, with
      // the items numbered part by part.  Lane k < K holds part k's chunk
      // count; an inclusive wave scan gives the first item after each part.
      int nc = 0;
      if (lw < K) {
        int as = 0, ae = 0;
        if (active) a_row(pr->part[lw], i, as, ae);
        nc = (ae - as + kWave - 1) / kWave;
      }
      int incl = nc;
#pragma unroll
      for (int off = 1; off < SPG_MAX_PARTS; off <<= 1) {
        const int y = __shfl_up(incl, off);
        if (lw >= off) incl += y;
      }
      const int total = __shfl(incl, K - 1);
      for (int j = w; j < total; j += NWV) {
        // part of item j: the number of parts whose items all precede j
        // wave-uniform: keeps the part's pointers in scalar registers
        const int k = __builtin_amdgcn_readfirstlane(__popcll(__ballot(lw < K && incl <= j)));
        const int before = __builtin_amdgcn_readfirstlane(k > 0 ? __shfl(incl, k - 1) : 0);
        part_products<false, VALUES, kWave, U, VT>(pr->part[k], i, active, lw, lS, sw, f,
                                                   j - before, 1 << 24);
      }
    }
    group_sync<true>();
    return;
  }
  for (int k = 0; k < K; ++k)
    part_products<BLOCK, VALUES, G, U, VT>(pr->part[k], i, active, l, lS, st, f);
}

// Adapter for per-product callbacks: f(col, val) for each valid product.
template <typename F>
struct EachProduct {
  F f;
  template <int N, typename VT>
  __device__ __forceinline__ void batch(const int (&col)[N], const VT (&v)[N]) {
#pragma unroll
    for (int u = 0; u < N; ++u)
      if (col[u] >= 0) f(col[u], v[u]);
  }
};
template <typename F>
__device__ __forceinline__ EachProduct<F> each_product(F f) {
  return EachProduct<F>{f};
}

}  // namespace spg

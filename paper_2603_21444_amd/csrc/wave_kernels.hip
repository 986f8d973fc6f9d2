// One-row-per-wave kernels of the symbolic (a3) and numeric (a5) passes with
// a software pipeline across rows.
//
// A row's work starts with a chain of dependent loads (row id -> A row
// pointers -> A entries -> B row bounds) before its products can be
// gathered.  With one row in flight per wave and the number of waves per CU
// capped by LDS, that chain was exposed on every row.  Here each wave walks
// the chain of its NEXT row one link per phase of the current row (after the
// table clear, after the inserts, after the output), so by the time the next
// row starts its A entries and B row bounds are already in registers: lane e
// holds entry e of the first 64 entries of the row's first block product.
// Entries beyond the first 64, and further block products (K > 1), are
// staged inline as in the generic kernels.  All row-level values are
// wave-uniform and live in scalar registers.
#include "internal.hpp"
#include "rowops.hpp"

namespace spg {

#ifndef SPG_WAVE_UNROLL
#define SPG_WAVE_UNROLL 2
#endif
#ifndef SPG_SYMW_UNROLL
#define SPG_SYMW_UNROLL 1
#endif
#ifndef SPG_WAVE_WAVES
#define SPG_WAVE_WAVES 8
#endif

constexpr int kWU = SPG_WAVE_UNROLL;   // products per lane per batch, numeric
constexpr int kSWU = SPG_SYMW_UNROLL;  // the same for the symbolic count

__device__ __forceinline__ int ufl(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Prefetched head of a row: uniform row data plus lane-held entry data.
template <typename VT>
struct RowHead {
  int i, as, nA, rs, re;  // uniform
  int b0, len;            // entry `lane` of the first chunk of part 0
  VT a;
};

// Products of entries [0, nE) staged in LDS, S lanes per entry, handed to
// ins.batch<U> (same enumeration as for_each_product).
// p[0..3] with one 16-byte load (p needs only 4-byte alignment)
__device__ __forceinline__ int4 load_int4(const SPG_GLOBAL int32_t *p) {
  int4 v;
  __builtin_memcpy(&v, p, sizeof(v));
  return v;
}

// Columns of entries [0, nE) for the count with four lanes per entry: each
// lane takes four consecutive elements of its entry's B row per pass, one
// 16-byte load for all four (a row's last partial group reads element by
// element from in-range positions).
template <typename F>
__device__ __forceinline__ void enum_cols_v4(const SPG_GLOBAL int32_t *bcol, int nE, int lane,
                                             const int *sb, const int *sl, F &ins) {
  const int sg = lane >> 2, q0 = 4 * (lane & 3);
  for (int t0 = sg; t0 < nE; t0 += kWave / 4) {
    const int b0 = sb[t0], len = sl[t0];
    for (int q = q0; q < len; q += 16) {
      int c[4];
      const float v[4] = {0.f, 0.f, 0.f, 0.f};
      if (q + 4 <= len) {
        const int4 cc = load_int4(bcol + b0 + q);
        c[0] = cc.x;
        c[1] = cc.y;
        c[2] = cc.z;
        c[3] = cc.w;
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int qq = q + t < len ? q + t : q;
          c[t] = bcol[b0 + qq];
          c[t] = q + t < len ? c[t] : -1;
        }
      }
      ins.template batch<4>(c, v);
    }
  }
}

template <bool VALUES, int U, typename VT, typename F>
__device__ __forceinline__ void enum_staged(const SPG_GLOBAL int32_t *bcol,
                                            const SPG_GLOBAL VT *bval, int nE, int lane, int lS,
                                            const int *sb, const int *sl, const VT *sa, F &ins) {
  if constexpr (!VALUES) {
    if (lS == 2) {
      enum_cols_v4(bcol, nE, lane, sb, sl, ins);
      return;
    }
  }
  const int S = 1 << lS, ES = kWave >> lS, sg = lane >> lS, q0 = lane & (S - 1);
  for (int t0 = sg; t0 < nE; t0 += ES * U) {
    // all LDS reads first, then all global loads, then the products: no
    // consumer sits between the U loads, so they are in flight together
    int col[U], b0[U], len[U];
    VT v[U], a[U], bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ee = t0 + ES * u;
      const int ec = ee < nE ? ee : 0;
      b0[u] = sb[ec];
      len[u] = ee < nE ? sl[ec] : 0;
      if (VALUES) a[u] = sa[ec];
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
    ins.template batch<U>(col, v);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      for (int q = q0 + S; q < len[u]; q += S) {
        const int idx = b0[u] + q;
        int c1[1] = {bcol[idx]};
        VT v1[1] = {VALUES ? a[u] * bval[idx] : VT(0)};
        ins.template batch<1>(c1, v1);
      }
    }
  }
}

// Stage entries [c0, c0+64) of part P's row i (inline path) and enumerate.
template <bool VALUES, int U, typename VT, typename F>
__device__ __forceinline__ void chunk_inline(const Part &P, int i, int as, int c0, int nA, int lane,
                                             int lS, int *sb, int *sl, VT *sa, F &ins) {
  const int e = c0 + lane;
  if (e < nA) {
    int r;
    VT a = VT(1);
    if (P.a_identity) {
      r = i;
    } else {
      r = gp(P.acol)[as + e];
      if (VALUES) a = gp(static_cast<const VT *>(P.aval))[as + e];
    }
    const int b0 = gp(P.brp)[r];
    sb[lane] = b0;
    sl[lane] = gp(P.brp)[r + 1] - b0;
    if (VALUES) sa[lane] = a;
  }
  group_sync<false>();
  enum_staged<VALUES, U, VT>(gp(P.bcol), gp(static_cast<const VT *>(P.bval)), min(kWave, nA - c0),
                             lane, lS, sb, sl, sa, ins);
  group_sync<false>();
}

// All products of a row whose head is prefetched.
template <bool VALUES, int U, typename VT, typename F>
__device__ __forceinline__ void row_products(const Problem *__restrict__ pr, const RowHead<VT> &h,
                                             int lane, int lS, int *sb, int *sl, VT *sa, F &ins) {
  const Part &P0 = pr->part[0];
  sb[lane] = h.b0;
  sl[lane] = h.len;
  if (VALUES) sa[lane] = h.a;
  group_sync<false>();
  enum_staged<VALUES, U, VT>(gp(P0.bcol), gp(static_cast<const VT *>(P0.bval)), min(kWave, h.nA),
                             lane, lS, sb, sl, sa, ins);
  group_sync<false>();
  for (int c0 = kWave; c0 < h.nA; c0 += kWave)
    chunk_inline<VALUES, U, VT>(P0, h.i, h.as, c0, h.nA, lane, lS, sb, sl, sa, ins);
  const int K = pr->K;
  for (int k = 1; k < K; ++k) {
    const Part &P = pr->part[k];
    int as, ae;
    a_row(P, h.i, as, ae);
    as = ufl(as);
    ae = ufl(ae);
    for (int c0 = 0; c0 < ae - as; c0 += kWave)
      chunk_inline<VALUES, U, VT>(P, h.i, as, c0, ae - as, lane, lS, sb, sl, sa, ins);
  }
}

// Links of the prefetch chain of the next row.
template <typename VT>
struct NextRow {
  bool has = false;
  int i = 0;
  int as = 0, ae = 0, rs = 0, re = 0;
  int r;
  VT a;
  __device__ __forceinline__ void link_row(const int32_t *rows, int start, int ri, int count) {
    has = ri < count;
    i = has ? ufl(rows[start + ri]) : 0;
  }
  __device__ __forceinline__ void link_ptrs(const Part &P0, const int32_t *crp) {
    if (!has) return;
    if (P0.a_identity) {
      as = 0;
      ae = 1;
    } else {
      as = ufl(gp(P0.arp)[i]);
      ae = ufl(gp(P0.arp)[i + 1]);
    }
    if (crp) {
      rs = ufl(crp[i]);
      re = ufl(crp[i + 1]);
    }
  }
  template <bool VALUES>
  __device__ __forceinline__ void link_entry(const Part &P0, int lane) {
    r = -1;
    a = VT(1);
    if (!has || lane >= ae - as) return;
    if (P0.a_identity) {
      r = i;
    } else {
      r = gp(P0.acol)[as + lane];
      if (VALUES) a = gp(static_cast<const VT *>(P0.aval))[as + lane];
    }
  }
  __device__ __forceinline__ RowHead<VT> link_b(const Part &P0) const {
    RowHead<VT> h;
    h.i = i;
    h.as = as;
    h.nA = has ? ae - as : 0;
    h.rs = rs;
    h.re = re;
    h.b0 = 0;
    h.len = 0;
    h.a = a;
    if (r >= 0) {
      h.b0 = gp(P0.brp)[r];
      h.len = gp(P0.brp)[r + 1] - h.b0;
    }
    return h;
  }
};

// Symbolic insert (same as the generic kernel's).
struct WSymInsert {
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

__global__ __launch_bounds__(256, SPG_WAVE_WAVES) void k_sym_wave(
    const Problem *__restrict__ pr, const int32_t *__restrict__ rows,
    const WsHeader *__restrict__ hdr, int bin, int lS, int log2T, int32_t *__restrict__ cnt) {
  extern __shared__ __align__(16) int smem[];
  const int T = 1 << log2T;
  const int w = ufl(threadIdx.x / kWave), lane = lane_id();
  int *tab = smem + w * T;
  int *sb = smem + 4 * T + w * kWave;
  int *sl = smem + 4 * T + 4 * kWave + w * kWave;
  if (hdr->status) return;
  const int count = hdr->bin_count[bin];
  const int start = hdr->bin_start[bin];
  const int stride = gridDim.x * 4;
  const Part &P0 = pr->part[0];
  int ri = blockIdx.x * 4 + w;
  // pipeline: n1 = next row (pointers known), n2 = row after (index known),
  // n3 = the one after that (index being fetched)
  NextRow<float> n1, n2, n3;
  n1.link_row(rows, start, ri, count);
  n1.link_ptrs(P0, nullptr);
  n1.template link_entry<false>(P0, lane);
  RowHead<float> cur = n1.link_b(P0);
  n1.link_row(rows, start, ri + stride, count);
  n1.link_ptrs(P0, nullptr);
  n2.link_row(rows, start, ri + 2 * stride, count);
  for (; ri < count; ri += stride) {
    int4 *t4 = reinterpret_cast<int4 *>(tab);
    for (int s = lane; s < T / 4; s += kWave) t4[s] = make_int4(kEmpty, kEmpty, kEmpty, kEmpty);
    group_sync<false>();
    n1.template link_entry<false>(P0, lane);
    WSymInsert ins{tab, T, log2T, 0};
    row_products<false, kSWU, float>(pr, cur, lane, lS, sb, sl, nullptr, ins);
    const RowHead<float> nh = n1.link_b(P0);
    n2.link_ptrs(P0, nullptr);
    n3.link_row(rows, start, ri + 3 * stride, count);
    int fresh = ins.fresh;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) fresh += __shfl_xor(fresh, off);
    if (lane == 0) cnt[cur.i] = fresh;
    group_sync<false>();
    cur = nh;
    n1 = n2;
    n2 = n3;
  }
}

template <typename VT, bool PACK>
struct WNumInsert {
  using KC = KeyCode<PACK>;
  int *key;
  VT *val;
  int *adj;
  int *flag;
  uint32_t mul;
  int maxwin;
  template <int N>
  __device__ __forceinline__ void batch(const int (&col)[N], const VT (&v)[N]) {
    int h[N], old[N], d[N];
#pragma unroll
    for (int u = 0; u < N; ++u) {
      h[u] = (int)mono_slot((uint32_t)col[u], mul);
      old[u] = col[u] >= 0 ? atomicCAS(&key[h[u]], kEmpty, KC::make(col[u])) : kEmpty;
    }
#pragma unroll
    for (int u = 0; u < N; ++u) {
      d[u] = 0;
      if (col[u] < 0) continue;
      while (old[u] != kEmpty && KC::col(old[u]) != col[u]) {
        if (d[u] == maxwin) {
          *flag = 1;
          d[u] = -1;
          break;
        }
        ++d[u];
        ++h[u];
        old[u] = atomicCAS(&key[h[u]], kEmpty, KC::make(col[u]));
      }
    }
#pragma unroll
    for (int u = 0; u < N; ++u)
      if (col[u] >= 0 && d[u] >= 0 && old[u] == kEmpty) val[h[u]] = v[u];
    group_sync<false>();
#pragma unroll
    for (int u = 0; u < N; ++u)
      if (col[u] >= 0 && d[u] >= 0 && old[u] != kEmpty) lds_add(&val[h[u]], v[u]);
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

template <typename VT, bool PACK>
__global__ __launch_bounds__(256, SPG_WAVE_WAVES) void k_num_wave(
    const Problem *__restrict__ pr, const int32_t *__restrict__ rows, WsHeader *__restrict__ hdr,
    int bin, int lS, int TT, uint32_t mul, int maxwin, const int32_t *__restrict__ crp,
    int32_t *__restrict__ ccol, VT *__restrict__ cval, int32_t *__restrict__ fb_rows) {
  using KC = KeyCode<PACK>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int rowflag[4];
  const int w = ufl(threadIdx.x / kWave), lane = lane_id();
  VT *val = reinterpret_cast<VT *>(smem_raw) + (size_t)w * TT;
  VT *sa = reinterpret_cast<VT *>(smem_raw) + (size_t)4 * TT + w * kWave;
  int *key = reinterpret_cast<int *>(reinterpret_cast<VT *>(smem_raw) + (size_t)4 * (TT + kWave)) +
             (size_t)w * TT;
  int *adj = key + (size_t)4 * TT;  // only when !PACK
  int *sb = key + (size_t)(PACK ? 4 : 8) * TT - (size_t)w * TT + w * kWave;
  int *sl = sb + 4 * kWave;
  if (hdr->status) return;
  const int count = hdr->bin_count[bin];
  const int start = hdr->bin_start[bin];
  const int stride = gridDim.x * 4;
  const Part &P0 = pr->part[0];
  const uint64_t below = lanes_below();
  int ri = blockIdx.x * 4 + w;
  NextRow<VT> n1, n2, n3;
  n1.link_row(rows, start, ri, count);
  n1.link_ptrs(P0, crp);
  n1.template link_entry<true>(P0, lane);
  RowHead<VT> cur = n1.link_b(P0);
  n1.link_row(rows, start, ri + stride, count);
  n1.link_ptrs(P0, crp);
  n2.link_row(rows, start, ri + 2 * stride, count);
  for (; ri < count; ri += stride) {
    {
      int4 *k4 = reinterpret_cast<int4 *>(key);
      for (int s = lane; s < TT / 4; s += kWave) k4[s] = make_int4(kEmpty, kEmpty, kEmpty, kEmpty);
      if (!PACK) {
        int4 *a4 = reinterpret_cast<int4 *>(adj);
        for (int s = lane; s < TT / 4; s += kWave) a4[s] = make_int4(0, 0, 0, 0);
      }
    }
    if (lane == 0) rowflag[w] = 0;
    group_sync<false>();
    n1.template link_entry<true>(P0, lane);
    WNumInsert<VT, PACK> ins{key, val, adj, &rowflag[w], mul, maxwin};
    row_products<true, kWU, VT>(pr, cur, lane, lS, sb, sl, sa, ins);
    const RowHead<VT> nh = n1.link_b(P0);
    n2.link_ptrs(P0, crp);
    n3.link_row(rows, start, ri + 3 * stride, count);
    const bool ok = rowflag[w] == 0;
    const int nnz = cur.re - cur.rs;
    SPG_GLOBAL int32_t *cb = gpw(ccol) + cur.rs;
    SPG_GLOBAL VT *vb = gpw(cval) + cur.rs;
    int base = 0;
    for (int s0 = 0; s0 < TT; s0 += kWave) {
      const int s = s0 + lane;
      const int kw = key[s];
      const uint64_t m = __ballot(kw != kEmpty);
      if (ok && kw != kEmpty && nnz > 0) {
        int rr = base + __popcll(m & below) + (PACK ? KC::adj(kw) : adj[s]);
        rr = rr < 0 ? 0 : (rr >= nnz ? nnz - 1 : rr);  // in bounds even for a changed pattern
        cb[(uint32_t)rr] = KC::col(kw);
        vb[(uint32_t)rr] = val[s];
      }
      base += __popcll(m);
    }
    if (ok && lane == 0 && base != nnz) atomicOr(&hdr->status, kStatInvalid);
    if (!ok && lane == 0) fb_rows[atomicAdd(&hdr->fallback_count, 1)] = cur.i;
    group_sync<false>();
    cur = nh;
    n1 = n2;
    n2 = n3;
  }
}

// ---------------------------------------------------------------------------
// Numeric pass by bucketing (rows of at most 256 distinct columns, n <= 2^24).
//
// Instead of a hash table with probing, every product is dropped into the
// bucket of its order-preserving home slot floor(col * T / n) (buckets are
// in column order), taking a ticket from the bucket's counter with one
// integer LDS atomic; the product is staged in LDS with its ticket.  A wave
// scan of the T counters gives each bucket's start and every product moves
// to start + ticket.  A row without repeated columns (as many products as
// output entries, known from the symbolic pass) then writes each product at
// its bucket's start plus the number of smaller columns in the bucket; other
// rows sort each (small) bucket in place by column, and the first of each
// run of equal columns sums the run and writes it, at a rank given by one
// ballot per 64 positions.
// There are no probe loops, no compare-and-swap retries and no rank-counter
// walks, which is where the hash kernel spends its scalar instructions.
// Rows with more products than the staging area holds, or a bucket with more
// than 255 products, go to the sort-based fallback kernel.
constexpr int kBucketMaxJ = 4;  // staged products per lane (capacity 256)

template <typename VT>
struct BucketInsert {
  uint32_t *cnt;   // T/2 words: two 16-bit bucket counters per word
  uint32_t *ikey;  // [cap] col | ticket << 24
  VT *ival;        // [cap]
  int *wcount;     // products staged so far (LDS, per wave)
  uint32_t mul;
  int cap;
  bool over;
  template <int N>
  __device__ __forceinline__ void batch(const int (&col)[N], const VT (&v)[N]) {
    uint32_t old[N], sh[N];
#pragma unroll
    for (int u = 0; u < N; ++u) {
      const uint32_t b = mono_slot((uint32_t)col[u], mul);
      sh[u] = (b & 1u) << 4;
      old[u] = col[u] >= 0 ? atomicAdd(&cnt[b >> 1], 1u << sh[u]) : 0u;
    }
    // staging indices: one LDS atomic per wave and call (correct for any set
    // of active lanes, also inside divergent code)
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

template <typename VT>
__global__ __launch_bounds__(256, SPG_WAVE_WAVES) void k_num_bucket(
    const Problem *__restrict__ pr, const int32_t *__restrict__ rows, WsHeader *__restrict__ hdr,
    int bin, int lS, int T, int cap, uint32_t mul, const int32_t *__restrict__ crp,
    int32_t *__restrict__ ccol, VT *__restrict__ cval, int32_t *__restrict__ fb_rows) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int wcount[4];
  const int w = ufl(threadIdx.x / kWave), lane = lane_id();
  const int TW = T / 2;  // counter words per wave
  uint32_t *cnt_all = reinterpret_cast<uint32_t *>(smem_raw);
  uint32_t *ikey_all = cnt_all + 4 * TW;
  VT *ival_all = reinterpret_cast<VT *>(ikey_all + 4 * cap);
  int *sb_all = reinterpret_cast<int *>(ival_all + 4 * cap);
  int *sl_all = sb_all + 4 * kWave;
  VT *sa_all = reinterpret_cast<VT *>(sl_all + 4 * kWave);
  uint32_t *cnt = cnt_all + w * TW;
  uint32_t *ikey = ikey_all + w * cap;
  VT *ival = ival_all + w * cap;
  int *sb = sb_all + w * kWave;
  int *sl = sl_all + w * kWave;
  VT *sa = sa_all + w * kWave;
  if (hdr->status) return;
  const int count = hdr->bin_count[bin];
  const int start = hdr->bin_start[bin];
  const int stride = gridDim.x * 4;
  const Part &P0 = pr->part[0];
  const uint64_t below = lanes_below();
  const int wpl = TW / kWave;  // counter words per lane (T >= 128)
  int ri = blockIdx.x * 4 + w;
  NextRow<VT> n1, n2, n3;
  n1.link_row(rows, start, ri, count);
  n1.link_ptrs(P0, crp);
  n1.template link_entry<true>(P0, lane);
  RowHead<VT> cur = n1.link_b(P0);
  n1.link_row(rows, start, ri + stride, count);
  n1.link_ptrs(P0, crp);
  n2.link_row(rows, start, ri + 2 * stride, count);
  for (; ri < count; ri += stride) {
    {
      int4 *c4 = reinterpret_cast<int4 *>(cnt);
      for (int s = lane; s < TW / 4; s += kWave) c4[s] = make_int4(0, 0, 0, 0);
    }
    if (lane == 0) wcount[w] = 0;
    group_sync<false>();
    n1.template link_entry<true>(P0, lane);
    BucketInsert<VT> ins{cnt, ikey, ival, &wcount[w], mul, cap, false};
    row_products<true, kWU, VT>(pr, cur, lane, lS, sb, sl, sa, ins);
    const RowHead<VT> nh = n1.link_b(P0);
    n2.link_ptrs(P0, crp);
    n3.link_row(rows, start, ri + 3 * stride, count);
    const int P = ufl(wcount[w]);
    const int nnz = cur.re - cur.rs;
    if (__any(ins.over) || P > cap) {  // staging overflow: the fallback redoes this row
      if (lane == 0) fb_rows[atomicAdd(&hdr->fallback_count, 1)] = cur.i;
      group_sync<false>();
      cur = nh;
      n1 = n2;
      n2 = n3;
      continue;
    }
    SPG_GLOBAL int32_t *cb = gpw(ccol) + cur.rs;
    SPG_GLOBAL VT *vb = gpw(cval) + cur.rs;
    // 1. bucket starts: exclusive scan of the 16-bit counters, in place;
    //    the largest bucket decides how buckets are sorted
    int bigmax = 0;
    {
      uint32_t wv[4];
      int loc = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        wv[j] = j < wpl ? cnt[lane * wpl + j] : 0u;
        loc += (int)(wv[j] & 0xffffu) + (int)(wv[j] >> 16);
        bigmax = max(bigmax, (int)max(wv[j] & 0xffffu, wv[j] >> 16));
      }
#pragma unroll
      for (int off = kWave / 2; off > 0; off >>= 1) bigmax = max(bigmax, __shfl_xor(bigmax, off));
      int x = loc;
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
      }
      int run = x - loc;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (j < wpl) {
          const uint32_t lo = (uint32_t)run;
          run += (int)(wv[j] & 0xffffu);
          const uint32_t hi = (uint32_t)run;
          run += (int)(wv[j] >> 16);
          cnt[lane * wpl + j] = lo | (hi << 16);
        }
      }
    }
    // 2. every product to start[bucket] + ticket
    uint32_t kk[kBucketMaxJ];
    VT vv[kBucketMaxJ];
#pragma unroll
    for (int j = 0; j < kBucketMaxJ; ++j) {
      const int p = lane + j * kWave;
      kk[j] = p < P ? ikey[p] : 0u;
      vv[j] = p < P ? ival[p] : VT(0);
    }
    group_sync<false>();
#pragma unroll
    for (int j = 0; j < kBucketMaxJ; ++j) {
      if (lane + j * kWave < P) {
        const uint32_t c = kk[j] & 0xffffffu;
        const uint32_t b = mono_slot(c, mul);
        const int st0 = (int)((cnt[b >> 1] >> ((b & 1u) << 4)) & 0xffffu);
        const int pos = st0 + (int)(kk[j] >> 24);
        ikey[pos] = c;
        ival[pos] = vv[j];
      }
    }
    const bool big = bigmax > kBigBucket;
    if (P == nnz && !big) {
      // no repeated column: a product's rank is its bucket's start plus the
      // number of smaller columns in the (small) bucket
      group_sync<false>();
      for (int p = lane; p < P; p += kWave) {
        const uint32_t c = ikey[p];
        const uint32_t b = mono_slot(c, mul);
        const int s0 = (int)((cnt[b >> 1] >> ((b & 1u) << 4)) & 0xffffu);
        const int s1 = b + 1 < (uint32_t)T
                           ? (int)((cnt[(b + 1) >> 1] >> (((b + 1) & 1u) << 4)) & 0xffffu)
                           : P;
        int r = s0;
        for (int q = s0; q < s1; ++q) r += ikey[q] < c ? 1 : 0;
        cb[r] = (int)c;
        vb[r] = ival[p];
      }
      group_sync<false>();
      cur = nh;
      n1 = n2;
      n2 = n3;
      continue;
    }
    group_sync<false>();
    // 3. sort every bucket of two or more products by column (insertion sort
    //    by one lane per bucket), or the whole row when a bucket is large
    if (big) lds_sort_pairs<false, kWave, VT>(ikey, ival, P, lane);
    for (int b = big ? T : lane; b < T; b += kWave) {
      const int s0 = (int)((cnt[b >> 1] >> ((b & 1) << 4)) & 0xffffu);
      const int s1 = b + 1 < T ? (int)((cnt[(b + 1) >> 1] >> (((b + 1) & 1) << 4)) & 0xffffu) : P;
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
    group_sync<false>();
    // 4. runs of equal columns: the first of each run sums it and writes
    int base = 0;
    for (int p0 = 0; p0 < P; p0 += kWave) {
      const int p = p0 + lane;
      const uint32_t c = p < P ? ikey[p] : 0xffffffffu;
      const uint32_t cp = p > 0 && p < P ? ikey[p - 1] : 0xfffffffeu;
      const bool first = p < P && c != cp;
      const uint64_t m = __ballot(first);
      if (first) {
        VT sum = ival[p];
        for (int q = p + 1; q < P && ikey[q] == c; ++q) sum += ival[q];
        const int d = base + __popcll(m & below);
        if (d < nnz) {  // the symbolic count bounds the row (a changed pattern is flagged)
          cb[d] = (int)c;
          vb[d] = sum;
        }
      }
      base += __popcll(m);
    }
    if (lane == 0 && base != nnz) atomicOr(&hdr->status, kStatInvalid);
    group_sync<false>();
    cur = nh;
    n1 = n2;
    n2 = n3;
  }
}

// Staging capacity and LDS of the bucket kernel for bin b (T = 2 * edge
// buckets, edge staged products: the rows of a bin never have more
// products than its edge, whatever thresholds the tuning picks).
int bucket_cap(int b) { return 8 << b; }
bool bucket_ok(int b) {
  const int T = bin_slots(b);
  return T >= 128 && T <= 512 && bucket_cap(b) <= kBucketMaxJ * kWave;
}
size_t bucket_lds_bytes(int b, size_t vbytes) {
  return (size_t)4 * (bin_slots(b) / 2) * 4 + (size_t)4 * bucket_cap(b) * (4 + vbytes) +
         (size_t)4 * kWave * (8 + vbytes);
}

// ---------------------------------------------------------------------------

// Slots of the count's table per row: four times the bin's upper edge (load
// <= 1/4, fewer probe round trips per insert).  Four waves' tables still fit
// eight blocks per CU; eight times the edge would halve the resident waves.
static int sym_wave_slots(int b) { return 2 * bin_slots(b); }
size_t sym_wave_lds_bytes(int b) { return (size_t)4 * sym_wave_slots(b) * 4 + (size_t)8 * kWave * 4; }

int num_wave_slots(int b) {
  const int need = bin_slots(b) + kTail;
  return (need + kWave - 1) / kWave * kWave;
}

size_t num_wave_lds_bytes(int b, size_t vbytes, bool pack) {
  const size_t TT = (size_t)num_wave_slots(b);
  return (size_t)4 * (TT + kWave) * vbytes + (size_t)4 * TT * (pack ? 4 : 8) +
         (size_t)8 * kWave * 4;
}

static int wave_grid(int count, size_t lds, int cap_waves_per_cu) {
  const DevInfo &D = dev_info();
  int per_cu = (int)(D.lds_per_cu / (lds ? lds : 1));
  const int by_waves = cap_waves_per_cu / 4;
  if (per_cu > by_waves) per_cu = by_waves;
  if (per_cu < 1) per_cu = 1;
  int grid = D.cus * per_cu;
  if (count >= 0) {
    const int need = (count + 3) / 4;
    if (need < grid) grid = need;
  }
  return grid < 1 ? 1 : grid;
}

void launch_sym_wave(const Problem *dpr, const int32_t *rows, const WsHeader *hdr, int bin,
                     int lS, int count, int32_t *cnt, hipStream_t st) {
  const size_t lds = sym_wave_lds_bytes(bin);
  int lt = 0;
  while ((1 << lt) < sym_wave_slots(bin)) ++lt;
  hipLaunchKernelGGL(k_sym_wave, dim3(wave_grid(count, lds, 4 * SPG_WAVE_WAVES)), dim3(256), lds, st,
                     dpr, rows, hdr, bin, lS, lt, cnt);
}

template <typename VT>
void launch_num_wave_t(const Problem *dpr, const int32_t *rows, WsHeader *hdr, int bin, int lS,
                       int count, uint32_t mul, int maxwin, bool pack, const int32_t *crp,
                       int32_t *ccol, VT *cval, int32_t *fb, hipStream_t st) {
  if (pack && bucket_ok(bin)) {
    const size_t lds = bucket_lds_bytes(bin, sizeof(VT));
    const int grid = wave_grid(count, lds, 4 * SPG_WAVE_WAVES);
    hipLaunchKernelGGL((k_num_bucket<VT>), dim3(grid), dim3(256), lds, st, dpr, rows, hdr, bin, lS,
                       bin_slots(bin), bucket_cap(bin), mul, crp, ccol, cval, fb);
    return;
  }
  const int TT = num_wave_slots(bin);
  const size_t lds = num_wave_lds_bytes(bin, sizeof(VT), pack);
  const int grid = wave_grid(count, lds, 4 * SPG_WAVE_WAVES);
  if (pack)
    hipLaunchKernelGGL((k_num_wave<VT, true>), dim3(grid), dim3(256), lds, st, dpr, rows, hdr, bin,
                       lS, TT, mul, maxwin, crp, ccol, cval, fb);
  else
    hipLaunchKernelGGL((k_num_wave<VT, false>), dim3(grid), dim3(256), lds, st, dpr, rows, hdr, bin,
                       lS, TT, mul, maxwin, crp, ccol, cval, fb);
}

void launch_num_wave(const Problem *dpr, const int32_t *rows, WsHeader *hdr, int bin, int lS,
                     int count, uint32_t mul, int maxwin, bool pack, const int32_t *crp,
                     int32_t *ccol, void *cval, bool f64, int32_t *fb, hipStream_t st) {
  if (f64)
    launch_num_wave_t<double>(dpr, rows, hdr, bin, lS, count, mul, maxwin, pack, crp, ccol,
                              static_cast<double *>(cval), fb, st);
  else
    launch_num_wave_t<float>(dpr, rows, hdr, bin, lS, count, mul, maxwin, pack, crp, ccol,
                             static_cast<float *>(cval), fb, st);
}

hipError_t configure_wave_lds(size_t lds_max) {
  const void *ks[] = {
      reinterpret_cast<const void *>(&k_sym_wave),
      reinterpret_cast<const void *>(&k_num_wave<float, true>),
      reinterpret_cast<const void *>(&k_num_wave<float, false>),
      reinterpret_cast<const void *>(&k_num_wave<double, true>),
      reinterpret_cast<const void *>(&k_num_wave<double, false>),
      reinterpret_cast<const void *>(&k_num_bucket<float>),
      reinterpret_cast<const void *>(&k_num_bucket<double>),
  };
  for (const void *k : ks) {
    hipError_t e =
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace spg

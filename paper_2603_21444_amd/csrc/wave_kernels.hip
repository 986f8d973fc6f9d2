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
#ifndef SPG_WAVE_WAVES
#define SPG_WAVE_WAVES 8
#endif

constexpr int kWU = SPG_WAVE_UNROLL;

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
template <bool VALUES, int U, typename VT, typename F>
__device__ __forceinline__ void enum_staged(const SPG_GLOBAL int32_t *bcol,
                                            const SPG_GLOBAL VT *bval, int nE, int lane, int lS,
                                            const int *sb, const int *sl, const VT *sa, F &ins) {
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
    row_products<false, kWU, float>(pr, cur, lane, lS, sb, sl, nullptr, ins);
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

size_t sym_wave_lds_bytes(int b) { return (size_t)4 * bin_slots(b) * 4 + (size_t)8 * kWave * 4; }

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
  while ((1 << lt) < bin_slots(bin)) ++lt;
  hipLaunchKernelGGL(k_sym_wave, dim3(wave_grid(count, lds, 4 * SPG_WAVE_WAVES)), dim3(256), lds, st,
                     dpr, rows, hdr, bin, lS, lt, cnt);
}

template <typename VT>
void launch_num_wave_t(const Problem *dpr, const int32_t *rows, WsHeader *hdr, int bin, int lS,
                       int count, uint32_t mul, int maxwin, bool pack, const int32_t *crp,
                       int32_t *ccol, VT *cval, int32_t *fb, hipStream_t st) {
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
  };
  for (const void *k : ks) {
    hipError_t e =
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace spg

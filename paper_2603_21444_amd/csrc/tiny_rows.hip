// Rows of very few products (at most 16), one thread per row: the symbolic
// count (a3) and the numeric pass (a5) of the first row bin.
//
// Such rows come from products whose right operand has about one entry per
// row, as a multigrid restriction operator (paper §5.4): there a group of
// lanes per row leaves most lanes idle and spends its time on table set-up.
// Here a thread gathers its row's products into its own column of an LDS
// staging array (slot n of thread t at n * blockDim + t, so the 64 lanes of
// a wave hit 64 banks), loads them into registers, sorts them with a
// bitonic network whose indices are all compile-time constants (the arrays
// stay in registers), and walks the sorted keys once: the count of distinct
// columns, or the sums of the runs of equal columns written in order.
#include "internal.hpp"
#include "rowops.hpp"

namespace spg {

constexpr int kTinyBlock = 256;

template <int N, typename VT>
__device__ __forceinline__ void tiny_sort(uint32_t (&key)[N], VT (&val)[N]) {
#pragma unroll
  for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          const uint32_t a = key[i], b = key[l];
          const bool sw = up ? (a > b) : (a < b);
          key[i] = sw ? b : a;
          key[l] = sw ? a : b;
          const VT va = val[i], vb = val[l];
          val[i] = sw ? vb : va;
          val[l] = sw ? va : vb;
        }
      }
    }
  }
}

// Stages the products of row i (at most N) in the thread's LDS column;
// returns their number.  VALUES: also the products a_ik * b_kj.
template <int N, bool VALUES, typename VT>
__device__ __forceinline__ int tiny_stage(const Problem *__restrict__ pr, int i, uint32_t *skey,
                                          VT *sval) {
  const int t = threadIdx.x;
  int n = 0;
  for (int k = 0; k < pr->K; ++k) {
    const Part &P = pr->part[k];
    int as, ae;
    a_row(P, i, as, ae);
    const SPG_GLOBAL int32_t *brp = gp(P.brp);
    const SPG_GLOBAL int32_t *bcol = gp(P.bcol);
    const SPG_GLOBAL VT *bval = gp(static_cast<const VT *>(P.bval));
    for (int p = as; p < ae; ++p) {
      int brow;
      VT a = VT(0);
      if (VALUES) a_entry<VT>(P, i, p, brow, a);
      else brow = a_entry_row(P, i, p);
      const int bs = brp[brow], be = brp[brow + 1];
      for (int q = bs; q < be && n < N; ++q, ++n) {
        skey[n * kTinyBlock + t] = (uint32_t)bcol[q];
        if (VALUES) sval[n * kTinyBlock + t] = a * bval[q];
      }
    }
  }
  return n;
}

template <int N>
__global__ __launch_bounds__(kTinyBlock) void k_sym_tiny(const Problem *__restrict__ pr,
                                                         const int32_t *__restrict__ rows,
                                                         const WsHeader *__restrict__ hdr, int bin,
                                                         int32_t *__restrict__ cnt) {
  __shared__ uint32_t skey[N * kTinyBlock];
  if (hdr->status) return;
  const int count = hdr->bin_count[bin];
  const int start = hdr->bin_start[bin];
  const int t = threadIdx.x;
  for (int ri = blockIdx.x * kTinyBlock + t; ri < count; ri += gridDim.x * kTinyBlock) {
    const int i = rows[start + ri];
    const int n = tiny_stage<N, false, float>(pr, i, skey, nullptr);
    uint32_t key[N];
    float dummy[N];
#pragma unroll
    for (int u = 0; u < N; ++u) {
      key[u] = u < n ? skey[u * kTinyBlock + t] : 0xffffffffu;
      dummy[u] = 0.f;
    }
    tiny_sort<N, float>(key, dummy);
    int d = n > 0 ? 1 : 0;
#pragma unroll
    for (int u = 1; u < N; ++u) d += (u < n && key[u] != key[u - 1]) ? 1 : 0;
    cnt[i] = d;
  }
}

template <int N, typename VT>
__global__ __launch_bounds__(kTinyBlock) void k_num_tiny(const Problem *__restrict__ pr,
                                                         const int32_t *__restrict__ rows,
                                                         WsHeader *__restrict__ hdr, int bin,
                                                         const int32_t *__restrict__ crp,
                                                         int32_t *__restrict__ ccol,
                                                         VT *__restrict__ cval) {
  __shared__ uint32_t skey[N * kTinyBlock];
  __shared__ VT sval[N * kTinyBlock];
  if (hdr->status) return;
  const int count = hdr->bin_count[bin];
  const int start = hdr->bin_start[bin];
  const int t = threadIdx.x;
  for (int ri = blockIdx.x * kTinyBlock + t; ri < count; ri += gridDim.x * kTinyBlock) {
    const int i = rows[start + ri];
    const int n = tiny_stage<N, true, VT>(pr, i, skey, sval);
    uint32_t key[N];
    VT val[N];
#pragma unroll
    for (int u = 0; u < N; ++u) {
      key[u] = u < n ? skey[u * kTinyBlock + t] : 0xffffffffu;
      val[u] = u < n ? sval[u * kTinyBlock + t] : VT(0);
    }
    tiny_sort<N, VT>(key, val);
    const int rs = crp[i], re = crp[i + 1];
    SPG_GLOBAL int32_t *cb = gpw(ccol);
    SPG_GLOBAL VT *vb = gpw(cval);
    // runs of equal columns: each run's sum is written when the run ends
    int o = rs;
    VT acc = val[0];
#pragma unroll
    for (int u = 1; u <= N; ++u) {
      const int un = u < N ? u : N - 1;  // a constant index; unused for u == N
      const bool ends = u - 1 < n && (u == N || u == n || key[un] != key[u - 1]);
      if (ends) {
        if (o < re) {  // the symbolic count bounds the row (a changed pattern is flagged)
          cb[o] = (int)key[u - 1];
          vb[o] = acc;
        }
        ++o;
      }
      if (u < N) acc = ends ? val[un] : acc + val[un];
    }
    if (o != re) atomicOr(&hdr->status, kStatInvalid);
  }
}

constexpr int kTinyN = 16;  // bin 1: at most 16 products per row

static int tiny_grid(int count, bool known) {
  const DevInfo &D = dev_info();
  const int cap = D.cus * 8;
  if (!known) return cap;
  const int need = (count + kTinyBlock - 1) / kTinyBlock;
  return need < 1 ? 1 : (need < cap ? need : cap);
}

void launch_sym_tiny(const Problem *dpr, const int32_t *rows, const WsHeader *hdr, int bin,
                     int count, bool known, int32_t *cnt, hipStream_t st) {
  const int grid = tiny_grid(count, known);
  hipLaunchKernelGGL(k_sym_tiny<kTinyN>, dim3(grid), dim3(kTinyBlock), 0, st, dpr, rows, hdr,
                     bin, cnt);
}

void launch_num_tiny(const Problem *dpr, const int32_t *rows, WsHeader *hdr, int bin, int count,
                     bool known, const int32_t *crp, int32_t *ccol, void *cval, bool f64,
                     hipStream_t st) {
  const int grid = tiny_grid(count, known);
#define SPG_TINY(N, VT)                                                                      \
  hipLaunchKernelGGL((k_num_tiny<N, VT>), dim3(grid), dim3(kTinyBlock), 0, st, dpr, rows, hdr, \
                     bin, crp, ccol, static_cast<VT *>(cval))
  if (f64) SPG_TINY(kTinyN, double);
  else SPG_TINY(kTinyN, float);
#undef SPG_TINY
}

}  // namespace spg

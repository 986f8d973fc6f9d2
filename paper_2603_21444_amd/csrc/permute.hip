// Permutation of a CSR matrix: B[prow[i], pcol[j]] = A[i, j] (paper §5.3:
// rows and columns of a structured matrix permuted uniformly at random as a
// light preprocessing step before the product; with prow = pcol it is the
// symmetric permutation P A P^T).
//
// Steps: the inverse row permutation (each new row reads its old row), with
// a check that both arrays are permutations; the new row lengths, their scan
// into B's row pointer, and lists of the new rows by length class; then
// every new row gathers its old row, maps the columns and writes them in
// ascending order.  The new columns of a row are distinct, so an element's
// output slot is the number of the row's elements with a smaller new
// column: short rows count it over the row's columns staged in LDS (group of
// G lanes, up to 4 elements per lane; one kernel per length class, each over
// its own list), rows longer than 4096 entries go through column panels (a
// bitmap of the panel's columns, a block scan of its words, then each
// element writes at its rank).
#include <algorithm>

#include "internal.hpp"
#include "rowops.hpp"

namespace spg {

constexpr int kPermE = 4;          // elements per lane in the short-row kernels
constexpr int kPermLong = 4096;    // rows longer than this take the panel kernel
constexpr int kPermPanelBits = 32768;  // columns per panel (one bitmap word per thread)

__global__ __launch_bounds__(256) void k_perm_clear(int32_t *a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = -1;
}

// inv[p[i]] = i; a value out of range or taken twice raises kStatInvalid.
__global__ __launch_bounds__(256) void k_perm_inverse(const int32_t *__restrict__ p, int n,
                                                      int32_t *__restrict__ inv, WsHeader *hdr) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int v = p[i];
    if (v < 0 || v >= n) bad = true;
    else if (atomicCAS(&inv[v], -1, (int)i) != -1) bad = true;
  }
  if (bad) atomicOr(&hdr->status, kStatInvalid);
}

// Length classes of the new rows: (0, 64], (64, 256], (256, 1024],
// (1024, 4096] (group kernels of 16, 64, 256, 1024 lanes) and longer (the
// panel kernel); empty rows need no work.
constexpr int kPermClasses = 5;

__device__ __forceinline__ int perm_class(int len) {
  return len <= 0 ? -1 : len <= 64 ? 0 : len <= 256 ? 1 : len <= 1024 ? 2 : len <= kPermLong ? 3 : 4;
}

// Length of every new row, and the row in its class's list (class c's list
// holds at most m rows at lists + c * m; its length is hdr->bin_count[c]).
// Each wave takes one atomic per class for its rows.
__global__ __launch_bounds__(256) void k_perm_len(const int32_t *__restrict__ arp,
                                                  const int32_t *__restrict__ rinv, int m,
                                                  int32_t *__restrict__ cnt,
                                                  int32_t *__restrict__ lists, WsHeader *hdr) {
  if (hdr->status) return;
  const uint64_t below = lanes_below();
  // whole waves step together, so the ballots below see every lane
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r0 = (int64_t)blockIdx.x * blockDim.x; r0 < m; r0 += stride) {
    const int64_t r = r0 + threadIdx.x;
    int cls = -1;
    if (r < m) {
      const int old = rinv ? rinv[r] : (int)r;
      const int len = arp[old + 1] - arp[old];
      cnt[r] = len;
      cls = perm_class(len);
    }
#pragma unroll
    for (int c = 0; c < kPermClasses; ++c) {
      const uint64_t mk = __ballot(cls == c);
      if (mk == 0) continue;
      const int leader = __ffsll((unsigned long long)mk) - 1;
      int base = 0;
      if (lane_id() == leader) base = atomicAdd(&hdr->bin_count[c], __popcll(mk));
      base = __shfl(base, leader);
      if (cls == c) lists[(int64_t)c * m + base + __popcll(mk & below)] = (int)r;
    }
  }
}

// Rows of length class `cls` (at most 4G entries): G lanes per row, elements
// e = l + t G.
template <int G, typename VT>
__global__ __launch_bounds__(G <= kWave ? 256 : G) void k_perm_rows(
    const int32_t *__restrict__ arp, const int32_t *__restrict__ acol,
    const VT *__restrict__ aval, const int32_t *__restrict__ rinv,
    const int32_t *__restrict__ pcol, const int32_t *__restrict__ list, int cls,
    const int32_t *__restrict__ brp, int32_t *__restrict__ bcol, VT *__restrict__ bval,
    const WsHeader *hdr) {
  constexpr int WG = G <= kWave ? 256 : G;
  constexpr int R = WG / G;
  constexpr int CAP = kPermE * G;
  __shared__ int skey[R * CAP];
  if (hdr->status) return;
  const int count = hdr->bin_count[cls];
  const int rslot = threadIdx.x / G, l = threadIdx.x % G;
  int *key_s = skey + rslot * CAP;
  const int ngroups = gridDim.x * R;
  for (int r0 = blockIdx.x * R; r0 < count; r0 += ngroups) {
    const int idx = r0 + rslot;
    int len = 0, s = 0, r = 0;
    if (idx < count) {
      r = list[idx];
      const int old = rinv ? rinv[r] : r;
      s = arp[old];
      len = arp[old + 1] - s;
    }
    const bool mine = idx < count && len <= CAP;
    int key[kPermE];
    VT v[kPermE];
#pragma unroll
    for (int t = 0; t < kPermE; ++t) {
      const int e = l + t * G;
      key[t] = -1;
      v[t] = VT(0);
      if (mine && e < len) {
        const int c = acol[s + e];
        key[t] = pcol ? pcol[c] : c;
        if (aval) v[t] = aval[s + e];
        key_s[e] = key[t];
      }
    }
    if (G > kWave) __syncthreads();
    else group_sync<false>();
    if (mine) {
      const int o = brp[r];
#pragma unroll
      for (int t = 0; t < kPermE; ++t) {
        if (key[t] < 0) continue;
        int rank = 0;
        for (int u = 0; u < len; ++u) rank += key_s[u] < key[t] ? 1 : 0;
        bcol[o + rank] = key[t];
        if (bval) bval[o + rank] = v[t];
      }
    }
    if (G > kWave) __syncthreads();
    else group_sync<false>();
  }
}

// Rows longer than kPermLong: one block per row, panels of kPermPanelBits
// new columns; in each panel a bitmap marks the row's columns, a block scan
// of the bitmap words gives each word's starting rank, and every element
// writes at that rank plus the marks below it in its word (columns are
// distinct).
template <typename VT>
__global__ __launch_bounds__(1024) void k_perm_long(
    const int32_t *__restrict__ arp, const int32_t *__restrict__ acol,
    const VT *__restrict__ aval, const int32_t *__restrict__ rinv,
    const int32_t *__restrict__ pcol, int ncols, const int32_t *__restrict__ longrows,
    int cls, const int32_t *__restrict__ brp, int32_t *__restrict__ bcol, VT *__restrict__ bval,
    const WsHeader *hdr) {
  static_assert(kPermPanelBits / 32 == 1024, "one bitmap word per thread");
  __shared__ uint32_t bm[kPermPanelBits / 32];
  __shared__ int wpre[kPermPanelBits / 32];
  __shared__ int wtot[1024 / kWave];
  if (hdr->status) return;
  const int count = hdr->bin_count[cls];
  const int tid = threadIdx.x;
  for (int li = blockIdx.x; li < count; li += gridDim.x) {
    const int r = longrows[li];
    const int old = rinv ? rinv[r] : r;
    const int s = arp[old], len = arp[old + 1] - s;
    int base = brp[r];
    for (int plo = 0; plo < ncols; plo += kPermPanelBits) {
      bm[tid] = 0u;
      __syncthreads();
      for (int e = tid; e < len; e += 1024) {
        const int c0 = acol[s + e];
        const uint32_t c = (uint32_t)((pcol ? pcol[c0] : c0) - plo);
        if (c < (uint32_t)kPermPanelBits) atomicOr(&bm[c >> 5], 1u << (c & 31));
      }
      __syncthreads();
      int total;
      wpre[tid] = group_excl_scan<true, 1024>(__popc(bm[tid]), tid, wtot, total);
      __syncthreads();
      for (int e = tid; e < len; e += 1024) {
        const int c0 = acol[s + e];
        const int cn = pcol ? pcol[c0] : c0;
        const uint32_t c = (uint32_t)(cn - plo);
        if (c < (uint32_t)kPermPanelBits) {
          const int w = (int)(c >> 5);
          const int pos = base + wpre[w] + __popc(bm[w] & ((1u << (c & 31)) - 1u));
          bcol[pos] = cn;
          if (bval) bval[pos] = aval[s + e];
        }
      }
      __syncthreads();
      base += total;
    }
  }
}

size_t perm_workspace_bytes(int64_t m, int64_t n, size_t *rinv_off, size_t *cinv_off,
                            size_t *long_off, size_t *scan_off) {
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t o = 4096;  // header
  *rinv_off = o;
  o = al(o + 4 * (size_t)(m > 0 ? m : 1));
  *cinv_off = o;
  o = al(o + 4 * (size_t)(n > 0 ? n : 1));
  *long_off = o;  // the row lists of the length classes
  o = al(o + 4 * (size_t)kPermClasses * (size_t)(m > 0 ? m : 1));
  *scan_off = o;
  o = al(o + 8 * (size_t)((m + 2047) / 2048 + 1));
  return o;
}

template <int G, typename VT>
static void perm_rows_launch(const int32_t *arp, const int32_t *acol, const void *aval,
                             const int32_t *rinv, const int32_t *pcol, int m,
                             const int32_t *lists, int cls, const int32_t *brp, int32_t *bcol,
                             void *bval, const WsHeader *hdr, int cus, hipStream_t st) {
  constexpr int WG = G <= kWave ? 256 : G;
  constexpr int R = WG / G;
  // a persistent grid over the class's list (its length is on the device)
  const int need = (m + R - 1) / R;
  const int grid = std::max(1, std::min(need, cus * (2048 / WG)));
  hipLaunchKernelGGL((k_perm_rows<G, VT>), dim3(grid), dim3(WG), 0, st, arp, acol,
                     static_cast<const VT *>(aval), rinv, pcol, lists + (size_t)cls * m, cls,
                     brp, bcol, static_cast<VT *>(bval), hdr);
}

template <typename VT>
static hipError_t permute_impl(const int32_t *arp, const int32_t *acol, const void *aval,
                               const int32_t *rinv, const int32_t *pcol, int m, int n,
                               const int32_t *brp, int32_t *bcol, void *bval,
                               const int32_t *longrows, const WsHeader *hdr, hipStream_t st) {
  const DevInfo &D = dev_info();
  static_assert(kPermE * 16 == 64 && kPermE * 64 == 256 && kPermE * 256 == 1024 &&
                    kPermE * 1024 == kPermLong,
                "the length classes match the group sizes");
  perm_rows_launch<16, VT>(arp, acol, aval, rinv, pcol, m, longrows, 0, brp, bcol, bval, hdr,
                           D.cus, st);
  perm_rows_launch<64, VT>(arp, acol, aval, rinv, pcol, m, longrows, 1, brp, bcol, bval, hdr,
                           D.cus, st);
  perm_rows_launch<256, VT>(arp, acol, aval, rinv, pcol, m, longrows, 2, brp, bcol, bval, hdr,
                            D.cus, st);
  perm_rows_launch<1024, VT>(arp, acol, aval, rinv, pcol, m, longrows, 3, brp, bcol, bval, hdr,
                             D.cus, st);
  hipLaunchKernelGGL((k_perm_long<VT>), dim3(D.cus), dim3(1024), 0, st, arp, acol,
                     static_cast<const VT *>(aval), rinv, pcol, n,
                     longrows + (size_t)4 * m, 4, brp, bcol,
                     static_cast<VT *>(bval), hdr);
  return hipGetLastError();
}

hipError_t launch_permute(const spg_csr &A, const int32_t *prow, const int32_t *pcol,
                          int dtype, int32_t *brp, int32_t *bcol, void *bval, char *ws,
                          hipStream_t st) {
  const int m = A.nrows, n = A.ncols;
  size_t ro, co, lo, so;
  (void)perm_workspace_bytes(m, n, &ro, &co, &lo, &so);
  WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
  int32_t *rinv = prow ? reinterpret_cast<int32_t *>(ws + ro) : nullptr;
  int32_t *cinv = reinterpret_cast<int32_t *>(ws + co);
  int32_t *longrows = reinterpret_cast<int32_t *>(ws + lo);
  const DevInfo &D = dev_info();
  const int g = D.cus * 4;
  if (prow) {
    hipLaunchKernelGGL(k_perm_clear, dim3(g), dim3(256), 0, st, rinv, (int64_t)m);
    hipLaunchKernelGGL(k_perm_inverse, dim3(g), dim3(256), 0, st, prow, m, rinv, hdr);
  }
  if (pcol) {  // the inverse itself is not needed, only the check
    hipLaunchKernelGGL(k_perm_clear, dim3(g), dim3(256), 0, st, cinv, (int64_t)n);
    hipLaunchKernelGGL(k_perm_inverse, dim3(g), dim3(256), 0, st, pcol, n, cinv, hdr);
  }
  hipLaunchKernelGGL(k_perm_len, dim3(g), dim3(256), 0, st, A.row_ptr, rinv, m, brp, longrows,
                     hdr);
  WsLayout L{};
  L.scanpart = so;
  hipError_t e = launch_scan(brp, m, -1, L, ws, st);
  if (e != hipSuccess) return e;
  if (dtype == SPG_F64)
    return permute_impl<double>(A.row_ptr, A.col_idx, A.vals, rinv, pcol, m, n, brp, bcol, bval,
                                longrows, hdr, st);
  return permute_impl<float>(A.row_ptr, A.col_idx, A.vals, rinv, pcol, m, n, brp, bcol, bval,
                             longrows, hdr, st);
}

}  // namespace spg

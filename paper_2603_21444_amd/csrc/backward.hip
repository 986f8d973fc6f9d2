// Backward pass of C = A B at fixed sparsity (a9): for a loss L with
// W = dL/dC on S(C),
//   dA_ik = sum_{j in S(B)_k} W_ij b_kj     for (i,k) in S(A)
//   dB_kj = sum_{i : k in S(A)_i} a_ik W_ij  for (k,j) in S(B).
// Not in the paper; the definition is the derivative of the bilinear map
// (A, B) -> A B restricted to the given patterns.
//
// One pass over the forward product set.  Per row i of C the W values go
// into an LDS hash keyed by column (FP32: column and value in one 64-bit
// slot; rows beyond the LDS tables use a dense row in the heavy-slot
// scratch instead).  Every product (p, q) looks up
// w = W_i,col(q); dA_p collects w * b_q in an LDS accumulator of its A
// entry, and a_p * w is added to dB_q with a device-scope float atomic, so
// the summation order of a dB entry is not fixed.
//
// Deterministic dB: the terms a_p * w (each rounded in the dtype, as in
// the float path) are added into fixed-point integers, one per B entry,
// where 2^E bounds every |a_p * w| (E from the largest |a| and |w|, taken
// with order-free integer maxima).  FP64: 128-bit integers with the unit
// 2^(E - 90), so a term loses less than 2^-90 of the largest term of the
// whole product and a sum of up to 2^31 terms still fits.  FP32: 64-bit
// integers with the unit 2^(E - 62 + L), 2^L >= the rows of A (the most
// terms a dB entry can have), so a sum always fits and a term loses less
// than 2^(L - 62) <= 2^-31 of the largest term, far below FP32 rounding;
// one atomic per term, as in the float path.  Integer addition is
// associative, so every run gives the same bits.  A last pass converts the
// integers to the dtype.
#include <vector>

#include "internal.hpp"
#include "rowops.hpp"

namespace spg {

// Deterministic dB: the fixed-point accumulators (lo: low 64 bits, hi: high
// 64 bits of FP64 sums, two's complement) and the scale words (largest |a|
// and |w| as bit patterns, then the shift S: a term v counts as v 2^S).
// lo == NULL: float atomics.
struct DetAcc {
  unsigned long long *lo;
  long long *hi;
  unsigned long long *mx;  // [0] max |a| bits, [1] max |w| bits, [2] S
};

__device__ __forceinline__ unsigned long long abs_bits(float v) {
  return __float_as_uint(v) & 0x7fffffffu;
}
__device__ __forceinline__ unsigned long long abs_bits(double v) {
  return (unsigned long long)__double_as_longlong(v) & 0x7fffffffffffffffull;
}

// Adds the term v (already rounded in the dtype) to accumulator q.
__device__ __forceinline__ void det_add(const DetAcc &d, int S, int64_t q, float v) {
  const long long x = (long long)ldexp((double)v, S);  // |x| < 2^(62 - L)
  if (x) atomicAdd(&d.lo[q], (unsigned long long)x);
}
__device__ __forceinline__ void det_add(const DetAcc &d, int S, int64_t q, double v) {
  double x = ldexp(v, S);  // |x| < 2^91
  const bool neg = x < 0.0;
  x = fabs(x);
  unsigned long long hm = (unsigned long long)floor(ldexp(x, -64));
  unsigned long long lm = (unsigned long long)(x - ldexp((double)hm, 64));  // below 2^64, exact
  unsigned long long lo = lm, hi = hm;
  if (neg) {  // two's complement of the 128-bit magnitude
    lo = ~lm + 1ull;
    hi = ~hm + (lm == 0ull ? 1ull : 0ull);
  }
  if (lo == 0ull && hi == 0ull) return;
  const unsigned long long old = atomicAdd(&d.lo[q], lo);
  const unsigned long long carry = old + lo < old ? 1ull : 0ull;
  if (hi + carry) atomicAdd(reinterpret_cast<unsigned long long *>(&d.hi[q]), hi + carry);
}

#ifndef SPG_BWD_UNROLL
#define SPG_BWD_UNROLL 2
#endif
constexpr int kBwdUnroll = SPG_BWD_UNROLL;

template <typename VT>
__global__ void k_fill_zero(VT *p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride)
    p[t] = VT(0);
}

// Products of row i, S lanes per A entry: f(col, b, idx, e) handles product
// (entry e, B position idx) and returns its contribution to dA_e, which the
// entry's S lanes sum in registers and reduce with shuffles into sd[e].
// Chunks of G entries of the A row are staged in LDS; `done(c0, nE)` runs
// after each chunk (group-synchronised).
template <bool BLOCK, int G, typename VT, typename F, typename D>
__device__ __forceinline__ void for_each_product_e(const Part &P, int i, int l, int lS, int *sb,
                                                   int *sl, VT *sa, VT *sd, F &&f, D &&done) {
  const int S = 1 << lS;
  const int ES = G >> lS;
  const int sg = l >> lS;
  const int q0 = l & (S - 1);
  const SPG_GLOBAL int32_t *brp = gp(P.brp);
  const SPG_GLOBAL int32_t *bcol = gp(P.bcol);
  const SPG_GLOBAL VT *bval = gp(static_cast<const VT *>(P.bval));
  const int as = gp(P.arp)[i], nA = gp(P.arp)[i + 1] - as;
  for (int c0 = 0; c0 < nA; c0 += G) {
    const int e = c0 + l;
    if (e < nA) {
      const int r = gp(P.acol)[as + e];
      const int b0 = brp[r];
      sb[l] = b0;
      sl[l] = brp[r + 1] - b0;
      sa[l] = gp(static_cast<const VT *>(P.aval))[as + e];
    }
    const int nE = min(G, nA - c0);
    group_sync<BLOCK>();
    // kBwdUnroll entries at a time: the loads of their first positions are
    // in flight together before any product is looked up
    for (int e0 = sg; e0 < nE; e0 += ES * kBwdUnroll) {
      int len[kBwdUnroll], b0[kBwdUnroll], col[kBwdUnroll];
      VT part[kBwdUnroll], bv[kBwdUnroll];
#pragma unroll
      for (int u = 0; u < kBwdUnroll; ++u) {
        const int ee = e0 + u * ES;
        len[u] = ee < nE ? sl[ee] : 0;
        b0[u] = ee < nE ? sb[ee] : 0;
        part[u] = VT(0);
      }
#pragma unroll
      for (int u = 0; u < kBwdUnroll; ++u) {
        col[u] = 0;
        bv[u] = VT(0);
        if (q0 < len[u]) {
          col[u] = bcol[b0[u] + q0];
          bv[u] = bval[b0[u] + q0];
        }
      }
#pragma unroll
      for (int u = 0; u < kBwdUnroll; ++u) {
        const int ee = e0 + u * ES;
        if (q0 < len[u]) part[u] += f(col[u], bv[u], b0[u] + q0, ee);
        for (int q = q0 + S; q < len[u]; q += S) {
          const int idx = b0[u] + q;
          part[u] += f(bcol[idx], bval[idx], idx, ee);
        }
      }
      // the S lanes of an entry hold its partial sums: reduce, one store
#pragma unroll
      for (int u = 0; u < kBwdUnroll; ++u) {
        for (int off = S / 2; off > 0; off >>= 1) part[u] += __shfl_xor(part[u], off, S);
        const int ee = e0 + u * ES;
        if (q0 == 0 && ee < nE) sd[ee] = part[u];
      }
    }
    group_sync<BLOCK>();
    done(as + c0, nE);
    group_sync<BLOCK>();
  }
}

template <int G>
struct BGeom {
  static constexpr bool BLOCK = G > kWave;
  static constexpr int WG = BLOCK ? G : 256;
  static constexpr int R = WG / G;
};

template <int G, typename VT>
__global__ __launch_bounds__(BGeom<G>::WG) void k_bwd_rows(
    const Problem *__restrict__ pr, const int32_t *__restrict__ rows,
    WsHeader *__restrict__ hdr, int bin, int lS, int log2T, const int32_t *__restrict__ crp,
    const int32_t *__restrict__ ccol, const VT *__restrict__ w, VT *__restrict__ dA,
    VT *__restrict__ dB, DetAcc det) {
  using GM = BGeom<G>;
  // FP32: column and W value in one 64-bit slot, so a lookup is one LDS
  // read per probe; FP64: a key array beside the value array
  constexpr bool PK = sizeof(VT) == 4;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int T = 1 << log2T;
  const int rslot = threadIdx.x / G, l = threadIdx.x % G;
  unsigned long long *slot = reinterpret_cast<unsigned long long *>(smem_raw) + (size_t)rslot * T;
  VT *wv = reinterpret_cast<VT *>(smem_raw) + (size_t)rslot * T;
  int *key = reinterpret_cast<int *>(reinterpret_cast<VT *>(smem_raw) + (size_t)GM::R * T) +
             (size_t)rslot * T;
  unsigned char *rest = smem_raw + (size_t)GM::R * T * (sizeof(VT) + 4);
  VT *sa = reinterpret_cast<VT *>(rest) + rslot * G;
  VT *sd = sa + (size_t)GM::R * G;
  int *sb = reinterpret_cast<int *>(reinterpret_cast<VT *>(rest) + (size_t)2 * GM::R * G) +
            rslot * G;
  int *sl = sb + (size_t)GM::R * G;
  if (hdr->status) return;
  const int count = hdr->bin_count[bin];
  const int start = hdr->bin_start[bin];
  const Part &P = pr->part[0];
  const int E = det.lo ? (int)(int32_t)(uint32_t)det.mx[2] : 0;
  for (int ri = blockIdx.x * GM::R + rslot; ri < count; ri += gridDim.x * GM::R) {
    int i = rows[start + ri];
    if (G >= kWave) i = __builtin_amdgcn_readfirstlane(i);
    for (int s = l; s < T; s += G) {
      if (PK) slot[s] = kEmptySlot;
      else key[s] = kEmpty;
    }
    group_sync<GM::BLOCK>();
    const int rs = crp[i], re = crp[i + 1];
    for (int t = rs + l; t < re; t += G) {
      const int col = ccol[t];
      uint32_t h = scramble_slot((uint32_t)col, log2T);
      int probes = 0;
      if constexpr (PK) {
        const unsigned long long sv = slot_make(col, (float)w[t]);
        while (atomicCAS(&slot[h], kEmptySlot, sv) != kEmptySlot) {
          if (++probes > T) {  // row longer than the plan's C row: pattern mismatch
            atomicOr(&hdr->status, kStatInvalid);
            break;
          }
          h = (h + 1) & (T - 1);
        }
      } else {
        while (atomicCAS(&key[h], kEmpty, col) != kEmpty) {
          if (++probes > T) {  // row longer than the plan's C row: pattern mismatch
            atomicOr(&hdr->status, kStatInvalid);
            break;
          }
          h = (h + 1) & (T - 1);
        }
        if (probes <= T) wv[h] = w[t];
      }
    }
    group_sync<GM::BLOCK>();
    // products: S lanes per A entry, kBwdUnroll entries at a time.  For
    // each round of positions the B loads of all entries are issued first,
    // then all first probes of the W lookups, then the dA terms, and the dB
    // atomics last, so no load waits behind an atomic.
    const SPG_GLOBAL int32_t *brp = gp(P.brp);
    const SPG_GLOBAL int32_t *bcol = gp(P.bcol);
    const SPG_GLOBAL VT *bval = gp(static_cast<const VT *>(P.bval));
    const int S = 1 << lS, ES = G >> lS, sg = l >> lS, q0 = l & (S - 1);
    const int as = gp(P.arp)[i], nA = gp(P.arp)[i + 1] - as;
    bool miss = false;
    for (int c0 = 0; c0 < nA; c0 += G) {
      const int e = c0 + l;
      if (e < nA) {
        const int r = gp(P.acol)[as + e];
        const int b0 = brp[r];
        sb[l] = b0;
        sl[l] = brp[r + 1] - b0;
        sa[l] = gp(static_cast<const VT *>(P.aval))[as + e];
      }
      const int nE = min(G, nA - c0);
      group_sync<GM::BLOCK>();
      for (int e0 = sg; e0 < nE; e0 += ES * kBwdUnroll) {
        int len[kBwdUnroll], b0[kBwdUnroll];
        VT av[kBwdUnroll], part[kBwdUnroll];
        int mlen = 0;
#pragma unroll
        for (int u = 0; u < kBwdUnroll; ++u) {
          const int ee = e0 + u * ES;
          len[u] = ee < nE ? sl[ee] : 0;
          b0[u] = ee < nE ? sb[ee] : 0;
          av[u] = ee < nE ? sa[ee] : VT(0);
          part[u] = VT(0);
          mlen = max(mlen, len[u]);
        }
        for (int q = q0; q < mlen; q += S) {
          int col[kBwdUnroll];
          VT bv[kBwdUnroll], wij[kBwdUnroll];
#pragma unroll
          for (int u = 0; u < kBwdUnroll; ++u) {
            col[u] = -1;
            bv[u] = VT(0);
            if (q < len[u]) {
              col[u] = bcol[b0[u] + q];
              bv[u] = bval[b0[u] + q];
            }
          }
          // W lookups: first probes of all entries, then the rare longer
          // probe paths (bounded by T; a column missing from the row is a
          // pattern mismatch)
          uint32_t h[kBwdUnroll];
          unsigned long long sv[kBwdUnroll];
          int kw[kBwdUnroll];
#pragma unroll
          for (int u = 0; u < kBwdUnroll; ++u) {
            h[u] = scramble_slot((uint32_t)max(col[u], 0), log2T);
            if (PK) sv[u] = slot[h[u]];
            else kw[u] = key[h[u]];
          }
#pragma unroll
          for (int u = 0; u < kBwdUnroll; ++u) {
            wij[u] = VT(0);
            if (col[u] < 0) continue;
            int k = PK ? slot_key(sv[u]) : kw[u];
            for (int pr2 = 0; k != col[u] && k != kEmpty && pr2 < T; ++pr2) {
              h[u] = (h[u] + 1) & (T - 1);
              if (PK) {
                sv[u] = slot[h[u]];
                k = slot_key(sv[u]);
              } else {
                k = key[h[u]];
              }
            }
            if (k != col[u]) {
              miss = true;
              col[u] = -1;
            } else {
              wij[u] = PK ? (VT)slot_val(sv[u]) : wv[h[u]];
            }
          }
#pragma unroll
          for (int u = 0; u < kBwdUnroll; ++u) {
            part[u] += wij[u] * bv[u];
            // keeps the dA terms (and their wait for the B values) ahead of
            // the dB atomics: a wait placed after the atomics would also
            // wait for them
            asm volatile("" : "+v"(part[u]));
          }
          if (dB) {
#pragma unroll
            for (int u = 0; u < kBwdUnroll; ++u) {
              if (col[u] < 0) continue;
              if (det.lo) det_add(det, E, b0[u] + q, av[u] * wij[u]);
              else global_add(&dB[b0[u] + q], av[u] * wij[u]);
            }
          }
        }
        // the S lanes of an entry hold its partial sums: reduce, one store
#pragma unroll
        for (int u = 0; u < kBwdUnroll; ++u) {
          for (int off = S / 2; off > 0; off >>= 1) part[u] += __shfl_xor(part[u], off, S);
          const int ee = e0 + u * ES;
          if (q0 == 0 && ee < nE) sd[ee] = part[u];
        }
      }
      group_sync<GM::BLOCK>();
      if (dA && l < nE) dA[as + c0 + l] = sd[l];
      group_sync<GM::BLOCK>();
    }
    if (miss) atomicOr(&hdr->status, kStatInvalid);  // product outside the given pattern
  }
}

// Heavy rows: W row scattered densely into the slot's scratch row.
template <typename VT>
__global__ __launch_bounds__(1024) void k_bwd_heavy(const Problem *__restrict__ pr,
                                                    const int32_t *__restrict__ rows,
                                                    WsHeader *__restrict__ hdr, int blo, int lS,
                                                    VT *gacc, const int32_t *__restrict__ crp,
                                                    const int32_t *__restrict__ ccol,
                                                    const VT *__restrict__ w,
                                                    VT *__restrict__ dA, VT *__restrict__ dB,
                                                    DetAcc det) {
  __shared__ int sb[1024], sl[1024];
  __shared__ VT sa[1024], sd[1024];
  const int n = pr->n;
  VT *dense = gacc + (size_t)blockIdx.x * n;
  if (hdr->status) return;
  const int start = hdr->bin_start[blo];
  const int count = hdr->bin_start[kHeavyBin + 1] - start;
  const int tid = threadIdx.x;
  const Part &P = pr->part[0];
  const int E = det.lo ? (int)(int32_t)(uint32_t)det.mx[2] : 0;
  __shared__ int item;
  for (int ri = block_next(&hdr->queue[kQueueHeavy], &item); ri < count;
       ri = block_next(&hdr->queue[kQueueHeavy], &item)) {
    const int i = rows[start + ri];
    const int rs = crp[i], re = crp[i + 1];
    for (int t = rs + tid; t < re; t += 1024) dense[ccol[t]] = w[t];
    __threadfence();
    __syncthreads();
    for_each_product_e<true, 1024, VT>(
        P, i, tid, lS, sb, sl, sa, sd,
        [&](int col, VT b, int idx, int ee) {
          const VT wij = dense[col];
          if (dB) {
            if (det.lo) det_add(det, E, idx, sa[ee] * wij);
            else global_add(&dB[idx], sa[ee] * wij);
          }
          return wij * b;
        },
        [&](int p0, int nE) {
          if (dA && tid < nE) dA[p0 + tid] = sd[tid];
        });
    __threadfence();
    __syncthreads();
  }
}

template <int G, typename VT>
static void bwd_launch(const Problem *dpr, const int32_t *rows, WsHeader *hdr, int bin, int lS,
                       int log2T, const int32_t *crp, const int32_t *ccol, const VT *w, VT *dA,
                       VT *dB, const DetAcc &det, int grid, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL((k_bwd_rows<G, VT>), dim3(grid), dim3(BGeom<G>::WG), lds, st, dpr, rows, hdr,
                     bin, lS, log2T, crp, ccol, w, dA, dB, det);
}

// Deterministic dB, before the product pass: the largest |a| and |w|
// (integer maxima of the bit patterns of non-negative values, so no order
// matters), then E with |a w| < 2^E for every term.
template <typename VT>
__global__ void k_det_absmax(const VT *__restrict__ a, int64_t na, const VT *__restrict__ w,
                             int64_t nw, unsigned long long *mx) {
  unsigned long long ma = 0, mw = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t t = t0; t < na; t += stride) ma = max(ma, abs_bits(a[t]));
  int64_t t = t0;
  for (; t + 3 * stride < nw; t += 4 * stride) {  // four loads in flight
    const VT w0 = w[t], w1 = w[t + stride], w2 = w[t + 2 * stride], w3 = w[t + 3 * stride];
    mw = max(mw, max(max(abs_bits(w0), abs_bits(w1)), max(abs_bits(w2), abs_bits(w3))));
  }
  for (; t < nw; t += stride) mw = max(mw, abs_bits(w[t]));
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    ma = max(ma, (unsigned long long)__shfl_xor(ma, off));
    mw = max(mw, (unsigned long long)__shfl_xor(mw, off));
  }
  __shared__ unsigned long long red[2][8];
  if (lane_id() == 0) {
    red[0][threadIdx.x / kWave] = ma;
    red[1][threadIdx.x / kWave] = mw;
  }
  __syncthreads();
  if (threadIdx.x == 0) {  // one atomic per block and word
    for (int w8 = 1; w8 < (int)blockDim.x / kWave; ++w8) {
      ma = max(ma, red[0][w8]);
      mw = max(mw, red[1][w8]);
    }
    if (ma) atomicMax(&mx[0], ma);
    if (mw) atomicMax(&mx[1], mw);
  }
}

template <typename VT>
__global__ void k_det_exponent(unsigned long long *mx, int m, WsHeader *hdr) {
  if (threadIdx.x != 0) return;
  VT ma, mw;
  if (sizeof(VT) == 4) {
    ma = (VT)__uint_as_float((uint32_t)mx[0]);
    mw = (VT)__uint_as_float((uint32_t)mx[1]);
  } else {
    ma = (VT)__longlong_as_double((long long)mx[0]);
    mw = (VT)__longlong_as_double((long long)mx[1]);
  }
  int E = 0;
  if (!isfinite((double)ma) || !isfinite((double)mw)) {
    atomicOr(&hdr->status, kStatInvalid);  // a fixed-point unit needs finite values
  } else if (ma > VT(0) && mw > VT(0)) {
    E = ilogb((double)ma) + ilogb((double)mw) + 2;  // |a| < 2^(ilogb+1), same for |w|
  }
  int L = 1;
  while (L < 31 && (1 << L) < m) ++L;
  const int S = sizeof(VT) == 8 ? 90 - E : 62 - L - E;
  mx[2] = (unsigned long long)(uint32_t)S;
}

template <typename VT>
__global__ void k_det_finish(const unsigned long long *__restrict__ lo,
                             const long long *__restrict__ hi,
                             const unsigned long long *__restrict__ mx, VT *__restrict__ dB,
                             int64_t n, const WsHeader *__restrict__ hdr) {
  if (hdr->status) return;
  const int S = (int)(int32_t)(uint32_t)mx[2];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
    if (sizeof(VT) == 4) {  // 64-bit sums
      dB[q] = (VT)ldexp((double)(long long)lo[q], -S);
      continue;
    }
    unsigned long long l = lo[q], h = (unsigned long long)hi[q];
    const bool neg = (long long)h < 0;
    if (neg) {  // magnitude of the two's complement value
      l = ~l + 1ull;
      h = ~h + (l == 0ull ? 1ull : 0ull);
    }
    const double mag = ldexp((double)h, 64) + (double)l;
    dB[q] = (VT)ldexp(neg ? -mag : mag, -S);
  }
}

size_t bwd_lds_bytes(int b, int G, size_t vbytes) {
  const int WG = G <= kWave ? 256 : G, R = WG / G;
  const size_t T = (size_t)bin_slots(b);
  return (size_t)R * T * (vbytes + 4) + (size_t)R * G * (2 * vbytes + 8);
}

template <typename VT>
static hipError_t backward_impl(const Problem *dpr, const BinPlan &bp, const WsLayout &L,
                                char *ws, const int32_t *crp, const int32_t *ccol, const VT *w,
                                int64_t nnzC, const VT *aval, VT *dA, int64_t nnzA, VT *dB,
                                int64_t nnzB, void *detws, hipStream_t st) {
  WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
  const int32_t *rows = reinterpret_cast<const int32_t *>(ws + L.rows);
  const DevInfo &D = dev_info();
  DetAcc det{nullptr, nullptr, nullptr};
  if (dB && detws) {
    det.mx = static_cast<unsigned long long *>(detws);
    det.lo = det.mx + 4;
    det.hi = reinterpret_cast<long long *>(det.lo + nnzB);
    // zero fills by kernel (capture-safe), then the exponent
    hipLaunchKernelGGL(k_fill_zero<unsigned long long>, dim3(D.cus * 4), dim3(256), 0, st,
                       det.mx, (int64_t)4 + (sizeof(VT) == 8 ? 2 : 1) * nnzB);
    hipLaunchKernelGGL(k_det_absmax<VT>, dim3(D.cus * 4), dim3(256), 0, st, aval, nnzA, w, nnzC,
                       det.mx);
    hipLaunchKernelGGL(k_det_exponent<VT>, dim3(1), dim3(64), 0, st, det.mx, bp.m, hdr);
  }
  if (dA && nnzA > 0)
    hipLaunchKernelGGL(k_fill_zero<VT>, dim3(D.cus * 4), dim3(256), 0, st, dA, nnzA);
  if (dB && nnzB > 0 && !det.lo)
    hipLaunchKernelGGL(k_fill_zero<VT>, dim3(D.cus * 4), dim3(256), 0, st, dB, nnzB);
  for (int b = 1; b <= bp.maxbin; ++b) {
    if (bp.known && bp.count[b] == 0) continue;
    // Groups of at most a wave take half the forward pass's lanes per row
    // and per A entry: a backward product costs more (W lookup, dB atomic)
    // than a forward one, and two rows per wave keep two chains of
    // dependent loads in flight (2^18 rows of 256 products: 0.72 against
    // 0.78 ms with the forward's 64 lanes and 16 per entry).
    const bool half = bp.lanes[b] <= kWave;
    int G = half ? bp.lanes[b] / 2 : bp.lanes[b];
    if (G < 8) G = 8;  // no one-thread-per-row backward kernel
    while (G < 1024 && bwd_lds_bytes(b, G, sizeof(VT)) > D.lds_per_block) G *= 2;
    const int WG = G <= kWave ? 256 : G;
    const int R = WG / G;
    const size_t lds = bwd_lds_bytes(b, G, sizeof(VT));
    int cap = D.cus * (int)std::max<size_t>(1, std::min<size_t>(D.lds_per_cu / lds, 2048 / WG));
    int grid = cap;
    if (bp.known) grid = std::min(cap, (bp.count[b] + R - 1) / R);
    int lt = 0;
    while ((1 << lt) < bin_slots(b)) ++lt;
    int S = bp.sub[b] > 0 ? bp.sub[b] : 16;
    if (half && S > 1) S /= 2;
    if (S > G) S = G;
    int lS = 0;
    while ((1 << lS) < S) ++lS;
    switch (G) {
#define SPG_BWD_CASE(g) \
  case g: bwd_launch<g, VT>(dpr, rows, hdr, b, lS, lt, crp, ccol, w, dA, dB, det, grid, lds, st); break;
      SPG_BWD_CASE(8)
      SPG_BWD_CASE(16)
      SPG_BWD_CASE(32)
      SPG_BWD_CASE(64)
      SPG_BWD_CASE(128)
      SPG_BWD_CASE(256)
      SPG_BWD_CASE(512)
      default: bwd_launch<1024, VT>(dpr, rows, hdr, b, lS, lt, crp, ccol, w, dA, dB, det, grid, lds, st);
#undef SPG_BWD_CASE
    }
  }
  int hc = -1;
  if (bp.known) {
    hc = 0;
    for (int b = bp.maxbin + 1; b <= kHeavyBin; ++b) hc += bp.count[b];
  }
  if (hc != 0) {
    int grid = bp.heavy_slots;
    if (hc > 0 && hc < grid) grid = hc;
    int S = bp.sub[kHeavyBin] > 0 ? bp.sub[kHeavyBin] : 16;
    int lS = 0;
    while ((1 << lS) < S) ++lS;
    hipLaunchKernelGGL(k_bwd_heavy<VT>, dim3(grid), dim3(1024), 0, st, dpr, rows, hdr,
                       bp.maxbin + 1, lS, reinterpret_cast<VT *>(ws + L.heavyacc), crp, ccol, w,
                       dA, dB, det);
  }
  if (det.lo && nnzB > 0)
    hipLaunchKernelGGL(k_det_finish<VT>, dim3(D.cus * 4), dim3(256), 0, st, det.lo, det.hi, det.mx,
                       dB, nnzB, hdr);
  return hipGetLastError();
}

hipError_t launch_backward(const Problem *dpr, const BinPlan &bp, const WsLayout &L, char *ws,
                           const int32_t *crp, const int32_t *ccol, const void *w, int64_t nnzC,
                           const void *aval, void *dA, int64_t nnzA, void *dB, int64_t nnzB,
                           void *detws, int dtype, hipStream_t st) {
  if (dtype == SPG_F64)
    return backward_impl<double>(dpr, bp, L, ws, crp, ccol, static_cast<const double *>(w), nnzC,
                                 static_cast<const double *>(aval), static_cast<double *>(dA),
                                 nnzA, static_cast<double *>(dB), nnzB, detws, st);
  return backward_impl<float>(dpr, bp, L, ws, crp, ccol, static_cast<const float *>(w), nnzC,
                              static_cast<const float *>(aval), static_cast<float *>(dA), nnzA,
                              static_cast<float *>(dB), nnzB, detws, st);
}

size_t det_workspace_bytes(int64_t nnzB) { return (size_t)(4 + 2 * (nnzB > 0 ? nnzB : 0)) * 8; }

hipError_t configure_backward_lds(size_t lds_max) {
  const void *ks[] = {
#define SPG_BWD_K(g) reinterpret_cast<const void *>(&k_bwd_rows<g, float>), \
                     reinterpret_cast<const void *>(&k_bwd_rows<g, double>),
      SPG_BWD_K(8) SPG_BWD_K(16) SPG_BWD_K(32) SPG_BWD_K(64) SPG_BWD_K(128) SPG_BWD_K(256)
      SPG_BWD_K(512) SPG_BWD_K(1024)
#undef SPG_BWD_K
  };
  for (const void *k : ks) {
    hipError_t e =
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace spg

/*
 * Oracle for the per-GPU SpGEMM hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct CPU implementations in FP64 of what the GPU
 * path computes.  Only the tests, the package smoke check and the benchmark's
 * CPU-baseline leg may load this file's library; the product path never does.
 * It shares no code, header or table with the HIP library.
 *
 * Definitions followed (paper sections, not the GPU design):
 *  - §2, problem statement: C = A B for A (m x k) and B (k x n), all in CSR
 *    (row pointer of length m+1, column indices and values of length nnz).
 *    The pattern of C is structural: (i,j) is stored iff some k has
 *    (i,k) in S(A) and (k,j) in S(B); exact cancellations stay stored.
 *    Output rows are canonical (columns strictly ascending).
 *  - §3.3.1, Alg. 1 and Eq. (1)/(2): a process accumulates C_ij over rounds
 *    r of partial products A_ir B_rj; §4.4: the partial products are summed
 *    into one sparse matrix (union of patterns, values added).
 *  - §5.7: Markov clustering iterates expansion (squaring by SpGEMM),
 *    column normalisation, pruning of small entries and an element-wise
 *    power (inflation).  Both step orders are here: the synthetic
 *    workload's (inflate, normalise, prune, top-k, renormalise) and the
 *    paper's own (normalise, prune, element-wise power).  Both hold
 *    X = M^T so that rows of X are columns of M.
 *  - Differentiation at fixed sparsity (not in the paper): for the bilinear
 *    loss L = sum_{(i,j) in S(C)} W_ij C_ij, dL/da_ik = sum_j W_ij b_kj over
 *    (k,j) in S(B), dL/db_kj = sum_i a_ik W_ij over (i,k) in S(A).
 *
 * Algorithm: row-by-row Gustavson with a dense accumulator (a "mark" array
 * of row stamps and an FP64 "acc" array of width n).  Products of two FP32
 * inputs are exact in FP64; the only rounding is in the FP64 sums, taken in
 * A's stored order, then B's stored order.  Row-parallel variants use one
 * private accumulator per OpenMP thread and give the same bits as the serial
 * loop because each row is summed by one thread in the same order.
 *
 * Return codes: 0 ok, 1 invalid input (index out of range), 2 int32
 * overflow of nnz(C), 3 allocation failure, 4 a gradient is requested at an
 * entry whose product is not in the supplied pattern of C.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_INVALID 1
#define ORC_OVERFLOW 2
#define ORC_NOMEM 3
#define ORC_PATTERN 4

/* record an error from inside a parallel region */
#define SETERR(v) do { _Pragma("omp atomic write") err = (v); } while (0)

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/* ---------------------------------------------------------------------- */
/* Row flop upper bound: ub_i = sum over k in S(A)_i of |S(B)_k|.          */
/* This is the number of scalar products row i of C = A B receives (§2).  */
int oracle_rowub(int64_t m, int64_t k, const int64_t *arp, const int32_t *acol,
                 const int64_t *brp, int64_t *ub) {
  for (int64_t i = 0; i < m; ++i) {
    int64_t s = 0;
    for (int64_t p = arp[i]; p < arp[i + 1]; ++p) {
      int32_t c = acol[p];
      if (c < 0 || c >= k) return ORC_INVALID;
      s += brp[c + 1] - brp[c];
    }
    ub[i] = s;
  }
  return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Sum of K block products, C = sum_k A_k B_k (all C_k of one shape m x n).
 * K = 1 is the plain product of §2.  Row i of C accumulates, in ascending
 * k, every product a_ip b_pj of A_k row i with B_k row p -- the rounds of
 * Alg. 1 accumulated into one C row (§3.3.1).
 * Pass 1 (cval == NULL): fills crp[m+1] with the row pointer of C.
 * Pass 2: fills ccol/cval (and cabs = sum |a||b| per entry if non-NULL). */
static int gustavson_batched(int K, int64_t m, int64_t n, const int64_t *kdim,
                             const int64_t *const *arp, const int32_t *const *acol,
                             const double *const *aval, const int64_t *const *brp,
                             const int32_t *const *bcol, const double *const *bval,
                             int64_t *crp, int32_t *ccol, double *cval, double *cabs) {
  int err = ORC_OK;
  int64_t *rowcnt = NULL;
  if (!cval) {
    rowcnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    if (!rowcnt) return ORC_NOMEM;
  }
#pragma omp parallel
  {
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    double *acc = cval ? (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1)) : NULL;
    double *aab = cabs ? (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1)) : NULL;
    int ok = mark && touched && (!cval || acc) && (!cabs || aab);
    if (!ok) {
      SETERR(ORC_NOMEM);
    } else {
      for (int64_t j = 0; j < n; ++j) mark[j] = -1;
    }
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i) {
      if (!ok) continue;
      int64_t nt = 0;
      for (int kk = 0; kk < K; ++kk) {
        for (int64_t p = arp[kk][i]; p < arp[kk][i + 1]; ++p) {
          int32_t r = acol[kk][p];
          if (r < 0 || r >= kdim[kk]) { SETERR(ORC_INVALID); continue; }
          double a = cval ? aval[kk][p] : 0.0;
          for (int64_t q = brp[kk][r]; q < brp[kk][r + 1]; ++q) {
            int32_t j = bcol[kk][q];
            if (j < 0 || j >= n) { SETERR(ORC_INVALID); continue; }
            if (mark[j] != (int32_t)i) {
              mark[j] = (int32_t)i;
              touched[nt++] = j;
              if (acc) acc[j] = 0.0;
              if (aab) aab[j] = 0.0;
            }
            if (acc) acc[j] += a * bval[kk][q];
            if (aab) aab[j] += fabs(a) * fabs(bval[kk][q]);
          }
        }
      }
      if (!cval) {
        rowcnt[i] = nt;
      } else {
        qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
        int64_t o = crp[i];
        if (crp[i + 1] - o != nt) { SETERR(ORC_INVALID); continue; }
        for (int64_t t = 0; t < nt; ++t) {
          int32_t j = touched[t];
          ccol[o + t] = j;
          cval[o + t] = acc[j];
          if (cabs) cabs[o + t] = aab[j];
        }
      }
    }
    free(mark); free(touched); free(acc); free(aab);
  }
  if (!cval && err == ORC_OK) {
    int64_t s = 0;
    crp[0] = 0;
    for (int64_t i = 0; i < m; ++i) { s += rowcnt[i]; crp[i + 1] = s; }
    if (s > INT32_MAX) err = ORC_OVERFLOW;
  }
  free(rowcnt);
  return err;
}

int oracle_spgemm_count(int64_t m, int64_t k, int64_t n, const int64_t *arp,
                        const int32_t *acol, const int64_t *brp, const int32_t *bcol,
                        int64_t *crp) {
  return gustavson_batched(1, m, n, &k, &arp, &acol, NULL, &brp, &bcol, NULL, crp,
                           NULL, NULL, NULL);
}

int oracle_spgemm_fill(int64_t m, int64_t k, int64_t n, const int64_t *arp,
                       const int32_t *acol, const double *aval, const int64_t *brp,
                       const int32_t *bcol, const double *bval, const int64_t *crp,
                       int32_t *ccol, double *cval, double *cabs) {
  return gustavson_batched(1, m, n, &k, &arp, &acol, &aval, &brp, &bcol, &bval,
                           (int64_t *)crp, ccol, cval, cabs);
}

int oracle_batched_count(int K, int64_t m, int64_t n, const int64_t *kdim,
                         const int64_t *const *arp, const int32_t *const *acol,
                         const int64_t *const *brp, const int32_t *const *bcol,
                         int64_t *crp) {
  return gustavson_batched(K, m, n, kdim, arp, acol, NULL, brp, bcol, NULL, crp, NULL,
                           NULL, NULL);
}

int oracle_batched_fill(int K, int64_t m, int64_t n, const int64_t *kdim,
                        const int64_t *const *arp, const int32_t *const *acol,
                        const double *const *aval, const int64_t *const *brp,
                        const int32_t *const *bcol, const double *const *bval,
                        const int64_t *crp, int32_t *ccol, double *cval, double *cabs) {
  return gustavson_batched(K, m, n, kdim, arp, acol, aval, brp, bcol, bval,
                           (int64_t *)crp, ccol, cval, cabs);
}

/* ---------------------------------------------------------------------- */
/* Sparse sum of K same-shape matrices, C = sum_k C_k (§4.4, the sum of the
 * partial products; §3.3.1 Alg. 1 accumulation).  S(C) = union of S(C_k);
 * values added in ascending k; zeros kept.  Written as a union-sum directly,
 * independent of the product code above. */
int oracle_merge(int K, int64_t m, int64_t n, const int64_t *const *rp,
                 const int32_t *const *col, const double *const *val, int64_t *crp,
                 int32_t *ccol, double *cval, double *cabs) {
  int err = ORC_OK;
  int64_t *rowcnt = NULL;
  if (!cval) {
    rowcnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    if (!rowcnt) return ORC_NOMEM;
  }
#pragma omp parallel
  {
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    double *acc = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *aab = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int ok = mark && touched && acc && aab;
    if (!ok) {
      SETERR(ORC_NOMEM);
    } else {
      for (int64_t j = 0; j < n; ++j) mark[j] = -1;
    }
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i) {
      if (!ok) continue;
      int64_t nt = 0;
      for (int kk = 0; kk < K; ++kk) {
        for (int64_t p = rp[kk][i]; p < rp[kk][i + 1]; ++p) {
          int32_t j = col[kk][p];
          if (j < 0 || j >= n) { SETERR(ORC_INVALID); continue; }
          if (mark[j] != (int32_t)i) {
            mark[j] = (int32_t)i; touched[nt++] = j; acc[j] = 0.0; aab[j] = 0.0;
          }
          if (cval) { acc[j] += val[kk][p]; aab[j] += fabs(val[kk][p]); }
        }
      }
      if (!cval) { rowcnt[i] = nt; continue; }
      qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
      int64_t o = crp[i];
      if (crp[i + 1] - o != nt) { SETERR(ORC_INVALID); continue; }
      for (int64_t t = 0; t < nt; ++t) {
        ccol[o + t] = touched[t];
        cval[o + t] = acc[touched[t]];
        if (cabs) cabs[o + t] = aab[touched[t]];
      }
    }
    free(mark); free(touched); free(acc); free(aab);
  }
  if (!cval && err == ORC_OK) {
    int64_t s = 0;
    crp[0] = 0;
    for (int64_t i = 0; i < m; ++i) { s += rowcnt[i]; crp[i + 1] = s; }
    if (s > INT32_MAX) err = ORC_OVERFLOW;
  }
  free(rowcnt);
  return err;
}

/* ---------------------------------------------------------------------- */
/* One Markov-clustering iteration on selected rows of X = M^T (§5.7; the
 * step order and parameters of the synthetic workload):
 *   1. E = X X (row c of E is column c of M M);
 *   2. inflation: e <- e^r (integer r >= 1, by repeated multiplication);
 *   3. divide the row by its sum;
 *   4. prune: drop entries with e < prune (strictly less);
 *   5. if more than topk remain, keep the topk largest, ties going to the
 *      smaller column index;
 *   6. if nothing remains, keep the largest entry of step 3 (ties to the
 *      smaller column index);
 *   7. divide the row by its new sum.
 * Output row t (for input row rows[t]) goes to out_col/out_val at offset
 * t*cap with cap = min(topk, n) entries of room, columns ascending;
 * out_cnt[t] holds its length.  Rows are independent, so any subset can be
 * checked on its own. */
typedef struct { double v; int32_t j; } vj_t;

static int cmp_vj_desc(const void *a, const void *b) {
  const vj_t *x = (const vj_t *)a, *y = (const vj_t *)b;
  if (x->v > y->v) return -1;
  if (x->v < y->v) return 1;
  return (x->j > y->j) - (x->j < y->j);
}

int oracle_mcl_rows(int64_t n, const int64_t *xrp, const int32_t *xcol, const double *xval,
                    int64_t nsel, const int64_t *rows, int r, double prune, int64_t topk,
                    int64_t cap, int32_t *out_cnt, int32_t *out_col, double *out_val) {
  int err = ORC_OK;
  if (r < 1 || topk < 1) return ORC_INVALID;
#pragma omp parallel
  {
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    double *acc = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    vj_t *cand = (vj_t *)malloc(sizeof(vj_t) * (size_t)(n > 0 ? n : 1));
    int ok = mark && touched && acc && cand;
    if (!ok) {
      SETERR(ORC_NOMEM);
    } else {
      for (int64_t j = 0; j < n; ++j) mark[j] = -1;
    }
#pragma omp for schedule(dynamic, 16)
    for (int64_t t = 0; t < nsel; ++t) {
      if (!ok) continue;
      int64_t i = rows[t];
      if (i < 0 || i >= n) { SETERR(ORC_INVALID); continue; }
      int64_t nt = 0;
      /* 1. expansion */
      for (int64_t p = xrp[i]; p < xrp[i + 1]; ++p) {
        int32_t kk = xcol[p];
        double a = xval[p];
        for (int64_t q = xrp[kk]; q < xrp[kk + 1]; ++q) {
          int32_t j = xcol[q];
          if (mark[j] != (int32_t)t) { mark[j] = (int32_t)t; touched[nt++] = j; acc[j] = 0.0; }
          acc[j] += a * xval[q];
        }
      }
      int32_t *oc = out_col + t * cap;
      double *ov = out_val + t * cap;
      if (nt == 0) { out_cnt[t] = 0; continue; }
      qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
      /* 2. inflation and 3. normalisation */
      double s = 0.0;
      for (int64_t u = 0; u < nt; ++u) {
        double e = acc[touched[u]], p = e;
        for (int q = 1; q < r; ++q) p *= e;
        acc[touched[u]] = p;
        s += p;
      }
      int64_t best = 0;
      for (int64_t u = 0; u < nt; ++u) {
        acc[touched[u]] /= s;
        if (acc[touched[u]] > acc[touched[best]]) best = u; /* first max = smallest col */
      }
      /* 4. prune */
      int64_t nc = 0;
      for (int64_t u = 0; u < nt; ++u) {
        double e = acc[touched[u]];
        if (!(e < prune)) { cand[nc].v = e; cand[nc].j = touched[u]; ++nc; }
      }
      /* 5. top-k with ties to the smaller column, 6. never empty */
      if (nc > topk) {
        qsort(cand, (size_t)nc, sizeof(vj_t), cmp_vj_desc);
        nc = topk;
        /* back to column order */
        for (int64_t u = 0; u < nc; ++u) touched[u] = cand[u].j;
        qsort(touched, (size_t)nc, sizeof(int32_t), cmp_i32);
        for (int64_t u = 0; u < nc; ++u) { cand[u].j = touched[u]; cand[u].v = acc[touched[u]]; }
      }
      if (nc == 0) { cand[0].j = touched[best]; cand[0].v = acc[touched[best]]; nc = 1; }
      if (nc > cap) { SETERR(ORC_INVALID); continue; }
      /* 7. renormalise */
      double s2 = 0.0;
      for (int64_t u = 0; u < nc; ++u) s2 += cand[u].v;
      for (int64_t u = 0; u < nc; ++u) { oc[u] = cand[u].j; ov[u] = cand[u].v / s2; }
      out_cnt[t] = (int32_t)nc;
    }
    free(mark); free(touched); free(acc); free(cand);
  }
  return err;
}

/* ---------------------------------------------------------------------- */
/* One Markov-clustering iteration in the order the paper describes for its
 * own runs (§5.7): expansion by squaring, normalisation of the columns,
 * pruning of the entries below a threshold, then an element-wise power of
 * what remains (the paper squares; r is the exponent).  The columns are not
 * normalised again afterwards: the next iteration's normalisation does it.
 * On selected rows of X = M^T:
 *   1. E = X X;
 *   2. divide the row by its sum;
 *   3. prune: drop entries with e < prune (strictly less);
 *   4. if more than topk remain, keep the topk largest, ties going to the
 *      smaller column (with prune > 0 at most 1/prune entries can remain, so
 *      topk >= 1/prune leaves this step inactive);
 *   5. if nothing remains, keep the largest entry of step 2 (ties to the
 *      smaller column);
 *   6. e <- e^r for every kept entry.
 * Same output layout as oracle_mcl_rows. */
int oracle_mcl_rows_paper(int64_t n, const int64_t *xrp, const int32_t *xcol,
                          const double *xval, int64_t nsel, const int64_t *rows, int r,
                          double prune, int64_t topk, int64_t cap, int32_t *out_cnt,
                          int32_t *out_col, double *out_val) {
  int err = ORC_OK;
  if (r < 1 || topk < 1) return ORC_INVALID;
#pragma omp parallel
  {
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    double *acc = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    vj_t *cand = (vj_t *)malloc(sizeof(vj_t) * (size_t)(n > 0 ? n : 1));
    int ok = mark && touched && acc && cand;
    if (!ok) {
      SETERR(ORC_NOMEM);
    } else {
      for (int64_t j = 0; j < n; ++j) mark[j] = -1;
    }
#pragma omp for schedule(dynamic, 16)
    for (int64_t t = 0; t < nsel; ++t) {
      if (!ok) continue;
      int64_t i = rows[t];
      if (i < 0 || i >= n) { SETERR(ORC_INVALID); continue; }
      int64_t nt = 0;
      /* 1. expansion */
      for (int64_t p = xrp[i]; p < xrp[i + 1]; ++p) {
        int32_t kk = xcol[p];
        double a = xval[p];
        for (int64_t q = xrp[kk]; q < xrp[kk + 1]; ++q) {
          int32_t j = xcol[q];
          if (mark[j] != (int32_t)t) { mark[j] = (int32_t)t; touched[nt++] = j; acc[j] = 0.0; }
          acc[j] += a * xval[q];
        }
      }
      int32_t *oc = out_col + t * cap;
      double *ov = out_val + t * cap;
      if (nt == 0) { out_cnt[t] = 0; continue; }
      qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
      /* 2. normalisation */
      double s = 0.0;
      for (int64_t u = 0; u < nt; ++u) s += acc[touched[u]];
      int64_t best = 0;
      for (int64_t u = 0; u < nt; ++u) {
        acc[touched[u]] /= s;
        if (acc[touched[u]] > acc[touched[best]]) best = u; /* first max = smallest col */
      }
      /* 3. prune */
      int64_t nc = 0;
      for (int64_t u = 0; u < nt; ++u) {
        double e = acc[touched[u]];
        if (!(e < prune)) { cand[nc].v = e; cand[nc].j = touched[u]; ++nc; }
      }
      /* 4. top-k, ties to the smaller column */
      if (nc > topk) {
        qsort(cand, (size_t)nc, sizeof(vj_t), cmp_vj_desc);
        nc = topk;
        for (int64_t u = 0; u < nc; ++u) touched[u] = cand[u].j;
        qsort(touched, (size_t)nc, sizeof(int32_t), cmp_i32);
        for (int64_t u = 0; u < nc; ++u) { cand[u].j = touched[u]; cand[u].v = acc[touched[u]]; }
      }
      /* 5. never empty */
      if (nc == 0) { cand[0].j = touched[best]; cand[0].v = acc[touched[best]]; nc = 1; }
      if (nc > cap) { SETERR(ORC_INVALID); continue; }
      /* 6. element-wise power of the kept entries */
      for (int64_t u = 0; u < nc; ++u) {
        double e = cand[u].v, p = e;
        for (int q = 1; q < r; ++q) p *= e;
        oc[u] = cand[u].j;
        ov[u] = p;
      }
      out_cnt[t] = (int32_t)nc;
    }
    free(mark); free(touched); free(acc); free(cand);
  }
  return err;
}

/* ---------------------------------------------------------------------- */
/* Permutation of rows and columns (§5.3: a structured matrix is permuted
 * uniformly at random before the product): B[prow[i], pcol[j]] = A[i, j],
 * each row of B in ascending column order.  prow / pcol NULL means the
 * identity; an array that is not a permutation is an error (1). */
typedef struct { int32_t j; double v; } jv_t;

static int cmp_jv(const void *a, const void *b) {
  int32_t x = ((const jv_t *)a)->j, y = ((const jv_t *)b)->j;
  return (x > y) - (x < y);
}

static int is_permutation(int64_t n, const int32_t *p) {
  if (!p) return 1;
  char *seen = (char *)calloc((size_t)(n > 0 ? n : 1), 1);
  if (!seen) return 0;
  int ok = 1;
  for (int64_t i = 0; i < n && ok; ++i) {
    if (p[i] < 0 || p[i] >= n || seen[p[i]]) ok = 0;
    else seen[p[i]] = 1;
  }
  free(seen);
  return ok;
}

int oracle_permute(int64_t m, int64_t n, const int64_t *arp, const int32_t *acol,
                   const double *aval, const int32_t *prow, const int32_t *pcol,
                   int64_t *brp, int32_t *bcol, double *bval) {
  if (!is_permutation(m, prow) || !is_permutation(n, pcol)) return ORC_INVALID;
  int64_t *from = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
  if (!from) return ORC_NOMEM;
  /* new row prow[i] comes from old row i */
  for (int64_t i = 0; i < m; ++i) from[prow ? prow[i] : i] = i;
  brp[0] = 0;
  for (int64_t r = 0; r < m; ++r) brp[r + 1] = brp[r] + (arp[from[r] + 1] - arp[from[r]]);
  int err = ORC_OK;
  jv_t *row = NULL;
  int64_t cap = 0;
  for (int64_t r = 0; r < m && err == ORC_OK; ++r) {
    int64_t i = from[r], len = arp[i + 1] - arp[i];
    if (len > cap) {
      free(row);
      cap = len;
      row = (jv_t *)malloc(sizeof(jv_t) * (size_t)cap);
      if (!row) { err = ORC_NOMEM; break; }
    }
    for (int64_t t = 0; t < len; ++t) {
      int32_t j = acol[arp[i] + t];
      if (j < 0 || j >= n) { err = ORC_INVALID; break; }
      row[t].j = pcol ? pcol[j] : j;
      row[t].v = aval ? aval[arp[i] + t] : 0.0;
    }
    if (err) break;
    qsort(row, (size_t)len, sizeof(jv_t), cmp_jv);
    for (int64_t t = 0; t < len; ++t) {
      bcol[brp[r] + t] = row[t].j;
      if (bval) bval[brp[r] + t] = row[t].v;
    }
  }
  free(row);
  free(from);
  return err;
}

/* ---------------------------------------------------------------------- */
/* Gradient of L = sum_{(i,j) in S(C)} W_ij C_ij at fixed sparsity, C = A B.
 *   dA_ik = sum_{j in S(B)_k} W_ij b_kj   for (i,k) in S(A)
 *   dB_kj = sum_{i : k in S(A)_i} a_ik W_ij  for (k,j) in S(B)
 * w is scattered densely per row of C; every j reached through S(A)_i and
 * S(B)_k lies in S(C)_i when S(C) is the product pattern, else error 4.
 * Serial over rows so the dB sums run in a fixed order. */
int oracle_backward(int64_t m, int64_t k, int64_t n, const int64_t *arp, const int32_t *acol,
                    const double *aval, const int64_t *brp, const int32_t *bcol,
                    const double *bval, const int64_t *crp, const int32_t *ccol,
                    const double *w, double *da, double *db) {
  int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  double *wd = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  if (!mark || !wd) { free(mark); free(wd); return ORC_NOMEM; }
  for (int64_t j = 0; j < n; ++j) mark[j] = -1;
  if (db) memset(db, 0, sizeof(double) * (size_t)brp[k]);
  int err = ORC_OK;
  for (int64_t i = 0; i < m && err == ORC_OK; ++i) {
    for (int64_t t = crp[i]; t < crp[i + 1]; ++t) { mark[ccol[t]] = (int32_t)i; wd[ccol[t]] = w[t]; }
    for (int64_t p = arp[i]; p < arp[i + 1]; ++p) {
      int32_t kk = acol[p];
      if (kk < 0 || kk >= k) { err = ORC_INVALID; break; }
      double s = 0.0;
      for (int64_t q = brp[kk]; q < brp[kk + 1]; ++q) {
        int32_t j = bcol[q];
        if (j < 0 || j >= n || mark[j] != (int32_t)i) { err = ORC_PATTERN; break; }
        s += wd[j] * bval[q];
        if (db) db[q] += aval[p] * wd[j];
      }
      if (da) da[p] = s;
    }
  }
  free(mark); free(wd);
  return err;
}

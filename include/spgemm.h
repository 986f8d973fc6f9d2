/*
 * spgemm.h -- C ABI of the MI355X (gfx950) local SpGEMM library.
 *
 * The library computes the per-GPU hot path of a distributed sparse matrix
 * product: the local block product C = A B of CSR matrices (paper §2,
 * problem statement), the accumulation of several block products into one C
 * over the rounds of the outer algorithm (§3.3.1, Alg. 1 and Eq. (1)/(2)),
 * the sparse sum of partial products (§4.4), one Markov-clustering
 * iteration (§5.7), and the gradient of a product at fixed sparsity.
 *
 * Conventions shared by every call
 *  - Array arguments inside spg_csr and every buffer argument are DEVICE
 *    pointers on the device that owns `stream`; scalars, handles and the
 *    spg_csr structs themselves are host memory.
 *  - CSR: row_ptr has nrows+1 int32 entries with row_ptr[0] = 0, non-
 *    decreasing, row_ptr[nrows] = nnz; col_idx has nnz int32 entries in
 *    [0, ncols) with no repeated column inside a row; vals has nnz entries
 *    of the call's dtype.  Column order inside a row of A or B may be
 *    arbitrary; every output row is canonical (columns strictly ascending).
 *  - The output pattern is structural: an entry that cancels to 0.0 stays
 *    stored.
 *  - The caller owns all memory: outputs and the workspace.  The library
 *    allocates no device memory and frees none of the caller's.  A plan
 *    holds host metadata and pointers into the caller's workspace and
 *    C row pointer, which must outlive the plan's use.
 *  - Work is queued on `stream` (a hipStream_t; NULL = the null stream).
 *    Calls return once the work is queued, except where a call says it
 *    synchronises.
 *  - Every call returns an spg_status; no exception crosses the ABI and the
 *    library prints nothing.  Asynchronous device faults surface as
 *    SPG_ERR_HIP from a later call.
 */
#ifndef SPGEMM_H_
#define SPGEMM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPG_OK = 0,
  SPG_ERR_INVALID = 1,     /* malformed CSR (with validation on) or bad value */
  SPG_ERR_SHAPE = 2,       /* operand shapes do not line up */
  SPG_ERR_OVERFLOW = 3,    /* nnz of an output exceeds 2^31-1 */
  SPG_ERR_CAPACITY = 4,    /* output larger than the capacity given */
  SPG_ERR_WORKSPACE = 5,   /* workspace missing or too small */
  SPG_ERR_HIP = 6,         /* a HIP runtime call failed */
  SPG_ERR_UNSUPPORTED = 7, /* argument combination not supported */
  SPG_ERR_ARG = 8,         /* NULL pointer or out-of-range scalar argument */
  SPG_ERR_SCRATCH = 9      /* too large for the library's static scratch (no-allocation call) */
} spg_status;

typedef enum { SPG_F32 = 0, SPG_F64 = 1 } spg_dtype;

typedef struct {
  int32_t nrows, ncols;
  int64_t nnz;
  const int32_t *row_ptr; /* device [nrows+1] */
  const int32_t *col_idx; /* device [nnz] */
  const void *vals;       /* device [nnz] of the call's dtype; unused by pattern-only steps */
} spg_csr;

typedef struct spg_plan_s *spg_plan;

/* Maximum number of block products / merge operands in one call. */
#define SPG_MAX_PARTS 16

/* Plan flags (spgemm_plan_create). */
#define SPG_FLAG_VALIDATE 1u  /* check CSR well-formedness on the device (one extra pass) */

/* ------------------------------------------------------------------------
 * Plans and workspace
 * --------------------------------------------------------------------- */

/* Create an empty plan.  flags: SPG_FLAG_*.  Host only. */
int spgemm_plan_create(uint32_t flags, spg_plan *plan_out);

/* Release a plan (host metadata only; no device memory is touched). */
void spgemm_plan_destroy(spg_plan plan);

/* Bytes of device workspace needed by a product with m output rows, n
 * output columns and kmax = the largest inner dimension among its blocks
 * (for a merge pass kmax = m).  Host only; depends on shapes alone, so it
 * can be sized before any device work (and before a graph capture). */
int spgemm_workspace_size(int32_t m, int32_t n, int32_t kmax, size_t *bytes);

/* Status word that device kernels raise in capture-safe mode (overflow,
 * capacity), read back on the host (synchronises the plan's last stream).
 * *device_status_host receives an spg_status.
 * The word lives in the workspace header.  Eager calls clear it when they
 * start.  Capture-safe calls clear it only the first time the plan uses a
 * workspace; afterwards it is sticky: once raised, every later kernel of
 * every capture-safe call on that workspace exits without touching its
 * operands or outputs, so an error raised by any call of a captured
 * sequence (a stage graph, several MCL iterations) is still there at the
 * end of the sequence and no later call reads an output that was never
 * written. */
int spgemm_plan_status(spg_plan plan, int32_t *device_status_host);

/* Queue a clear of the status word of the plan's current workspace on
 * `stream` (capture-safe: one small kernel, no host synchronisation).  A
 * captured sequence starts with it so that every replay reports only its
 * own errors.  SPG_ERR_WORKSPACE if the plan has not been given a workspace
 * yet. */
int spgemm_plan_clear_status(spg_plan plan, void *stream);

/* Last known nnz of the plan's output (after a synchronising symbolic call
 * or after spgemm_plan_status), and the number of scalar products. */
int spgemm_plan_info(spg_plan plan, int64_t *nnz, int64_t *products);

const char *spgemm_status_string(int status);

/* Rows per bin after an eager symbolic call (host arrays of SPG_NBINS),
 * bins by products per row.  The numeric pass reuses the symbolic bins (a
 * row's products bound its nnz, so a table sized for them holds the row):
 * num_counts equals sym_counts.  Bin b >= 1 holds rows with key in
 * (e[b-1], e[b]] with e[b] = 8*2^b by default (bin 1: 1..16) or the tuned
 * spg_tuning.bin_edge, bin 0 empty rows, bin 12 the rows beyond every LDS
 * table of the pass in question.
 * SPG_ERR_ARG if the counts were not read back (capture-safe call). */
int spgemm_plan_bins(spg_plan plan, int32_t *sym_counts, int32_t *num_counts);

/* ------------------------------------------------------------------------
 * Product  C = sum_{k<K} A_k B_k   (K = 1: the plain block product, §2;
 * K > 1: the per-round partial products of §3.3.1 Alg. 1 accumulated into
 * one C without materialising the partials, the fused form of §4.4's sum).
 * All A_k share nrows = m, all B_k share ncols = n, A_k.ncols = B_k.nrows.
 * --------------------------------------------------------------------- */

/* Symbolic pass: per-row products (flop upper bound), row binning, exact
 * distinct-column count per row and the exclusive scan into C_row_ptr.
 *   C_row_ptr   device [m+1], written.
 *   C_nnz_host  non-NULL: the call synchronises `stream` and stores nnz(C)
 *               (eager mode).  NULL: nothing is read back (capture-safe
 *               mode); nnz(C) > capacity raises SPG_ERR_CAPACITY in the
 *               device status word and the numeric pass then writes nothing.
 *   capacity    capture-safe mode only: entries the caller allocated for C.
 *   workspace   device, at least spgemm_workspace_size(m, n, max_k k_k).
 * Errors: SPG_ERR_SHAPE, SPG_ERR_ARG, SPG_ERR_WORKSPACE, SPG_ERR_OVERFLOW
 * (eager: returned; capture-safe: device status), SPG_ERR_INVALID (with
 * validation on), SPG_ERR_HIP. */
int spgemm_symbolic(spg_plan plan, int32_t K, const spg_csr *A, const spg_csr *B,
                    int32_t *C_row_ptr, int64_t *C_nnz_host, int64_t capacity,
                    void *workspace, size_t ws_bytes, void *stream);

/* Symbolic pass that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  It is spgemm_symbolic in capture-safe
 * mode (nothing is read back; nnz(C) > capacity raises SPG_ERR_CAPACITY in
 * the device status word) whose workspace is a static device array inside
 * the library, SPG_SCRATCH_BYTES per device, instead of a caller argument.
 * The caller still passes the operands, C_row_ptr [m+1] and, afterwards,
 * C_col_idx / C_vals [capacity] to spgemm_numeric on the same plan (which
 * then also works in that array).  The library takes the array's device
 * address once per device, on that device's first call.
 *  - Limit: a problem whose workspace (spgemm_workspace_size with fewer
 *    concurrent heavy rows, at least one) exceeds SPG_SCRATCH_BYTES returns
 *    SPG_ERR_SCRATCH before any work is queued; about 9 m + 8 n bytes with
 *    one heavy row, so m = n = 2^22 is beyond it.
 *  - Sharing: every such call on a device uses that device's one array and
 *    leaves its contents behind (the kernels clear what they need).  Calls
 *    that overlap on one device race, including a symbolic call of one plan
 *    between the symbolic and numeric calls of another: serialise them (one
 *    stream, or events).
 *  - Status: as for other capture-safe calls, the status word (in the
 *    array) is cleared on a plan's first use of the array and is sticky
 *    afterwards; spgemm_plan_clear_status clears it, spgemm_plan_status
 *    reads it.
 * Errors: as spgemm_symbolic, plus SPG_ERR_SCRATCH, and SPG_ERR_HIP if the
 * array's device address cannot be obtained. */
#define SPG_SCRATCH_BYTES (128u << 20)
int spgemm_symbolic_noalloc(spg_plan plan, int32_t K, const spg_csr *A, const spg_csr *B,
                            int32_t *C_row_ptr, int64_t capacity, void *stream);

/* Numeric pass: values and canonical column order of C, for the same K
 * operand patterns as the plan's symbolic call (values may differ: the plan
 * is reusable at fixed sparsity).  Patterns that differ from the symbolic
 * call's are the caller's error: a count that no longer matches is flagged
 * (SPG_ERR_INVALID), but a change that keeps every row's product and
 * column counts can go unseen; C is then unspecified, and every write still
 * stays inside C_col_idx and C_vals.
 *   C_col_idx  device [nnz(C)] int32, written.
 *   C_vals     device [nnz(C)] of dtype, written.
 * Accumulation is in dtype (FP32 or FP64). */
int spgemm_numeric(spg_plan plan, int32_t K, const spg_csr *A, const spg_csr *B,
                   spg_dtype dtype, int32_t *C_col_idx, void *C_vals, void *stream);

/* ------------------------------------------------------------------------
 * Sparse sum  C = sum_{k<K} P_k  of same-shape matrices (§4.4: the partial
 * products of the rounds summed into one C; union of patterns, values
 * added).  The P_k need not be canonical.  Two phases share the plan:
 * first call with C_col_idx == NULL and C_vals == NULL to build C_row_ptr
 * (and nnz, as in spgemm_symbolic), then call again with the output
 * buffers to fill them.
 * --------------------------------------------------------------------- */
int spgemm_merge(spg_plan plan, int32_t K, const spg_csr *P, spg_dtype dtype,
                 int32_t *C_row_ptr, int64_t *C_nnz_host, int64_t capacity,
                 int32_t *C_col_idx, void *C_vals, void *workspace, size_t ws_bytes,
                 void *stream);

/* ------------------------------------------------------------------------
 * Backward at fixed sparsity of C = A B (K = 1) for a loss L with
 * dL/dC = dC on S(C):
 *   dA = (dC B^T) restricted to S(A),  dB = (A^T dC) restricted to S(B).
 *   dC         CSR with the pattern the plan's numeric pass produced; its
 *              vals are dL/dC_ij.
 *   dA_vals    device [nnz(A)] or NULL (not computed), written.
 *   dB_vals    device [nnz(B)] or NULL, written (zeroed first, then
 *              accumulated with device float atomics: the summation order
 *              of a dB entry is not fixed; spgemm_backward_deterministic
 *              below fixes the result).
 * Not in the paper; the definition is the derivative of the bilinear map
 * (A, B) -> A B at a fixed pattern. */
int spgemm_backward(spg_plan plan, const spg_csr *A, const spg_csr *B, const spg_csr *dC,
                    spg_dtype dtype, void *dA_vals, void *dB_vals, void *stream);

/* The same backward with dB_vals the same bits on every run: each term
 * a_ik * dC_ij (rounded in dtype, as in spgemm_backward) is added into a
 * fixed-point integer per B entry, with 2^E above every |a_ik| * |dC_ij|
 * (E from the largest |a| and |dC| of the call); integer addition does not
 * depend on the order.  FP64: 128-bit sums with the unit 2^(E - 90) (a term
 * loses less than 2^-90 times the largest term of the call).  FP32: 64-bit
 * sums with the unit 2^(E - 62 + L), 2^L >= the rows of A (a term loses
 * less than 2^(L - 62) <= 2^-31 times the largest term).  Each sum is
 * converted to dtype once.  dA_vals is computed as
 * by spgemm_backward (each dA entry has one summing lane group: already
 * deterministic).
 *   workspace  device, 8-byte aligned, at least
 *              spgemm_backward_deterministic_workspace_size(nnz(B)) bytes
 *              (unused when dB_vals is NULL); the caller owns it.
 * Non-finite values in A or dC raise SPG_ERR_INVALID in the plan's device
 * status word, and dB_vals is then not written.  Capture-safe: every fill
 * is a kernel, nothing is read back. */
int spgemm_backward_deterministic_workspace_size(int64_t nnzB, size_t *bytes);
int spgemm_backward_deterministic(spg_plan plan, const spg_csr *A, const spg_csr *B,
                                  const spg_csr *dC, spg_dtype dtype, void *dA_vals,
                                  void *dB_vals, void *workspace, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Permutation B = P_r A P_c^T, i.e. B[row_perm[i], col_perm[j]] = A[i, j]
 * (§5.3: the rows and columns of a structured matrix are permuted uniformly
 * at random as a light preprocessing step, which turns diagonal bands into
 * unstructured sparsity; row_perm == col_perm is the symmetric permutation,
 * under which (P A P^T)^2 = P A^2 P^T).
 *   A          CSR, any column order; nrows m, ncols n.
 *   row_perm   device int32 [m], a permutation of 0..m-1, or NULL (identity).
 *   col_perm   device int32 [n], a permutation of 0..n-1, or NULL (identity).
 *   B_row_ptr  device [m+1], written.
 *   B_col_idx  device [nnz(A)], written, every row in ascending order.
 *   B_vals     device [nnz(A)] of dtype, written, or NULL (pattern only).
 *   workspace  device, at least spgemm_permute_workspace_size(m, n).
 * Capture-safe: nothing is read back.  An array that is not a permutation
 * raises SPG_ERR_INVALID in the plan's device status word
 * (spgemm_plan_status; cleared on the plan's first use of the workspace,
 * sticky afterwards) and nothing more is written.  Values are copied, not
 * computed. */
int spgemm_permute_workspace_size(int32_t m, int32_t n, size_t *bytes);
int spgemm_permute(spg_plan plan, const spg_csr *A, const int32_t *row_perm,
                   const int32_t *col_perm, spg_dtype dtype, int32_t *B_row_ptr,
                   int32_t *B_col_idx, void *B_vals, void *workspace, size_t ws_bytes,
                   void *stream);

/* ------------------------------------------------------------------------
 * One Markov-clustering iteration (§5.7) on X = M^T (row c of X is
 * column c of M, so (M M)^T = X X):
 *   E = X X; e <- e^r; divide each row by its sum; drop e < prune;
 *   keep the topk largest (ties to the smaller column); an emptied row
 *   keeps its largest entry; divide each row by its new sum.
 * The unpruned product is never stored.
 *   Y_row_ptr  device [n+1], written.
 *   Y_col_idx, Y_vals  device, capacity entries each (capacity >= the
 *              output nnz; n*min(topk,n) always suffices), written.
 *   capacity   entries of Y_col_idx / Y_vals; an output larger than it
 *              raises SPG_ERR_CAPACITY and nothing is written to them.
 *              Eager mode may pass -1 (unchecked: the caller sized the
 *              buffers for n*min(topk,n)).
 *   Y_nnz_host non-NULL: synchronises and returns nnz(Y) (or the error);
 *              NULL: capture-safe, errors go to the device status word.
 *   workspace  device, at least spgemm_mcl_workspace_size(n, topk).
 * FP32 only (dtype SPG_F32); inflation exponent r in 1..8; n <= 2^24
 * (SPG_ERR_UNSUPPORTED above).  X must be canonical (columns ascending
 * within a row, no repeats) with finite values, as MCL iterates on a
 * stochastic matrix and this call's own output is canonical: rows whose
 * columns do not fit the largest LDS table are swept in column order and
 * rely on it.  Such rows accumulate exactly-rounded products in 64-bit fixed
 * point scaled per row, so their sums do not depend on the order of the
 * adds; rows held in an LDS table (up to twice that table's product bin)
 * add in FP32, in no fixed order. */
int spgemm_mcl_workspace_size(int32_t n, int32_t topk, size_t *bytes);
int spgemm_mcl_iteration(spg_plan plan, const spg_csr *X, int32_t r, float prune,
                         int32_t topk, int32_t *Y_row_ptr, int32_t *Y_col_idx,
                         float *Y_vals, int64_t capacity, int64_t *Y_nnz_host,
                         void *workspace, size_t ws_bytes, void *stream);

/* The same iteration in either step order.
 *   SPG_MCL_INFLATE_FIRST  as spgemm_mcl_iteration above.
 *   SPG_MCL_PAPER          the order §5.7 describes for the paper's own runs:
 *                          E = X X; divide each row by its sum; drop
 *                          e < prune; keep the topk largest (ties to the
 *                          smaller column); an emptied row keeps its largest
 *                          entry; e <- e^r for every kept entry, with no
 *                          second normalisation (the next iteration's
 *                          normalisation does it).  With prune > 0 at most
 *                          1/prune entries survive per row, so topk =
 *                          floor(1/prune) leaves the top-k step inactive and
 *                          sizes the capacity (the paper's 0.002: 500).
 * Arguments, capacity, workspace and errors as for spgemm_mcl_iteration. */
#define SPG_MCL_INFLATE_FIRST 0
#define SPG_MCL_PAPER 1
int spgemm_mcl_iteration_order(spg_plan plan, const spg_csr *X, int32_t order, int32_t r,
                               float prune, int32_t topk, int32_t *Y_row_ptr,
                               int32_t *Y_col_idx, float *Y_vals, int64_t capacity,
                               int64_t *Y_nnz_host, void *workspace, size_t ws_bytes,
                               void *stream);

/* ------------------------------------------------------------------------
 * Tuning (chosen by the autotuner outside any graph capture).
 * --------------------------------------------------------------------- */
#define SPG_NBINS 16

typedef struct {
  int32_t lanes[SPG_NBINS];     /* threads cooperating on one row, per bin (power of 2, 8..1024;
                                   bin 1 also 1: one thread per row, products sorted in
                                   registers) */
  int32_t sub[SPG_NBINS];       /* threads sharing one A entry's B row, per bin (power of 2, <= 64) */
  int32_t sym_sub[SPG_NBINS];   /* the same for the symbolic count (power of 2, <= 64) */
  int32_t heavy_slots;          /* concurrent heavy rows (0 = as many as the workspace holds) */
  int32_t max_window;           /* longest hash probe kept in the fast numeric kernel (1..32) */
  int32_t bin_edge[SPG_NBINS];  /* upper products-per-row key of LDS bin b of the product
                                   passes, 1..8*2^b, or 0 for 8*2^b (the bin's table size / 2).
                                   Rows with keys in (bin_edge[b], 8*2^b] go to bin b+1, whose
                                   tables are twice as large: the edge sets both the bin
                                   threshold and the table load factor of those rows.
                                   Effective edges are made non-decreasing; the last LDS bin
                                   always keeps its full edge.  MCL keeps the default edges. */
} spg_tuning;

int spgemm_default_tuning(spg_tuning *t);
int spgemm_plan_set_tuning(spg_plan plan, const spg_tuning *t);

#ifdef __cplusplus
}
#endif
#endif /* SPGEMM_H_ */

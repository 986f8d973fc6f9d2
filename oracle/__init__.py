"""FP64 CPU oracle for the local SpGEMM hot path -- TEST INFRASTRUCTURE ONLY.

Only tests, the package smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps oracle/oracle.c (plain C, FP64, row-by-row
Gustavson with a dense accumulator) through ctypes and never touches the HIP
library.  Inputs are any objects with `shape`, `indptr`, `indices` and
`data` attributes (host numpy arrays); values are upcast to float64, which
is exact for float32 inputs.

Functions and the paper passages they follow:
  rowub     -- products per row of C = A B (§2 problem statement)
  spgemm    -- C = A B in canonical CSR, structural pattern (§2)
  batched   -- C = sum_k A_k B_k accumulated per row over the rounds
               (§3.3.1, Alg. 1 and Eq. (1)/(2))
  merge     -- C = sum_k C_k, union pattern, values added (§4.4)
  mcl_rows  -- one Markov-clustering iteration on selected rows of X = M^T
               (§5.7; order="workload": inflate, normalise, prune, top-k,
               renormalise; order="paper": normalise, prune, element-wise
               power, the order the paper describes for its runs)
  backward  -- dA, dB of L = <W, C> at fixed sparsity (not in the paper)
  permute   -- B[prow[i], pcol[j]] = A[i, j], rows in ascending column
               order (§5.3: random permutation as preprocessing)
"""
from __future__ import annotations

import ctypes as C
import os
import types

import numpy as np

from . import build as _build

_lib = None
_P = C.c_void_p
_I64 = C.c_int64

ERRORS = {1: "invalid input", 2: "nnz(C) overflows int32", 3: "out of memory",
          4: "product outside the given pattern of C"}


class OracleError(RuntimeError):
    pass


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(path)
        for name in ["oracle_rowub", "oracle_spgemm_count", "oracle_spgemm_fill",
                     "oracle_batched_count", "oracle_batched_fill", "oracle_merge",
                     "oracle_mcl_rows", "oracle_mcl_rows_paper", "oracle_backward", "oracle_permute",
                     "oracle_num_threads"]:
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise OracleError(ERRORS.get(rc, f"error {rc}"))


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(_P) if a is not None else None


class CSR(types.SimpleNamespace):
    """Host CSR result: shape, indptr (int64), indices (int32), data (float64)."""

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])


def _csr(shape, indptr, indices, data):
    return CSR(shape=tuple(shape), indptr=indptr, indices=indices, data=data)


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_threads(t: int) -> None:
    lib().oracle_set_threads(C.c_int(t))


def rowub(A, B) -> np.ndarray:
    m, k = A.shape
    arp, acol, brp = _i64(A.indptr), _i32(A.indices), _i64(B.indptr)
    ub = np.zeros(m, dtype=np.int64)
    _check(lib().oracle_rowub(_I64(m), _I64(k), _p(arp), _p(acol), _p(brp), _p(ub)))
    return ub


def spgemm(A, B, with_abs: bool = False):
    """C = A B (FP64).  Returns a CSR namespace; with_abs also returns
    S_ij = sum_k |a_ik||b_kj| used to scale tolerances."""
    m, k = A.shape
    k2, n = B.shape
    if k != k2:
        raise OracleError("inner dimensions differ")
    arp, acol, aval = _i64(A.indptr), _i32(A.indices), _f64(A.data)
    brp, bcol, bval = _i64(B.indptr), _i32(B.indices), _f64(B.data)
    crp = np.zeros(m + 1, dtype=np.int64)
    L = lib()
    _check(L.oracle_spgemm_count(_I64(m), _I64(k), _I64(n), _p(arp), _p(acol), _p(brp),
                                 _p(bcol), _p(crp)))
    nnz = int(crp[-1])
    ccol = np.zeros(nnz, dtype=np.int32)
    cval = np.zeros(nnz, dtype=np.float64)
    cabs = np.zeros(nnz, dtype=np.float64) if with_abs else None
    _check(L.oracle_spgemm_fill(_I64(m), _I64(k), _I64(n), _p(arp), _p(acol), _p(aval),
                                _p(brp), _p(bcol), _p(bval), _p(crp), _p(ccol), _p(cval),
                                _p(cabs)))
    Cm = _csr((m, n), crp, ccol, cval)
    return (Cm, cabs) if with_abs else Cm


def _ptrs(arrs):
    return (_P * len(arrs))(*[a.ctypes.data for a in arrs])


def batched(pairs, with_abs: bool = False):
    """C = sum_k A_k B_k, accumulated per row of C in ascending k."""
    K = len(pairs)
    m = pairs[0][0].shape[0]
    n = pairs[0][1].shape[1]
    kdim = np.array([A.shape[1] for A, _ in pairs], dtype=np.int64)
    for A, B in pairs:
        if A.shape[0] != m or B.shape[1] != n or A.shape[1] != B.shape[0]:
            raise OracleError("block shapes do not line up")
    arp = [_i64(A.indptr) for A, _ in pairs]
    acol = [_i32(A.indices) for A, _ in pairs]
    aval = [_f64(A.data) for A, _ in pairs]
    brp = [_i64(B.indptr) for _, B in pairs]
    bcol = [_i32(B.indices) for _, B in pairs]
    bval = [_f64(B.data) for _, B in pairs]
    crp = np.zeros(m + 1, dtype=np.int64)
    L = lib()
    _check(L.oracle_batched_count(C.c_int(K), _I64(m), _I64(n), _p(kdim), _ptrs(arp),
                                  _ptrs(acol), _ptrs(brp), _ptrs(bcol), _p(crp)))
    nnz = int(crp[-1])
    ccol = np.zeros(nnz, dtype=np.int32)
    cval = np.zeros(nnz, dtype=np.float64)
    cabs = np.zeros(nnz, dtype=np.float64) if with_abs else None
    _check(L.oracle_batched_fill(C.c_int(K), _I64(m), _I64(n), _p(kdim), _ptrs(arp),
                                 _ptrs(acol), _ptrs(aval), _ptrs(brp), _ptrs(bcol),
                                 _ptrs(bval), _p(crp), _p(ccol), _p(cval), _p(cabs)))
    Cm = _csr((m, n), crp, ccol, cval)
    return (Cm, cabs) if with_abs else Cm


def merge(parts, with_abs: bool = False):
    """C = sum_k C_k over same-shape CSR matrices (union pattern)."""
    K = len(parts)
    m, n = parts[0].shape
    for P in parts:
        if tuple(P.shape) != (m, n):
            raise OracleError("merge operands differ in shape")
    rp = [_i64(P.indptr) for P in parts]
    col = [_i32(P.indices) for P in parts]
    val = [_f64(P.data) for P in parts]
    crp = np.zeros(m + 1, dtype=np.int64)
    L = lib()
    _check(L.oracle_merge(C.c_int(K), _I64(m), _I64(n), _ptrs(rp), _ptrs(col), _ptrs(val),
                          _p(crp), None, None, None))
    nnz = int(crp[-1])
    ccol = np.zeros(nnz, dtype=np.int32)
    cval = np.zeros(nnz, dtype=np.float64)
    cabs = np.zeros(nnz, dtype=np.float64) if with_abs else None
    _check(L.oracle_merge(C.c_int(K), _I64(m), _I64(n), _ptrs(rp), _ptrs(col), _ptrs(val),
                          _p(crp), _p(ccol), _p(cval), _p(cabs)))
    Cm = _csr((m, n), crp, ccol, cval)
    return (Cm, cabs) if with_abs else Cm


def mcl_rows(X, rows, r: int = 2, prune: float = 1e-4, topk: int = 1000,
             order: str = "workload", flat: bool = False):
    """One MCL iteration on the given rows of X = M^T.  Returns
    (counts[nsel], cols list, vals list) with rows in canonical order, or
    with flat=True (counts, all columns, all values) concatenated."""
    n = X.shape[0]
    rows = _i64(rows)
    cap = int(min(topk, n))
    nsel = rows.size
    xrp, xcol, xval = _i64(X.indptr), _i32(X.indices), _f64(X.data)
    cnt = np.zeros(nsel, dtype=np.int32)
    oc = np.zeros(max(nsel * cap, 1), dtype=np.int32)
    ov = np.zeros(max(nsel * cap, 1), dtype=np.float64)
    if order == "workload":
        fn = lib().oracle_mcl_rows
    elif order == "paper":
        fn = lib().oracle_mcl_rows_paper
    else:
        raise ValueError(f"unknown MCL step order {order!r}")
    _check(fn(_I64(n), _p(xrp), _p(xcol), _p(xval), _I64(nsel), _p(rows), C.c_int(r),
              C.c_double(prune), _I64(topk), _I64(cap), _p(cnt), _p(oc), _p(ov)))
    if flat:
        keep = (np.arange(cap)[None, :] < cnt[:, None]).reshape(-1)
        return cnt, oc[:nsel * cap][keep], ov[:nsel * cap][keep]
    cols = [oc[t * cap: t * cap + cnt[t]].copy() for t in range(nsel)]
    vals = [ov[t * cap: t * cap + cnt[t]].copy() for t in range(nsel)]
    return cnt, cols, vals


def mcl_step(X, r: int = 2, prune: float = 1e-4, topk: int = 1000, order: str = "workload"):
    """One MCL iteration on every row; returns the new X as CSR (FP64)."""
    n = X.shape[0]
    cnt, cols, vals = mcl_rows(X, np.arange(n), r, prune, topk, order, flat=True)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt, out=indptr[1:])
    return _csr((n, n), indptr, cols.astype(np.int32), vals)


def backward(A, B, Cpat, W):
    """(dA, dB) of L = sum_{S(C)} W_ij C_ij, C = A B, on S(A) and S(B).
    W is aligned with Cpat's stored entries."""
    m, k = A.shape
    _, n = B.shape
    arp, acol, aval = _i64(A.indptr), _i32(A.indices), _f64(A.data)
    brp, bcol, bval = _i64(B.indptr), _i32(B.indices), _f64(B.data)
    crp, ccol, w = _i64(Cpat.indptr), _i32(Cpat.indices), _f64(W)
    da = np.zeros(arp[-1], dtype=np.float64)
    db = np.zeros(brp[-1], dtype=np.float64)
    _check(lib().oracle_backward(_I64(m), _I64(k), _I64(n), _p(arp), _p(acol), _p(aval),
                                 _p(brp), _p(bcol), _p(bval), _p(crp), _p(ccol), _p(w),
                                 _p(da), _p(db)))
    return da, db


def permute(A, prow=None, pcol=None):
    """B[prow[i], pcol[j]] = A[i, j] (None = identity), rows sorted."""
    m, n = A.shape
    arp, acol = _i64(A.indptr), _i32(A.indices)
    aval = None if A.data is None else _f64(A.data)
    pr = None if prow is None else _i32(prow)
    pc = None if pcol is None else _i32(pcol)
    brp = np.zeros(m + 1, dtype=np.int64)
    bcol = np.zeros(max(int(arp[-1]), 1), dtype=np.int32)
    bval = None if aval is None else np.zeros(max(int(arp[-1]), 1), dtype=np.float64)
    _check(lib().oracle_permute(_I64(m), _I64(n), _p(arp), _p(acol), _p(aval), _p(pr), _p(pc),
                                _p(brp), _p(bcol), _p(bval)))
    nnz = int(brp[-1])
    return _csr((m, n), brp, bcol[:nnz], None if bval is None else bval[:nnz])

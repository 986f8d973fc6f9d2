"""Seeded synthetic CSR inputs for the local SpGEMM hot path.

This module is shared by the tests, the benchmark and the oracle checks.  It
only draws random sparsity patterns and values; it holds none of the
product's arithmetic (no products, sums, scans or normalisation of results).

Matrices are stored in CSR as in the paper's problem statement (§2: a row
pointer of length m+1, a column-index array and a value array, both of
length nnz).  Indices are int32, row pointers int64 on the host (the device
boundary uses int32 and converts).

Workload shapes follow the paper's regime of unstructured matrices (§1, §5.2
Table 2: near-uniform nonzero distribution, imbalance ~1.02) with an R-MAT
variant standing in for its skewed matrices (imbalance 4.6-20.6).
Random numbers are numpy PCG64 streams spawned from a SeedSequence, so the
same seed gives the same matrix on every machine.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "HostCSR", "rng_for", "uniform_csr", "varnnz_csr", "rmat_csr",
    "mcl_matrix", "identity_csr", "permutation_csr", "draw_values",
    "column_blocks", "split_inner", "shuffle_rows",
    "batched_uniform_blocks", "batched_rmat_blocks", "aggregation_csr", "banded_csr",
    "random_permutation",
]


@dataclasses.dataclass
class HostCSR:
    """Host CSR triple (scipy-style attribute names)."""
    shape: tuple
    indptr: np.ndarray   # int64 [m+1]
    indices: np.ndarray  # int32 [nnz]
    data: np.ndarray     # float32/float64 [nnz] (may be None for a pattern)

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def row(self, i):
        s, e = int(self.indptr[i]), int(self.indptr[i + 1])
        return self.indices[s:e], (None if self.data is None else self.data[s:e])

    def with_data(self, data) -> "HostCSR":
        return HostCSR(self.shape, self.indptr, self.indices, data)

    def astype(self, dtype) -> "HostCSR":
        return self.with_data(self.data.astype(dtype))


def rng_for(seed: int, stream: int = 0) -> np.random.Generator:
    """PCG64 generator for (seed, stream): independent streams per matrix."""
    ss = np.random.SeedSequence(seed)
    child = ss.spawn(stream + 1)[stream]
    return np.random.Generator(np.random.PCG64(child))


def draw_values(rng, n: int, kind: str, dtype) -> np.ndarray:
    """Values of the stored entries.

    kind: 'u01'    uniform in (0,1], drawn as 1-U[0,1) in float64;
          'normal' N(0,1) drawn in float64;
          'int'    small nonzero integers in {-4..4}\\{0} (every partial sum
                   is exactly representable, so any summation order gives the
                   same bits);
          'pos_int' small integers in {1..4};
          'one'    all ones.
    Values are rounded to `dtype` once, after drawing.
    """
    if kind == "u01":
        v = 1.0 - rng.random(n)
    elif kind == "normal":
        v = rng.standard_normal(n)
    elif kind == "int":
        v = rng.integers(1, 5, size=n) * rng.choice(np.array([-1, 1]), size=n)
        v = v.astype(np.float64)
    elif kind == "pos_int":
        v = rng.integers(1, 5, size=n).astype(np.float64)
    elif kind == "one":
        v = np.ones(n)
    else:
        raise ValueError(f"unknown value kind {kind!r}")
    return v.astype(dtype)


def _distinct_rows(rng, m: int, n: int, d: int) -> np.ndarray:
    """[m, d] int64 matrix whose rows hold d distinct columns in [0, n)."""
    if d > n:
        raise ValueError(f"cannot draw {d} distinct columns out of {n}")
    if d == 0 or m == 0:
        return np.zeros((m, d), dtype=np.int64)
    if 4 * d > n:  # dense-ish: per-row permutation prefix
        return np.stack([rng.permutation(n)[:d] for _ in range(m)]).astype(np.int64)
    cols = rng.integers(0, n, size=(m, d), dtype=np.int64)
    s = np.sort(cols, axis=1)
    bad = np.nonzero((s[:, 1:] == s[:, :-1]).any(axis=1))[0]
    for i in bad:  # keep the first copy of each column, redraw the repeats
        row = cols[i]
        _, first = np.unique(row, return_index=True)
        keep = np.zeros(d, dtype=bool)
        keep[first] = True
        have = set(row[keep].tolist())
        for p in np.nonzero(~keep)[0]:
            while True:
                c = int(rng.integers(0, n))
                if c not in have:
                    have.add(c)
                    row[p] = c
                    break
    return cols


def _csr_from_rows(m, n, cols_md, lens, vals_rng, values, dtype, sort_rows):
    """Pack the first lens[i] entries of row i of cols_md into CSR."""
    d = cols_md.shape[1]
    keep = np.arange(d)[None, :] < lens[:, None]
    if sort_rows:
        big = np.where(keep, cols_md, np.iinfo(np.int64).max)
        cols_md = np.sort(big, axis=1)
        keep = np.arange(d)[None, :] < lens[:, None]
    indices = cols_md[keep].astype(np.int32)
    indptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lens, out=indptr[1:])
    data = None if values is None else draw_values(vals_rng, indices.size, values, dtype)
    return HostCSR((m, n), indptr, indices, data)


def uniform_csr(m: int, n: int, d: int, seed: int, dtype=np.float32,
                values: str | None = "u01", stream: int = 0,
                sort_rows: bool = True) -> HostCSR:
    """m x n CSR with exactly d distinct uniform-random columns per row."""
    rng = rng_for(seed, stream)
    cols = _distinct_rows(rng, m, n, d)
    lens = np.full(m, d, dtype=np.int64)
    return _csr_from_rows(m, n, cols, lens, rng, values, dtype, sort_rows)


def varnnz_csr(m: int, n: int, dmin: int, dmax: int, seed: int,
               dtype=np.float32, values: str | None = "normal", stream: int = 0,
               sort_rows: bool = True) -> HostCSR:
    """m x n CSR whose row i holds len_i ~ U{dmin..dmax} distinct uniform columns."""
    rng = rng_for(seed, stream)
    lens = rng.integers(dmin, dmax + 1, size=m).astype(np.int64)
    cols = _distinct_rows(rng, m, n, dmax)
    return _csr_from_rows(m, n, cols, lens, rng, values, dtype, sort_rows)


def rmat_csr(scale: int, edge_factor: int, abcd=(0.57, 0.19, 0.19, 0.05),
             seed: int = 0, dtype=np.float32, values: str | None = "normal",
             stream: int = 0) -> HostCSR:
    """R-MAT graph as a 2^scale square CSR.

    edge_factor * 2^scale directed edge draws, each choosing one quadrant per
    level with probabilities (a, b, c, d); duplicate draws collapse to one
    entry, self-loops are kept, no relabelling and no noise.
    """
    a, b, c, d = abcd
    rng = rng_for(seed, stream)
    n = 1 << scale
    ne = edge_factor * n
    row = np.zeros(ne, dtype=np.int64)
    col = np.zeros(ne, dtype=np.int64)
    for _ in range(scale):
        r = rng.random(ne)
        rbit = r >= a + b
        cbit = ((r >= a) & (r < a + b)) | (r >= a + b + c)
        row = (row << 1) | rbit
        col = (col << 1) | cbit
    key = np.unique(row * n + col)
    rows = key // n
    indices = (key % n).astype(np.int32)
    counts = np.bincount(rows, minlength=n)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    data = None if values is None else draw_values(rng, indices.size, values, dtype)
    return HostCSR((n, n), indptr, indices, data)


def mcl_matrix(n: int, d: int, seed: int, dtype=np.float32, stream: int = 0) -> HostCSR:
    """X = M^T for a Markov-clustering input M (column-stochastic).

    Column c of M (row c of X) holds d distinct uniform-random off-diagonal
    rows plus the diagonal self-loop; weights are 1-U[0,1) and each column is
    scaled to sum to one (in float64, then rounded to dtype).  This is input
    preparation, not part of the iteration itself.
    """
    rng = rng_for(seed, stream)
    cols = _distinct_rows(rng, n, n - 1, d)
    # shift draws >= c up by one so the diagonal is never drawn twice
    cols = cols + (cols >= np.arange(n)[:, None])
    cols = np.concatenate([cols, np.arange(n)[:, None]], axis=1)
    cols = np.sort(cols, axis=1)
    w = 1.0 - rng.random(cols.shape)
    w = w / w.sum(axis=1, keepdims=True)
    indptr = np.arange(n + 1, dtype=np.int64) * (d + 1)
    return HostCSR((n, n), indptr, cols.reshape(-1).astype(np.int32),
                   w.reshape(-1).astype(dtype))


def identity_csr(n: int, dtype=np.float64) -> HostCSR:
    return HostCSR((n, n), np.arange(n + 1, dtype=np.int64),
                   np.arange(n, dtype=np.int32), np.ones(n, dtype=dtype))


def permutation_csr(n: int, seed: int, dtype=np.float64) -> HostCSR:
    """P with P[i, perm[i]] = 1, so (P B) row i = B row perm[i]."""
    perm = rng_for(seed).permutation(n).astype(np.int32)
    return HostCSR((n, n), np.arange(n + 1, dtype=np.int64), perm,
                   np.ones(n, dtype=dtype))


def shuffle_rows(M: HostCSR, seed: int) -> HostCSR:
    """Same matrix with the entries of every row stored in random order."""
    rng = rng_for(seed, 99)
    m = M.shape[0]
    lens = np.diff(M.indptr)
    rowid = np.repeat(np.arange(m), lens)
    key = rng.random(M.nnz)
    order = np.lexsort((key, rowid))
    data = None if M.data is None else M.data[order]
    return HostCSR(M.shape, M.indptr.copy(), M.indices[order].copy(), data)


def column_blocks(n: int, K: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """K contiguous uneven blocks of [0, n): widths drawn U[lo, hi] then scaled
    to sum to n.  Returns the K+1 boundaries."""
    rng = rng_for(seed, 7)
    w = rng.integers(lo, hi + 1, size=K).astype(np.float64)
    b = np.floor(np.cumsum(w) / w.sum() * n).astype(np.int64)
    b[-1] = n
    return np.concatenate([[0], b])


def split_inner(A: HostCSR, B: HostCSR, bounds: np.ndarray):
    """Split A by column blocks and B by the matching row blocks, so that
    A @ B equals the sum over k of A[:, K_k] @ B[K_k, :]."""
    parts = []
    for k in range(len(bounds) - 1):
        lo, hi = int(bounds[k]), int(bounds[k + 1])
        lens = np.diff(A.indptr)
        rowid = np.repeat(np.arange(A.shape[0]), lens)
        sel = (A.indices >= lo) & (A.indices < hi)
        cnt = np.bincount(rowid[sel], minlength=A.shape[0])
        ip = np.zeros(A.shape[0] + 1, dtype=np.int64)
        np.cumsum(cnt, out=ip[1:])
        Ak = HostCSR((A.shape[0], hi - lo), ip, (A.indices[sel] - lo).astype(np.int32),
                     None if A.data is None else A.data[sel])
        s, e = int(B.indptr[lo]), int(B.indptr[hi])
        Bk = HostCSR((hi - lo, B.shape[1]), B.indptr[lo:hi + 1] - s,
                     B.indices[s:e].copy(), None if B.data is None else B.data[s:e].copy())
        parts.append((Ak, Bk))
    return parts


# ---------------------------------------------------------------------------
# The benchmark workloads' inputs, shared by the benchmark and the full-size
# parity tests so that both see the same matrices.

WORKLOAD_SEED = 20260321


def batched_uniform_blocks(seed: int = WORKLOAD_SEED + 3, m: int = 1 << 18, n: int = 1 << 20,
                           K: int = 8, kmin: int = 1 << 18, kmax: int = 1 << 20):
    """Batched stage sequence, uniform variant: K block products A_k B_k
    with A_k m x K_k and B_k K_k x n, inner sizes K_k ~ U[kmin, kmax], rows of
    U{4..32} distinct uniform columns, values N(0,1) in FP32."""
    rng = rng_for(seed, 11)
    kdims = rng.integers(kmin, kmax + 1, size=K)
    pairs = []
    for k in range(K):
        Ak = varnnz_csr(m, int(kdims[k]), 4, 32, seed, np.float32, "normal", stream=2 * k)
        Bk = varnnz_csr(int(kdims[k]), n, 4, 32, seed, np.float32, "normal", stream=2 * k + 1)
        pairs.append((Ak, Bk))
    return pairs


def batched_rmat_blocks(seed: int = WORKLOAD_SEED + 6, scale: int = 20, K: int = 8):
    """Batched stage sequence, power-law variant: A = R-MAT(0.57, 0.19, 0.19,
    0.05) of the given scale with edge factor 16, B 2^scale x 2^scale with
    U{4..32} uniform columns per row (FP32 N(0,1)), split into K contiguous
    uneven inner blocks.  Returns (A, B, pairs)."""
    n = 1 << scale
    A = rmat_csr(scale, 16, seed=seed, dtype=np.float32, values="normal", stream=0)
    Bm = varnnz_csr(n, n, 4, 32, seed, np.float32, "normal", stream=1)
    bounds = column_blocks(n, K, n // 16, n // 4, seed)
    return A, Bm, split_inner(A, Bm, bounds)


def aggregation_csr(n: int, nc: int, seed: int, dtype=np.float32, values: str = "one",
                    stream: int = 0) -> HostCSR:
    """Rectangular aggregation operator R (n x nc) of an algebraic-multigrid
    setup: row i holds one entry, in column agg[i], the aggregate of fine
    point i.  Aggregates are drawn as a random permutation of (i mod nc), so
    every aggregate gets n/nc points (one more for the first n mod nc)
    scattered uniformly, as for an unstructured fine matrix.  Values: 'one'
    (piecewise-constant aggregation) or any kind of draw_values."""
    if not (1 <= nc <= n):
        raise ValueError("need 1 <= nc <= n")
    rng = rng_for(seed, stream)
    agg = (rng.permutation(n) % nc).astype(np.int32)
    data = draw_values(rng, n, values, dtype)
    return HostCSR((n, nc), np.arange(n + 1, dtype=np.int64), agg, data)


def banded_csr(n: int, d: int, offsets, halfwidth: int, seed: int, dtype=np.float32,
               values: str = "u01", stream: int = 0) -> HostCSR:
    """Structured n x n matrix made of diagonal bands: row i holds d distinct
    columns drawn uniformly from the union of the windows
    [i + o - halfwidth, i + o + halfwidth] (clipped to [0, n)) over the band
    offsets o, so its nonzeros sit on a few diagonals, as in the structured
    matrices that the paper permutes at random before multiplying."""
    rng = rng_for(seed, stream)
    offsets = np.asarray(offsets, dtype=np.int64)
    w = 2 * halfwidth + 1
    span = offsets.size * w
    if d > span:
        raise ValueError("more entries per row than the bands hold")
    # d distinct slots of the row's band windows (slot s: band s // w, step s % w)
    slots = _distinct_rows(rng, n, span, d)
    cols = np.arange(n)[:, None] + offsets[slots // w] + (slots % w) - halfwidth
    # clip into [0, n) by reflecting at the edges, then drop repeats
    cols = np.where(cols < 0, -cols - 1, cols)
    cols = np.where(cols >= n, 2 * n - 1 - cols, cols)
    cols = np.sort(cols, axis=1)
    keep = np.ones_like(cols, dtype=bool)
    keep[:, 1:] = cols[:, 1:] != cols[:, :-1]
    lens = keep.sum(axis=1).astype(np.int64)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=indptr[1:])
    indices = cols[keep].astype(np.int32)
    data = draw_values(rng, indices.size, values, dtype)
    return HostCSR((n, n), indptr, indices, data)


def random_permutation(n: int, seed: int, stream: int = 0) -> np.ndarray:
    """A uniformly random permutation p of [0, n) (int32): the symmetric
    permutation maps entry (i, j) to (p[i], p[j])."""
    return rng_for(seed, stream).permutation(n).astype(np.int32)

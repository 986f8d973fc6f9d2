"""Small host helpers shared by the tests (no GPU, no oracle arithmetic)."""
from __future__ import annotations

import json
import os

import numpy as np

from paper_2603_21444_amd.synth import HostCSR

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def csr_from_json(d, dtype=np.float64) -> HostCSR:
    return HostCSR(tuple(d["shape"]), np.array(d["indptr"], dtype=np.int64),
                   np.array(d["indices"], dtype=np.int32),
                   np.array(d["data"], dtype=dtype))


def dense(M) -> np.ndarray:
    out = np.zeros(M.shape, dtype=np.float64)
    rows = np.repeat(np.arange(M.shape[0]), np.diff(M.indptr))
    np.add.at(out, (rows, M.indices), np.asarray(M.data, dtype=np.float64))
    return out


def mask(M) -> np.ndarray:
    out = np.zeros(M.shape, dtype=np.int64)
    rows = np.repeat(np.arange(M.shape[0]), np.diff(M.indptr))
    out[rows, M.indices] = 1
    return out


def row_ids(M) -> np.ndarray:
    return np.repeat(np.arange(M.shape[0]), np.diff(M.indptr))


def assert_canonical(M):
    """Columns strictly ascending within every row, indices in range."""
    rid = row_ids(M)
    if M.indices.size:
        assert M.indices.min() >= 0 and M.indices.max() < M.shape[1]
        same = rid[1:] == rid[:-1]
        assert np.all(M.indices[1:][same] > M.indices[:-1][same])


def row_subset(M, rows) -> HostCSR:
    """Rows `rows` of M (in that order) as a new CSR with the same columns."""
    rows = np.asarray(rows, dtype=np.int64)
    indptr = np.asarray(M.indptr, dtype=np.int64)
    lens = indptr[rows + 1] - indptr[rows]
    ip = np.zeros(rows.size + 1, dtype=np.int64)
    np.cumsum(lens, out=ip[1:])
    # entry t of the subset is entry indptr[row] + (t - ip[slot]) of M
    idx = np.arange(ip[-1], dtype=np.int64) + np.repeat(indptr[rows] - ip[:-1], lens)
    return HostCSR((rows.size, M.shape[1]), ip, M.indices[idx].astype(np.int32),
                   None if M.data is None else M.data[idx])


def tol_for(dtype) -> float:
    """Value tolerance relative to S_ij = sum_k |a_ik||b_kj| against the FP64
    oracle: 1e-12 for FP64, 1e-5 for FP32 accumulation."""
    return 1e-12 if np.dtype(dtype) == np.float64 else 1e-5


def assert_same_csr(got, ref, S, dtype, exact=False, what=""):
    """Bit-exact row_ptr and col_idx; values exact or within tol*S."""
    assert tuple(got.shape) == tuple(ref.shape), what
    assert np.array_equal(np.asarray(got.indptr, np.int64), np.asarray(ref.indptr, np.int64)), f"{what}: row_ptr differs"
    assert np.array_equal(got.indices, ref.indices), f"{what}: col_idx differs"
    g = np.asarray(got.data, dtype=np.float64)
    if exact:
        assert np.array_equal(g, ref.data), f"{what}: values differ"
    else:
        err = np.abs(g - ref.data)
        bad = err > tol_for(dtype) * S
        assert not bad.any(), f"{what}: {int(bad.sum())} values out of tolerance, worst {float((err / np.maximum(S, 1e-300)).max()):.3e}"

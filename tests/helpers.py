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

"""GPU parity of the restriction-operator product C = A R of an algebraic-
multigrid setup (paper §5.4): R rectangular (n x n_c) with one entry per row,
so each row of C is the row of A merged by aggregate; few products per row
(the low-flop regime).  Patterns bit-exact, values within tolerance (exact
on small integers)."""
import numpy as np
import pytest

import oracle
from paper_2603_21444_amd import synth
from helpers import assert_same_csr

pytestmark = pytest.mark.gpu

SEED = synth.WORKLOAD_SEED


@pytest.fixture(scope="module")
def B():
    import torch
    from paper_2603_21444_amd import binding
    assert torch.cuda.is_available()
    binding.lib()
    return binding


@pytest.mark.parametrize("dtype,avals,rvals", [(np.float32, "u01", "one"), (np.float32, "normal", "u01"),
                                               (np.float64, "int", "int")])
def test_restriction_product(B, dtype, avals, rvals):
    n, nc = 1 << 16, 1 << 13
    A = synth.uniform_csr(n, n, 16, 41, dtype, avals)
    R = synth.aggregation_csr(n, nc, 41, dtype, rvals)
    got = B.spgemm(B.to_device(A), B.to_device(R)).to_host()
    ref, S = oracle.spgemm(A.astype(np.float64), R.astype(np.float64), with_abs=True)
    assert_same_csr(got, ref, S, dtype, exact=(avals == "int"), what="A R")


def test_restriction_of_power_law_rows(B):
    """R-MAT rows (hubs with thousands of entries, empty rows) times an
    aggregation to 1/4 of the points."""
    n = 1 << 15
    A = synth.rmat_csr(15, 16, seed=42, dtype=np.float32, values="normal")
    R = synth.aggregation_csr(n, n // 4, 42, np.float32, "u01")
    got = B.spgemm(B.to_device(A), B.to_device(R)).to_host()
    ref, S = oracle.spgemm(A.astype(np.float64), R.astype(np.float64), with_abs=True)
    assert_same_csr(got, ref, S, np.float32, what="R-MAT A R")


@pytest.mark.slow
def test_restriction_full_size(B):
    """The benchmark's restriction workload: A 2^20 x 2^20 with 16 uniform
    columns per row (FP32 in (0,1]) times R 2^20 x 2^17 (aggregates of 8),
    every row checked."""
    n, nc = 1 << 20, 1 << 17
    A = synth.uniform_csr(n, n, 16, SEED + 1, np.float32, "u01", stream=0)
    R = synth.aggregation_csr(n, nc, SEED + 7, np.float32, "u01")
    got = B.spgemm(B.to_device(A), B.to_device(R)).to_host()
    ref, S = oracle.spgemm(A.astype(np.float64), R.astype(np.float64), with_abs=True)
    assert_same_csr(got, ref, S, np.float32, what="2^20 A R")

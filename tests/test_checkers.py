"""The stepwise MCL checker itself, on the CPU: it accepts the oracle's own
output and rejects outputs with a planted mistake (a dropped entry far from
the thresholds, a wrong value, a value renormalised over the wrong set)."""
import numpy as np
import pytest

import oracle
from paper_2603_21444_amd import synth
from mcl_check import check_mcl_step


def _as_host(Y, dtype=np.float32):
    return synth.HostCSR(Y.shape, Y.indptr.copy(), Y.indices.copy(), Y.data.astype(dtype))


@pytest.mark.parametrize("order,r,prune,topk", [("workload", 2, 1e-4, 1000), ("workload", 2, 1e-3, 20),
                                                ("paper", 2, 0.002, 500), ("paper", 2, 0.01, 30)])
def test_checker_accepts_the_oracle(order, r, prune, topk):
    X = synth.mcl_matrix(2000, 20, 3, np.float32)
    Y = oracle.mcl_step(X.astype(np.float64), r, prune, topk, order=order)
    assert check_mcl_step(X, _as_host(Y), r, prune, topk, order=order) == 0
    rows = np.arange(0, 2000, 7)
    assert check_mcl_step(X, _as_host(Y), r, prune, topk, rows=rows, order=order) == 0


@pytest.mark.parametrize("order", ["workload", "paper"])
def test_checker_rejects_planted_mistakes(order):
    r, prune, topk = 2, 1e-3, 1000
    X = synth.mcl_matrix(1000, 20, 5, np.float32)
    Y = oracle.mcl_step(X.astype(np.float64), r, prune, topk, order=order)
    # 1. a value off by 1e-3 relative
    bad = _as_host(Y)
    bad.data[17] *= 1.001
    with pytest.raises(AssertionError):
        check_mcl_step(X, bad, r, prune, topk, order=order)
    # 2. the largest entry of a row dropped (far outside the band)
    i = 3
    s, e = int(Y.indptr[i]), int(Y.indptr[i + 1])
    j = s + int(np.argmax(Y.data[s:e]))
    keep = np.ones(Y.indices.size, dtype=bool)
    keep[j] = False
    ip = Y.indptr.copy()
    ip[i + 1:] -= 1
    bad = synth.HostCSR(Y.shape, ip, Y.indices[keep], Y.data[keep].astype(np.float32))
    with pytest.raises(AssertionError):
        check_mcl_step(X, bad, r, prune, topk, order=order)
    # 3. rows left un-normalised (workload) / renormalised (paper)
    bad = _as_host(Y)
    rid = np.repeat(np.arange(1000), np.diff(Y.indptr))
    sums = np.bincount(rid, weights=Y.data, minlength=1000)
    if order == "workload":
        bad.data = (Y.data * 1.01).astype(np.float32)
    else:
        bad.data = (Y.data / sums[rid]).astype(np.float32)
    with pytest.raises(AssertionError):
        check_mcl_step(X, bad, r, prune, topk, order=order)

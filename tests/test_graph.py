"""Captured stage graphs: every replay matches the eager result (several
replays, with eager work and synchronisation between them)."""
import numpy as np
import pytest

import oracle
from paper_2603_21444_amd import synth
from helpers import assert_same_csr, row_ids
from mcl_check import check_mcl_step

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    from paper_2603_21444_amd import binding
    assert torch.cuda.is_available()
    binding.lib()
    return binding


def _pairs(dtype, kind, seed=3, K=5):
    m, kk, n = 4000, 30000, 12000
    A = synth.varnnz_csr(m, kk, 4, 32, seed, dtype, kind, stream=0)
    Bm = synth.varnnz_csr(kk, n, 4, 32, seed, dtype, kind, stream=1)
    bounds = synth.column_blocks(kk, K, kk // 10, kk // 3, seed)
    return synth.split_inner(A, Bm, bounds)


def test_stage_graph_replays_match_eager_exactly(B):
    import torch
    from paper_2603_21444_amd.graph import StageGraph
    pairs = _pairs(np.float64, "int")
    dp = [(B.to_device(a), B.to_device(b)) for a, b in pairs]
    eager = B.batched(dp).to_host()
    g = StageGraph(dp)
    for rep in range(4):
        g.replay()
        got = g.result().to_host()
        assert np.array_equal(got.indptr, eager.indptr), rep
        assert np.array_equal(got.indices, eager.indices), rep
        assert np.array_equal(got.data, eager.data), rep  # integer values: exact
        # eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        float((x * x).sum())
        B.spgemm(*dp[0])
        torch.cuda.synchronize()


def test_stage_graph_fp32_against_oracle(B):
    from paper_2603_21444_amd.graph import StageGraph
    pairs = _pairs(np.float32, "normal", seed=5, K=8)
    dp = [(B.to_device(a), B.to_device(b)) for a, b in pairs]
    g = StageGraph(dp)
    ref, S = oracle.batched([(a.astype(np.float64), b.astype(np.float64)) for a, b in pairs],
                            with_abs=True)
    for _ in range(3):
        g.replay()
        assert_same_csr(g.result().to_host(), ref, S, np.float32, what="graph")


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_stage_graph_power_law_heavy_rows(B, dtype):
    """R-MAT rows (scale 15, edge factor 16) split into 8 uneven inner blocks:
    hub rows beyond every LDS table, empty rows and all LDS bins, captured
    once and replayed; every replay matches the oracle (heavy rows add in
    no fixed order, so replays are compared by tolerance, not bit for bit)."""
    from paper_2603_21444_amd.graph import StageGraph
    n = 1 << 15
    A = synth.rmat_csr(15, 16, seed=23, dtype=dtype, values="normal")
    Bm = synth.varnnz_csr(n, n, 4, 32, 23, dtype, "normal", stream=3)
    f64 = lambda M: M.with_data(M.data.astype(np.float64))
    ub = oracle.rowub(f64(A), f64(Bm))
    assert ub.max() > 20000 and (ub == 0).any()
    ref, S = oracle.spgemm(f64(A), f64(Bm), with_abs=True)
    bounds = synth.column_blocks(n, 8, n // 16, n // 4, 23)
    dp = [(B.to_device(a), B.to_device(b)) for a, b in synth.split_inner(A, Bm, bounds)]
    g = StageGraph(dp)
    for rep in range(3):
        g.replay()
        assert_same_csr(g.result().to_host(), ref, S, dtype, what=f"power-law graph, replay {rep}")


def test_stage_graph_capacity_error_surfaces(B):
    from paper_2603_21444_amd.graph import StageGraph
    pairs = _pairs(np.float32, "normal", seed=7, K=3)
    dp = [(B.to_device(a), B.to_device(b)) for a, b in pairs]
    g = StageGraph(dp, capacity=1000)
    g.replay()
    with pytest.raises(B.SpgError) as e:
        g.result()
    assert e.value.code == B.SPG_ERR_CAPACITY


def test_mcl_graph_fixed_point_and_replays(B):
    import torch
    from paper_2603_21444_amd.graph import MCLGraph
    b, nb = 32, 12
    n = b * nb
    perm = synth.rng_for(9).permutation(n)
    rows, cols = [], []
    for blk in perm.reshape(nb, b):
        for i in blk:
            for j in blk:
                rows.append(i); cols.append(j)
    rows, cols = np.array(rows), np.array(cols)
    order = np.lexsort((cols, rows))
    ip = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=ip[1:])
    X = synth.HostCSR((n, n), ip, cols[order].astype(np.int32), np.full(n * b, 1.0 / b, np.float32))
    g = MCLGraph(B.to_device(X), iters=10)
    for _ in range(3):
        g.replay()
        H = g.result().to_host()
        assert np.array_equal(H.indptr, X.indptr)
        assert np.array_equal(H.indices, X.indices)
        assert np.array_equal(H.data, X.data)
        torch.cuda.synchronize()


@pytest.mark.parametrize("iters", [1, 2, 10])
def test_mcl_graph_last_step_matches_oracle(B, iters):
    """An MCL graph of `iters` iterations on a random input: after each of
    two replays, the last iteration's output is checked stepwise against the
    oracle run on the previous iteration's output (the input itself for one
    iteration), on every row; column sums and row lengths hold."""
    import torch
    from paper_2603_21444_amd.graph import MCLGraph
    n = 5000
    X = synth.mcl_matrix(n, 16, 13, np.float32)
    dX = B.to_device(X)
    g = MCLGraph(dX, iters=iters)
    for rep in range(2):
        g.replay()
        got = g.result().to_host()
        prev = X if iters == 1 else g.buffer(iters - 2).to_host()
        check_mcl_step(prev, got, 2, 1e-4, 1000)
        sums = np.bincount(row_ids(got), weights=got.data.astype(np.float64), minlength=n)
        assert np.allclose(sums, 1.0, atol=1e-5)
        lens = np.diff(got.indptr)
        assert lens.max() <= 1000 and lens.min() >= 1
        # eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        float((x * x).sum())
        torch.cuda.synchronize()


def test_mcl_graph_error_in_an_early_iteration_reaches_the_end(B):
    """A capacity too small for the first iteration's output: the error is
    raised in iteration 1, every later iteration skips its work (so nothing
    reads the unwritten buffer), and result() reports it after the replay.
    An eager iteration on the same plan afterwards works and clears it."""
    from paper_2603_21444_amd.graph import MCLGraph
    X = synth.mcl_matrix(3000, 12, 17, np.float32)
    dX = B.to_device(X)
    g = MCLGraph(dX, iters=6, capacity=1000)
    for _ in range(2):
        g.replay()
        with pytest.raises(B.SpgError) as e:
            g.result()
        assert e.value.code == B.SPG_ERR_CAPACITY
    Y = B.mcl_iteration(dX, plan=g.plan).to_host()
    check_mcl_step(X, Y, 2, 1e-4, 1000)
    assert g.plan.status() == B.SPG_OK


def test_stage_graph_status_clears_per_replay(B):
    """The stage graph clears the status word at its start: a replay after
    an eager call that failed on the same plan reports only its own result."""
    from paper_2603_21444_amd.graph import StageGraph
    pairs = _pairs(np.float32, "normal", seed=9, K=3)
    dp = [(B.to_device(a), B.to_device(b)) for a, b in pairs]
    g = StageGraph(dp)
    ref, S = oracle.batched([(a.astype(np.float64), b.astype(np.float64)) for a, b in pairs],
                            with_abs=True)
    rp, _ = g.plan.symbolic(g.As, g.Bs, capacity=10, rp=g.row_ptr)  # raises capacity in the device
    assert g.plan.status() == B.SPG_ERR_CAPACITY
    g.replay()
    assert_same_csr(g.result().to_host(), ref, S, np.float32, what="graph after a failed call")

"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (captured graphs replayed), against the FP64 oracle.

  batched stage sequence, uniform: 8 block products A_k B_k (m = 2^18,
      n = 2^20, inner K_k ~ U[2^18, 2^20], U{4..32} per row, FP32 N(0,1))
      summed into one C by the fused product, captured once, replayed twice;
      every row of C checked (row_ptr, col_idx bit-exact; values within
      1e-5 * sum |a||b|).
  batched stage sequence, R-MAT: A = R-MAT scale 20, edge factor 16 split
      into 8 uneven inner blocks, same checks on every row.
  MCL, n = 2^19 (24 + 1 per column, FP32), r = 2, prune < 1e-4, top-1000:
      ten eager iterations, each checked stepwise (oracle input = the GPU's
      previous output): iteration 1 on every row, later iterations on 4096
      sampled rows plus the 16 longest; then the ten iterations captured as
      one graph, whose last step is checked stepwise on 4096 sampled rows.
Inputs come from the same generators and seeds as the benchmark."""
import sys

import numpy as np
import pytest

import oracle
from paper_2603_21444_amd import synth
from helpers import assert_same_csr, row_ids
from mcl_check import check_mcl_step

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

SEED = synth.WORKLOAD_SEED


def say(msg):
    print(f"[full-size] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def B():
    import torch
    from paper_2603_21444_amd import binding
    assert torch.cuda.is_available()
    binding.lib()
    return binding


def _f64(M):
    return M.with_data(M.data.astype(np.float64))


def _graph_vs_oracle(B, hpairs, what):
    import torch
    from paper_2603_21444_amd.graph import StageGraph
    dp = [(B.to_device(a), B.to_device(b)) for a, b in hpairs]
    say(f"{what}: blocks on the device")
    g = StageGraph(dp)
    ref, S = oracle.batched([(_f64(a), _f64(b)) for a, b in hpairs], with_abs=True)
    say(f"{what}: oracle done, nnz(C) = {ref.nnz}")
    for rep in range(2):
        g.replay()
        got = g.result().to_host()
        assert_same_csr(got, ref, S, np.float32, what=f"{what}, replay {rep}")
        say(f"{what}: replay {rep} matches the oracle on every row")
        del got
    del g
    torch.cuda.empty_cache()


def test_stage_graph_uniform_batched_full_size(B):
    _graph_vs_oracle(B, synth.batched_uniform_blocks(SEED + 3), "uniform batched graph")


def test_stage_graph_rmat_batched_full_size(B):
    A, Bm, hpairs = synth.batched_rmat_blocks(SEED + 6)
    ub = oracle.rowub(_f64(A), _f64(Bm))
    assert ub.max() > 10 ** 5  # hub rows far beyond every LDS table
    _graph_vs_oracle(B, hpairs, "R-MAT batched graph")


def _sample(n, k, seed, lens):
    rows = synth.rng_for(seed, 13).choice(n, k, replace=False)
    longest = np.argsort(lens, kind="stable")[-16:]
    return np.unique(np.concatenate([rows, longest]))


def test_mcl_2p19_stepwise_eager_and_graph(B):
    import torch
    from paper_2603_21444_amd.graph import MCLGraph
    n, r, prune, topk = 1 << 19, 2, 1e-4, 1000
    X = synth.mcl_matrix(n, 24, SEED + 4, np.float32)
    dX = B.to_device(X)
    plan = B.Plan()
    prev_h, Y = X, dX
    flips = 0
    for it in range(1, 11):
        Y = B.mcl_iteration(Y, r, prune, topk, plan=plan)
        got = Y.to_host()
        rows = None if it == 1 else _sample(n, 4096, it, np.diff(prev_h.indptr))
        flips += check_mcl_step(prev_h, got, r, prune, topk, rows)
        sums = np.bincount(row_ids(got), weights=got.data.astype(np.float64), minlength=n)
        assert np.allclose(sums, 1.0, atol=1e-5)
        lens = np.diff(got.indptr)
        assert lens.max() <= topk and lens.min() >= 1
        say(f"MCL eager iteration {it}: nnz {got.nnz}, "
            f"{'every row' if rows is None else f'{rows.size} rows'} match, {flips} band flips so far")
        prev_h = got
    del Y
    torch.cuda.empty_cache()
    g = MCLGraph(dX, iters=10)
    g.replay()
    last = g.result().to_host()
    before = g.buffer(8).to_host()
    rows = _sample(n, 4096, 99, np.diff(before.indptr))
    check_mcl_step(before, last, r, prune, topk, rows)
    sums = np.bincount(row_ids(last), weights=last.data.astype(np.float64), minlength=n)
    assert np.allclose(sums, 1.0, atol=1e-5)
    say(f"MCL graph: iteration 10 matches on {rows.size} rows")

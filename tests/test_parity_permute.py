"""GPU parity of the random-permutation preprocessing (paper §5.3):
B[row_perm[i], col_perm[j]] = A[i, j] with rows in ascending column order,
against the oracle, bit for bit (values are copied, not computed)."""
import numpy as np
import pytest

import oracle
from paper_2603_21444_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    from paper_2603_21444_amd import binding
    assert torch.cuda.is_available()
    binding.lib()
    return binding


def _dev_perm(p):
    import torch
    return None if p is None else torch.from_numpy(np.ascontiguousarray(p, dtype=np.int32)).cuda()


def _check(B, A, p, q, dtype=np.float32, pattern_only=False):
    import torch
    dA = B.to_device(A, dtype=None if pattern_only else dtype)
    if pattern_only:
        dA.vals = None
    plan = B.Plan()
    got = B.permute(dA, _dev_perm(p), _dev_perm(q), plan=plan)
    torch.cuda.synchronize()
    assert plan.status() == B.SPG_OK
    h = got.to_host()
    ref = oracle.permute(A.with_data(None) if pattern_only else A.astype(np.float64), p, q)
    assert np.array_equal(h.indptr, ref.indptr), "row_ptr"
    assert np.array_equal(h.indices, ref.indices), "col_idx"
    if not pattern_only:
        assert np.array_equal(h.data.astype(np.float64), ref.data), "values"
    return h


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_symmetric_permutation_of_banded_matrix(B, dtype):
    n = 1 << 16
    A = synth.banded_csr(n, 16, [0, n // 8, -n // 8], 64, 3, dtype)
    p = synth.random_permutation(n, 3)
    _check(B, A, p, p, dtype)


def test_rows_of_every_length_class(B):
    """Row lengths 0..5000 (every short-row group size and the panel kernel),
    unsorted input rows, rectangular, separate row and column permutations,
    a column space of several panels."""
    m, n = 3000, 100000
    A = synth.shuffle_rows(synth.varnnz_csr(m, n, 0, 300, 7, np.float32, "normal"), 7)
    rng = synth.rng_for(7, 9)
    ip, ind, dat = [0], [], []
    for i in range(m):
        c, v = A.row(i)
        if i % 997 == 5:  # long rows: the panel kernel
            c = rng.choice(n, 5000 + 3000 * (i // 997), replace=False).astype(np.int32)
            v = rng.standard_normal(c.size).astype(np.float32)
        elif i % 211 == 3:  # rows of 1025..4096 entries: 1024-lane groups
            c = rng.choice(n, 1025 + 13 * i % 3000, replace=False).astype(np.int32)
            v = rng.standard_normal(c.size).astype(np.float32)
        ind.append(c); dat.append(v); ip.append(ip[-1] + c.size)
    A = synth.HostCSR((m, n), np.array(ip, np.int64), np.concatenate(ind).astype(np.int32),
                      np.concatenate(dat).astype(np.float32))
    lens = np.diff(A.indptr)
    assert lens.max() > 4096 and ((lens > 1024) & (lens <= 4096)).any() and (lens == 0).any()
    p, q = synth.random_permutation(m, 11), synth.random_permutation(n, 12)
    _check(B, A, p, q)
    _check(B, A, None, q)
    _check(B, A, p, None)
    _check(B, A, None, None)
    _check(B, A, p, q, pattern_only=True)


def test_power_law_rows(B):
    n = 1 << 15
    A = synth.rmat_csr(15, 16, seed=5, dtype=np.float64, values="normal")
    p = synth.random_permutation(n, 13)
    _check(B, A, p, p, np.float64)


def test_not_a_permutation_is_reported(B):
    import torch
    A = synth.varnnz_csr(500, 500, 1, 10, 8, np.float32, "normal")
    dA = B.to_device(A)
    p = np.arange(500, dtype=np.int32)
    p[10] = 11  # 11 twice, 10 never
    plan = B.Plan()
    rp = torch.full((501,), -7, dtype=torch.int32, device="cuda")
    col = torch.zeros(A.nnz, dtype=torch.int32, device="cuda")
    vals = torch.zeros(A.nnz, dtype=torch.float32, device="cuda")
    B.permute(dA, _dev_perm(p), None, plan=plan, out=(rp, col, vals))
    assert plan.status() == B.SPG_ERR_INVALID
    assert int((rp != -7).sum().item()) == 0 and int(col.abs().sum().item()) == 0
    plan.clear_status()
    q = np.arange(500, dtype=np.int32)
    q[0] = 500  # out of range
    B.permute(dA, None, _dev_perm(q), plan=plan, out=(rp, col, vals))
    assert plan.status() == B.SPG_ERR_INVALID


def test_permutation_in_a_captured_graph(B):
    """Permute + product captured together, replayed three times: every
    replay equals (P A P^T)^2 from the oracle (small integers: exact)."""
    import torch
    n = 4096
    A = synth.banded_csr(n, 8, [0, 512], 16, 9, np.float64, "int")
    p = synth.random_permutation(n, 14)
    dA, dp = B.to_device(A), _dev_perm(p)
    pplan = B.Plan()
    PA = B.permute(dA, dp, dp, plan=pplan)
    plan = B.Plan()
    rp, nnz = plan.symbolic([PA], [PA])
    col = torch.empty(nnz, dtype=torch.int32, device="cuda")
    vals = torch.empty(nnz, dtype=torch.float64, device="cuda")
    plan.numeric([PA], [PA], rp, nnz, col=col, vals=vals)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.graph(g, stream=s):
        pplan.clear_status(s)
        plan.clear_status(s)
        B.permute(dA, dp, dp, plan=pplan, stream=s, out=(PA.row_ptr, PA.col_idx, PA.vals))
        plan.symbolic([PA], [PA], capacity=nnz, stream=s, rp=rp)
        plan.numeric([PA], [PA], rp, nnz, col=col, vals=vals, stream=s)
    Ph = oracle.permute(A.astype(np.float64), p, p)
    Phh = synth.HostCSR(Ph.shape, Ph.indptr, Ph.indices, Ph.data)
    ref = oracle.spgemm(Phh, Phh)
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert pplan.status() == B.SPG_OK and plan.status() == B.SPG_OK
        assert np.array_equal(rp.cpu().numpy(), ref.indptr)
        assert np.array_equal(col.cpu().numpy(), ref.indices)
        assert np.array_equal(vals.cpu().numpy(), ref.data)
        x = torch.randn(1 << 18, device="cuda")
        float((x * x).sum())

"""The symbolic call that allocates nothing (static scratch inside the
library) against the same product through the caller-workspace entry point:
two calls in a row, the second on a smaller input, each followed by the
ordinary numeric call on the same plan.  Patterns bit-exact, values within
the FP32 tolerance of the oracle (and bit-exact on small integers)."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2603_21444_amd import synth
from helpers import assert_same_csr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    from paper_2603_21444_amd import binding
    assert torch.cuda.is_available()
    binding.lib()
    return binding


def _inputs(m, k, n, seed, kind, dtype, heavy_rows=()):
    A = synth.varnnz_csr(m, k, 0, 40, seed, dtype, kind, stream=0)
    Bm = synth.varnnz_csr(k, n, 0, 48, seed, dtype, kind, stream=1)
    if heavy_rows:  # a few long rows of A: products beyond every LDS table
        rng = synth.rng_for(seed, 4)
        ip, ind, dat = [0], [], []
        for i in range(m):
            c, v = A.row(i)
            if i in heavy_rows:
                c = np.sort(rng.choice(k, 3000, replace=False)).astype(np.int32)
                v = synth.draw_values(rng, c.size, kind, dtype)
            ind.append(c); dat.append(v); ip.append(ip[-1] + c.size)
        A = synth.HostCSR((m, k), np.array(ip, np.int64), np.concatenate(ind).astype(np.int32),
                          np.concatenate(dat).astype(dtype))
    return A, Bm


def _run(B, A, Bm, noalloc):
    import torch
    dA, dB = B.to_device(A), B.to_device(Bm)
    plan = B.Plan()
    m = A.shape[0]
    ref_plan = B.Plan()
    _, nnz = ref_plan.symbolic([dA], [dB])  # eager count: the capacity to allocate
    rp = torch.empty(m + 1, dtype=torch.int32, device="cuda")
    if noalloc:
        plan.symbolic_noalloc([dA], [dB], rp, nnz)
    else:
        plan.symbolic([dA], [dB], capacity=nnz, rp=rp)
    col, vals = plan.numeric([dA], [dB], rp, nnz)
    torch.cuda.synchronize()
    assert plan.status() == B.SPG_OK
    return B.DeviceCSR((m, Bm.shape[1]), rp, col, vals).to_host()


@pytest.mark.parametrize("kind,dtype", [("normal", np.float32), ("int", np.float64)])
def test_noalloc_matches_workspace_entry_point_twice(B, kind, dtype):
    cases = [(6000, 9000, 70000, 31, (5, 4321)), (2500, 3000, 4000, 32, ())]
    for m, k, n, seed, heavy in cases:  # second call smaller
        A, Bm = _inputs(m, k, n, seed, kind, dtype, heavy)
        got = _run(B, A, Bm, noalloc=True)
        ref_ws = _run(B, A, Bm, noalloc=False)
        assert np.array_equal(got.indptr, ref_ws.indptr)
        assert np.array_equal(got.indices, ref_ws.indices)
        ref, S = oracle.spgemm(A.astype(np.float64), Bm.astype(np.float64), with_abs=True)
        assert_same_csr(got, ref, S, dtype, exact=(kind == "int"), what=f"no-alloc m={m}")
        if kind == "int":
            assert np.array_equal(got.data, ref_ws.data)


def test_noalloc_capacity_error_and_limit(B):
    import torch
    A, Bm = _inputs(2000, 2000, 3000, 33, "normal", np.float32)
    dA, dB = B.to_device(A), B.to_device(Bm)
    plan = B.Plan()
    rp = torch.empty(2001, dtype=torch.int32, device="cuda")
    plan.symbolic_noalloc([dA], [dB], rp, 10)
    col = torch.zeros(10, dtype=torch.int32, device="cuda")
    vals = torch.zeros(10, dtype=torch.float32, device="cuda")
    plan.numeric([dA], [dB], rp, 10, col=col, vals=vals)
    assert plan.status() == B.SPG_ERR_CAPACITY
    assert int(col.abs().sum().item()) == 0
    plan.clear_status()
    assert plan.status() == B.SPG_OK
    # beyond the scratch: rejected on the host, nothing queued
    big = B.SpgCsr(1 << 23, 1 << 23, 0, rp.data_ptr(), None, None)
    L = B.lib()
    arrA, arrB = (B.SpgCsr * 1)(big), (B.SpgCsr * 1)(big)
    rc = L.spgemm_symbolic_noalloc(plan.h, 1, arrA, arrB, C.c_void_p(rp.data_ptr()), 0,
                                   C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == B.SPG_ERR_SCRATCH

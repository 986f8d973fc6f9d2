"""GPU parity of the sparse sum of partial products (merge), the fused
batched sum of block products, and the backward pass at fixed sparsity,
against the FP64 oracle.  Calls go through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_2603_21444_amd import synth
from helpers import assert_same_csr, dense, row_ids, tol_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    from paper_2603_21444_amd import binding
    assert torch.cuda.is_available()
    binding.lib()
    return binding


def _f64(M):
    return M.with_data(M.data.astype(np.float64))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_merge_matches_oracle(B, dtype):
    parts = [synth.varnnz_csr(3000, 5000, 0, 40, 100 + k, dtype, "normal") for k in range(5)]
    parts.append(synth.shuffle_rows(synth.varnnz_csr(3000, 5000, 0, 40, 199, dtype, "normal"), 3))
    got = B.merge([B.to_device(P) for P in parts]).to_host()
    ref, S = oracle.merge([_f64(P) for P in parts], with_abs=True)
    assert_same_csr(got, ref, S, dtype, what="merge")


def test_merge_exact_cancellation_and_single_operand(B):
    P = synth.varnnz_csr(2000, 3000, 0, 30, 7, np.float64, "int")
    got = B.merge([B.to_device(P), B.to_device(P.with_data(-P.data))]).to_host()
    assert np.array_equal(got.indptr, P.indptr)
    assert np.array_equal(got.indices, P.indices)  # P has sorted rows
    assert np.all(got.data == 0.0)
    one = B.merge([B.to_device(P)]).to_host()
    assert np.array_equal(one.indices, P.indices) and np.array_equal(one.data, P.data)


def test_merge_heavy_rows(B):
    parts = [synth.varnnz_csr(50, 40000, 1, 3000, 300 + k, np.float32, "normal") for k in range(8)]
    got = B.merge([B.to_device(P) for P in parts]).to_host()
    ref, S = oracle.merge([_f64(P) for P in parts], with_abs=True)
    assert_same_csr(got, ref, S, np.float32, what="merge heavy")


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_batched_sum_of_uneven_blocks(B, dtype):
    """C = sum_k A_k B_k over 6 uneven inner blocks, fused in one pass,
    equals the oracle's round-by-round accumulation and A B itself."""
    m, kk, n = 3000, 20000, 9000
    A = synth.varnnz_csr(m, kk, 4, 32, 11, dtype, "normal", stream=0)
    Bm = synth.varnnz_csr(kk, n, 4, 32, 11, dtype, "normal", stream=1)
    bounds = synth.column_blocks(kk, 6, kk // 12, kk // 3, 11)
    pairs = synth.split_inner(A, Bm, bounds)
    got = B.batched([(B.to_device(a), B.to_device(b)) for a, b in pairs]).to_host()
    ref, S = oracle.batched([(_f64(a), _f64(b)) for a, b in pairs], with_abs=True)
    assert_same_csr(got, ref, S, dtype, what="batched")
    full = oracle.spgemm(_f64(A), _f64(Bm))
    assert np.array_equal(ref.indices, full.indices)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_rmat_product_and_batched(B, dtype):
    """Power-law rows (R-MAT (0.57, 0.19, 0.19, 0.05), scale 15, edge factor
    16): empty rows, every LDS bin and hub rows beyond the LDS tables.  The
    plain product and the sum of its 8 uneven inner blocks in one pass both
    match the oracle."""
    n = 1 << 15
    A = synth.rmat_csr(15, 16, seed=21, dtype=dtype, values="normal")
    Bm = synth.varnnz_csr(n, n, 4, 32, 21, dtype, "normal", stream=3)
    ub = oracle.rowub(_f64(A), _f64(Bm))
    assert ub.max() > 20000 and (ub == 0).any()  # heavy rows and empty rows
    ref, S = oracle.spgemm(_f64(A), _f64(Bm), with_abs=True)
    got = B.spgemm(B.to_device(A), B.to_device(Bm)).to_host()
    assert_same_csr(got, ref, S, dtype, what="R-MAT product")
    bounds = synth.column_blocks(n, 8, n // 16, n // 4, 21)
    pairs = synth.split_inner(A, Bm, bounds)
    got = B.batched([(B.to_device(a), B.to_device(b)) for a, b in pairs]).to_host()
    assert_same_csr(got, ref, S, dtype, what="R-MAT batched")


def test_rmat_batched_full_size_sampled(B):
    """The R-MAT batched workload at full size (scale 20, edge factor 16, B
    with 4..32 uniform columns per row, 8 uneven inner blocks, FP32 N(0,1)):
    row_ptr of the fused sum against the oracle's count on every row;
    columns and values on the 16 heaviest rows and 2000 sampled ones."""
    import ctypes as C
    n = 1 << 20
    A = synth.rmat_csr(20, 16, seed=20260324, dtype=np.float32, values="normal", stream=0)
    Bm = synth.varnnz_csr(n, n, 4, 32, 20260324, np.float32, "normal", stream=1)
    bounds = synth.column_blocks(n, 8, n // 16, n // 4, 20260324)
    pairs = synth.split_inner(A, Bm, bounds)
    got = B.batched([(B.to_device(a), B.to_device(b)) for a, b in pairs]).to_host()
    Af, Bf = _f64(A), _f64(Bm)
    ref_rp = np.zeros(n + 1, dtype=np.int64)
    rc = oracle.lib().oracle_spgemm_count(
        C.c_int64(n), C.c_int64(n), C.c_int64(n), Af.indptr.ctypes.data_as(C.c_void_p),
        Af.indices.ctypes.data_as(C.c_void_p), Bf.indptr.ctypes.data_as(C.c_void_p),
        Bf.indices.ctypes.data_as(C.c_void_p), ref_rp.ctypes.data_as(C.c_void_p))
    assert rc == 0
    assert np.array_equal(got.indptr.astype(np.int64), ref_rp)
    ub = oracle.rowub(Af, Bf)
    heavy = np.argsort(ub)[-16:]
    rows = np.unique(np.concatenate([heavy, synth.rng_for(5, 5).choice(n, 2000, replace=False)]))
    from helpers import row_subset
    ref, S = oracle.spgemm(row_subset(Af, rows), Bf, with_abs=True)
    assert_same_csr(row_subset(got, rows), ref, S, np.float32, what="R-MAT 2^20 sampled rows")


def test_batched_equals_merge_of_products_exactly(B):
    pairs = [(synth.varnnz_csr(1500, 2000 + 100 * k, 0, 20, 40 + k, np.float64, "int", stream=0),
              synth.varnnz_csr(2000 + 100 * k, 2500, 0, 20, 40 + k, np.float64, "int", stream=1))
             for k in range(4)]
    dpairs = [(B.to_device(a), B.to_device(b)) for a, b in pairs]
    fused = B.batched(dpairs).to_host()
    partials = [B.spgemm(a, b) for a, b in dpairs]
    merged = B.merge(partials).to_host()
    assert np.array_equal(fused.indptr, merged.indptr)
    assert np.array_equal(fused.indices, merged.indices)
    assert np.array_equal(fused.data, merged.data)


def _grad_scales(A, Bm, C, W):
    """sum_j |W_ij||b_kj| per A entry and sum_i |a_ik||W_ij| per B entry."""
    return oracle.backward(A.with_data(np.abs(A.data)), Bm.with_data(np.abs(Bm.data)), C, np.abs(W))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_backward_matches_oracle_gradient(B, dtype):
    import torch
    A = synth.uniform_csr(8192, 8192, 16, 5, dtype, "normal", stream=0)
    Bm = synth.uniform_csr(8192, 8192, 16, 5, dtype, "normal", stream=1)
    dA_, dB_ = B.to_device(A), B.to_device(Bm)
    plan = B.Plan()
    rp, nnz = plan.symbolic([dA_], [dB_])
    col, vals = plan.numeric([dA_], [dB_], rp, nnz)
    Cg = B.DeviceCSR((8192, 8192), rp, col, vals).to_host()
    W = synth.draw_values(synth.rng_for(5, 9), nnz, "normal", dtype)
    dC = B.DeviceCSR((8192, 8192), rp, col, torch.from_numpy(W).cuda())
    gA, gB = plan.backward(dA_, dB_, dC)
    gA, gB = gA.cpu().numpy(), gB.cpu().numpy()
    Cp = synth.HostCSR(Cg.shape, Cg.indptr, Cg.indices, None)
    rA, rB = oracle.backward(_f64(A), _f64(Bm), Cp, W.astype(np.float64))
    sA, sB = _grad_scales(_f64(A), _f64(Bm), Cp, W.astype(np.float64))
    t = tol_for(dtype)
    assert np.all(np.abs(gA - rA) <= t * sA + 1e-300)
    assert np.all(np.abs(gB - rB) <= t * sB + 1e-300)


def test_backward_heavy_and_empty_rows(B):
    import torch
    A = synth.varnnz_csr(200, 3000, 0, 10, 8, np.float64, "normal", stream=0)
    dense_rows = synth.uniform_csr(3, 3000, 2000, 8, np.float64, "normal", stream=2)
    rows = [5, 60, 199]
    out = []
    for i in range(200):
        c, v = (dense_rows.row(rows.index(i)) if i in rows else A.row(i))
        out.append((c, v))
    ip = np.zeros(201, dtype=np.int64)
    np.cumsum([len(c) for c, _ in out], out=ip[1:])
    A = synth.HostCSR(A.shape, ip, np.concatenate([c for c, _ in out]).astype(np.int32),
                      np.concatenate([v for _, v in out]))
    Bm = synth.varnnz_csr(3000, 50000, 0, 24, 8, np.float64, "normal", stream=1)
    dA_, dB_ = B.to_device(A), B.to_device(Bm)
    plan = B.Plan()
    rp, nnz = plan.symbolic([dA_], [dB_])
    col, vals = plan.numeric([dA_], [dB_], rp, nnz)
    W = synth.draw_values(synth.rng_for(8, 9), nnz, "normal", np.float64)
    dC = B.DeviceCSR(A.shape[:1] + (50000,), rp, col, torch.from_numpy(W).cuda())
    gA, gB = plan.backward(dA_, dB_, dC)
    Cg = B.DeviceCSR((200, 50000), rp, col, vals).to_host()
    Cp = synth.HostCSR(Cg.shape, Cg.indptr, Cg.indices, None)
    rA, rB = oracle.backward(A, Bm, Cp, W)
    sA, sB = _grad_scales(A, Bm, Cp, W)
    assert np.all(np.abs(gA.cpu().numpy() - rA) <= 1e-12 * sA + 1e-300)
    assert np.all(np.abs(gB.cpu().numpy() - rB) <= 1e-12 * sB + 1e-300)


def _backward_case(B, A, Bm, seed, dtype, kind="normal"):
    import torch
    dA_, dB_ = B.to_device(A), B.to_device(Bm)
    plan = B.Plan()
    rp, nnz = plan.symbolic([dA_], [dB_])
    col, vals = plan.numeric([dA_], [dB_], rp, nnz)
    Cg = B.DeviceCSR((A.shape[0], Bm.shape[1]), rp, col, vals).to_host()
    W = synth.draw_values(synth.rng_for(seed, 9), nnz, kind, dtype)
    dC = B.DeviceCSR((A.shape[0], Bm.shape[1]), rp, col, torch.from_numpy(W).cuda())
    Cp = synth.HostCSR(Cg.shape, Cg.indptr, Cg.indices, None)
    return plan, dA_, dB_, dC, Cp, W


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_backward_deterministic_dB(B, dtype):
    """The deterministic backward: dB within tolerance of the oracle, the
    same bits on repeated runs, dA identical to the float-atomic path."""
    A = synth.uniform_csr(8192, 8192, 16, 15, dtype, "normal", stream=0)
    Bm = synth.uniform_csr(8192, 8192, 16, 15, dtype, "normal", stream=1)
    plan, dA_, dB_, dC, Cp, W = _backward_case(B, A, Bm, 15, dtype)
    gA, gB = plan.backward(dA_, dB_, dC, deterministic=True)
    gA2, gB2 = plan.backward(dA_, dB_, dC, deterministic=True)
    fA, _ = plan.backward(dA_, dB_, dC)
    assert plan.status() == B.SPG_OK
    gA, gB, gA2, gB2, fA = (x.cpu().numpy() for x in (gA, gB, gA2, gB2, fA))
    assert np.array_equal(gB.view(np.uint8), gB2.view(np.uint8))  # bit for bit
    assert np.array_equal(gA.view(np.uint8), gA2.view(np.uint8))
    assert np.array_equal(gA, fA)
    rA, rB = oracle.backward(_f64(A), _f64(Bm), Cp, W.astype(np.float64))
    sA, sB = _grad_scales(_f64(A), _f64(Bm), Cp, W.astype(np.float64))
    t = tol_for(dtype)
    assert np.all(np.abs(gB - rB) <= t * sB + 1e-300)
    assert np.all(np.abs(gA - rA) <= t * sA + 1e-300)


def test_backward_deterministic_exact_on_integers_with_heavy_rows(B):
    """Small-integer values: every term and sum is exact in the fixed-point
    units, so dB equals the oracle exactly, heavy rows and empty rows
    included."""
    A = synth.varnnz_csr(200, 3000, 0, 10, 18, np.float64, "int", stream=0)
    dense_rows = synth.uniform_csr(3, 3000, 2000, 18, np.float64, "int", stream=2)
    rows = [5, 60, 199]
    out = [(dense_rows.row(rows.index(i)) if i in rows else A.row(i)) for i in range(200)]
    ip = np.zeros(201, dtype=np.int64)
    np.cumsum([len(c) for c, _ in out], out=ip[1:])
    A = synth.HostCSR(A.shape, ip, np.concatenate([c for c, _ in out]).astype(np.int32),
                      np.concatenate([v for _, v in out]))
    Bm = synth.varnnz_csr(3000, 50000, 0, 24, 18, np.float64, "int", stream=1)
    plan, dA_, dB_, dC, Cp, W = _backward_case(B, A, Bm, 18, np.float64, "int")
    gA, gB = plan.backward(dA_, dB_, dC, deterministic=True)
    assert plan.status() == B.SPG_OK
    rA, rB = oracle.backward(A, Bm, Cp, W)
    assert np.array_equal(gB.cpu().numpy(), rB)
    assert np.array_equal(gA.cpu().numpy(), rA)


def _unaligned(t, off):
    """A copy of the 1-D tensor t whose data starts off elements past a
    16-byte boundary."""
    import torch
    buf = torch.zeros(t.numel() + off, dtype=t.dtype, device=t.device)
    buf[off:] = t
    return buf[off:]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_backward_deterministic_unaligned_values(B, dtype):
    """A and W values that start off a 16-byte boundary, with the largest
    |w| and |a| in the first (unaligned) or the last elements: the scale
    of the fixed-point sums sees them, and dA, dB are the bits of the
    aligned run."""
    A = synth.uniform_csr(3000, 3000, 12, 21, dtype, "normal", stream=0)
    Bm = synth.uniform_csr(3000, 3000, 12, 21, dtype, "normal", stream=1)
    plan, dA_, dB_, dC, Cp, W = _backward_case(B, A, Bm, 21, dtype)
    offs = [1, 3] if dtype == np.float32 else [1]
    for where in (0, -1):
        Wd = dC.vals.clone()
        Wd[where] = 1e3
        Ad = dA_.vals.clone()
        Ad[where] = -1e3
        ref = plan.backward(B.DeviceCSR(dA_.shape, dA_.row_ptr, dA_.col_idx, Ad), dB_,
                            B.DeviceCSR(dC.shape, dC.row_ptr, dC.col_idx, Wd), deterministic=True)
        ref = [x.cpu().numpy() for x in ref]
        for off in offs:
            got = plan.backward(
                B.DeviceCSR(dA_.shape, dA_.row_ptr, dA_.col_idx, _unaligned(Ad, off)), dB_,
                B.DeviceCSR(dC.shape, dC.row_ptr, dC.col_idx, _unaligned(Wd, off)),
                deterministic=True)
            assert plan.status() == B.SPG_OK
            for g, r in zip(got, ref):
                assert np.array_equal(g.cpu().numpy().view(np.uint8), r.view(np.uint8))
        A2 = A.with_data(Ad.cpu().numpy())
        W2 = Wd.cpu().numpy()
        rA, rB = oracle.backward(_f64(A2), _f64(Bm), Cp, W2.astype(np.float64))
        sA, sB = _grad_scales(_f64(A2), _f64(Bm), Cp, W2.astype(np.float64))
        t = tol_for(dtype)
        assert np.all(np.abs(ref[1] - rB) <= t * sB + 1e-300)
        assert np.all(np.abs(ref[0] - rA) <= t * sA + 1e-300)


def test_backward_deterministic_rejects_non_finite(B):
    import torch
    A = synth.uniform_csr(500, 500, 8, 19, np.float32, "normal", stream=0)
    Bm = synth.uniform_csr(500, 500, 8, 19, np.float32, "normal", stream=1)
    plan, dA_, dB_, dC, Cp, W = _backward_case(B, A, Bm, 19, np.float32)
    W[3] = np.inf
    dC = B.DeviceCSR(dC.shape, dC.row_ptr, dC.col_idx, torch.from_numpy(W).cuda())
    plan.backward(dA_, dB_, dC, deterministic=True)
    assert plan.status() == B.SPG_ERR_INVALID


@pytest.mark.parametrize("det", [False, True])
def test_autograd_function_and_euler_identity(B, det):
    """loss = <W, C>: autograd gradients equal the oracle's, and
    <A, dA> = L = <B, dB> (bilinearity); with the deterministic backward a
    second pass gives the same bits."""
    import torch
    from paper_2603_21444_amd.autograd import SpGEMMPattern, spgemm_values
    A = synth.uniform_csr(4096, 4096, 16, 12, np.float64, "normal", stream=0)
    Bm = synth.uniform_csr(4096, 4096, 16, 12, np.float64, "normal", stream=1)
    Ap, Bp = B.to_device(A), B.to_device(Bm)
    pat = SpGEMMPattern(Ap, Bp, deterministic=det)
    a = Ap.vals.clone().requires_grad_(True)
    b = Bp.vals.clone().requires_grad_(True)
    c = spgemm_values(a, b, Ap, Bp, pat)
    W = torch.from_numpy(synth.draw_values(synth.rng_for(12, 3), pat.nnz, "normal", np.float64)).cuda()
    loss = (W * c).sum()
    loss.backward()
    L = float(loss)
    assert abs(float((a.detach() * a.grad).sum()) - L) <= 1e-10 * (1 + abs(L))
    assert abs(float((b.detach() * b.grad).sum()) - L) <= 1e-10 * (1 + abs(L))
    Cp = synth.HostCSR((4096, 4096), pat.row_ptr.cpu().numpy().astype(np.int64),
                       pat.col_idx.cpu().numpy(), None)
    rA, rB = oracle.backward(A, Bm, Cp, W.cpu().numpy())
    sA, sB = _grad_scales(A, Bm, Cp, W.cpu().numpy())
    assert np.all(np.abs(a.grad.cpu().numpy() - rA) <= 1e-12 * sA + 1e-300)
    assert np.all(np.abs(b.grad.cpu().numpy() - rB) <= 1e-12 * sB + 1e-300)
    if det:
        b2 = Bp.vals.clone().requires_grad_(True)
        (W * spgemm_values(a.detach(), b2, Ap, Bp, pat)).sum().backward()
        assert torch.equal(b2.grad, b.grad)

"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test checks the oracle against something fixed by the paper's
definitions or by mathematics: hand-worked examples, brute force on tiny
inputs, dense numpy products, closed forms, invariants and special cases.
"""
from fractions import Fraction
from itertools import product as iproduct

import numpy as np
import pytest

import oracle
from paper_2603_21444_amd import synth
from helpers import (assert_canonical, csr_from_json, dense, load_golden, mask,
                     row_ids)

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# --------------------------------------------------------------- §2 product
def test_hand_worked_golden():
    g = load_golden("spgemm_hand.json")
    A, B, Cx = csr_from_json(g["A"]), csr_from_json(g["B"]), csr_from_json(g["C"])
    C = oracle.spgemm(A, B)
    assert np.array_equal(C.indptr, Cx.indptr)
    assert np.array_equal(C.indices, Cx.indices)
    assert np.array_equal(C.data, Cx.data)
    assert np.array_equal(oracle.rowub(A, B), np.array(g["ub"]))


def _brute(A, B):
    """Every (i, k, j) triple with a_ik and b_kj stored, in exact Fractions."""
    Ad, Bd = dense(A), dense(B)
    Am, Bm = mask(A), mask(B)
    m, k = A.shape
    n = B.shape[1]
    out = {}
    for i, kk, j in iproduct(range(m), range(k), range(n)):
        if Am[i, kk] and Bm[kk, j]:
            out[(i, j)] = out.get((i, j), Fraction(0)) + Fraction(Ad[i, kk]) * Fraction(Bd[kk, j])
    return out


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("kind", ["int", "u01"])
def test_brute_force_tiny(seed, kind):
    A = synth.varnnz_csr(13, 11, 0, 5, seed, np.float64, kind, stream=0)
    B = synth.varnnz_csr(11, 9, 0, 4, seed, np.float64, kind, stream=1)
    C = oracle.spgemm(A, B)
    ref = _brute(A, B)
    got = {(int(i), int(j)): v for i, j, v in zip(row_ids(C), C.indices, C.data)}
    assert set(got) == set(ref)
    for key, v in ref.items():
        if kind == "int":
            assert got[key] == float(v)
        else:
            assert abs(got[key] - float(v)) <= 1e-15 * max(1.0, abs(float(v))) * 8
    assert_canonical(C)
    assert np.array_equal(oracle.rowub(A, B),
                          np.array([sum(1 for (i2, kk, j) in iproduct([i], range(11), range(9))
                                        if mask(A)[i2, kk] and mask(B)[kk, j])
                                    for i in range(13)]))


@pytest.mark.parametrize("seed", [5, 6])
def test_pattern_is_boolean_product(seed):
    """S(C) equals the boolean product of the patterns, cancellation or not."""
    A = synth.uniform_csr(200, 150, 6, seed, np.float64, "int", stream=0)
    B = synth.uniform_csr(150, 170, 5, seed, np.float64, "int", stream=1)
    C = oracle.spgemm(A, B)
    bool_prod = (mask(A) @ mask(B)) > 0
    assert np.array_equal(mask(C).astype(bool), bool_prod)
    # integer values: every partial sum is exact, so values match dense exactly
    assert np.array_equal(dense(C), dense(A) @ dense(B))
    # exact cancellations happen and stay stored
    assert np.sum(C.data == 0.0) > 0
    assert_canonical(C)


def test_dense_fp64_positive():
    A = synth.uniform_csr(300, 256, 9, 11, np.float64, "u01", stream=0)
    B = synth.uniform_csr(256, 280, 7, 11, np.float64, "u01", stream=1)
    C, S = oracle.spgemm(A, B, with_abs=True)
    D = dense(A) @ dense(B)
    assert np.array_equal(mask(C).astype(bool), D > 0)
    rid = row_ids(C)
    assert np.allclose(C.data, D[rid, C.indices], rtol=1e-14, atol=0)
    # positive inputs: S_ij equals C_ij
    assert np.allclose(S, C.data, rtol=1e-14, atol=0)


def test_row_sum_invariant_and_scipy():
    A = synth.varnnz_csr(2000, 1500, 0, 12, 21, np.float64, "normal", stream=0)
    B = synth.varnnz_csr(1500, 1800, 0, 12, 21, np.float64, "normal", stream=1)
    C, S = oracle.spgemm(A, B, with_abs=True)
    ones = np.ones(B.shape[1])
    lhs = np.bincount(row_ids(C), weights=C.data, minlength=C.shape[0])
    Bd, Ad = dense(B), dense(A)
    rhs = Ad @ (Bd @ ones)
    bound = np.bincount(row_ids(C), weights=S, minlength=C.shape[0])
    assert np.all(np.abs(lhs - rhs) <= 1e-13 * (bound + 1e-300))
    # scipy cross-check of the values on the structural pattern
    import scipy.sparse as sp
    a = sp.csr_matrix((A.data, A.indices, A.indptr), shape=A.shape)
    b = sp.csr_matrix((B.data, B.indices, B.indptr), shape=B.shape)
    c = (a @ b).toarray()
    assert np.all(np.abs(c[row_ids(C), C.indices] - C.data) <= 1e-13 * S + 1e-300)


def test_column_stochastic_closure():
    X = synth.mcl_matrix(500, 7, 3, np.float64)       # rows of X = columns of M
    M = synth.HostCSR(X.shape, X.indptr, X.indices, X.data)
    # C^T = X X, and column sums of M M are row sums of X X
    C = oracle.spgemm(M, M)
    sums = np.bincount(row_ids(C), weights=C.data, minlength=500)
    assert np.allclose(sums, 1.0, rtol=0, atol=1e-14)


def test_identity_and_permutation_exact():
    B = synth.varnnz_csr(400, 350, 0, 9, 31, np.float64, "normal")
    I = synth.identity_csr(400)
    C = oracle.spgemm(I, B)
    assert np.array_equal(C.indptr, B.indptr)
    assert np.array_equal(C.indices, B.indices)
    assert np.array_equal(C.data, B.data)
    P = synth.permutation_csr(400, 7)
    C = oracle.spgemm(P, B)
    perm = P.indices
    lens = np.diff(B.indptr)
    assert np.array_equal(np.diff(C.indptr), lens[perm])
    for i in range(0, 400, 37):
        cols, vals = B.row(perm[i])
        s, e = C.indptr[i], C.indptr[i + 1]
        assert np.array_equal(C.indices[s:e], cols)
        assert np.array_equal(C.data[s:e], vals)
    # A B with B = identity returns A
    C = oracle.spgemm(B, synth.identity_csr(350))
    assert np.array_equal(C.indices, B.indices) and np.array_equal(C.data, B.data)


def test_input_order_does_not_matter():
    A = synth.uniform_csr(300, 300, 10, 41, np.float64, "int", stream=0)
    B = synth.uniform_csr(300, 300, 10, 41, np.float64, "int", stream=1)
    C1 = oracle.spgemm(A, B)
    C2 = oracle.spgemm(synth.shuffle_rows(A, 1), synth.shuffle_rows(B, 2))
    assert np.array_equal(C1.indptr, C2.indptr)
    assert np.array_equal(C1.indices, C2.indices)
    assert np.array_equal(C1.data, C2.data)


def test_empty_shapes():
    A = synth.uniform_csr(0, 5, 0, 1, np.float64)
    B = synth.uniform_csr(5, 7, 2, 1, np.float64)
    C = oracle.spgemm(A, B)
    assert C.indptr.tolist() == [0] and C.indices.size == 0
    A = synth.uniform_csr(6, 5, 0, 1, np.float64)
    C = oracle.spgemm(A, B)
    assert C.indptr.tolist() == [0] * 7
    with pytest.raises(oracle.OracleError):
        oracle.spgemm(B, B)


def test_threads_do_not_change_bits():
    A = synth.varnnz_csr(3000, 2000, 0, 20, 51, np.float64, "normal", stream=0)
    B = synth.varnnz_csr(2000, 2500, 0, 20, 51, np.float64, "normal", stream=1)
    t0 = oracle.num_threads()
    try:
        oracle.set_threads(1)
        C1 = oracle.spgemm(A, B)
        oracle.set_threads(max(2, t0))
        C2 = oracle.spgemm(A, B)
    finally:
        oracle.set_threads(t0)
    assert np.array_equal(C1.indices, C2.indices)
    assert np.array_equal(C1.data, C2.data)


# ------------------------------------------------------ §4.4 merge, Alg. 1 sums
def test_merge_against_dense_and_cancellation():
    parts = [synth.varnnz_csr(120, 90, 0, 8, 60 + k, np.float64, "normal") for k in range(4)]
    C = oracle.merge(parts)
    D = sum(dense(P) for P in parts)
    U = sum(mask(P) for P in parts) > 0
    assert np.array_equal(mask(C).astype(bool), U)
    assert np.allclose(dense(C), D, rtol=1e-15, atol=1e-15)
    assert_canonical(C)
    P = parts[0]
    Z = oracle.merge([P, P.with_data(-P.data)])
    assert np.array_equal(Z.indices, P.indices) and np.all(Z.data == 0.0)


def test_merge_disjoint_is_concatenation():
    P = synth.varnnz_csr(50, 64, 0, 10, 70, np.float64, "normal")
    # split each row's entries by column parity into two disjoint matrices
    sel = P.indices % 2 == 0
    rid = row_ids(P)

    def take(s):
        ip = np.zeros(51, dtype=np.int64)
        np.cumsum(np.bincount(rid[s], minlength=50), out=ip[1:])
        return synth.HostCSR(P.shape, ip, P.indices[s], P.data[s])

    C = oracle.merge([take(sel), take(~sel)])
    assert np.array_equal(C.indptr, P.indptr)
    assert np.array_equal(C.indices, P.indices)
    assert np.array_equal(C.data, P.data)


def test_batched_equals_merge_of_products_and_full_product():
    A = synth.varnnz_csr(256, 1000, 4, 32, 81, np.float64, "int", stream=0)
    B = synth.varnnz_csr(1000, 700, 4, 32, 81, np.float64, "int", stream=1)
    bounds = synth.column_blocks(1000, 5, 100, 400, 81)
    pairs = synth.split_inner(A, B, bounds)
    Cb = oracle.batched(pairs)
    Cm = oracle.merge([oracle.spgemm(a, b) for a, b in pairs])
    Cf = oracle.spgemm(A, B)
    for X in (Cm, Cf):
        assert np.array_equal(Cb.indptr, X.indptr)
        assert np.array_equal(Cb.indices, X.indices)
        assert np.array_equal(Cb.data, X.data)  # integer values: exact
    assert np.array_equal(dense(Cb), dense(A) @ dense(B))


# ------------------------------------------------------------- §5.7 MCL step
def test_mcl_hand_worked_golden():
    g = load_golden("mcl_hand.json")
    X = csr_from_json(g["X"])
    for case in g["cases"]:
        cnt, cols, vals = oracle.mcl_rows(X, np.arange(3), 2, case["prune"], case["topk"])
        for t, (ecols, evals) in enumerate(case["rows"]):
            assert cols[t].tolist() == ecols
            want = [p / q for p, q in evals]
            assert np.allclose(vals[t], want, rtol=1e-15, atol=0)


@pytest.mark.parametrize("b", [4, 8, 64])
def test_mcl_block_fixed_point(b):
    """Block-diagonal M with all entries 1/b is idempotent and survives
    inflation + normalisation unchanged: exact fixed point."""
    nb = 6
    n = b * nb
    perm = synth.rng_for(b).permutation(n)
    blocks = perm.reshape(nb, b)
    rows, cols = [], []
    for blk in blocks:
        for i in blk:
            for j in blk:
                rows.append(i); cols.append(j)
    rows, cols = np.array(rows), np.array(cols)
    order = np.lexsort((cols, rows))
    ip = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=ip[1:])
    X = synth.HostCSR((n, n), ip, cols[order].astype(np.int32), np.full(n * b, 1.0 / b))
    Y = X
    for _ in range(10):
        Y = oracle.mcl_step(Y, 2, 1e-4, 1000)
    assert np.array_equal(Y.indptr, X.indptr)
    assert np.array_equal(Y.indices, X.indices)
    assert np.array_equal(Y.data, X.data)


def test_mcl_topk_ties_go_to_smaller_column():
    """All entries of a block are equal: top-2 keeps the two smallest
    columns of the block, renormalised to 1/2 each."""
    b, nb = 4, 5
    n = b * nb
    rows = np.repeat(np.arange(n), b)
    cols = (rows // b) * b + np.tile(np.arange(b), n)
    ip = np.arange(n + 1, dtype=np.int64) * b
    X = synth.HostCSR((n, n), ip, cols.astype(np.int32), np.full(n * b, 1.0 / b))
    Y = oracle.mcl_step(X, 2, 1e-4, 2)
    for i in range(n):
        s, e = Y.indptr[i], Y.indptr[i + 1]
        assert Y.indices[s:e].tolist() == [(i // b) * b, (i // b) * b + 1]
        assert Y.data[s:e].tolist() == [0.5, 0.5]


def test_mcl_no_prune_matches_dense():
    X = synth.mcl_matrix(300, 6, 9, np.float64)
    Y = oracle.mcl_step(X, 2, 0.0, 10 ** 6)
    E = dense(X) @ dense(X)
    E = E ** 2
    E = E / E.sum(axis=1, keepdims=True)
    assert np.array_equal(mask(Y).astype(bool), E > 0)
    assert np.allclose(dense(Y), E, rtol=1e-13, atol=0)


def test_mcl_invariants_and_topk():
    X = synth.mcl_matrix(400, 12, 13, np.float64)
    for prune, topk in [(1e-4, 1000), (2e-3, 50), (0.0, 7), (0.5, 3)]:
        Y = oracle.mcl_step(X, 2, prune, topk)
        sums = np.bincount(row_ids(Y), weights=Y.data, minlength=400)
        assert np.allclose(sums, 1.0, atol=1e-14, rtol=0)
        lens = np.diff(Y.indptr)
        assert lens.max() <= topk and lens.min() >= 1
        assert_canonical(Y)
        # which entries survive: the kept set is the top of the pruned,
        # normalised, inflated expansion (checked densely)
        E = (dense(X) @ dense(X)) ** 2
        E = E / E.sum(axis=1, keepdims=True)
        for i in range(0, 400, 23):
            row = E[i]
            nz = np.nonzero(row)[0]
            keep = nz[row[nz] >= prune]
            if keep.size > topk:
                order = np.lexsort((keep, -row[keep]))
                keep = np.sort(keep[order[:topk]])
            if keep.size == 0:
                keep = np.array([nz[np.argmax(row[nz])]])
            s, e = Y.indptr[i], Y.indptr[i + 1]
            assert np.array_equal(Y.indices[s:e], keep)


# -------------------------------------------------------------- backward pins
def test_backward_hand_worked_golden():
    g = load_golden("spgemm_hand.json")
    A, B, Cx = csr_from_json(g["A"]), csr_from_json(g["B"]), csr_from_json(g["C"])
    W = np.array(g["backward"]["W"], dtype=np.float64)
    dA, dB = oracle.backward(A, B, Cx, W)
    assert dA.tolist() == g["backward"]["dA"]
    assert dB.tolist() == g["backward"]["dB"]
    assert float(np.dot(W, oracle.spgemm(A, B).data)) == g["backward"]["L"]


def test_backward_dense_formula_and_euler():
    A = synth.uniform_csr(120, 100, 6, 91, np.float64, "normal", stream=0)
    B = synth.uniform_csr(100, 110, 5, 91, np.float64, "normal", stream=1)
    C = oracle.spgemm(A, B)
    W = synth.draw_values(synth.rng_for(91, 5), C.nnz, "normal", np.float64)
    dA, dB = oracle.backward(A, B, C, W)
    Wd = np.zeros(C.shape)
    Wd[row_ids(C), C.indices] = W
    dAd = Wd @ dense(B).T
    dBd = dense(A).T @ Wd
    assert np.allclose(dA, dAd[row_ids(A), A.indices], rtol=1e-12, atol=1e-13)
    assert np.allclose(dB, dBd[row_ids(B), B.indices], rtol=1e-12, atol=1e-13)
    L = float(np.dot(W, C.data))
    assert abs(np.dot(A.data, dA) - L) <= 1e-12 * (1 + abs(L))
    assert abs(np.dot(B.data, dB) - L) <= 1e-12 * (1 + abs(L))


def test_backward_identity_b():
    A = synth.uniform_csr(64, 64, 5, 93, np.float64, "normal")
    I = synth.identity_csr(64)
    C = oracle.spgemm(A, I)
    W = synth.draw_values(synth.rng_for(93, 2), C.nnz, "normal", np.float64)
    dA, dB = oracle.backward(A, I, C, W)
    assert np.array_equal(dA, W)


def test_backward_central_fd():
    """L is bilinear in (A, B): central differences are exact in real
    arithmetic for any step, so only FP64 rounding of L remains.  L is
    evaluated densely (numpy), independent of the oracle."""
    A = synth.uniform_csr(512, 512, 16, 95, np.float64, "normal", stream=0)
    B = synth.uniform_csr(512, 512, 16, 95, np.float64, "normal", stream=1)
    C = oracle.spgemm(A, B)
    W = synth.draw_values(synth.rng_for(95, 3), C.nnz, "normal", np.float64)
    dA, dB = oracle.backward(A, B, C, W)
    Wd = np.zeros(C.shape)
    Wd[row_ids(C), C.indices] = W
    Ad, Bd = dense(A), dense(B)

    def loss(Am, Bm):
        return float(np.sum(Wd * (Am @ Bm)))

    h = 0.5
    rng = synth.rng_for(95, 4)
    ra, rb = row_ids(A), row_ids(B)
    for p in rng.choice(A.nnz, 24, replace=False):
        E = np.zeros_like(Ad)
        E[ra[p], A.indices[p]] = h
        fd = (loss(Ad + E, Bd) - loss(Ad - E, Bd)) / (2 * h)
        assert abs(fd - dA[p]) <= 1e-8 * (1 + abs(dA[p]))
    for q in rng.choice(B.nnz, 24, replace=False):
        E = np.zeros_like(Bd)
        E[rb[q], B.indices[q]] = h
        fd = (loss(Ad, Bd + E) - loss(Ad, Bd - E)) / (2 * h)
        assert abs(fd - dB[q]) <= 1e-8 * (1 + abs(dB[q]))


def test_backward_rejects_foreign_pattern():
    A = synth.uniform_csr(20, 20, 3, 97, np.float64, "normal", stream=0)
    B = synth.uniform_csr(20, 20, 3, 97, np.float64, "normal", stream=1)
    C = oracle.spgemm(A, B)
    C2 = synth.HostCSR(C.shape, C.indptr, (C.indices + 1) % 20, C.data)
    with pytest.raises(oracle.OracleError):
        oracle.backward(A, B, C2, np.ones(C.nnz))


# ------------------------------------- §5.7 MCL step in the paper's own order
def test_mcl_paper_order_hand_worked_golden():
    g = load_golden("mcl_paper_hand.json")
    X = csr_from_json(g["X"])
    for case in g["cases"]:
        cnt, cols, vals = oracle.mcl_rows(X, np.arange(3), case["r"], case["prune"], case["topk"],
                                          order="paper")
        for t, (ecols, evals) in enumerate(case["rows"]):
            assert cols[t].tolist() == ecols, (case, t)
            want = [p / q for p, q in evals]
            assert np.allclose(vals[t], want, rtol=1e-15, atol=0), (case, t)


@pytest.mark.parametrize("b", [4, 8, 64])
def test_mcl_paper_order_block_fixed_point(b):
    """Blocks of 1/b: the first iteration gives blocks of 1/b^2 (normalised
    back to 1/b, then squared); from then on E has entries 1/b^3, which
    normalise to 1/b and square to 1/b^2 again.  Exact for b a power of 2."""
    nb = 5
    n = b * nb
    perm = synth.rng_for(b, 3).permutation(n)
    rows, cols = [], []
    for blk in perm.reshape(nb, b):
        for i in blk:
            for j in blk:
                rows.append(i); cols.append(j)
    rows, cols = np.array(rows), np.array(cols)
    order = np.lexsort((cols, rows))
    ip = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=ip[1:])
    X = synth.HostCSR((n, n), ip, cols[order].astype(np.int32), np.full(n * b, 1.0 / b))
    Y = X
    for _ in range(10):
        Y = oracle.mcl_step(Y, 2, 0.002, 500, order="paper")
        assert np.array_equal(Y.indptr, X.indptr)
        assert np.array_equal(Y.indices, X.indices)
        assert np.all(Y.data == 1.0 / (b * b))


@pytest.mark.parametrize("r", [1, 2, 3])
def test_mcl_paper_order_no_prune_matches_dense(r):
    X = synth.mcl_matrix(300, 6, 19, np.float64)
    Y = oracle.mcl_step(X, r, 0.0, 10 ** 6, order="paper")
    E = dense(X) @ dense(X)
    E = (E / E.sum(axis=1, keepdims=True)) ** r
    assert np.array_equal(mask(Y).astype(bool), E > 0)
    assert np.allclose(dense(Y), E, rtol=1e-13, atol=0)


def test_mcl_paper_order_prune_keeps_the_large_entries():
    """With the paper's threshold 0.002: kept entries are exactly those whose
    normalised expansion value is >= 0.002 (dense check), at most 500 per
    row, each output is that value squared, and no row is empty."""
    X = synth.mcl_matrix(600, 40, 23, np.float64)
    Y = oracle.mcl_step(X, 2, 0.002, 500, order="paper")
    E = dense(X) @ dense(X)
    N = E / E.sum(axis=1, keepdims=True)
    keep = N >= 0.002
    empty = ~keep.any(axis=1)
    keep[empty, np.argmax(N[empty], axis=1)] = True
    assert np.array_equal(mask(Y).astype(bool), keep)
    assert np.allclose(dense(Y)[keep], N[keep] ** 2, rtol=1e-13, atol=0)
    lens = np.diff(Y.indptr)
    assert lens.max() <= 500 and lens.min() >= 1
    assert_canonical(Y)


# ------------------------------------- §5.3 random permutation preprocessing
def test_permute_identity_and_inverse():
    A = synth.shuffle_rows(synth.varnnz_csr(300, 250, 0, 30, 4, np.float64, "normal"), 4)
    I = oracle.permute(A)
    rid = np.repeat(np.arange(300), np.diff(A.indptr))
    order = np.lexsort((A.indices, rid))  # A with every row sorted (numpy, not the oracle)
    ref = synth.HostCSR(A.shape, A.indptr, A.indices[order], A.data[order])
    assert np.array_equal(I.indptr, ref.indptr) and np.array_equal(I.indices, ref.indices)
    assert np.array_equal(I.data, ref.data)
    p, q = synth.random_permutation(300, 1), synth.random_permutation(250, 2)
    Bp = oracle.permute(A, p, q)
    back = oracle.permute(synth.HostCSR(Bp.shape, Bp.indptr, Bp.indices, Bp.data),
                          np.argsort(p).astype(np.int32), np.argsort(q).astype(np.int32))
    assert np.array_equal(back.indptr, ref.indptr) and np.array_equal(back.indices, ref.indices)
    assert np.array_equal(back.data, ref.data)


def test_permute_matches_dense_permutation_matrices():
    A = synth.varnnz_csr(120, 90, 0, 20, 5, np.float64, "normal")
    p, q = synth.random_permutation(120, 3), synth.random_permutation(90, 4)
    Bp = oracle.permute(A, p, q)
    Pr = np.zeros((120, 120)); Pr[p, np.arange(120)] = 1.0
    Pc = np.zeros((90, 90)); Pc[q, np.arange(90)] = 1.0
    assert np.array_equal(dense(Bp), Pr @ dense(A) @ Pc.T)
    assert np.array_equal(mask(Bp), (Pr @ mask(A) @ Pc.T).astype(np.int64))
    assert_canonical(Bp)


def test_symmetric_permutation_commutes_with_squaring():
    A = synth.banded_csr(400, 6, [0, 100, -100], 5, 6, np.float64, "int")
    p = synth.random_permutation(400, 5)
    PA = oracle.permute(A, p, p)
    PAh = synth.HostCSR(PA.shape, PA.indptr, PA.indices, PA.data)
    lhs = oracle.spgemm(PAh, PAh)
    rhs = oracle.permute(oracle.spgemm(A, A), p, p)
    assert np.array_equal(lhs.indptr, rhs.indptr) and np.array_equal(lhs.indices, rhs.indices)
    assert np.array_equal(lhs.data, rhs.data)  # small integers: exact


def test_permute_rejects_non_permutations():
    A = synth.varnnz_csr(10, 10, 1, 3, 6, np.float64, "normal")
    bad = np.arange(10, dtype=np.int32)
    bad[3] = 4
    with pytest.raises(oracle.OracleError):
        oracle.permute(A, bad, None)
    with pytest.raises(oracle.OracleError):
        oracle.permute(A, None, np.arange(1, 11, dtype=np.int32))


def test_banded_generator_has_bands():
    A = synth.banded_csr(5000, 12, [0, 1000, -1000], 20, 7, np.float32)
    rid = np.repeat(np.arange(5000), np.diff(A.indptr))
    off = A.indices.astype(np.int64) - rid
    near = np.min(np.abs(off[:, None] - np.array([0, 1000, -1000])[None, :]), axis=1)
    inner = (rid >= 1100) & (rid < 3900)  # rows whose windows stay inside [0, n)
    assert np.all(near[inner] <= 20)
    assert_canonical(A)


# ------------------------------- §5.4 restriction operator product C = A R
@pytest.mark.parametrize("values", ["one", "int"])
def test_restriction_product_is_a_row_merge_by_aggregate(values):
    """R has one entry per row (fine point k -> aggregate agg[k], weight
    w_k), so row i of C = A R holds, for every aggregate j reached from A_i,
    the sum of a_ik w_k over the k of A_i in aggregate j.  Built here by a
    segmented sum in numpy, independently of the oracle's product."""
    m, n, nc = 700, 900, 111
    A = synth.varnnz_csr(m, n, 0, 25, 31, np.float64, "int")
    R = synth.aggregation_csr(n, nc, 31, np.float64, values)
    assert np.all(np.diff(R.indptr) == 1) and np.bincount(R.indices, minlength=nc).min() >= n // nc
    C = oracle.spgemm(A, R)
    rid = np.repeat(np.arange(m), np.diff(A.indptr))
    agg = R.indices[A.indices]
    contrib = A.data * R.data[A.indices]
    order = np.lexsort((agg, rid))
    rid, agg, contrib = rid[order], agg[order], contrib[order]
    first = np.ones(rid.size, dtype=bool)
    first[1:] = (rid[1:] != rid[:-1]) | (agg[1:] != agg[:-1])
    starts = np.nonzero(first)[0]
    sums = np.add.reduceat(contrib, starts) if starts.size else np.zeros(0)
    ip = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rid[starts], minlength=m), out=ip[1:])
    assert np.array_equal(C.indptr, ip)
    assert np.array_equal(C.indices, agg[starts])
    assert np.array_equal(C.data, sums)  # small integers: exact in any order

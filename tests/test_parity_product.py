"""GPU parity of the product C = A B (symbolic + numeric) against the FP64
oracle: bit-exact row_ptr and col_idx, values within tolerance (or exact
for small-integer values).  Calls go through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_2603_21444_amd import synth
from helpers import assert_same_csr, row_subset

pytestmark = pytest.mark.gpu

SEED = 20260321


@pytest.fixture(scope="module")
def B():
    import torch
    from paper_2603_21444_amd import binding
    assert torch.cuda.is_available()
    binding.lib()
    return binding


def gpu_product(binding, A, Bm, dtype):
    dA = binding.to_device(A, dtype=dtype)
    dB = binding.to_device(Bm, dtype=dtype)
    C = binding.spgemm(dA, dB)
    return C.to_host()


def check(binding, A, Bm, dtype, exact=False, what=""):
    got = gpu_product(binding, A, Bm, dtype)
    Af = A.with_data(A.data.astype(dtype).astype(np.float64))
    Bf = Bm.with_data(Bm.data.astype(dtype).astype(np.float64))
    ref, S = oracle.spgemm(Af, Bf, with_abs=True)
    assert_same_csr(got, ref, S, dtype, exact, what)
    return got


def test_square_4096_fp64(B):
    """C = A A, n = 4096, exactly 8 uniform distinct columns per row, FP64 in (0,1]."""
    A = synth.uniform_csr(4096, 4096, 8, SEED, np.float64, "u01")
    check(B, A, A, np.float64, what="A*A n=4096")


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_small_integers_exact(B, dtype):
    A = synth.uniform_csr(3000, 2500, 12, 3, dtype, "int", stream=0)
    Bm = synth.uniform_csr(2500, 2700, 12, 3, dtype, "int", stream=1)
    got = check(B, A, Bm, dtype, exact=True, what="integers")
    assert np.sum(got.data == 0) > 0  # cancellations stay stored


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_ragged_rows_span_all_lds_bins(B, dtype):
    """Row lengths 0..200 times 0..64 give 0..~8000 products per row, so every
    LDS bin and the empty bin are hit, with ragged tails everywhere."""
    A = synth.varnnz_csr(6000, 4000, 0, 200, 5, dtype, "normal", stream=0)
    Bm = synth.varnnz_csr(4000, 30000, 0, 64, 5, dtype, "normal", stream=1)
    check(B, A, Bm, dtype, what="ragged")


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_heavy_rows_lds_bitmap(B, dtype):
    """A few dense A rows push rows past every LDS table into the heavy path."""
    n = 60000
    A = synth.varnnz_csr(300, 5000, 1, 40, 7, dtype, "normal", stream=0)
    dense_rows = synth.uniform_csr(4, 5000, 2500, 7, dtype, "normal", stream=2)
    A = _replace_rows(A, [3, 77, 150, 299], dense_rows)
    Bm = synth.varnnz_csr(5000, n, 4, 32, 7, dtype, "normal", stream=1)
    check(B, A, Bm, dtype, what="heavy")


def test_heavy_rows_global_bitmap(B):
    """More than 2^20 output columns: heavy rows use the global bitmap."""
    n = (1 << 20) + 4097
    A = synth.varnnz_csr(64, 3000, 1, 30, 9, np.float32, "normal", stream=0)
    dense_rows = synth.uniform_csr(2, 3000, 1500, 9, np.float32, "normal", stream=2)
    A = _replace_rows(A, [5, 40], dense_rows)
    Bm = synth.varnnz_csr(3000, n, 8, 24, 9, np.float32, "normal", stream=1)
    check(B, A, Bm, np.float32, what="heavy, wide")


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_heavy_rows_beyond_the_staging_area(B, dtype):
    """Heavy rows with more products than the output has columns (+4): the
    column-range kernel cannot stage them and adds them densely instead;
    the other heavy rows of the same launch take the range path."""
    n = 40000
    A = synth.varnnz_csr(200, 4000, 1, 20, 13, dtype, "normal", stream=0)
    dense_rows = synth.uniform_csr(3, 4000, 3000, 13, dtype, "normal", stream=2)
    A = _replace_rows(A, [7, 100, 199], dense_rows)  # ~60000 products > n + 4: dense
    mid_rows = synth.uniform_csr(2, 4000, 1000, 14, dtype, "normal", stream=3)
    A = _replace_rows(A, [50, 51], mid_rows)  # ~20000 products: heavy, staged by range
    Bm = synth.varnnz_csr(4000, n, 10, 30, 13, dtype, "normal", stream=1)
    check(B, A, Bm, dtype, what="heavy beyond staging")


def _band_rows(k, n, width, step, seed, dtype):
    """k x n matrix whose row r holds `width` consecutive columns from
    (r * step) mod n: products of nearby rows pile up on the same columns."""
    rows = np.repeat(np.arange(k), width)
    cols = ((rows * step) % n + np.tile(np.arange(width), k)) % n
    order = np.lexsort((cols, rows))
    vals = synth.draw_values(synth.rng_for(seed), cols.size, "normal", dtype)
    return synth.HostCSR((k, n), np.arange(k + 1, dtype=np.int64) * width,
                         cols[order].astype(np.int32), vals)


def _rows_from(A, lists, seed, dtype):
    """A with row i replaced by the columns lists[i] (for i in lists)."""
    out_rows = []
    rng = synth.rng_for(seed, 9)
    for i in range(A.shape[0]):
        if i in lists:
            c = np.sort(np.asarray(lists[i], dtype=np.int32))
            out_rows.append((c, synth.draw_values(rng, c.size, "normal", dtype)))
        else:
            out_rows.append(A.row(i))
    ip = np.zeros(A.shape[0] + 1, dtype=np.int64)
    np.cumsum([len(c) for c, _ in out_rows], out=ip[1:])
    return synth.HostCSR(A.shape, ip, np.concatenate([c for c, _ in out_rows]).astype(np.int32),
                         np.concatenate([v for _, v in out_rows]))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_split_rows_clustered_columns(B, dtype):
    """Rows beyond the LDS tables whose products pile up on few columns:
    column ranges with more products than a sorted segment (dense panel),
    ranges alone with large buckets (whole-segment sort), grouped ranges,
    and a long row over every range, in one launch."""
    k, n = 20000, 60000
    Bm = _band_rows(k, n, 48, 3, 31, dtype)
    A = synth.varnnz_csr(400, k, 1, 30, 31, dtype, "normal")
    lists = {
        5: np.arange(2000, 2400),                    # 19200 products on ~1250 columns
        17: np.arange(0, 20000, 10),                 # 96000 products over every range
        40: np.concatenate([np.arange(s, s + 60) for s in (100, 5000, 9000, 15000)]),
        41: np.concatenate([np.arange(s, s + 30) for s in range(0, 20000, 600)]),
        60: np.arange(0, 20000, 100),                # ~1300 products per range: grouped
    }
    A = _rows_from(A, lists, 31, dtype)
    check(B, A, Bm, dtype, what="split rows, clustered")


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_split_rows_with_a_small_staging_area(B, dtype):
    """One heavy slot: the staging area holds about n * 2/3 products, so the
    first heavy rows to reserve it are split over many blocks and the others
    stay with the one-block kernels, in the same launch."""
    n = 60000
    A = synth.varnnz_csr(300, 5000, 1, 40, 37, dtype, "normal", stream=0)
    dense_rows = synth.uniform_csr(8, 5000, 1200, 37, dtype, "normal", stream=2)
    A = _replace_rows(A, [3, 50, 77, 120, 150, 200, 250, 299], dense_rows)
    Bm = synth.varnnz_csr(5000, n, 4, 32, 37, dtype, "normal", stream=1)
    t = B.default_tuning()
    t.heavy_slots = 1
    plan = B.Plan(tuning=t)
    got = B.spgemm(B.to_device(A, dtype=dtype), B.to_device(Bm, dtype=dtype), plan=plan).to_host()
    f = lambda M: M.with_data(M.data.astype(dtype).astype(np.float64))
    ref, S = oracle.spgemm(f(A), f(Bm), with_abs=True)
    assert_same_csr(got, ref, S, dtype, what="split and one-block heavy rows")


@pytest.mark.parametrize("n", [100, 8192, 8193])
def test_split_rows_few_columns(B, n):
    """Rows of more than 4096 products over few output columns (one or two
    8192-column ranges, a range ending past n): dense-panel and bucket
    segments at the matrix's right edge; small integers, so exact."""
    A = synth.varnnz_csr(64, 3000, 1, 20, 41, np.float64, "int", stream=0)
    dense_rows = synth.uniform_csr(3, 3000, 1500, 41, np.float64, "int", stream=2)
    A = _replace_rows(A, [0, 31, 63], dense_rows)
    Bm = synth.varnnz_csr(3000, n, 1, min(n, 12), 41, np.float64, "int", stream=1)
    check(B, A, Bm, np.float64, exact=True, what=f"split rows, n={n}")



def _planted_repeats(dtype, kind, seed, planted=48, entries=(20, 200)):
    """Rows over 2^22 columns, so chance repeats are rare, plus planted
    ones: B rows 0..planted-1 all hold column c1 and the first half of them
    also column c2, and A row i takes the first d_i of those rows
    (d_i = i mod planted) among its entries, next to `entries` random ones.
    Rows then repeat 0, a few, or many products, with columns repeated two
    to `planted` times in the middle of the row's column range."""
    k, n, m = 4000, 1 << 22, 480
    c1, c2 = n // 2 + 7, n // 3
    rng = synth.rng_for(seed, 3)
    brows = []
    for r in range(k):
        c = rng.choice(n, size=int(rng.integers(8, 25)), replace=False)
        if r < planted:
            c = np.append(c, c1)
        if r < planted // 2:
            c = np.append(c, c2)
        brows.append(np.unique(c))
    bp = np.zeros(k + 1, dtype=np.int64)
    np.cumsum([len(c) for c in brows], out=bp[1:])
    bc = np.concatenate(brows).astype(np.int32)
    Bm = synth.HostCSR((k, n), bp, bc, synth.draw_values(rng, bc.size, kind, dtype))
    arows = []
    for i in range(m):
        d = i % planted
        extra = rng.choice(np.arange(planted, k), size=int(rng.integers(*entries)),
                           replace=False)
        arows.append(np.unique(np.concatenate([np.arange(d), extra])))
    ap = np.zeros(m + 1, dtype=np.int64)
    np.cumsum([len(c) for c in arows], out=ap[1:])
    ac = np.concatenate(arows).astype(np.int32)
    A = synth.HostCSR((m, k), ap, ac, synth.draw_values(rng, ac.size, kind, dtype))
    return A, Bm


@pytest.mark.parametrize("dtype,kind", [(np.float64, "int"), (np.float32, "normal")])
def test_block_rows_with_few_repeated_columns(B, dtype, kind):
    """Block-bucket rows ranked in their buckets with a list of repeats
    (1..32 repeated products), next to rows without repeats and rows that
    sort (more than 32)."""
    A, Bm = _planted_repeats(dtype, kind, 43)
    check(B, A, Bm, dtype, exact=(kind == "int"), what="planted repeats")


@pytest.mark.parametrize("dtype,kind", [(np.float64, "int"), (np.float32, "normal")])
def test_split_rows_with_few_repeated_columns(B, dtype, kind):
    """Rows of about 4150..6200 products over 2^22 columns, split over many
    blocks: their segments (ranges grouped to at most 4096 products) repeat
    no product (in-bucket ranks), a few or many (bucket sort and runs)."""
    A, Bm = _planted_repeats(dtype, kind, 53, planted=48, entries=(260, 330))
    check(B, A, Bm, dtype, exact=(kind == "int"), what="planted repeats, split rows")


@pytest.mark.parametrize("dtype,kind", [(np.float64, "int"), (np.float32, "normal")])
def test_wave_rows_with_few_repeated_columns(B, dtype, kind):
    """Rows of about 30..420 products (the one-row-per-wave bins and their
    neighbours) with 0..21 repeated products: in-bucket ranks without
    repeats, bucket sort and runs with them."""
    A, Bm = _planted_repeats(dtype, kind, 47, planted=16, entries=(2, 10))
    check(B, A, Bm, dtype, exact=(kind == "int"), what="planted repeats, short rows")

def _replace_rows(A, rows, R):
    """A with rows `rows` replaced by the rows of R (same column count)."""
    rows = list(rows)
    out_rows = []
    for i in range(A.shape[0]):
        if i in rows:
            c, v = R.row(rows.index(i))
        else:
            c, v = A.row(i)
        out_rows.append((c, v))
    ip = np.zeros(A.shape[0] + 1, dtype=np.int64)
    np.cumsum([len(c) for c, _ in out_rows], out=ip[1:])
    return synth.HostCSR(A.shape, ip, np.concatenate([c for c, _ in out_rows]).astype(np.int32),
                         np.concatenate([v for _, v in out_rows]))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_clustered_columns_take_the_sort_fallback(B, dtype):
    """Banded B rows give long runs of adjacent output columns: rows whose
    runs exceed the in-place rank window go through the sort fallback."""
    k, n = 3000, 3000
    rows = np.repeat(np.arange(k), 48)
    cols = (rows + np.tile(np.arange(48), k)) % n
    ip = np.arange(k + 1, dtype=np.int64) * 48
    order = np.lexsort((cols, rows))
    vals = synth.draw_values(synth.rng_for(11), cols.size, "normal", dtype)
    Bm = synth.HostCSR((k, n), ip, cols[order].astype(np.int32), vals)
    A = synth.varnnz_csr(2000, k, 1, 40, 11, dtype, "normal")
    check(B, A, Bm, dtype, what="banded")


def test_unsorted_input_rows(B):
    A = synth.shuffle_rows(synth.uniform_csr(2000, 3000, 20, 13, np.float64, "int", stream=0), 1)
    Bm = synth.shuffle_rows(synth.uniform_csr(3000, 2000, 20, 13, np.float64, "int", stream=1), 2)
    check(B, A, Bm, np.float64, exact=True, what="unsorted inputs")


def test_identity_and_permutation(B):
    Bm = synth.varnnz_csr(5000, 7000, 0, 50, 17, np.float32, "normal")
    got = gpu_product(B, synth.identity_csr(5000, np.float32), Bm, np.float32)
    assert np.array_equal(got.indptr, Bm.indptr)
    assert np.array_equal(got.indices, Bm.indices)
    assert np.array_equal(got.data, Bm.data)
    P = synth.permutation_csr(5000, 3, np.float32)
    got = gpu_product(B, P, Bm, np.float32)
    ref = oracle.spgemm(P, Bm)
    assert np.array_equal(got.indices, ref.indices)
    assert np.array_equal(got.data.astype(np.float64), ref.data)


def test_degenerate_shapes(B):
    # no rows
    A = synth.uniform_csr(0, 10, 0, 1, np.float32)
    Bm = synth.uniform_csr(10, 10, 3, 1, np.float32)
    got = gpu_product(B, A, Bm, np.float32)
    assert got.indptr.tolist() == [0] and got.nnz == 0
    # all rows empty
    A = synth.uniform_csr(100, 10, 0, 1, np.float32)
    got = gpu_product(B, A, Bm, np.float32)
    assert got.indptr.tolist() == [0] * 101
    # a single output column: every product lands on column 0
    A = synth.uniform_csr(1000, 500, 50, 2, np.float64, "int")
    Bm = synth.HostCSR((500, 1), np.arange(501, dtype=np.int64), np.zeros(500, np.int32),
                       synth.draw_values(synth.rng_for(2, 3), 500, "int", np.float64))
    check(B, A, Bm, np.float64, exact=True, what="n=1")
    # one row, one column inner dimension
    A = synth.HostCSR((1, 1), np.array([0, 1]), np.array([0], np.int32), np.array([2.0]))
    Bm = synth.HostCSR((1, 3), np.array([0, 2]), np.array([0, 2], np.int32), np.array([1.5, -1.0]))
    check(B, A, Bm, np.float64, exact=True, what="1x1")


def test_repeat_gives_identical_pattern(B):
    A = synth.varnnz_csr(4000, 4000, 0, 60, 19, np.float32, "normal", stream=0)
    Bm = synth.varnnz_csr(4000, 4000, 0, 60, 19, np.float32, "normal", stream=1)
    g1 = gpu_product(B, A, Bm, np.float32)
    g2 = gpu_product(B, A, Bm, np.float32)
    assert np.array_equal(g1.indptr, g2.indptr)
    assert np.array_equal(g1.indices, g2.indices)


def test_validation_flags_bad_columns(B):
    import torch
    A = synth.uniform_csr(100, 50, 5, 23, np.float32)
    Bm = synth.uniform_csr(50, 60, 5, 23, np.float32, stream=1)
    dA = B.to_device(A)
    dB = B.to_device(Bm)
    dB.col_idx[7] = 60  # out of range
    plan = B.Plan(validate=True)
    with pytest.raises(B.SpgError) as e:
        plan.symbolic([dA], [dB])
    assert e.value.code == B.SPG_ERR_INVALID
    dB.col_idx[7] = 3
    dB.row_ptr[10] = dB.row_ptr[9] - 1  # decreasing row pointer
    with pytest.raises(B.SpgError) as e:
        plan.symbolic([dA], [dB])
    assert e.value.code == B.SPG_ERR_INVALID
    torch.cuda.synchronize()


def test_nnz_overflow_is_reported(B):
    """A (4096 x 1, all ones) times one dense row of 2^20 columns has 2^32
    output entries: the symbolic pass must report the int32 overflow."""
    import torch
    m, n = 4096, 1 << 20
    A = synth.HostCSR((m, 1), np.arange(m + 1, dtype=np.int64), np.zeros(m, np.int32),
                      np.ones(m, np.float32))
    Bm = synth.HostCSR((1, n), np.array([0, n], dtype=np.int64), np.arange(n, dtype=np.int32),
                       np.ones(n, np.float32))
    plan = B.Plan()
    with pytest.raises(B.SpgError) as e:
        plan.symbolic([B.to_device(A)], [B.to_device(Bm)])
    assert e.value.code == B.SPG_ERR_OVERFLOW
    torch.cuda.synchronize()


def test_capacity_mode_reports_too_small_output(B):
    import torch
    A = synth.uniform_csr(500, 500, 8, 29, np.float32)
    dA = B.to_device(A)
    plan = B.Plan()
    rp, _ = plan.symbolic([dA], [dA], capacity=100)
    col = torch.zeros(100, dtype=torch.int32, device="cuda")
    vals = torch.zeros(100, dtype=torch.float32, device="cuda")
    plan.numeric([dA], [dA], rp, 100, col=col, vals=vals)
    assert plan.status() == B.SPG_ERR_CAPACITY
    assert int(col.abs().sum().item()) == 0  # nothing written


@pytest.mark.slow
def test_uniform_2p20_fp32_full_size(B):
    """One GPU's block share: A, B independent 2^20 x 2^20, 16 uniform columns
    per row, FP32 in (0,1] (the benchmark's plain workload, same seed):
    row_ptr and col_idx bit-exact on every row, every value within
    1e-5 * sum |a||b| of the FP64 oracle's."""
    n = 1 << 20
    A = synth.uniform_csr(n, n, 16, SEED + 1, np.float32, "u01", stream=0)
    Bm = synth.uniform_csr(n, n, 16, SEED + 1, np.float32, "u01", stream=1)
    got = gpu_product(B, A, Bm, np.float32)
    ref, S = oracle.spgemm(A.astype(np.float64), Bm.astype(np.float64), with_abs=True)
    assert_same_csr(got, ref, S, np.float32, what="2^20 uniform, every row")


@pytest.mark.parametrize("d,dtype,kind", [(16, np.float64, "int"), (16, np.float32, "normal"),
                                          (24, np.float32, "normal"), (48, np.float64, "int"),
                                          (48, np.float32, "u01")])
def test_banded_products(B, d, dtype, kind):
    """Columns clustered on three diagonal bands (a structured matrix, as
    the ones the paper permutes before multiplying): the products of a row
    fall into a few buckets of the order-preserving bucketing, which the
    bucket kernels then sort as a whole row.  Rows of 256, ~576 and ~2300
    products: the one-wave kernel and two block-group sizes."""
    n = 1 << 14
    A = synth.banded_csr(n, d, [0, n // 8, -n // 8], 64, 51 + d, dtype, kind)
    check(B, A, A, dtype, exact=(kind == "int"), what=f"banded d={d}")

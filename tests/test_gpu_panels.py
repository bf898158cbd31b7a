"""GPU parity of the column-panel product y = A x (x staged in LDS by
panels of 64 KB of doubles or 112 KB of floats, rows cut into strided pieces of
at most 32 entries, each piece's entries in a panel summed serially by one
lane, four column groups per row range added in order): bit-exact against the
oracle on integer data, within the dot-product bound on float data, bitwise
repeatable, with ragged panels, fewer panels than groups, empty rows and
panels, long segments, large blocks, and the fallbacks (unsorted columns, a
misaligned x, ranges with too many pieces, blocks that would be mostly
padding) that keep the row-block kernel."""
import numpy as np
import pytest
import torch

import oracle
from paper_1211_1581_amd import inputs as I
from gpu_util import U32, check_f64, dense_abs_product, gamma, spcg, to_dev

pytestmark = pytest.mark.gpu


def with_panels(A, dtype=torch.float64):
    S = spcg()
    old = S.column_panels("on")
    try:
        M = S.CsrMatrix.from_host(A, dtype=dtype)
    finally:
        S.column_panels(old)
    return M


def product(M, x, dtype=torch.float64, mode="on"):
    S = spcg()
    old = S.column_panels(mode)
    try:
        y = S.spmv_csr(M, to_dev(x, dtype))
        torch.cuda.synchronize()
    finally:
        S.column_panels(old)
    return y.cpu().numpy()


def width(dtype):
    return 8192 if dtype == torch.float64 else 28672


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nc", [70001, 28672, 5000])
def test_panels_integer_bit_exact(seed, dtype, nc):
    # sorted columns over n_cols that is ragged against the panel width (and
    # odd: the last 16-byte unit of x is partial), a multiple of it, or below
    # it (one panel); empty rows, rows of one entry, long rows
    A, x = I.random_csr_small(6000, nc, seed, max_len=60, integer=True,
                              long_rows=[(7, 3000), (5999, 2000)])
    M = with_panels(A, dtype)
    info = M.panel_info()
    assert info is not None and info[1] == -(-nc // width(dtype))
    # blocks of whole rounds of 1024 lanes, padding within the build limit
    assert A.nnz <= info[2] <= 2 * A.nnz + (1 << 24) and info[2] % 1024 == 0
    y = product(M, x, dtype)
    assert np.array_equal(y.astype(np.float64), oracle.spmv(A, x))
    # the row-block kernel on the same handle agrees exactly on integer data
    assert np.array_equal(product(M, x, dtype, "off"), y)


def test_panels_empty_panels_and_rows():
    # columns only in panels 0 and 3 of 5, and a run of empty rows
    rng = np.random.default_rng(4)
    W = width(torch.float64)
    n, nc = 3000, 4 * W + 123
    lens = rng.integers(0, 30, n)
    lens[1000:1500] = 0
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    pool = np.concatenate([np.arange(0, W), np.arange(3 * W, 4 * W)])
    col = np.concatenate([np.sort(rng.choice(pool, l, replace=False)) for l in lens]).astype(np.int32)
    A = I.CSR(n, nc, rp.astype(np.int32), col, rng.integers(-4, 5, rp[-1]).astype(np.float64))
    x = rng.integers(-4, 5, nc).astype(np.float64)
    M = with_panels(A)
    assert M.panel_info()[1] == 5
    assert np.array_equal(product(M, x), oracle.spmv(A, x))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_panels_lognormal_float_and_repeatable(dtype):
    A, x = I.lognormal_irregular(n=50000, seed=9)
    M = with_panels(A, dtype)
    assert M.panel_info() is not None
    ys = [product(M, x, dtype) for _ in range(3)]
    assert all(np.array_equal(ys[0], y) for y in ys[1:])
    if dtype == torch.float64:
        check_f64(ys[0], oracle.spmv(A, x), A, x, "panels")
    else:
        v32, x32 = A.vals.astype(np.float32), x.astype(np.float32)
        ref = oracle.spmv_f32in(A, v32, x32)
        absax = dense_abs_product(I.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col,
                                        v32.astype(np.float64)), x32)
        lens = np.diff(A.row_ptr).astype(np.float64)
        bound = gamma(lens + 1, U32) * absax * 1.0001 + 1e-30
        assert np.all(np.abs(ys[0].astype(np.float64) - ref) <= bound)


def test_panels_full_size_lognormal():
    A, x = I.lognormal_irregular()
    M = with_panels(A)
    y = product(M, x)
    check_f64(y, oracle.spmv(A, x), A, x, "lognormal panels")
    M32 = with_panels(A, torch.float32)
    y32 = product(M32, x, torch.float32)
    ref64 = oracle.spmv(A, x)
    assert np.linalg.norm(y32 - ref64) / np.linalg.norm(ref64) < 1e-5


def test_panels_fallbacks():
    S = spcg()
    # unsorted columns: no panels; the product still runs (row blocks)
    A, x = I.random_csr_small(3000, 30000, 2, max_len=40, integer=True, unsorted=True)
    M = with_panels(A)
    assert M.panel_info() is None
    assert np.array_equal(product(M, x), oracle.spmv(A, x))
    # a misaligned x (8 bytes past a 16-byte boundary): row blocks, same values
    B, xb = I.random_csr_small(3000, 30000, 3, max_len=40, integer=True)
    MB = with_panels(B)
    assert MB.panel_info() is not None
    buf = to_dev(np.concatenate([[0.0], xb]))
    old = S.column_panels("on")
    try:
        y = S.spmv_csr(MB, buf[1:])
        torch.cuda.synchronize()
    finally:
        S.column_panels(old)
    assert np.array_equal(y.cpu().numpy(), oracle.spmv(B, xb))


def test_panels_not_built_for_crowded_ranges():
    # 3 M rows of one entry: every range holds far more than 10240 pieces, so
    # the panels are not built and the product keeps the row-block kernel
    rng = np.random.default_rng(11)
    n = 3 << 20
    rp = np.arange(n + 1, dtype=np.int32)
    col = rng.integers(0, n, n).astype(np.int32)
    A = I.CSR(n, n, rp, col, rng.integers(-3, 4, n).astype(np.float64))
    x = rng.integers(-3, 4, n).astype(np.float64)
    M = with_panels(A)
    assert M.panel_info() is None
    assert np.array_equal(product(M, x), x[col] * A.vals)


def test_panels_long_segments_banded():
    # rows of 41 consecutive columns: two pieces of 21 and 20 entries, each in
    # one or two panels, so segments are long and the lanes' height is set by
    # them (padding)
    A = I.banded_spd(20000, 41)
    x = np.random.default_rng(5).integers(-4, 5, A.n_cols).astype(np.float64)
    M = with_panels(A)
    info = M.panel_info()
    assert info is not None and info[2] > A.nnz  # some padding
    assert np.array_equal(product(M, x), oracle.spmv(A, x))


def test_panels_not_built_for_narrow_x():
    # x narrower than one 16-byte unit of FP32: no panels
    A, x = I.random_csr_small(50, 3, 1, max_len=3, integer=True)
    M = with_panels(A, torch.float32)
    assert M.panel_info() is None
    assert np.array_equal(product(M, x, torch.float32).astype(np.float64), oracle.spmv(A, x))


def test_panels_products_on_two_streams():
    # products of one panel handle on two streams share its partial vectors:
    # the second waits for the first, so both results are right
    S = spcg()
    A, x1 = I.random_csr_small(20000, 60000, 5, max_len=80, integer=True)
    x2 = -x1[::-1].copy()
    M = with_panels(A)
    assert M.panel_info() is not None
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    xd1, xd2 = to_dev(x1), to_dev(x2)
    y1 = torch.empty(A.n_rows, dtype=torch.float64, device="cuda")
    y2 = torch.empty_like(y1)
    torch.cuda.synchronize()
    old = S.column_panels("on")
    try:
        for _ in range(5):
            with torch.cuda.stream(s1):
                S.spmv_csr(M, xd1, y1)
            with torch.cuda.stream(s2):
                S.spmv_csr(M, xd2, y2)
        torch.cuda.synchronize()
    finally:
        S.column_panels(old)
    assert np.array_equal(y1.cpu().numpy(), oracle.spmv(A, x1))
    assert np.array_equal(y2.cpu().numpy(), oracle.spmv(A, x2))


def test_panels_packing_retry():
    # 1536 rows of two entries per range, all in panel 0: each (range, panel)
    # block holds 3072 entries, so the lanes start at height 3, where a lane
    # fits one two-entry segment and 512 segments are left over; the packing
    # retries at height 4 and every block takes 4 rounds of 1024 lanes
    R = torch.cuda.get_device_properties(0).multi_processor_count // 4
    rng = np.random.default_rng(14)
    n, nc = 1536 * R, width(torch.float64)
    rp = (np.arange(n + 1, dtype=np.int64) * 2).astype(np.int32)
    col = np.sort(rng.integers(0, nc // 2, (n, 2)) * 2 + np.array([0, 1]), axis=1).astype(np.int32).ravel()
    A = I.CSR(n, nc, rp, col, rng.integers(-3, 4, 2 * n).astype(np.float64))
    x = rng.integers(-3, 4, nc).astype(np.float64)
    M = with_panels(A)
    info = M.panel_info()
    assert info is not None and info[0] == R and info[1] == 1
    assert info[2] == R * 4 * 1024
    assert np.array_equal(product(M, x), oracle.spmv(A, x))


def test_panels_large_blocks():
    # 1000 dense rows over 6000 columns (one FP64 panel): each range's block
    # holds about 94 000 entries (92 rounds of 1024 lanes, every segment 32
    # entries long)
    rng = np.random.default_rng(12)
    n, nc = 1000, 6000
    rp = (np.arange(n + 1, dtype=np.int64) * nc).astype(np.int32)
    col = np.tile(np.arange(nc, dtype=np.int32), n)
    A = I.CSR(n, nc, rp, col, rng.integers(-3, 4, n * nc).astype(np.float64))
    x = rng.integers(-3, 4, nc).astype(np.float64)
    M = with_panels(A)
    info = M.panel_info()
    assert info is not None and info[1] == 1 and info[2] >= A.nnz
    assert np.array_equal(product(M, x), oracle.spmv(A, x))


def test_panels_not_built_for_sparse_blocks():
    # 100 000 rows of two entries over 8 M columns (977 FP64 panels): a block
    # holds a few entries but takes a round of 1024 lanes, so the padded copy
    # would exceed twice the entries plus 2^24 and the panels are not built
    rng = np.random.default_rng(13)
    n, nc = 100_000, 8_000_000
    rp = (np.arange(n + 1, dtype=np.int64) * 2).astype(np.int32)
    col = np.sort(rng.integers(0, nc // 2, (n, 2)) * 2 + np.array([0, 1]), axis=1).astype(np.int32).ravel()
    A = I.CSR(n, nc, rp, col, rng.integers(-3, 4, 2 * n).astype(np.float64))
    x = rng.integers(-3, 4, nc).astype(np.float64)
    M = with_panels(A)
    assert M.panel_info() is None
    assert np.array_equal(product(M, x), oracle.spmv(A, x))


def test_panels_auto_policy():
    # the default policy builds panels only for long rows spread over a wide
    # x: the lognormal matrix (100 000 rows, 79 entries per row on average);
    # not for a stencil (short rows), a band (local columns), a matrix below
    # 65 536 rows, nor while row binning is on; products stay correct
    S = spcg()
    assert S.column_panels() == "auto"
    A, x = I.lognormal_irregular(n=100_000, seed=15)
    M = S.CsrMatrix.from_host(A)
    assert M.panel_info() is not None
    y = S.spmv_csr(M, to_dev(x))
    torch.cuda.synchronize()
    check_f64(y.cpu().numpy(), oracle.spmv(A, x), A, x, "auto panels")
    for B in (I.poisson3d(48), I.banded_spd(100_000, 41), I.lognormal_irregular(n=50_000, seed=16)[0]):
        assert S.CsrMatrix.from_host(B).panel_info() is None
    old = S.row_binning("on")
    try:
        assert S.CsrMatrix.from_host(A).panel_info() is None
    finally:
        S.row_binning(old)

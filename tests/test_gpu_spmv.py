"""GPU parity of y = A x (Sec. 3.2) against the FP64 oracle: bit-exact on
integer-valued inputs, 1e-12 normwise plus the componentwise dot-product bound
in FP64, the FP32 bound for FP32 values; full-size workloads; determinism;
edge cases (empty, ragged, long rows, unsorted, duplicates, invalid CSR)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1211_1581_amd import inputs as I
from gpu_util import U32, check_f64, dense_abs_product, gamma, lower_upper, spcg, to_dev

pytestmark = pytest.mark.gpu


def run(A, x, dtype=torch.float64, binning=None):
    """y = A x on the device with the column panels off (these tests are of
    the row-block, short-row and binned kernels; test_gpu_panels.py covers the
    panels).  binning: the row-binning policy in force while the handle is made
    and the product runs ("off": row-block kernel, "on": row-length bins),
    restored afterwards; None keeps the default (off)."""
    S = spcg()
    old = S.row_binning(binning) if binning is not None else None
    old_p = S.column_panels("off")
    try:
        M = S.CsrMatrix.from_host(A, dtype=dtype)
        y = S.spmv_csr(M, to_dev(x, dtype))
        torch.cuda.synchronize()
    finally:
        S.column_panels(old_p)
        if old is not None:
            S.row_binning(old)
    return y.cpu().numpy(), M


BOTH = pytest.mark.parametrize("binning", ["off", "on"])


@BOTH
@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_integer_valued_bit_exact(seed, dtype, binning):
    # several row blocks, a ragged tail, empty rows, long rows beyond the LDS
    # slab; with bins, rows in every bin including the long-row one
    A, x = I.random_csr_small(7001, 6000, seed, max_len=40, integer=True,
                              long_rows=[(5, 5000), (3000, 1900), (7000, 2500)],
                              unsorted=bool(seed % 2), duplicates=(seed == 2))
    y, M = run(A, x, dtype, binning)
    assert M.info()["n_long"] >= 2
    assert M.has_bins() == (binning == "on")
    assert np.array_equal(y.astype(np.float64), oracle.spmv(A, x))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_bins_every_length_class(dtype):
    # rows of every length from 0 to 600 (both sides of each bin edge 4, 8,
    # ..., 256), a 5000-entry row, empty rows last: bin counts equal the
    # histogram of the row lengths, and the binned product is bit-exact
    S = spcg()
    rng = np.random.default_rng(17)
    lens = np.concatenate([np.arange(0, 601), [5000], rng.integers(0, 40, 3000), [0, 0, 0]])
    rng.shuffle(lens[:-3])
    rp = np.zeros(len(lens) + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    nc = 6000
    col = np.concatenate([np.sort(rng.choice(nc, l, replace=False)) for l in lens]).astype(np.int32)
    A = I.CSR(len(lens), nc, rp.astype(np.int32), col,
              rng.integers(-4, 5, rp[-1]).astype(np.float64))
    x = rng.integers(-4, 5, nc).astype(np.float64)
    y, M = run(A, x, dtype, "on")
    edges = [4 << b for b in range(7)]
    want = np.bincount(np.searchsorted(edges, lens, side="left"), minlength=8)
    assert np.array_equal(M.bin_counts(), want)
    assert np.array_equal(y.astype(np.float64), oracle.spmv(A, x))


@BOTH
def test_edge_shapes(binning):
    S = spcg()
    old = S.row_binning(binning)
    try:
        _edge_shapes(S)
    finally:
        S.row_binning(old)


def _edge_shapes(S):
    # n = 1
    A = I.CSR(1, 1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([2.5]))
    assert run(A, np.array([4.0]))[0][0] == 10.0
    # every row empty (nnz = 0), in both precisions (one wide block per 2048 rows)
    E = I.CSR(300, 7, np.zeros(301, np.int32), np.zeros(0, np.int32), np.zeros(0))
    for dt in (torch.float64, torch.float32):
        y, M = run(E, np.ones(7), dt)
        assert np.array_equal(y, np.zeros(300))
        assert M.info()["n_wide_blocks"] == 1
    # empty matrix: no row blocks in either partition
    for dt in (torch.float64, torch.float32):
        Z = S.CsrMatrix(torch.zeros(1, dtype=torch.int32, device="cuda"),
                        torch.zeros(0, dtype=torch.int32, device="cuda"),
                        torch.zeros(0, dtype=dt, device="cuda"))
        y = S.spmv_csr(Z, torch.zeros(0, dtype=dt, device="cuda"))
        torch.cuda.synchronize()
        assert y.numel() == 0
        assert Z.info()["n_blocks"] == 0 and Z.info()["n_wide_blocks"] == 0
    # a single very long row and many tiny ones
    A, x = I.random_csr_small(50, 20000, 3, max_len=3, long_rows=[(49, 20000), (0, 12000)])
    y, M = run(A, x)
    check_f64(y, oracle.spmv(A, x), A, x, "long rows")


@pytest.mark.parametrize("n", [1, 5, 255, 257, 1000, 70001])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_short_rows_bit_exact(n, dtype):
    # every row at most 4 entries: the short-row kernel (empty rows, ragged
    # tail of a workgroup step, unsorted columns)
    A, x = I.random_csr_small(n, max(n, 7), n + 11, max_len=4, integer=True, unsorted=True)
    if A.nnz == 0:
        A, x = I.random_csr_small(n, max(n, 7), n + 12, max_len=4, integer=True, empty_frac=0.0)
    y, M = run(A, x, dtype)
    assert M.info()["max_row_len"] <= 4
    assert np.array_equal(y.astype(np.float64), oracle.spmv(A, x))


def test_short_rows_factor_pattern():
    # lower and upper triangles of the 7-point stencil (at most 4 per row),
    # and the 5-entry boundary case that stays on the row-block kernel
    A = I.poisson3d(24)
    L, U = lower_upper(A, np.random.default_rng(0).uniform(-1, 1, (A.nnz + A.n_rows) // 2))
    x = np.random.default_rng(1).uniform(-1, 1, A.n_rows)
    for F in (L, U):
        y, M = run(F, x)
        assert M.info()["max_row_len"] == 4
        check_f64(y, oracle.spmv(F, x), F, x, "factor pattern")
    B, xb = I.random_csr_small(3000, 3000, 5, max_len=5, empty_frac=0.0)
    y, M = run(B, xb)
    assert M.info()["max_row_len"] == 5
    check_f64(y, oracle.spmv(B, xb), B, xb, "len 5")


@pytest.mark.parametrize("n,maxlen", [(257, 5), (4099, 80), (20011, 300)])
def test_random_float(n, maxlen):
    A, x = I.random_csr_small(n, n, n, max_len=maxlen)
    y, _ = run(A, x)
    check_f64(y, oracle.spmv(A, x), A, x, f"n={n}")


def test_poisson_and_fv():
    for A in [I.poisson2d(64), I.poisson3d(40), I.fv_diffusion(20, 3)[0]]:
        x = I.uniform_vector(A.n_rows, 11)
        y, _ = run(A, x)
        check_f64(y, oracle.spmv(A, x), A, x)


def f32_check(A, x, y32):
    v32 = A.vals.astype(np.float32)
    x32 = x.astype(np.float32)
    ref = oracle.spmv_f32in(A, v32, x32)
    absax = dense_abs_product(I.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col,
                                    v32.astype(np.float64)), x32)
    lens = np.diff(A.row_ptr).astype(np.float64)
    bound = gamma(lens + 1, U32) * absax * 1.0001 + 1e-30
    err = np.abs(y32.astype(np.float64) - ref)
    assert np.all(err <= bound), float(np.max(err / bound))
    return ref


def test_f32_lognormal_small():
    A, x = I.lognormal_irregular(n=30000, seed=5)
    y, _ = run(A, x, torch.float32)
    f32_check(A, x, y)


def test_full_size_poisson128():
    A = I.poisson3d(128)
    x = I.uniform_vector(A.n_rows, 1)
    y, M = run(A, x)
    check_f64(y, oracle.spmv(A, x), A, x, "128^3")
    assert M.info()["n_blocks"] == (A.nnz + A.n_rows + 1535) // 1536  # 1536 merge items per row block


def test_poisson256_several_blocks_per_workgroup():
    # 87K row blocks: more than one launch's workgroups, so each workgroup walks
    # a range of blocks (the LDS slab is reused between them)
    A = I.poisson3d(256)
    x = I.uniform_vector(A.n_rows, 3)
    y, M = run(A, x)
    assert M.info()["n_blocks"] > 32768
    check_f64(y, oracle.spmv(A, x), A, x, "256^3")


def test_many_empty_rows_several_blocks_per_workgroup():
    # 48M rows, three in four empty, every 97th row with 6 entries (row-block
    # kernel, not the short-row one), columns in a small range
    n, nc = 48_000_000, 4096
    rng = np.random.default_rng(8)
    lens = np.zeros(n, np.int64)
    lens[::4] = 1
    lens[::97] = 6
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    nnz = int(rp[-1])
    col = rng.integers(0, nc, nnz).astype(np.int32)
    vals = rng.integers(-4, 5, nnz).astype(np.float64)
    A = I.CSR(n, nc, rp.astype(np.int32), col, vals)
    x = rng.integers(-3, 4, nc).astype(np.float64)
    y, M = run(A, x)
    assert M.info()["n_blocks"] > 32768 and M.info()["max_row_len"] == 6
    assert np.array_equal(y, oracle.spmv(A, x))


@pytest.fixture(scope="module")
def lognormal_200k():
    return I.lognormal_irregular()


@BOTH
def test_full_size_lognormal_f64(lognormal_200k, binning):
    A, x = lognormal_200k
    assert A.nnz == 15_788_355
    y, M = run(A, x, binning=binning)
    check_f64(y, oracle.spmv(A, x), A, x, "lognormal f64")
    assert M.info()["max_row_len"] == 4096


@BOTH
def test_full_size_lognormal_f32(lognormal_200k, binning):
    A, x = lognormal_200k
    y, _ = run(A, x, torch.float32, binning)
    ref = f32_check(A, x, y)
    # report-only: error against the FP64 product of the unrounded inputs
    ref64 = oracle.spmv(A, x)
    assert np.linalg.norm(y - ref64) / np.linalg.norm(ref64) < 1e-5
    assert np.linalg.norm(ref - ref64) / np.linalg.norm(ref64) < 1e-5


def test_full_size_fv160_both():
    A, _, xs = I.fv_diffusion(160, 3)
    y, _ = run(A, xs)
    check_f64(y, oracle.spmv(A, xs), A, xs, "fv160")
    y32, _ = run(A, xs, torch.float32)
    f32_check(A, xs, y32)


def test_deterministic_repeats():
    S = spcg()
    A, x = I.lognormal_irregular(n=50000, seed=9)
    old = S.row_binning("on")
    try:
        M = S.CsrMatrix.from_host(A)
        assert M.has_bins()
        xt = to_dev(x)
        ys = [S.spmv_csr(M, xt).cpu().numpy() for _ in range(3)]
    finally:
        S.row_binning(old)
    assert all(np.array_equal(ys[0], y) for y in ys[1:])
    # the row-block kernel on the same handle: its own fixed order, also
    # repeatable, and within the dot-product bound of the oracle
    zs = [S.spmv_csr(M, xt).cpu().numpy() for _ in range(2)]
    assert np.array_equal(zs[0], zs[1])
    check_f64(zs[0], oracle.spmv(A, x), A, x, "row blocks")
    check_f64(ys[0], oracle.spmv(A, x), A, x, "bins")


def test_invalid_csr_rejected_on_device():
    S = spcg()
    A, _ = I.random_csr_small(100, 50, 1)
    bad = A.col.copy()
    bad[7] = 50
    with pytest.raises(S.SpcgError) as e:
        S.CsrMatrix(to_dev(A.row_ptr), to_dev(bad), to_dev(A.vals), n_cols=50)
    assert e.value.status == S.INVALID_CSR
    rp = A.row_ptr.copy()
    rp[10], rp[11] = rp[11], rp[10] - 1
    with pytest.raises(S.SpcgError):
        S.CsrMatrix(to_dev(rp), to_dev(A.col), to_dev(A.vals), n_cols=50)


def test_dot_deterministic_and_bounded():
    S = spcg()
    rng = np.random.default_rng(4)
    for n in [0, 1, 4095, 4096, 1_000_003]:
        a, b = rng.standard_normal(n), rng.standard_normal(n)
        ta, tb = to_dev(a), to_dev(b)
        d1 = S.dot(ta, tb).item()
        d2 = S.dot(ta, tb).item()
        assert d1 == d2
        ref = oracle.dot(a, b)
        bound = 2 * gamma(max(n, 1), 2.0 ** -53) * np.sum(np.abs(a * b))
        assert abs(d1 - ref) <= bound + 1e-300


@pytest.mark.parametrize("L", [1535, 1536, 1537, 1775, 1776, 1777, 1792, 1793,
                               2047, 2048, 2049, 2287, 2288, 2289])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_rows_at_the_lds_slab_size(L, dtype):
    # each row of L entries opens its own row block: lengths around the
    # merge-coordinate span (1536) and the LDS slab (1776), and around the
    # wide partition's span (2048) and slab (2288) that the FP32 product
    # uses, below and above, then short rows after them
    lens = np.array([L, L, 3, L - 1, 0, 5] * 3, np.int64)
    rp = np.zeros(len(lens) + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    rng = np.random.default_rng(L)
    nc = 4000
    col = np.concatenate([np.sort(rng.choice(nc, l, replace=False)) for l in lens]).astype(np.int32)
    vals = rng.integers(-5, 6, rp[-1]).astype(np.float64)
    A = I.CSR(len(lens), nc, rp.astype(np.int32), col, vals)
    x = rng.integers(-3, 4, nc).astype(np.float64)
    for binning in ("off", "on"):
        y, M = run(A, x, dtype, binning)
        assert np.array_equal(y.astype(np.float64), oracle.spmv(A, x))


def test_wide_partition_f32():
    # an FP32 handle's own product runs over the handle's wide partition,
    # blocks of 2048 merge items (the FP64 products and the kernels with FP64
    # sums keep 1536; the mixed form's FP32 inner product uses the wide one
    # too, tested with the solver).  For rows of fewer than 8
    # entries each row's sum is taken in entry order whatever the partition,
    # so the product equals the one over the 1536-item blocks bit for bit
    # (taken here with run-compressed columns, which follow that partition);
    # both lie within the FP32 bound of the oracle's sum of the same inputs
    S = spcg()
    A = I.poisson3d(64)
    x = I.uniform_vector(A.n_rows, 4)
    y, M = run(A, x, torch.float32)
    info = M.info()
    assert info["n_blocks"] == (A.nnz + A.n_rows + 1535) // 1536
    assert info["n_wide_blocks"] == (A.nnz + A.n_rows + 2047) // 2048
    _, M64 = run(A, x)
    assert M64.info()["n_wide_blocks"] == info["n_wide_blocks"]
    old = S.run_columns("on")
    try:
        Mr = S.CsrMatrix.from_host(A, dtype=torch.float32)
        yr = S.spmv_csr(Mr, to_dev(x, torch.float32))
        torch.cuda.synchronize()
    finally:
        S.run_columns(old)
    assert Mr.run_info() is not None
    assert np.array_equal(y, yr.cpu().numpy())
    f32_check(A, x, y)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_arrays_at_odd_element_offsets(dtype):
    # the row-block product reads a lane's consecutive entries as one 16-byte
    # vector of values and one of columns: CSR arrays that start one element
    # past an aligned address (views into larger buffers) make those loads
    # misaligned; the products equal the aligned handle's bit for bit
    S = spcg()

    def shifted(a, dt):
        t = torch.as_tensor(a).to(dt)
        buf = torch.zeros(t.numel() + 1, dtype=dt, device="cuda")
        buf[1:] = t.to("cuda")
        return buf[1:]

    mats = [I.poisson3d(24), I.random_csr_small(20000, 30000, 5, max_len=40, integer=True)[0]]
    for A in mats:
        x = np.random.default_rng(A.nnz).integers(-3, 4, A.n_cols).astype(np.float64)
        M = S.CsrMatrix(shifted(A.row_ptr, torch.int32), shifted(A.col, torch.int32),
                        shifted(A.vals, dtype), n_cols=A.n_cols)
        assert M.col.data_ptr() % 16 != 0 and M.vals.data_ptr() % 16 != 0
        aligned = S.CsrMatrix.from_host(A, dtype=dtype)
        xd = to_dev(x, dtype)
        y1 = S.spmv_csr(M, xd)
        y0 = S.spmv_csr(aligned, xd)
        torch.cuda.synchronize()
        assert np.array_equal(y1.cpu().numpy(), y0.cpu().numpy())
        assert np.array_equal(y1.cpu().numpy().astype(np.float64), oracle.spmv(A, x))


def test_maximum_size():
    # nnz = 2^31 - 2^16 - 8 (the handle's limit is 2^31 - 2^16 - 1): 268M rows
    # of 8 entries and a last row of 6000 (reduced outside the LDS slab, at the
    # top of the index range).  The inputs are made on the device from closed
    # formulas; sampled rows are checked against the oracle, every row through
    # two weighted sums taken by torch.  Integer values keep all of it exact.
    S = spcg()
    lim = 2**31 - 2**16 - 1
    last = 6000
    nr = (lim - last) // 8 + 1
    nnz = 8 * (nr - 1) + last
    nc = 1 << 20
    dev = "cuda"
    rp = torch.empty(nr + 1, dtype=torch.int32, device=dev)
    rp[:nr] = (torch.arange(nr, device=dev, dtype=torch.int64) * 8).to(torch.int32)
    rp[nr] = nnz
    col = torch.empty(nnz, dtype=torch.int32, device=dev)
    vals = torch.empty(nnz, dtype=torch.float64, device=dev)
    ch = 1 << 28
    for a in range(0, nnz, ch):
        k = torch.arange(a, min(a + ch, nnz), device=dev, dtype=torch.int64)
        col[a:a + k.numel()] = ((k * 2654435761) % nc).to(torch.int32)
        vals[a:a + k.numel()] = (((k * 40503) >> 7) % 7 - 3).to(torch.float64)
        del k
    x = (torch.arange(nc, device=dev) % 5 - 2).to(torch.float64)

    def host_rows(rows):
        rows = np.asarray(rows, np.int64)
        starts = 8 * rows
        lens = np.where(rows == nr - 1, last, 8)
        sub_rp = np.zeros(len(rows) + 1, np.int64)
        np.cumsum(lens, out=sub_rp[1:])
        k = np.concatenate([np.arange(s, s + l) for s, l in zip(starts, lens)])
        c = ((k * 2654435761) % nc).astype(np.int32)
        v = (((k * 40503) >> 7) % 7 - 3).astype(np.float64)
        return I.CSR(len(rows), nc, sub_rp.astype(np.int32), c, v)

    rng = np.random.default_rng(31)
    rows = np.unique(np.concatenate([np.arange(10), nr - 1 - np.arange(10),
                                     rng.integers(0, nr, 2000)]))
    xh = (np.arange(nc) % 5 - 2).astype(np.float64)
    ref = oracle.spmv(host_rows(rows), xh)

    def weighted(w_of_row):
        # sum over k of w(row(k)) vals[k] x[col[k]], chunked, exact in FP64
        tot = 0.0
        for a in range(0, nnz, ch):
            k = torch.arange(a, min(a + ch, nnz), device=dev, dtype=torch.int64)
            r = torch.clamp(k // 8, max=nr - 1)
            t = w_of_row(r) * vals[a:a + k.numel()] * x[col[a:a + k.numel()].long()]
            tot += float(t.sum())
            del k, r, t
        return tot

    w1 = lambda r: (r % 7 + 1).to(torch.float64)
    w2 = lambda r: ((r * 31) % 11 + 1).to(torch.float64)
    s1, s2 = weighted(w1), weighted(w2)
    ridx = torch.arange(nr, device=dev, dtype=torch.int64)
    for dtype in (torch.float64, torch.float32):
        M = S.CsrMatrix(rp, col, vals.to(dtype), n_cols=nc)
        info = M.info()
        assert info["max_row_len"] == last and info["n_long"] >= 1
        y = S.spmv_csr(M, x.to(dtype))
        torch.cuda.synchronize()
        assert np.array_equal(y[torch.as_tensor(rows, device=dev)].double().cpu().numpy(), ref)
        yd = y.double()
        assert float((w1(ridx) * yd).sum()) == s1 and float((w2(ridx) * yd).sum()) == s2
        M.close()
        del y, yd, M

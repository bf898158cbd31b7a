"""Pins of the oracle's CSR SpMV (Sec. 3.2) against mathematics it does not use:
dense products, exact integer arithmetic, scipy.sparse, and the closed-form
eigenpairs and row sums of the Poisson operators."""
import math

import numpy as np
import pytest

import oracle
from paper_1211_1581_amd import inputs as I


def dense(A):
    M = np.zeros((A.n_rows, A.n_cols))
    for i in range(A.n_rows):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            M[i, A.col[k]] += A.vals[k]
    return M


@pytest.mark.parametrize("seed", range(6))
def test_integer_valued_is_exact(seed):
    # small integers: every product and partial sum is exact, so any correct
    # summation order gives the dense product bit for bit
    A, x = I.random_csr_small(57, 43, seed, max_len=30, integer=True,
                              long_rows=[(3, 43)], unsorted=bool(seed % 2),
                              duplicates=(seed == 4))
    y = oracle.spmv(A, x)
    assert np.array_equal(y, dense(A) @ x)


def test_edge_shapes():
    # n = 1, all-empty rows, a single long row
    A = I.CSR(1, 1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([2.5]))
    assert oracle.spmv(A, np.array([4.0]))[0] == 10.0
    E = I.CSR(5, 3, np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert np.array_equal(oracle.spmv(E, np.ones(3)), np.zeros(5))
    Z = I.CSR(0, 0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert oracle.spmv(Z, np.zeros(0)).size == 0


def test_last_row_and_overwrite():
    # all n rows are computed (the OpenMP listings stop at nrows-1) and y is
    # overwritten, not accumulated
    A, x = I.random_csr_small(20, 20, 7, integer=True, empty_frac=0.0)
    y = oracle.spmv(A, x)
    assert y[-1] == (dense(A) @ x)[-1] and A.row_ptr[-1] > A.row_ptr[-2]


@pytest.mark.parametrize("seed", range(3))
def test_matches_scipy_float(seed):
    A, x = I.random_csr_small(300, 300, seed, max_len=80)
    y = oracle.spmv(A, x)
    ref = A.to_scipy() @ x
    absax = np.abs(dense(A)) @ np.abs(x)
    lens = np.diff(A.row_ptr)
    u = 2.0 ** -53
    bound = 2 * lens * u / (1 - lens * u) * absax
    assert np.all(np.abs(y - ref) <= bound + 1e-300)


def test_transpose_and_f32in():
    A, x = I.random_csr_small(40, 31, 3, max_len=20)
    xt = np.random.default_rng(0).standard_normal(40)
    assert np.allclose(oracle.spmv_transpose(A, xt), dense(A).T @ xt, rtol=1e-14, atol=1e-14)
    v32 = A.vals.astype(np.float32)
    x32 = x.astype(np.float32)
    exact = dense(I.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, v32.astype(np.float64))) @ x32.astype(np.float64)
    assert np.allclose(oracle.spmv_f32in(A, v32, x32), exact, rtol=1e-15, atol=1e-15)


def test_poisson_row_sums():
    # A*1 counts Dirichlet neighbours: 2-D interior 0, edge 1, corner 2
    N = 9
    y = oracle.spmv(I.poisson2d(N), np.ones(N * N)).reshape(N, N)
    assert y[4, 4] == 0 and y[0, 4] == 1 and y[0, 0] == 2 and y[N - 1, N - 1] == 2
    y3 = oracle.spmv(I.poisson3d(N), np.ones(N ** 3)).reshape(N, N, N)
    assert y3[4, 4, 4] == 0 and y3[0, 4, 4] == 1 and y3[0, 0, 4] == 2 and y3[0, 0, 0] == 3
    assert I.poisson2d(64).nnz == 20224 and I.poisson3d(16).nnz == 7 * 16 ** 3 - 6 * 16 ** 2


@pytest.mark.parametrize("modes", [(1, 1, 1), (2, 5, 3), (7, 7, 1)])
def test_poisson3d_eigenpairs(modes):
    N = 12
    j, k, l = modes
    g = np.arange(1, N + 1) / (N + 1)
    vz, vy, vx = (np.sin(m * np.pi * g) for m in (l, k, j))
    v = (vz[:, None, None] * vy[None, :, None] * vx[None, None, :]).ravel()
    lam = sum(4 * math.sin(m * math.pi / (2 * (N + 1))) ** 2 for m in modes)
    Av = oracle.spmv(I.poisson3d(N), v)
    assert np.linalg.norm(Av - lam * v) <= 1e-14 * lam * np.linalg.norm(v) * 10


def test_poisson2d_eigenpair():
    N = 64
    g = np.arange(1, N + 1) / (N + 1)
    v = np.outer(np.sin(np.pi * g), np.sin(np.pi * g)).ravel()
    lam = 8 * math.sin(math.pi / (2 * (N + 1))) ** 2
    assert abs(lam - 4.671e-3) < 1e-6
    Av = oracle.spmv(I.poisson2d(N), v)
    assert np.linalg.norm(Av - lam * v) <= 1e-13 * np.linalg.norm(v)


def test_dot_blocked():
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal(10_001), rng.standard_normal(10_001)
    exact = math.fsum(a * b)  # products rounded, sum exact
    n = a.size
    assert abs(oracle.dot(a, b) - exact) <= n * 2.0 ** -53 * np.sum(np.abs(a * b)) * 1.01
    # fixed order: blocks of 4096, then block sums
    blocks = [sum((a[i:i + 4096] * b[i:i + 4096]).tolist(), 0.0) for i in range(0, n, 4096)]
    s = 0.0
    for t in blocks:
        s += t
    # python's sum adds left to right, the same order
    assert oracle.dot(a, b) == s
    assert oracle.dot(np.zeros(0), np.zeros(0)) == 0.0


def test_csr_check():
    A, _ = I.random_csr_small(10, 10, 0)
    assert oracle.csr_check(A) == oracle.OK
    bad = I.CSR(A.n_rows, A.n_cols, A.row_ptr.copy(), A.col.copy(), A.vals)
    bad.row_ptr[3], bad.row_ptr[4] = bad.row_ptr[4] + 1, bad.row_ptr[3]
    assert oracle.csr_check(bad) == oracle.INVALID_CSR
    bad2 = I.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col.copy(), A.vals)
    bad2.col[0] = 10
    assert oracle.csr_check(bad2) == oracle.INVALID_CSR
    bad3 = I.CSR(A.n_rows, A.n_cols, A.row_ptr.copy(), A.col, A.vals)
    bad3.row_ptr[0] = 1
    assert oracle.csr_check(bad3) == oracle.INVALID_CSR


def test_paper_table_shapes():
    # the generators reproduce the printed input tables (golden, Sec. 3.2 Table 1,
    # Sec. 3.4 Table 2)
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.txt")
    t1, t2, cur = [], [], None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            cur = line
            continue
        f = line.split()
        if cur == "[table1]":
            t1.append((int(f[0]), float(f[1])))
        else:
            t2.append((int(f[1]), int(f[2])))
    assert t1 == I.TABLE1_MOD2AS and t2 == I.TABLE2_CG
    for n, bw in t2[:4]:
        A = I.banded_spd(n, bw)
        h = (bw - 1) // 2
        assert A.nnz == n + 2 * sum(n - d for d in range(1, h + 1))
        assert np.all(np.linalg.eigvalsh(dense(A)) > 0)
    A, _ = I.random_fill(100, 3.5, 0)
    assert A.nnz == 100 * 4

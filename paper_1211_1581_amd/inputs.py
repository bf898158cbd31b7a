"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This module builds matrices and vectors only.  It holds none of the method's
arithmetic (no SpMV kernel, no CG step, no preconditioner, no network); the
right-hand sides ``b = A x*`` are formed by ``scipy.sparse`` so that neither
the oracle nor the HIP library is used to make its own inputs.

Every generator takes an explicit seed and draws from
``numpy.random.default_rng(seed)`` (PCG64) in a fixed, documented order.

Workloads (shapes follow the paper's problem statements):
  * CSR storage with three arrays -- values, column index per value, and the
    position of each row's first value (Sec. 3.2) -- int32 indices.
  * 2-D 5-point and 3-D 7-point Poisson operators with Dirichlet boundary,
    grid ordering idx = (z*N + y)*N + x (x fastest).
  * irregular CSR with lognormal row lengths.
  * 3-D cell-centred finite-volume diffusion with a log-normal Gaussian random
    coefficient field (harmonic face means, Dirichlet ghost cells).
  * banded symmetric matrices of the CG input table (Sec. 3.4, Table 2) and
    random square matrices of the SpMV input table (Sec. 3.2, Table 1).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "CSR", "poisson2d", "poisson3d", "lognormal_irregular", "grf_field",
    "fv_diffusion", "banded_spd", "random_fill", "uniform_vector",
    "rhs_from_solution", "rademacher_probes", "random_csr_small",
    "TABLE1_MOD2AS", "TABLE2_CG",
]


@dataclasses.dataclass
class CSR:
    """Square (or rectangular) CSR matrix: row_ptr int32[n+1], col int32[nnz], vals f64[nnz]."""

    n_rows: int
    n_cols: int
    row_ptr: np.ndarray
    col: np.ndarray
    vals: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.vals, self.col, self.row_ptr),
                             shape=(self.n_rows, self.n_cols))

    def astype(self, dtype) -> "CSR":
        return CSR(self.n_rows, self.n_cols, self.row_ptr, self.col,
                   self.vals.astype(dtype))


def _from_coo(n_rows, n_cols, rows, cols, vals) -> CSR:
    """Assemble CSR with rows ascending, columns sorted inside each row."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    vals = np.asarray(vals, dtype=np.float64)[order]
    counts = np.bincount(rows, minlength=n_rows)
    row_ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    assert row_ptr[-1] < 2**31
    return CSR(n_rows, n_cols, row_ptr.astype(np.int32), cols.astype(np.int32), vals)


def _grid_stencil(shape, diag, neigh_weight):
    """Dirichlet stencil on a tensor grid with x fastest.

    ``neigh_weight(axis, lo_idx)`` returns the (positive) coupling across the
    face between a cell and its +1 neighbour along ``axis``; off-diagonals are
    its negative.  ``diag`` is the full diagonal (flattened)."""
    dims = len(shape)
    n = int(np.prod(shape))
    idx = np.arange(n, dtype=np.int64).reshape(shape)
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [np.asarray(diag, dtype=np.float64).ravel()]
    for ax in range(dims):
        lo = [slice(None)] * dims
        hi = [slice(None)] * dims
        lo[ax] = slice(0, shape[ax] - 1)
        hi[ax] = slice(1, shape[ax])
        a = idx[tuple(lo)].ravel()
        b = idx[tuple(hi)].ravel()
        w = np.asarray(neigh_weight(ax, tuple(lo), tuple(hi)), dtype=np.float64).ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [-w, -w]
    return _from_coo(n, n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def poisson2d(N: int) -> CSR:
    """5-point Poisson on an N x N interior grid: A = I(x)T + T(x)I, T = tridiag(-1, 2, -1)."""
    shape = (N, N)  # (y, x), x fastest
    diag = np.full(shape, 4.0)
    return _grid_stencil(shape, diag, lambda ax, lo, hi: np.ones(shape)[lo])


def poisson3d(N: int) -> CSR:
    """7-point Poisson on an N^3 interior grid, diagonal 6, off-diagonals -1."""
    shape = (N, N, N)  # (z, y, x)
    diag = np.full(shape, 6.0)
    return _grid_stencil(shape, diag, lambda ax, lo, hi: np.ones(shape)[lo])


def grf_field(N: int, rng: np.random.Generator, corr_len: float = 8.0, std: float = 1.5,
              contrast: float = 1.0e4) -> np.ndarray:
    """Log-coefficient field g on an N^3 periodic grid (z, y, x order).

    Steps, in draw order: white noise N(0,1) of shape (N,N,N); Fourier filter
    with transfer exp(-s^2 |k|^2 / 2), s = corr_len / sqrt(2), which gives the
    covariance exp(-r^2 / (2 corr_len^2)); normalise to empirical mean 0 and
    std 1; scale by ``std``; clip to +-ln(contrast)/2 so max(k)/min(k) <= contrast.
    """
    w = rng.standard_normal((N, N, N))
    kf = 2.0 * np.pi * np.fft.fftfreq(N)
    kz, ky, kx = np.meshgrid(kf, kf, kf, indexing="ij")
    s = corr_len / math.sqrt(2.0)
    H = np.exp(-0.5 * s * s * (kx * kx + ky * ky + kz * kz))
    g = np.real(np.fft.ifftn(np.fft.fftn(w) * H))
    sd = g.std()
    g = (g - g.mean()) / sd if sd > 0 else np.zeros_like(g)
    g *= std
    lim = 0.5 * math.log(contrast)
    return np.clip(g, -lim, lim)


def fv_diffusion(N: int, seed: int, with_solution: bool = True, corr_len: float = 8.0):
    """3-D cell-centred finite-volume diffusion, h = 1, 7-point stencil.

    k = exp(g) with g from :func:`grf_field`.  Interior faces carry the
    harmonic mean T = 2 k_i k_j / (k_i + k_j); each boundary face carries
    T = k_i (homogeneous Dirichlet through a ghost cell at distance 1).
    Off-diagonal = -T, diagonal = sum of the cell's face T.  With k = 1 this is
    exactly :func:`poisson3d`.  Returns (A, k, x_star) where x_star ~ U[-1, 1]
    is drawn after the field from the same generator.  Grids much smaller than
    the correlation length need a shorter ``corr_len`` to carry any variation.
    """
    rng = np.random.default_rng(seed)
    g = grf_field(N, rng, corr_len=corr_len)
    kc = np.exp(g)
    return (*_fv_from_k(kc), (uniform_from(rng, N ** 3) if with_solution else None))


def _fv_from_k(kc: np.ndarray):
    shape = kc.shape
    diag = np.zeros(shape)
    faces = []
    for ax in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, shape[ax] - 1)
        hi[ax] = slice(1, shape[ax])
        ki, kj = kc[tuple(lo)], kc[tuple(hi)]
        T = 2.0 * ki * kj / (ki + kj)
        faces.append(T)
        diag[tuple(lo)] += T
        diag[tuple(hi)] += T
        # Dirichlet ghost faces on both ends of this axis
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[ax] = slice(0, 1)
        last[ax] = slice(shape[ax] - 1, shape[ax])
        diag[tuple(first)] += kc[tuple(first)]
        diag[tuple(last)] += kc[tuple(last)]
    A = _grid_stencil(shape, diag, lambda ax, lo, hi: faces[ax])
    return A, kc


def fv_from_coefficients(kc: np.ndarray) -> CSR:
    """FV operator of :func:`fv_diffusion` for a given cell-coefficient array."""
    return _fv_from_k(np.asarray(kc, dtype=np.float64))[0]


def uniform_from(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.uniform(-1.0, 1.0, n)


def uniform_vector(n: int, seed: int) -> np.ndarray:
    """x ~ U[-1, 1] of length n from default_rng(seed)."""
    return uniform_from(np.random.default_rng(seed), n)


def rhs_from_solution(A: CSR, x_star: np.ndarray) -> np.ndarray:
    """Manufactured right-hand side b = A x*, formed by scipy.sparse."""
    return np.asarray(A.to_scipy() @ x_star, dtype=np.float64)


def lognormal_irregular(n: int = 200_000, seed: int = 2, mu_len: float = 48.0,
                        sigma: float = 1.0, max_len: int = 4096):
    """Irregular square CSR.  One generator, drawing in this order:
    (1) row lengths L = clip(rint(lognormal(ln mu_len, sigma, n)), 1, max_len);
    (2) per row, sorted columns drawn uniformly without replacement;
    (3) values ~ N(0, 1) for all nonzeros;  (4) x ~ U[-1, 1].
    Returns (A, x)."""
    rng = np.random.default_rng(seed)
    L = np.clip(np.rint(rng.lognormal(math.log(mu_len), sigma, n)), 1, min(max_len, n)).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(L, out=row_ptr[1:])
    col = np.empty(int(row_ptr[-1]), dtype=np.int32)
    for i in range(n):
        col[row_ptr[i]:row_ptr[i + 1]] = np.sort(rng.choice(n, int(L[i]), replace=False))
    vals = rng.standard_normal(int(row_ptr[-1]))
    x = rng.uniform(-1.0, 1.0, n)
    return CSR(n, n, row_ptr.astype(np.int32), col, vals), x


def banded_spd(n: int, bw: int) -> CSR:
    """Banded symmetric matrix for the CG input table: total bandwidth bw = 2h+1
    (bw = 3 is tridiagonal), off-diagonals -1, diagonal bw.  Strict diagonal
    dominance (bw > bw - 1 >= row's off-diagonal count) makes it SPD."""
    h = (bw - 1) // 2
    rows, cols, vals = [], [], []
    i = np.arange(n, dtype=np.int64)
    rows.append(i); cols.append(i); vals.append(np.full(n, float(bw)))
    for d in range(1, h + 1):
        a = np.arange(n - d, dtype=np.int64)
        rows += [a, a + d]; cols += [a + d, a]; vals += [-np.ones(n - d), -np.ones(n - d)]
    return _from_coo(n, n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def random_fill(n: int, fill_percent: float, seed: int):
    """Square matrix of the SpMV input table: each row holds
    round(n * fill/100) distinct columns drawn uniformly, values ~ U[-1, 1].
    Returns (A, x) with x ~ U[-1, 1]."""
    rng = np.random.default_rng(seed)
    k = max(1, int(round(n * fill_percent / 100.0)))
    cols = np.empty(n * k, dtype=np.int32)
    for i in range(n):
        cols[i * k:(i + 1) * k] = np.sort(rng.choice(n, k, replace=False))
    vals = rng.uniform(-1.0, 1.0, n * k)
    row_ptr = (np.arange(n + 1, dtype=np.int64) * k).astype(np.int32)
    x = rng.uniform(-1.0, 1.0, n)
    return CSR(n, n, row_ptr, cols, vals), x


def random_csr_small(n_rows: int, n_cols: int, seed: int, max_len: int = 12,
                     empty_frac: float = 0.2, integer: bool = False,
                     long_rows: tuple = (), unsorted: bool = False,
                     duplicates: bool = False):
    """Small irregular CSR for edge cases: empty rows, chosen long rows,
    optional unsorted columns and duplicate (i, j) entries.  With
    ``integer=True`` values and x are small integers so every product and
    partial sum is exact in FP64 (and in FP32 while |sums| < 2^24).
    Returns (A, x)."""
    rng = np.random.default_rng(seed)
    L = rng.integers(0, max_len + 1, n_rows)
    L[rng.random(n_rows) < empty_frac] = 0
    for r, ln in long_rows:
        L[r] = ln
    if not duplicates:
        L = np.minimum(L, n_cols)
    row_ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(L, out=row_ptr[1:])
    col = np.empty(int(row_ptr[-1]), dtype=np.int32)
    for i in range(n_rows):
        if duplicates:
            c = rng.integers(0, n_cols, int(L[i]))
        else:
            c = rng.choice(n_cols, int(L[i]), replace=False)
        col[row_ptr[i]:row_ptr[i + 1]] = c if unsorted else np.sort(c)
    nnz = int(row_ptr[-1])
    if integer:
        vals = rng.integers(-4, 5, nnz).astype(np.float64)
        x = rng.integers(-4, 5, n_cols).astype(np.float64)
    else:
        vals = rng.standard_normal(nnz)
        x = rng.uniform(-1.0, 1.0, n_cols)
    return CSR(n_rows, n_cols, row_ptr.astype(np.int32), col, vals), x


def rademacher_probes(n: int, m: int, seed: int) -> np.ndarray:
    """m probe vectors with independent +-1 entries, shape (m, n), float64."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2, (m, n)).astype(np.float64) * 2.0 - 1.0


# SpMV input table of the paper (Sec. 3.2, Table 1): (n, fill in percent)
TABLE1_MOD2AS = [
    (100, 3.50), (200, 3.75), (256, 5.0), (400, 4.38), (500, 5.00), (512, 4.00),
    (960, 4.50), (1000, 5.00), (1024, 5.50), (2000, 7.50), (4096, 3.50),
    (4992, 4.00), (5000, 4.00), (9984, 4.50), (10000, 5.00), (10240, 5.72),
]

# CG input table of the paper (Sec. 3.4, Table 2): (n, bandwidth)
TABLE2_CG = [
    (128, 3), (128, 31), (128, 63), (256, 3), (256, 31), (256, 63), (256, 127),
    (512, 3), (512, 31), (512, 63), (512, 127), (512, 255),
    (1024, 3), (1024, 31), (1024, 63), (1024, 127), (1024, 255), (1024, 511),
]


def mpnn_init(spec, seed: int) -> np.ndarray:
    """Initial network weights as one flat float64 vector in the order of
    ``spec`` (a list of (name, shape)).  Matrices of shape (out, in) are drawn
    U(-1/sqrt(in), 1/sqrt(in)) from default_rng(seed) in spec order; biases
    are zero; every parameter whose name starts with ``head`` is zero, so the
    untrained network reproduces the Jacobi preconditioner exactly."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in spec:
        k = int(np.prod(shape))
        if name.startswith("head") or len(shape) == 1:
            parts.append(np.zeros(k))
        else:
            lim = 1.0 / math.sqrt(shape[1])
            parts.append(rng.uniform(-lim, lim, k))
    return np.concatenate(parts)


def normal_vector(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """N(0, scale^2) vector from default_rng(seed)."""
    return np.random.default_rng(seed).standard_normal(n) * scale

"""An independent numpy restatement of the mixed-precision CG (Sec. 3.4 CG loop
run in FP32 under FP64 residual replacement), used to pin the C oracle's FP32
inner arithmetic.

It is written from the method, not from the oracle's source: an FP32
Jacobi-PCG on fl32(A) with dinv32 = fl32(1 / a_ii); when the FP32 recursive
residual falls below delta times the residual of the last replacement (or to
tol, or at the pass cap) x64 += x32, r64 = b - A x64 in FP64, r32 = fl32(r64),
z and rho are recomputed and the direction is kept.

Every operation is spelled out so that its rounding is explicit:
  * row sums run over each row's entries in index order from zero, one
    rounding per product and one per addition (vectorised across rows only);
  * inner products are taken in one of two stated orders: "blocked" (blocks
    of 4096 summed in index order, then the block sums in order: the order
    the oracle documents) or "pairwise" (a balanced binary tree over the
    products, the shape of a GPU reduction);
  * FP32 steps use float32 arrays and scalars only, FP64 steps float64.
"""
from __future__ import annotations

import numpy as np

BLOCK = 4096


def row_sums(rp, col, vals, x, dtype):
    """y_i = sum over row i in index order, accumulated in `dtype`."""
    n = rp.size - 1
    lens = np.diff(rp)
    y = np.zeros(n, dtype=dtype)
    start = rp[:-1].astype(np.int64)
    for j in range(int(lens.max(initial=0))):
        m = lens > j
        e = start[m] + j
        y[m] = y[m] + vals[e] * x[col[e]]
    return y


def _seq_sum(v):
    """Sequential left-to-right sum in v's dtype (one rounding per addition)."""
    if v.size == 0:
        return v.dtype.type(0)
    return np.add.accumulate(v, dtype=v.dtype)[-1]


def dot(a, b, order="blocked"):
    """Inner product in the dtype of a and b with the stated summation order."""
    t = a.dtype.type
    prod = a * b
    n = prod.size
    if order == "blocked":
        nb = (n + BLOCK - 1) // BLOCK
        pad = np.zeros(nb * BLOCK, dtype=prod.dtype)
        pad[:n] = prod
        parts = np.add.accumulate(pad.reshape(nb, BLOCK), axis=1, dtype=prod.dtype)[:, -1] \
            if nb else np.zeros(0, prod.dtype)
        return t(_seq_sum(parts))
    if order == "pairwise":
        v = prod
        if v.size == 0:
            return t(0)
        while v.size > 1:
            if v.size & 1:
                v = np.concatenate([v, np.zeros(1, v.dtype)])
            v = v[0::2] + v[1::2]
        return t(v[0])
    raise ValueError(order)


def diag_of(rp, col, vals):
    n = rp.size - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    d = np.zeros(n)
    np.add.at(d, rows[col == rows], vals[col == rows])
    return d


def cg_mixed(A, b, x0=None, tol=1e-10, maxit=20000, delta=0.1, order="blocked"):
    """Returns dict(iters, n_updates, hist, x, true_relres).  `order` sets the
    summation order of the FP32 inner products only (FP64 ones stay blocked)."""
    f32, f64 = np.float32, np.float64
    rp = np.asarray(A.row_ptr, dtype=np.int64)
    col = np.asarray(A.col, dtype=np.int64)
    v64 = np.asarray(A.vals, dtype=f64)
    v32 = v64.astype(f32)
    b = np.asarray(b, dtype=f64)
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=f64)
    dinv32 = (1.0 / diag_of(rp, col, v64)).astype(f32)
    nb = np.sqrt(dot(b, b))
    hist = [np.nan] * (maxit + 1)

    r64 = b - row_sums(rp, col, v64, x, f64)
    rlast = np.sqrt(dot(r64, r64))
    hist[0] = rlast / nb
    r32 = r64.astype(f32)
    z = dinv32 * r32
    p = z.copy()
    x32 = np.zeros(n, dtype=f32)
    rho = dot(r32, z, order)
    k = 0
    updates = 0
    converged = rlast <= tol * nb
    while not converged and k < maxit:
        q = row_sums(rp, col, v32, p, f32)
        sigma = dot(p, q, order)
        assert sigma > f32(0)
        alpha = f32(rho / sigma)
        x32 = x32 + alpha * p
        r32 = r32 - alpha * q
        z = dinv32 * r32
        rho_new = dot(r32, z, order)
        rr = dot(r32, r32, order)
        beta = f32(rho_new / rho)
        p = z + beta * p
        rho = rho_new
        k += 1
        est = np.sqrt(f64(rr))
        hist[k] = est / nb
        if est < delta * rlast or est <= tol * nb or k == maxit:
            x = x + x32.astype(f64)
            x32 = np.zeros(n, dtype=f32)
            r64 = b - row_sums(rp, col, v64, x, f64)
            rlast = np.sqrt(dot(r64, r64))
            updates += 1
            hist[k] = rlast / nb
            r32 = r64.astype(f32)
            z = dinv32 * r32
            rho = dot(r32, z, order)
            converged = rlast <= tol * nb
    x = x + x32.astype(f64)
    r64 = b - row_sums(rp, col, v64, x, f64)
    return dict(iters=k, n_updates=updates, hist=np.array(hist[:k + 1]), x=x,
                true_relres=float(np.sqrt(dot(r64, r64)) / nb))

"""Correctness oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library
and the HIP library never imports it.

* ``liboracle.so`` (``oracle.c``): FP64 CSR SpMV, blocked inner products,
  CG / Jacobi-PCG / G G^T-PCG with Jacobi fallback, and the FP32-inner /
  FP64-outer reliable-update solver, all plain sequential-order C.
* ``oracle.mpnn``: the message-passing network that predicts G, its probe
  loss and gradients, in FP64 PyTorch on the CPU.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

OK, NOT_CONVERGED, FELL_BACK = 0, 1, 2
INVALID_ARG, INVALID_CSR, NOT_SPD, NON_FINITE = -1, -2, -4, -5
PRECOND_NONE, PRECOND_JACOBI, PRECOND_G = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc: FP64, no FMA contraction, OpenMP over rows."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.oracle_csr_check.argtypes = [i32, i32, i64, P, P]
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = ctypes.c_int
        L.oracle_spmv_csr.argtypes = [i32, P, P, P, P, P]
        L.oracle_spmv_csr.restype = None
        L.oracle_spmv_csr_f32in.argtypes = [i32, P, P, P, P, P]
        L.oracle_spmv_csr_f32in.restype = None
        L.oracle_spmv_csr_transpose.argtypes = [i32, i32, P, P, P, P, P]
        L.oracle_spmv_csr_transpose.restype = None
        L.oracle_dot.argtypes = [i64, P, P]
        L.oracle_dot.restype = f64
        L.oracle_jacobi_dinv.argtypes = [i32, P, P, P, P]
        L.oracle_pcg.argtypes = [i32, P, P, P, P, P, ctypes.c_int, P, P, P, P, f64, i32,
                                 P, P, P]
        L.oracle_pcg_learned.argtypes = [i32, P, P, P, P, P, P, P, P, f64, i32, i32,
                                         P, P, P, P, P]
        L.oracle_cg_mixed.argtypes = [i32, P, P, P, P, P, f64, i32, f64, ctypes.c_int, P, P,
                                      P, P]
        L.oracle_cg_single_reduction.argtypes = [i32, P, P, P, P, P, ctypes.c_int, f64, i32, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def csr_check(A) -> int:
    rp, c = _i32(A.row_ptr), _i32(A.col)
    if rp.size != A.n_rows + 1:
        return INVALID_CSR
    return lib().oracle_csr_check(A.n_rows, A.n_cols, c.size, _p(rp), _p(c))


def set_threads(n: int) -> int:
    """Threads of the OpenMP row loops (n <= 0: unchanged); returns the previous count."""
    return lib().oracle_set_threads(int(n))


def spmv(A, x) -> np.ndarray:
    """y = A x in FP64, each row summed from zero in index order."""
    rp, c, v, x = _i32(A.row_ptr), _i32(A.col), _f64(A.vals), _f64(x)
    assert x.size == A.n_cols
    y = np.empty(A.n_rows)
    lib().oracle_spmv_csr(A.n_rows, _p(rp), _p(c), _p(v), _p(x), _p(y))
    return y


def spmv_f32in(A, vals32, x32) -> np.ndarray:
    """FP64-accumulated row sums of FP32 values times FP32 x."""
    rp, c = _i32(A.row_ptr), _i32(A.col)
    v = np.ascontiguousarray(vals32, dtype=np.float32)
    x = np.ascontiguousarray(x32, dtype=np.float32)
    y = np.empty(A.n_rows)
    lib().oracle_spmv_csr_f32in(A.n_rows, _p(rp), _p(c), _p(v), _p(x), _p(y))
    return y


def spmv_transpose(A, x) -> np.ndarray:
    rp, c, v, x = _i32(A.row_ptr), _i32(A.col), _f64(A.vals), _f64(x)
    y = np.empty(A.n_cols)
    lib().oracle_spmv_csr_transpose(A.n_rows, A.n_cols, _p(rp), _p(c), _p(v), _p(x), _p(y))
    return y


def dot(a, b) -> float:
    a, b = _f64(a), _f64(b)
    return lib().oracle_dot(a.size, _p(a), _p(b))


def jacobi_dinv(A):
    rp, c, v = _i32(A.row_ptr), _i32(A.col), _f64(A.vals)
    d = np.empty(A.n_rows)
    st = lib().oracle_jacobi_dinv(A.n_rows, _p(rp), _p(c), _p(v), _p(d))
    return st, d


def pcg(A, b, x0=None, tol=1e-10, maxit=2000, precond="jacobi", G=None):
    """Returns dict(status, x, iters, hist, true_relres)."""
    kind = {"none": PRECOND_NONE, "jacobi": PRECOND_JACOBI, "g": PRECOND_G}[precond]
    rp, c, v, b = _i32(A.row_ptr), _i32(A.col), _f64(A.vals), _f64(b)
    x = np.zeros(A.n_rows) if x0 is None else _f64(x0).copy()
    hist = np.full(maxit + 1, np.nan)
    it = ctypes.c_int32(0)
    tr = ctypes.c_double(0.0)
    if G is not None:
        grp, gc, gv = _i32(G.row_ptr), _i32(G.col), _f64(G.vals)
    else:
        grp = gc = gv = None
    st = lib().oracle_pcg(A.n_rows, _p(rp), _p(c), _p(v), _p(b), _p(x), kind, None,
                          _p(grp), _p(gc), _p(gv), tol, maxit, ctypes.byref(it),
                          _p(hist), ctypes.byref(tr))
    k = it.value
    return dict(status=st, x=x, iters=k, hist=hist[:k + 1].copy(), true_relres=tr.value)


def cg_single_reduction(A, b, x0=None, tol=1e-10, maxit=2000, precond="jacobi"):
    """Chronopoulos-Gear single-reduction PCG.  Returns dict(status, x, iters,
    hist, true_relres)."""
    kind = {"none": PRECOND_NONE, "jacobi": PRECOND_JACOBI}[precond]
    rp, c, v, b = _i32(A.row_ptr), _i32(A.col), _f64(A.vals), _f64(b)
    x = np.zeros(A.n_rows) if x0 is None else _f64(x0).copy()
    hist = np.full(maxit + 1, np.nan)
    it = ctypes.c_int32(0)
    tr = ctypes.c_double(0.0)
    st = lib().oracle_cg_single_reduction(A.n_rows, _p(rp), _p(c), _p(v), _p(b), _p(x), kind,
                                          tol, maxit, ctypes.byref(it), _p(hist),
                                          ctypes.byref(tr))
    k = it.value
    return dict(status=st, x=x, iters=k, hist=hist[:k + 1].copy(), true_relres=tr.value)


def pcg_learned(A, b, G, x0=None, tol=1e-10, maxit=20000, budget=1000):
    rp, c, v, b = _i32(A.row_ptr), _i32(A.col), _f64(A.vals), _f64(b)
    grp, gc, gv = _i32(G.row_ptr), _i32(G.col), _f64(G.vals)
    x = np.zeros(A.n_rows) if x0 is None else _f64(x0).copy()
    hl = np.full(maxit + 1, np.nan)
    hf = np.full(maxit + 1, np.nan)
    il, ifb = ctypes.c_int32(0), ctypes.c_int32(0)
    tr = ctypes.c_double(0.0)
    st = lib().oracle_pcg_learned(A.n_rows, _p(rp), _p(c), _p(v), _p(b), _p(x), _p(grp),
                                  _p(gc), _p(gv), tol, maxit, budget, ctypes.byref(il),
                                  ctypes.byref(ifb), _p(hl), _p(hf), ctypes.byref(tr))
    return dict(status=st, x=x, iters_learned=il.value, iters_fallback=ifb.value,
                hist_learned=hl[:il.value + 1].copy(),
                hist_fallback=hf[:ifb.value + 1].copy(), true_relres=tr.value)


def cg_mixed(A, b, x0=None, tol=1e-10, maxit=20000, delta=0.1, dot_order="tree"):
    """FP32-inner / FP64-outer reliable-update CG.  dot_order: "tree" (FP32
    inner products as a balanced binary tree, the order of a data-parallel
    reduction) or "blocked" (blocks of 4096 in index order)."""
    order = {"blocked": 0, "tree": 1}[dot_order]
    rp, c, v, b = _i32(A.row_ptr), _i32(A.col), _f64(A.vals), _f64(b)
    x = np.zeros(A.n_rows) if x0 is None else _f64(x0).copy()
    hist = np.full(maxit + 1, np.nan)
    it, nu = ctypes.c_int32(0), ctypes.c_int32(0)
    tr = ctypes.c_double(0.0)
    st = lib().oracle_cg_mixed(A.n_rows, _p(rp), _p(c), _p(v), _p(b), _p(x), tol, maxit,
                               delta, order, ctypes.byref(it), ctypes.byref(nu), _p(hist),
                               ctypes.byref(tr))
    k = it.value
    return dict(status=st, x=x, iters=k, n_updates=nu.value, hist=hist[:k + 1].copy(),
                true_relres=tr.value)


def true_relres(A, b, x) -> float:
    """||b - A x||_2 / ||b||_2 in FP64, with the oracle's own SpMV and dot."""
    r = _f64(b) - spmv(A, x)
    nb = np.sqrt(dot(b, b))
    return float(np.sqrt(dot(r, r)) / nb) if nb > 0 else 0.0

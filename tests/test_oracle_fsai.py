"""Pins of the FSAI oracle (Kolotilina-Yeremin factorized sparse approximate
inverse on a lower pattern, M^-1 = G G^T): the 2x2 closed form, exactness on
the full lower pattern (G G^T = A^-1), the diagonal case G = D^-1/2, the unit
diagonal of G^T A G on a sparse pattern, and fewer CG passes than Jacobi."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle.fsai import fsai_values
from paper_1211_1581_amd import inputs as I


def csr(S):
    S = sp.csr_matrix(S)
    S.sort_indices()
    return I.CSR(S.shape[0], S.shape[1], S.indptr.astype(np.int32), S.indices.astype(np.int32),
                 S.data.astype(np.float64))


def lower_pattern(A):
    return csr(sp.tril(A.to_scipy()))


def dense_g(G, vals):
    return sp.csr_matrix((vals, G.col, G.row_ptr), shape=(G.n_rows, G.n_cols)).toarray()


def test_two_by_two_closed_form():
    a, b, c = 4.0, -1.5, 3.0
    A = csr(np.array([[a, b], [b, c]]))
    G = lower_pattern(A)
    g = dense_g(G, fsai_values(A, G))
    det = a * c - b * b
    want = np.array([[np.sqrt(c / det), 0.0], [-b / np.sqrt(c * det), 1.0 / np.sqrt(c)]])
    assert np.allclose(g, want, rtol=1e-14, atol=0)


def test_full_lower_pattern_is_exact():
    rng = np.random.default_rng(3)
    B = rng.standard_normal((12, 12))
    Ad = B @ B.T + 12 * np.eye(12)
    A = csr(Ad)
    G = lower_pattern(A)
    g = dense_g(G, fsai_values(A, G))
    assert np.allclose(g @ g.T, np.linalg.inv(Ad), rtol=1e-10, atol=1e-13)
    assert np.allclose(np.diag(g.T @ Ad @ g), 1.0, rtol=1e-13)


def test_diagonal_matrix_gives_inverse_square_root():
    d = np.array([1.0, 4.0, 9.0, 0.25, 2.0])
    A = csr(np.diag(d))
    G = lower_pattern(A)
    assert np.allclose(fsai_values(A, G), 1.0 / np.sqrt(d), rtol=1e-15)


def test_unit_diagonal_on_sparse_pattern():
    A, _, _ = I.fv_diffusion(8, 4, corr_len=2.0)
    G = lower_pattern(A)
    g = sp.csr_matrix((fsai_values(A, G), G.col, G.row_ptr), shape=(A.n_rows, A.n_rows))
    T = (g.T @ A.to_scipy() @ g).diagonal()
    assert np.allclose(T, 1.0, rtol=1e-12)
    assert np.all(np.tril(g.toarray()) == g.toarray())


def test_fsai_pcg_beats_jacobi_on_diffusion():
    # 3-D diffusion with a log-normal coefficient field: FSAI on tril(A) needs
    # roughly half the Jacobi-PCG passes
    A, _, xs = I.fv_diffusion(24, 100)
    b = I.rhs_from_solution(A, xs)
    G = lower_pattern(A)
    G.vals[:] = fsai_values(A, G)
    f = oracle.pcg(A, b, tol=1e-10, maxit=5000, precond="g", G=G)
    j = oracle.pcg(A, b, tol=1e-10, maxit=5000, precond="jacobi")
    assert f["status"] == 0 and f["true_relres"] <= 1e-10
    assert f["iters"] <= 0.7 * j["iters"], (f["iters"], j["iters"])


def test_missing_diagonal_is_rejected():
    A = csr(np.array([[2.0, 1.0], [1.0, 2.0]]))
    G = csr(np.array([[0.0, 0.0], [1.0, 1.0]]))   # column 0 without (0, 0)
    with pytest.raises(ValueError):
        fsai_values(A, G)

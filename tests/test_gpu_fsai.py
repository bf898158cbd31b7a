"""GPU parity of the factorized sparse approximate inverse (spcg_fsai_values)
against the FP64 oracle: factor values (one FP32 rounding apart), FSAI-PCG
pass counts and residuals, the full-lower-pattern case, a pattern with longer
columns, and the error paths."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle
from oracle.fsai import fsai_values
from paper_1211_1581_amd import inputs as I
from gpu_util import lower_upper, spcg, to_dev

pytestmark = pytest.mark.gpu


def within(k_gpu, k_or, frac=0.02, extra=2):
    return abs(k_gpu - k_or) <= frac * k_or + extra


def gpu_fsai(A):
    S = spcg()
    Lh, Uh = lower_upper(A)
    M = S.CsrMatrix.from_host(A)
    G = S.CsrMatrix.from_host(Lh, dtype=torch.float32)
    GT = S.CsrMatrix.from_host(Uh, dtype=torch.float32)
    S.fsai_values(M, G, GT)
    torch.cuda.synchronize()
    return M, G, GT, Lh, Uh


def check_values(dev_vals, ref):
    g = dev_vals.cpu().numpy().astype(np.float64)
    # FP64 arithmetic in both, then one rounding to FP32 on the device
    assert np.all(np.abs(g - ref) <= 2.0 ** -23 * np.abs(ref) + 1e-30), float(np.max(np.abs(g - ref)))


@pytest.mark.parametrize("case", ["fv", "poisson2d", "banded"])
def test_values_match_oracle(case):
    A = {"fv": lambda: I.fv_diffusion(20, 7)[0], "poisson2d": lambda: I.poisson2d(50),
         "banded": lambda: I.banded_spd(2000, 11)}[case]()
    M, G, GT, Lh, Uh = gpu_fsai(A)
    ref = fsai_values(A, Lh)
    check_values(G.vals, ref)
    # G^T carries the same numbers in its own order
    Ug = sp.csr_matrix((ref, Lh.col, Lh.row_ptr), shape=(A.n_rows, A.n_rows)).T.tocsr()
    Ug.sort_indices()
    check_values(GT.vals, Ug.data)


def test_full_lower_pattern_dense():
    rng = np.random.default_rng(5)
    B = rng.standard_normal((8, 8))
    Ad = B @ B.T + 8 * np.eye(8)
    S = sp.csr_matrix(Ad)
    A = I.CSR(8, 8, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data)
    M, G, GT, Lh, Uh = gpu_fsai(A)
    g = sp.csr_matrix((G.vals.cpu().numpy().astype(np.float64), Lh.col, Lh.row_ptr),
                      shape=(8, 8)).toarray()
    assert np.allclose(g @ g.T, np.linalg.inv(Ad), rtol=1e-6, atol=1e-8)


def test_fsai_pcg_matches_oracle():
    A, _, xs = I.fv_diffusion(24, 100)
    b = I.rhs_from_solution(A, xs)
    M, G, GT, Lh, Uh = gpu_fsai(A)
    Lh.vals[:] = fsai_values(A, Lh).astype(np.float32).astype(np.float64)
    ref = oracle.pcg(A, b, tol=1e-10, maxit=5000, precond="g", G=Lh)
    S = spcg()
    g = S.cg_solve(M, to_dev(b), tol=1e-10, maxit=5000, precond="learned", G=G, GT=GT)
    j = S.cg_solve(M, to_dev(b), tol=1e-10, maxit=5000, precond="jacobi")
    assert g["status"] == 0 and within(g["iters"], ref["iters"])
    assert oracle.true_relres(A, b, g["x"].cpu().numpy()) <= 1e-10
    assert g["iters"] <= 0.7 * j["iters"]


def test_error_paths():
    S = spcg()
    # a non-SPD local system (negative diagonal entry)
    A = I.poisson2d(8)
    A.vals[A.col == np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))] *= np.where(
        np.arange(A.n_rows) == 5, -1.0, 1.0)
    M, G, GT = (S.CsrMatrix.from_host(A),) + tuple(
        S.CsrMatrix.from_host(F, dtype=torch.float32) for F in lower_upper(A))
    with pytest.raises(S.SpcgError) as e:
        S.fsai_values(M, G, GT)
    assert e.value.status == S.NOT_SPD
    # columns longer than the supported set
    B = I.banded_spd(200, 19)
    MB, GB, GTB = (S.CsrMatrix.from_host(B),) + tuple(
        S.CsrMatrix.from_host(F, dtype=torch.float32) for F in lower_upper(B))
    with pytest.raises(S.SpcgError) as e:
        S.fsai_values(MB, GB, GTB)
    assert e.value.status == S.INVALID_ARG
    # G^T without its diagonal
    P = I.poisson2d(6)
    Lh, Uh = lower_upper(P)
    U = Uh.to_scipy().tolil()
    U.setdiag(0.0)
    U = sp.csr_matrix(U)
    U.eliminate_zeros()
    U.sort_indices()
    Lx = sp.csr_matrix(U.T)
    Lx.sort_indices()
    mk = lambda Q: S.CsrMatrix.from_host(I.CSR(Q.shape[0], Q.shape[1], Q.indptr.astype(np.int32),
                                                Q.indices.astype(np.int32), Q.data), dtype=torch.float32)
    with pytest.raises(S.SpcgError) as e:
        S.fsai_values(S.CsrMatrix.from_host(P), mk(Lx), mk(U))
    assert e.value.status == S.INVALID_ARG

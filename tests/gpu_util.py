"""Helpers shared by the GPU tests (marshal host CSR to the device, bounds)."""
import numpy as np
import scipy.sparse as sp
import torch

from paper_1211_1581_amd import inputs as I

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def spcg():
    from paper_1211_1581_amd import spcg as m
    return m


def to_dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def dense_abs_product(A, x):
    """(|A| |x|)_i with numpy/scipy (used only for error bounds)."""
    S = sp.csr_matrix((np.abs(np.asarray(A.vals, dtype=np.float64)), A.col, A.row_ptr),
                      shape=(A.n_rows, A.n_cols))
    return S @ np.abs(np.asarray(x, dtype=np.float64))


def gamma(k, u):
    k = np.asarray(k, dtype=np.float64)
    return k * u / (1.0 - k * u)


def check_f64(y, ref, A, x, label=""):
    """Normwise <= 1e-12 and componentwise |y - ref| <= 2 gamma_len |A||x| + tiny."""
    lens = np.diff(A.row_ptr).astype(np.float64)
    bound = 2.0 * gamma(lens + 1, U64) * dense_abs_product(A, x) + 1e-300
    err = np.abs(y - ref)
    assert np.all(err <= bound), (label, float(np.max(err / bound)))
    nr = np.linalg.norm(ref)
    if nr > 0:
        assert np.linalg.norm(y - ref) / nr <= 1e-12, label


def lower_upper(A, gvals=None):
    """G = tril(A) pattern (values gvals or zeros) and G^T, as host CSR objects."""
    S = A.to_scipy()
    L = sp.tril(S, format="csr")
    L.sort_indices()
    if gvals is not None:
        L.data[:] = gvals
    U = L.T.tocsr()
    U.sort_indices()
    mk = lambda M: I.CSR(M.shape[0], M.shape[1], M.indptr.astype(np.int32),
                         M.indices.astype(np.int32), M.data.astype(np.float64))
    return mk(L), mk(U)

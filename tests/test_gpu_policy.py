"""The load policy of the matrix streams (cache-allocating or non-temporal
loads, chosen from the matrix bytes against spcg_keep_bytes) changes only the
memory instructions: every product and solve must be bitwise identical under
both policies."""
import numpy as np
import pytest
import torch

from paper_1211_1581_amd import inputs as I
from gpu_util import lower_upper, spcg, to_dev

pytestmark = pytest.mark.gpu

BOTH = (0, 1 << 40)  # always non-temporal, always cache-allocating


@pytest.fixture(autouse=True)
def restore_policy():
    S = spcg()
    d = S.keep_bytes()
    yield
    S.keep_bytes(d)


def under_both(f):
    S = spcg()
    out = []
    for lim in BOTH:
        S.keep_bytes(lim)
        out.append(f())
        torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_spmv_bitwise_under_both_policies(dtype):
    S = spcg()
    A, x = I.random_csr_small(20011, 20011, 3, max_len=300, long_rows=[(7, 5000)])
    L, _ = lower_upper(I.poisson3d(20))  # short-row kernel
    for M in (A, L):
        H = S.CsrMatrix.from_host(M, dtype=dtype)
        xt = to_dev(I.uniform_vector(M.n_cols, 5), dtype)
        ys = under_both(lambda: S.spmv_csr(H, xt).cpu().numpy())
        assert np.array_equal(ys[0], ys[1])


@pytest.mark.parametrize("form", ["jacobi", "none", "mixed", "single_reduction", "learned"])
def test_cg_bitwise_under_both_policies(form):
    S = spcg()
    A, _, xs = I.fv_diffusion(24, 7)
    b = to_dev(I.rhs_from_solution(A, xs))
    M = S.CsrMatrix.from_host(A)
    kw = dict(tol=1e-10, maxit=5000, small_path=False)
    if form == "learned":
        Lh, _ = lower_upper(A)
        rows = np.repeat(np.arange(A.n_rows), np.diff(Lh.row_ptr))
        d = A.to_scipy().diagonal()
        gv = (np.where(Lh.col == rows, 1.0, 0.1) / np.sqrt(d[rows])).astype(np.float32).astype(np.float64)
        Lh2, Uh2 = lower_upper(A, gv)
        kw.update(precond="learned", G=S.CsrMatrix.from_host(Lh2, dtype=torch.float32),
                  GT=S.CsrMatrix.from_host(Uh2, dtype=torch.float32))
    elif form == "mixed":
        kw.update(precision="mixed")
    elif form == "single_reduction":
        kw.update(variant="single_reduction")
    else:
        kw.update(precond=form)
    rs = under_both(lambda: S.cg_solve(M, b, **kw))
    assert rs[0]["status"] == 0 and rs[0]["iters"] == rs[1]["iters"]
    assert np.array_equal(rs[0]["x"].cpu().numpy(), rs[1]["x"].cpu().numpy())
    assert np.array_equal(rs[0]["hist"], rs[1]["hist"])

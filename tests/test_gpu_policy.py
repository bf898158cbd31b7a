"""The load policy of the matrix streams (cache-allocating or non-temporal
loads, chosen from the matrix bytes against spcg_keep_bytes, and for a solve
whose matrix is above the limit a share of its row blocks kept all the same)
changes only the memory instructions: every product and solve must be bitwise
identical under every limit."""
import numpy as np
import pytest
import torch

from paper_1211_1581_amd import inputs as I
from gpu_util import lower_upper, spcg, to_dev

pytestmark = pytest.mark.gpu

# always non-temporal; partial keeps for the 24^3 test system (400 kB: 6/16 of
# the mixed form's compact FP32 copy, 1/16 of the FP64 matrix; 700 kB: 5/16 of
# the FP64 matrix, all of the compact copy); always cache-allocating
LIMITS = (0, 400_000, 700_000, 1 << 40)


@pytest.fixture(autouse=True)
def restore_policy():
    S = spcg()
    d = S.keep_bytes()
    yield
    S.keep_bytes(d)


def under_both(f):
    S = spcg()
    out = []
    for lim in LIMITS:
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
        assert all(np.array_equal(ys[0], y) for y in ys[1:])


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
    assert rs[0]["status"] == 0
    for r in rs[1:]:
        assert r["iters"] == rs[0]["iters"]
        assert np.array_equal(r["x"].cpu().numpy(), rs[0]["x"].cpu().numpy())
        assert np.array_equal(r["hist"], rs[0]["hist"])

"""cg_solve_static (the allocation-free entry point: workspace in the library's
static device scratch area) against cg_solve with a caller workspace: the
same kernels run, so pass counts, histories and solutions agree bit for bit.
Calls follow each other largest first, so every later call runs on an area
that still holds an earlier solve's contents."""
import numpy as np
import pytest
import torch

import oracle
from paper_1211_1581_amd import inputs as I
from gpu_util import spcg, to_dev

pytestmark = pytest.mark.gpu


def _both(A, b, **kw):
    S = spcg()
    M = S.CsrMatrix.from_host(A)
    bd = to_dev(b)
    ref = S.cg_solve(M, bd, **kw)
    got = S.cg_solve_static(M, bd, **kw)
    torch.cuda.synchronize()
    return ref, got


def _same(ref, got):
    for key in ("status", "iters", "iters_fallback", "n_updates", "n_restarts", "true_relres"):
        assert ref[key] == got[key], (key, ref[key], got[key])
    assert np.array_equal(ref["hist"], got["hist"])
    assert torch.equal(ref["x"], got["x"])


@pytest.mark.parametrize("form", ["jacobi", "mixed"])
def test_static_matches_cg_solve_twice_smaller_second(form):
    S = spcg()
    kw = dict(tol=1e-10, maxit=5000, precond="jacobi", small_path=False,
              precision="mixed" if form == "mixed" else "f64")
    first, second = (40, 3), (20, 6)
    for N, seed in (first, second):
        A, _, xs = I.fv_diffusion(N, seed)
        b = I.rhs_from_solution(A, xs)
        M = S.CsrMatrix.from_host(A)
        need = S.lib().spcg_cg_workspace_bytes(M.handle, S.cg_opts(**kw))
        assert need <= S.STATIC_WORK_BYTES
        ref, got = _both(A, b, **kw)
        _same(ref, got)
        assert got["status"] == 0
        assert oracle.true_relres(A, b, got["x"].cpu().numpy()) <= 1e-10


def test_static_full_size_poisson128_then_small():
    # the 128^3 Jacobi-PCG workspace (67.5 MB) fits the 96 MiB area; then a
    # 2-D system that takes the single-workgroup solver
    for A, seed in ((I.poisson3d(128), 1), (I.poisson2d(64), 0)):
        b = I.rhs_from_solution(A, I.uniform_vector(A.n_rows, seed))
        ref, got = _both(A, b, tol=1e-10, maxit=20000, precond="jacobi")
        _same(ref, got)
        assert got["status"] == 0
        assert oracle.true_relres(A, b, got["x"].cpu().numpy()) <= 1e-10


def test_static_rejects_workspace_beyond_area():
    S = spcg()
    A = I.poisson2d(16)
    M = S.CsrMatrix.from_host(A)
    b = to_dev(np.ones(A.n_rows))
    # a history of 20M + 1 entries needs 160 MB of workspace
    with pytest.raises(S.SpcgError) as e:
        S.cg_solve_static(M, b, maxit=20_000_000)
    assert e.value.status == S.TOO_LARGE
    assert "static scratch" in S.last_error()
    # timing mode creates events: refused
    with pytest.raises(S.SpcgError) as e:
        S.cg_solve_static(M, b, timing=1)
    assert e.value.status == S.INVALID_ARG
    # the area is still usable afterwards
    ref, got = _both(A, np.ones(A.n_rows), tol=1e-10, maxit=2000)
    _same(ref, got)

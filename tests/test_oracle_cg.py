"""Pins of the oracle's CG / PCG (Sec. 3.4) against dense direct solves,
scipy's independent CG, finite termination, the Poisson spectrum, manufactured
solutions and the solver's status contract."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from paper_1211_1581_amd import inputs as I


def csr_from_dense(M):
    S = sp.csr_matrix(M)
    S.sort_indices()
    return I.CSR(M.shape[0], M.shape[1], S.indptr.astype(np.int32), S.indices.astype(np.int32),
                 S.data.astype(np.float64))


def csr_from_scipy(S):
    S = sp.csr_matrix(S)
    S.sort_indices()
    return I.CSR(S.shape[0], S.shape[1], S.indptr.astype(np.int32), S.indices.astype(np.int32),
                 S.data.astype(np.float64))


@pytest.mark.parametrize("precond", ["none", "jacobi"])
@pytest.mark.parametrize("seed", range(3))
def test_tiny_spd_vs_direct(precond, seed):
    rng = np.random.default_rng(seed)
    n = 30
    B = rng.standard_normal((n, n))
    M = B @ B.T + n * np.eye(n)
    M[np.abs(M) < 2.0] = 0.0  # sparsify, keep SPD via the diagonal shift
    M = 0.5 * (M + M.T) + n * np.eye(n)
    A = csr_from_dense(M)
    b = rng.standard_normal(n)
    r = oracle.pcg(A, b, tol=1e-13, maxit=500, precond=precond)
    assert r["status"] == oracle.OK
    xd = np.linalg.solve(M, b)
    kappa = np.linalg.cond(M)
    assert np.linalg.norm(r["x"] - xd) / np.linalg.norm(xd) <= kappa * 1e-12
    assert r["true_relres"] <= 1e-13


def test_poisson2d_64_manufactured():
    A = I.poisson2d(64)
    xs = I.uniform_vector(A.n_rows, 0)
    b = I.rhs_from_solution(A, xs)
    r = oracle.pcg(A, b, tol=1e-10, maxit=2000, precond="none")
    assert r["status"] == oracle.OK and r["true_relres"] <= 1e-10
    # closed-form spectrum: lambda_min = 8 sin^2(pi/130), lambda_max = 8 cos^2(pi/130)
    lmin = 8 * math.sin(math.pi / 130) ** 2
    lmax = 8 * math.cos(math.pi / 130) ** 2
    kappa = lmax / lmin
    assert abs(kappa - 1711.7) < 0.1
    sk = math.sqrt(kappa)
    bound = math.ceil(math.log(2 * sk / 1e-10) / math.log((sk + 1) / (sk - 1)))
    # the residual bound from the Chebyshev estimate caps the iteration count
    assert r["iters"] <= bound and bound == 568
    # forward error <= kappa * relres
    assert np.linalg.norm(r["x"] - xs) / np.linalg.norm(xs) <= kappa * r["true_relres"]
    assert 190 <= r["iters"] <= 212  # observed 201, sanity band
    assert len(r["hist"]) == r["iters"] + 1 and r["hist"][0] == 1.0


def test_jacobi_equals_cg_on_constant_diagonal():
    A = I.poisson2d(32)
    b = I.rhs_from_solution(A, I.uniform_vector(A.n_rows, 5))
    a = oracle.pcg(A, b, tol=1e-10, maxit=2000, precond="none")
    j = oracle.pcg(A, b, tol=1e-10, maxit=2000, precond="jacobi")
    assert abs(a["iters"] - j["iters"]) <= 1
    k = min(a["iters"], j["iters"])
    assert np.allclose(a["hist"][:k], j["hist"][:k], rtol=1e-8, atol=1e-14)
    assert np.linalg.norm(a["x"] - j["x"]) <= 1e-9 * np.linalg.norm(a["x"])


def test_finite_termination():
    # m distinct eigenvalues -> at most m passes (exact arithmetic; loose tol)
    ev = np.repeat([1.0, 2.0, 5.0, 9.0], 25)
    A = csr_from_scipy(sp.diags(ev))
    b = np.random.default_rng(0).standard_normal(ev.size)
    r = oracle.pcg(A, b, tol=1e-12, maxit=100, precond="none")
    assert r["status"] == oracle.OK and r["iters"] <= 4
    # diagonal A: Jacobi-PCG exact after one pass
    d = np.random.default_rng(1).uniform(1, 100, 50)
    Ad = csr_from_scipy(sp.diags(d))
    r = oracle.pcg(Ad, b[:50], tol=1e-14, maxit=10, precond="jacobi")
    assert r["iters"] == 1 and r["status"] == oracle.OK
    # A = c I: plain CG exact after one pass
    r = oracle.pcg(csr_from_scipy(3.0 * sp.eye(40)), b[:40], tol=1e-14, maxit=10, precond="none")
    assert r["iters"] == 1
    # 1-D tridiag(-1, 2, -1) of size m has m distinct eigenvalues
    m = 24
    T = csr_from_scipy(sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1]))
    r = oracle.pcg(T, np.ones(m), tol=1e-12, maxit=100, precond="none")
    assert r["iters"] <= m


def test_vs_scipy_cg_iterations():
    A, _, xs = I.fv_diffusion(12, 7)
    b = I.rhs_from_solution(A, xs)
    S = A.to_scipy()
    count = [0]
    Dinv = sp.diags(1.0 / S.diagonal())
    x, info = spla.cg(S, b, rtol=1e-10, maxiter=5000, M=Dinv,
                      callback=lambda xk: count.__setitem__(0, count[0] + 1))
    r = oracle.pcg(A, b, tol=1e-10, maxit=5000, precond="jacobi")
    assert info == 0 and r["status"] == oracle.OK
    assert abs(count[0] - r["iters"]) <= 2
    assert np.linalg.norm(x - r["x"]) <= 1e-7 * np.linalg.norm(x)


def test_status_codes():
    A = I.poisson2d(8)
    n = A.n_rows
    # b = 0 -> x = 0, zero passes
    r = oracle.pcg(A, np.zeros(n), x0=np.ones(n), precond="jacobi")
    assert r["status"] == oracle.OK and r["iters"] == 0 and np.all(r["x"] == 0)
    # maxit hit
    b = np.ones(n)
    r = oracle.pcg(A, b, maxit=1, precond="jacobi")
    assert r["status"] == oracle.NOT_CONVERGED and r["iters"] == 1
    # non-finite input
    bn = b.copy(); bn[3] = np.nan
    assert oracle.pcg(A, bn)["status"] == oracle.NON_FINITE
    # indefinite matrix: p.Ap <= 0
    Mi = csr_from_scipy(sp.diags([1.0, -1.0, 2.0]))
    assert oracle.pcg(Mi, np.array([1.0, 1.0, 1.0]), precond="none")["status"] == oracle.NOT_SPD
    # non-positive diagonal with Jacobi
    assert oracle.pcg(Mi, np.array([1.0, 1.0, 1.0]), precond="jacobi")["status"] == oracle.NOT_SPD


def test_learned_form_zero_head_is_jacobi():
    # G = D^-1/2 (what a zero-initialised head produces): G G^T = D^-1
    A, _, xs = I.fv_diffusion(10, 3)
    b = I.rhs_from_solution(A, xs)
    S = A.to_scipy()
    G = csr_from_scipy(sp.diags(1.0 / np.sqrt(S.diagonal())))
    Gl = csr_from_scipy(sp.tril(S))  # lower pattern with D^-1/2 on the diagonal
    Gl.vals[:] = 0.0
    dpos = [np.flatnonzero(Gl.col[Gl.row_ptr[i]:Gl.row_ptr[i + 1]] == i)[0] + Gl.row_ptr[i]
            for i in range(A.n_rows)]
    Gl.vals[dpos] = G.vals
    j = oracle.pcg(A, b, tol=1e-10, maxit=2000, precond="jacobi")
    g = oracle.pcg(A, b, tol=1e-10, maxit=2000, precond="g", G=Gl)
    assert j["iters"] == g["iters"]
    assert np.allclose(j["hist"], g["hist"], rtol=1e-10, atol=0)
    # learned wrapper: converges without fallback, and falls back on a tiny budget
    L = oracle.pcg_learned(A, b, Gl, tol=1e-10, maxit=2000, budget=1000)
    assert L["status"] == oracle.OK and L["iters_fallback"] == 0
    L = oracle.pcg_learned(A, b, Gl, tol=1e-10, maxit=2000, budget=1)
    assert L["status"] == oracle.FELL_BACK and L["iters_learned"] == 1
    assert L["true_relres"] <= 1e-10


@pytest.mark.parametrize("order", ["tree", "blocked"])
def test_mixed_reliable_update(order):
    A, _, xs = I.fv_diffusion(16, 3)
    b = I.rhs_from_solution(A, xs)
    j = oracle.pcg(A, b, tol=1e-10, maxit=5000, precond="jacobi")
    m = oracle.cg_mixed(A, b, tol=1e-10, maxit=5000, delta=0.1, dot_order=order)
    assert m["status"] == oracle.OK
    assert oracle.true_relres(A, b, m["x"]) <= 1e-10
    assert m["n_updates"] >= 5
    # the kept direction keeps the inner count near the FP64 count
    assert m["iters"] <= 1.15 * j["iters"] + 5


# The mixed solver's inner loop is FP32 arithmetic (Sec. 3.4 CG loop in FP32
# under FP64 residual replacement).  Its pins: an independent numpy restatement
# with every rounding spelled out (tests/fp32_replay.py) reproduces it bit for
# bit, which a wider accumulator anywhere in the row sums or inner products
# would break; and the true residual at the first replacement sits at FP32
# attainable accuracy, which FP64 vectors would not.

@pytest.mark.parametrize("order", ["tree", "blocked"])
def test_mixed_first_passes_replay_bitwise(order):
    # 17^3 = 4913 rows: the blocked order spans two blocks.  Two passes, then
    # the pass cap forces a replacement: x = fl64(x32) after two FP32 passes,
    # hist[1] the FP32 recursive residual of pass 1.
    import fp32_replay as R
    A, _, xs = I.fv_diffusion(17, 3)
    b = I.rhs_from_solution(A, xs)
    ro = "pairwise" if order == "tree" else "blocked"
    o = oracle.cg_mixed(A, b, tol=1e-10, maxit=2, delta=1e-30, dot_order=order)
    r = R.cg_mixed(A, b, tol=1e-10, maxit=2, delta=1e-30, order=ro)
    assert o["iters"] == r["iters"] == 2 and o["n_updates"] == r["n_updates"] == 1
    assert np.array_equal(o["x"], r["x"])
    assert np.array_equal(o["hist"], r["hist"])
    # the FP32 correction is an FP32 vector: every entry of x is a float
    assert np.array_equal(o["x"].astype(np.float32).astype(np.float64), o["x"])


@pytest.mark.parametrize("N,seed,x0seed", [(16, 3, None), (20, 6, 77), (24, 5, None)])
@pytest.mark.parametrize("order", ["tree", "blocked"])
def test_mixed_full_solve_replay_bitwise(N, seed, x0seed, order):
    import fp32_replay as R
    A, _, xs = I.fv_diffusion(N, seed)
    b = I.rhs_from_solution(A, xs)
    x0 = None if x0seed is None else I.uniform_vector(A.n_rows, x0seed)
    ro = "pairwise" if order == "tree" else "blocked"
    o = oracle.cg_mixed(A, b, x0=x0, tol=1e-10, maxit=5000, delta=0.1, dot_order=order)
    r = R.cg_mixed(A, b, x0=x0, tol=1e-10, maxit=5000, delta=0.1, order=ro)
    assert o["status"] == oracle.OK
    assert (o["iters"], o["n_updates"]) == (r["iters"], r["n_updates"])
    assert np.array_equal(o["hist"], r["hist"]) and np.array_equal(o["x"], r["x"])
    assert o["true_relres"] == r["true_relres"]


def test_mixed_attainable_accuracy_is_fp32():
    # With delta tiny, the first replacement comes only when the FP32
    # recursion claims tol: the FP64 residual recomputed there is the FP32
    # solve's attainable accuracy (about u32 times the condition number), far
    # above tol; an inner loop in FP64 would track its recursion to ~1e-12.
    A, _, xs = I.fv_diffusion(16, 3)
    b = I.rhs_from_solution(A, xs)
    o = oracle.cg_mixed(A, b, tol=1e-10, maxit=400, delta=1e-30)
    h = o["hist"]
    jumps = np.flatnonzero(h[1:] > 10.0 * h[:-1]) + 1
    assert jumps.size > 0
    j = int(jumps[0])
    assert h[j - 1] <= 1e-9          # FP32 recursive residual near tol
    assert h[j] >= 1e-8              # FP64 true residual at FP32 accuracy
    assert np.all(h[1:j] < 1.0)      # the FP32 recursion descended until then


def test_mixed_inner_count_depends_on_fp32_sum_order():
    # From a nonzero initial guess on FV 20^3 the FP32 inner pass count moves
    # by more than 10 % between two valid summation orders of the FP32 inner
    # products (sequential blocks of 4096 against a tree), while each order's
    # count is reproduced exactly by the replay above: device reductions, which
    # are trees, are compared with the tree order.
    A, _, xs = I.fv_diffusion(20, 6)
    b = I.rhs_from_solution(A, xs)
    x0 = I.uniform_vector(A.n_rows, 77)
    t = oracle.cg_mixed(A, b, x0=x0, tol=1e-10, maxit=5000, dot_order="tree")
    k = oracle.cg_mixed(A, b, x0=x0, tol=1e-10, maxit=5000, dot_order="blocked")
    j = oracle.pcg(A, b, x0=x0, tol=1e-10, maxit=5000, precond="jacobi")
    assert t["status"] == k["status"] == oracle.OK
    assert abs(t["iters"] - k["iters"]) > 0.1 * t["iters"]
    assert abs(t["iters"] - j["iters"]) <= 2


# ------------------------------------------- single-reduction (Chronopoulos-Gear) --

@pytest.mark.parametrize("case,precond", [("poisson", "none"), ("poisson", "jacobi"),
                                           ("fv", "jacobi"), ("fv", "none")])
def test_single_reduction_matches_standard_cg(case, precond):
    # same Krylov iterates in exact arithmetic: residual histories agree while
    # rounding has not built up, and the pass counts match.  Plain CG on the
    # high-contrast diffusion matrix (kappa ~ 1e6) is the exception that shows
    # the rounding: both variants leave exact arithmetic after ~10 passes, so
    # only the pass count (within 5 %) and the true residual are compared.
    A = I.poisson2d(64) if case == "poisson" else I.fv_diffusion(12, 3, corr_len=2.0)[0]
    b = I.rhs_from_solution(A, I.uniform_vector(A.n_rows, 0 if case == "poisson" else 1))
    s = oracle.cg_single_reduction(A, b, tol=1e-10, maxit=5000, precond=precond)
    c = oracle.pcg(A, b, tol=1e-10, maxit=5000, precond=precond)
    assert s["status"] == 0 and c["status"] == 0 and s["true_relres"] <= 1e-10
    if case == "fv" and precond == "none":
        assert abs(s["iters"] - c["iters"]) <= 0.05 * c["iters"] + 2
        assert np.allclose(s["hist"][:8], c["hist"][:8], rtol=1e-10, atol=0)
        return
    assert abs(s["iters"] - c["iters"]) <= 2
    k = min(60, len(s["hist"]), len(c["hist"]))
    assert np.allclose(s["hist"][:k], c["hist"][:k], rtol=1e-8, atol=0)


def test_single_reduction_dense_solve_and_finite_termination():
    rng = np.random.default_rng(11)
    B = rng.standard_normal((30, 30))
    M = B @ B.T + 30 * np.eye(30)
    A = csr_from_dense(M)
    b = rng.standard_normal(30)
    s = oracle.cg_single_reduction(A, b, tol=1e-13, maxit=500, precond="jacobi")
    assert s["status"] == 0
    assert np.allclose(s["x"], np.linalg.solve(M, b), rtol=1e-10, atol=1e-12)
    # 6 distinct eigenvalues -> at most 6 passes
    D = csr_from_dense(np.diag(np.repeat([1.0, 2.0, 3.5, 5.0, 8.0, 13.0], 5)))
    r = oracle.cg_single_reduction(D, np.ones(30), tol=1e-12, maxit=100, precond="none")
    assert r["status"] == 0 and r["iters"] <= 6
    # diagonal A with Jacobi: one pass
    r = oracle.cg_single_reduction(D, np.arange(1.0, 31.0), tol=1e-12, maxit=100, precond="jacobi")
    assert r["status"] == 0 and r["iters"] == 1


def test_single_reduction_status_codes():
    A = csr_from_dense(np.array([[1.0, 2.0], [2.0, 1.0]]))   # indefinite
    r = oracle.cg_single_reduction(A, np.array([1.0, -0.5]), precond="none")
    assert r["status"] == oracle.NOT_SPD
    P = I.poisson2d(8)
    r = oracle.cg_single_reduction(P, np.zeros(P.n_rows))
    assert r["status"] == 0 and r["iters"] == 0 and not np.any(r["x"])

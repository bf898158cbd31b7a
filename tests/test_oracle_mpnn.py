"""Pins of the FP64 network oracle: central finite differences of the probe
loss, the closed-form gradient with respect to the factor values, the zero-head
identity with Jacobi scaling, and positive definiteness of G G^T."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import mpnn
from paper_1211_1581_amd import inputs as I


def random_params(seed, head_scale=0.3):
    flat = I.mpnn_init(mpnn.param_spec(), seed)
    rng = np.random.default_rng(seed + 1000)
    P = mpnn.unflatten(flat)
    for name in P:
        if name.startswith("head") or P[name].ndim == 1:
            P[name] = rng.uniform(-head_scale, head_scale, P[name].shape)
    return P


def test_param_count():
    assert mpnn.n_params() == 29442


def test_zero_head_is_jacobi_scaling():
    A, _, _ = I.fv_diffusion(5, 11, corr_len=1.5)
    P = mpnn.unflatten(I.mpnn_init(mpnn.param_spec(), 0))
    V = I.rademacher_probes(A.n_rows, 3, 1)
    out = mpnn.forward(P, A, V)
    S = A.to_scipy()
    d = S.diagonal()
    G = mpnn.g_csr(A, out["g_vals"])
    Gd = sp.csr_matrix((G.vals, G.col, G.row_ptr), shape=S.shape).toarray()
    assert np.array_equal(Gd, np.diag(1.0 / np.sqrt(d)))
    At = (sp.diags(d ** -0.5) @ S @ sp.diags(d ** -0.5)).toarray()
    ref = sum(np.sum((At @ v - v) ** 2) for v in V) / (A.n_rows * 3)
    assert abs(out["loss"] - ref) <= 1e-13 * ref


def test_factor_gradient_closed_form():
    # dL/dG_ij = sum_v u_i s_j + (A G s)_i v_j with w = G v, u = A w,
    # t = G^T u, s = 2 (t - v) / (n m)
    A, _, _ = I.fv_diffusion(4, 5, corr_len=1.5)
    rng = np.random.default_rng(3)
    gr = mpnn.graph(A)
    nl = int(gr["lower"].sum())
    gv = rng.uniform(0.2, 1.0, nl)
    V = I.rademacher_probes(A.n_rows, 2, 9)
    loss, grad = mpnn.probe_loss_grad_g(A, gv, V)
    S = A.to_scipy().toarray()
    G = mpnn.g_csr(A, gv)
    Gd = sp.csr_matrix((G.vals, G.col, G.row_ptr), shape=S.shape).toarray()
    n, m = A.n_rows, V.shape[0]
    ref = np.zeros_like(Gd)
    L = 0.0
    for v in V:
        u = S @ (Gd @ v)
        t = Gd.T @ u
        L += np.sum((t - v) ** 2)
        s = 2 * (t - v) / (n * m)
        ref += np.outer(u, s) + np.outer(S @ (Gd @ s), v)
    assert abs(loss - L / (n * m)) <= 1e-12 * loss
    rows = np.repeat(np.arange(n), np.diff(G.row_ptr))
    assert np.allclose(grad, ref[rows, G.col], rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("seed", [0, 1])
def test_weight_gradients_finite_differences(seed):
    A, _, _ = I.fv_diffusion(4, 20 + seed, corr_len=1.5)
    P = random_params(seed)
    V = I.rademacher_probes(A.n_rows, 2, 40 + seed)
    out = mpnn.forward(P, A, V, need_grad=True)
    flat = mpnn.flatten(P)
    g = out["grads"]
    rng = np.random.default_rng(seed)
    idx = rng.choice(flat.size, 60, replace=False)
    # include head and encoder entries explicitly
    idx = np.unique(np.concatenate([idx, [0, 100, flat.size - 1, flat.size - 33, flat.size - 34]]))
    h = 1e-6
    for k in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[k] += h
        fm[k] -= h
        lp = mpnn.forward(mpnn.unflatten(fp), A, V)["loss"]
        lm = mpnn.forward(mpnn.unflatten(fm), A, V)["loss"]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(g[k]), 1e-3 * np.abs(g).max()), (k, fd, g[k])


def test_factor_is_spd_for_any_output():
    A, _, _ = I.fv_diffusion(4, 1, corr_len=1.5)
    P = random_params(5, head_scale=0.5)
    out = mpnn.forward(P, A)
    G = mpnn.g_csr(A, out["g_vals"])
    Gd = sp.csr_matrix((G.vals, G.col, G.row_ptr), shape=(A.n_rows, A.n_rows)).toarray()
    assert np.allclose(Gd, np.tril(Gd)) and np.all(np.diag(Gd) > 0)
    np.linalg.cholesky(Gd @ Gd.T)

"""GPU parity of the learned-factor network (BF16 matrix-core MLPs, FP32
accumulation) with the FP64 oracle: factor pattern, the zero-head Jacobi
identity, forward factor values, probe loss and weight gradients, the Adam
step, and a CG solve with the predicted factor.

Tolerances: activations are stored in BF16 (unit roundoff 2^-9) before each of
the ~10 matrix products on the path to the head, so the forward outputs
carry relative errors of order 1e-2; the tests bound the normwise relative
error of the factor values by 2e-2 (measured: 3e-3 .. 6e-3), the loss by
1e-2, the gradient by 5e-2 (measured: 2e-3 .. 2.3e-2), and require cosine
similarity >= 0.9999 (factor) / 0.999 (gradients).  A wrong index, sign or
transposition gives O(1) errors."""
import ctypes

import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle
from oracle import mpnn
from paper_1211_1581_amd import inputs as I
from gpu_util import spcg, to_dev

pytestmark = pytest.mark.gpu


def weights(seed, head_scale=0.3):
    flat = I.mpnn_init(mpnn.param_spec(), seed)
    P = mpnn.unflatten(flat)
    rng = np.random.default_rng(seed + 7)
    for name in P:
        if name.startswith("head") or P[name].ndim == 1:
            P[name] = rng.uniform(-head_scale, head_scale, P[name].shape)
    return P


def graph(A, train=False):
    S = spcg()
    M = S.CsrMatrix.from_host(A)
    return M, S.MpnnGraph(M, train=train)


def cos(a, b):
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)))


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("N", [7, 45])
def test_factor_pattern_and_zero_head(N):
    # 45^3 rows span many chunks of the device scan that builds the patterns
    A, _, _ = I.fv_diffusion(N, 4, corr_len=2.0)
    M, g = graph(A)
    P0 = mpnn.unflatten(I.mpnn_init(mpnn.param_spec(), 0))
    w = torch.tensor(mpnn.flatten(P0), dtype=torch.float32, device="cuda")
    g.predict(w)
    rp, col, gv, gtv = g.factor_arrays()
    L = sp.tril(A.to_scipy(), format="csr")
    L.sort_indices()
    assert np.array_equal(rp, L.indptr) and np.array_equal(col, L.indices)
    d = A.to_scipy().diagonal()
    rows = np.repeat(np.arange(A.n_rows), np.diff(rp))
    diag = col == rows
    assert np.allclose(gv[diag], 1.0 / np.sqrt(d), rtol=2e-7)
    assert np.all(gv[~diag] == 0.0)
    # G^T values in G^T's CSR order equal the transpose of G
    Gs = sp.csr_matrix((gv.astype(np.float64), col, rp), shape=(A.n_rows,) * 2)
    U = Gs.T.tocsr()
    U.sort_indices()
    assert np.array_equal(U.data.astype(np.float32), gtv)


# N = 31: 202 771 edges, 6337 tiles of 32 with a ragged last one, more than the
# edge kernel keeps resident, so every wavefront runs its pipelined loop over
# several tiles
@pytest.mark.parametrize("N,seed", [(6, 1), (12, 2), (31, 5)])
def test_forward_matches_oracle(N, seed):
    A, _, _ = I.fv_diffusion(N, seed, corr_len=2.0)
    P = weights(seed)
    ref = mpnn.forward(P, A)["g_vals"]
    M, g = graph(A)
    g.predict(torch.tensor(mpnn.flatten(P), dtype=torch.float32, device="cuda"))
    _, _, gv, _ = g.factor_arrays()
    assert cos(gv, ref) >= 0.9999 and rel(gv, ref) <= 2e-2, (cos(gv, ref), rel(gv, ref))


@pytest.mark.parametrize("N,seed", [(12, 2), (31, 5)])
def test_inference_forward_equals_training_forward(N, seed):
    """Without training the first edge layer encodes the edge state itself; with
    training the encoder stores it. Both round each encoded value once to BF16
    from the same FP32 operations, so the two factors agree bit for bit."""
    A, _, _ = I.fv_diffusion(N, seed, corr_len=2.0)
    w = torch.tensor(mpnn.flatten(weights(seed)), dtype=torch.float32, device="cuda")
    _, gi = graph(A)
    _, gt = graph(A, train=True)
    gi.predict(w)
    # the training forward runs inside the loss (every layer's state stored)
    V = torch.tensor(I.rademacher_probes(A.n_rows, 2, seed), dtype=torch.float32, device="cuda")
    gt.loss_grad(w, V, want_loss=False)
    _, _, gv_i, gtv_i = gi.factor_arrays()
    _, _, gv_t, gtv_t = gt.factor_arrays()
    assert np.array_equal(gv_i, gv_t) and np.array_equal(gtv_i, gtv_t)


# N = 21: 62 181 edges, 1944 tiles with a ragged last one, more than the
# backward kernels' wavefronts, so their loops and per-wave partials cover
# several tiles each
@pytest.mark.parametrize("N,seed", [(6, 3), (10, 4), (21, 6)])
def test_loss_and_gradients_match_oracle(N, seed):
    A, _, _ = I.fv_diffusion(N, seed, corr_len=2.0)
    P = weights(seed)
    V = I.rademacher_probes(A.n_rows, 4, seed + 100)
    ref = mpnn.forward(P, A, V, need_grad=True)
    M, g = graph(A, train=True)
    w = torch.tensor(mpnn.flatten(P), dtype=torch.float32, device="cuda")
    grad = torch.zeros(spcg().MPNN_PARAMS, dtype=torch.float32, device="cuda")
    loss = g.loss_grad(w, torch.tensor(V, dtype=torch.float32, device="cuda"), grad)
    gr = grad.cpu().numpy().astype(np.float64)
    assert abs(loss - ref["loss"]) <= 1e-2 * ref["loss"], (loss, ref["loss"])
    assert cos(gr, ref["grads"]) >= 0.999, cos(gr, ref["grads"])
    assert rel(gr, ref["grads"]) <= 5e-2, rel(gr, ref["grads"])
    # each parameter block points the same way as the oracle's
    o = 0
    for name, shape in mpnn.param_spec():
        k = int(np.prod(shape))
        a, b = gr[o:o + k], ref["grads"][o:o + k]
        if np.linalg.norm(b) > 1e-3 * np.linalg.norm(ref["grads"]) and k > 1:
            assert cos(a, b) >= 0.95, (name, cos(a, b))
        o += k


def test_adam_step():
    S = spcg()
    rng = np.random.default_rng(0)
    w, gr = rng.standard_normal(1000), rng.standard_normal(1000)
    m, v = rng.standard_normal(1000) * 0.1, rng.random(1000) * 0.1
    t = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in (w, gr, m, v)]
    S.adam_step(*t, 3, lr=1e-2)
    b1, b2, eps = 0.9, 0.999, 1e-8
    m2 = b1 * m + (1 - b1) * gr
    v2 = b2 * v + (1 - b2) * gr * gr
    w2 = w - 1e-2 * (m2 / (1 - b1 ** 3)) / (np.sqrt(v2 / (1 - b2 ** 3)) + eps)
    assert np.allclose(t[0].cpu().numpy(), w2, rtol=1e-5, atol=1e-6)


def test_learned_cg_with_predicted_factor():
    A, _, xs = I.fv_diffusion(16, 9)
    b = I.rhs_from_solution(A, xs)
    P = weights(5, head_scale=0.02)
    M, g = graph(A)
    g.predict(torch.tensor(mpnn.flatten(P), dtype=torch.float32, device="cuda"))
    S = spcg()
    out = S.cg_solve(M, to_dev(b), tol=1e-10, maxit=5000, precond="learned", G=g.G, GT=g.GT,
                     budget=400)
    assert out["status"] in (S.OK, S.FELL_BACK)
    assert oracle.true_relres(A, b, out["x"].cpu().numpy()) <= 1e-10
    # the oracle's learned solve with the same (FP32) factor and budget: same
    # outcome, and each phase's pass count within the rounding band
    rp, col, gv, _ = g.factor_arrays()
    Gh = I.CSR(A.n_rows, A.n_rows, rp, col, gv.astype(np.float64))
    ro = oracle.pcg_learned(A, b, Gh, tol=1e-10, maxit=5000, budget=400)
    assert (out["status"] == S.FELL_BACK) == (ro["status"] == oracle.FELL_BACK)
    assert abs(out["iters"] - ro["iters_learned"]) <= 0.02 * ro["iters_learned"] + 2
    assert abs(out["iters_fallback"] - ro["iters_fallback"]) <= 0.02 * ro["iters_fallback"] + 2


def test_invalid_patterns_rejected():
    S = spcg()
    # unsymmetric pattern
    D = sp.csr_matrix(np.array([[2.0, 1.0, 0.0], [0.0, 2.0, 0.0], [0.0, 0.0, 2.0]]))
    A = I.CSR(3, 3, D.indptr.astype(np.int32), D.indices.astype(np.int32), D.data)
    M = S.CsrMatrix.from_host(A)
    with pytest.raises(S.SpcgError) as e:
        S.MpnnGraph(M)
    assert e.value.status == S.INVALID_CSR


def test_caller_workspace_rules():
    # the network calls run on a caller-owned workspace: too small or
    # misaligned is rejected before any work; a larger one shared by a smaller
    # graph gives the same factor as the graph's own
    S = spcg()
    A, _, _ = I.fv_diffusion(10, 3, corr_len=2.0)
    B, _, _ = I.fv_diffusion(6, 3, corr_len=2.0)
    w = torch.tensor(mpnn.flatten(weights(3)), dtype=torch.float32, device="cuda")
    MA, ga = graph(A)
    MB = S.CsrMatrix.from_host(B)
    gb_own = S.MpnnGraph(MB)
    gb_shared = S.MpnnGraph(MB, ws=ga.ws)
    gb_own.predict(w)
    gb_shared.predict(w)
    assert np.array_equal(gb_own.factor_arrays()[2], gb_shared.factor_arrays()[2])
    L = S.lib()
    need = L.spcg_mpnn_workspace_bytes(A.n_rows, ga.n_edges, 0)
    assert need == ga.ws.nbytes
    buf = ga.ws.buf
    assert L.spcg_mpnn_predict(ga._h, S._ptr(w), S._ptr(buf), need - 1,
                               S._stream()) == S.INVALID_ARG
    assert L.spcg_mpnn_predict(ga._h, S._ptr(w), ctypes.c_void_p(buf.data_ptr() + 8), need,
                               S._stream()) == S.INVALID_ARG
    # the training loss needs the training layout
    gt = S.MpnnGraph(MA, train=True)
    V = torch.ones((1, A.n_rows), dtype=torch.float32, device="cuda")
    with pytest.raises(S.SpcgError):
        gt.ws = ga.ws  # an inference-sized workspace
        gt.loss_grad(w, V)

"""What the trained network gains over the method without it: on held-out
48^3 diffusion matrices (seeds the training never saw), PCG with the factor
predicted by the committed weights needs far fewer passes than Jacobi-PCG,
while the untrained network (zero head) reproduces Jacobi-PCG; both reach
the 1e-10 FP64 residual, recomputed by the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1211_1581_amd import inputs as I
from paper_1211_1581_amd import train
from gpu_util import spcg

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed", [356, 361])
def test_trained_factor_beats_jacobi(seed):
    S = spcg()
    A, _, xs = I.fv_diffusion(48, seed)
    b_np = I.rhs_from_solution(A, xs)
    b = torch.as_tensor(b_np, device="cuda")
    M = S.CsrMatrix.from_host(A)
    g = S.MpnnGraph(M)
    w_trained, meta = train.load_weights()
    counts = {}
    for name, w in [("trained", w_trained), ("untrained", train.initial_weights(0))]:
        g.predict(torch.tensor(w, dtype=torch.float32, device="cuda"))
        r = S.cg_solve(M, b, tol=1e-10, maxit=5000, precond="learned", G=g.G, GT=g.GT)
        assert r["status"] == S.OK
        assert oracle.true_relres(A, b_np, r["x"].cpu().numpy()) <= 1e-10
        counts[name] = r["iters"]
    j = S.cg_solve(M, b, tol=1e-10, maxit=5000, precond="jacobi")
    assert abs(counts["untrained"] - j["iters"]) <= 2
    assert counts["trained"] <= 0.6 * j["iters"], (counts, j["iters"])
    # the weights file records a held-out loss well below Jacobi's
    assert meta["heldout_loss"] < 0.5 * meta["heldout_loss_jacobi"]

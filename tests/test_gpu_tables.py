"""The paper's own input tables on the built kernels (GPU parity against the
FP64 oracle): every SpMV configuration of Sec. 3.2 Table 1 (square matrices
of n rows with the stated fill, random sorted columns, U[-1, 1] values) and
every CG configuration of Sec. 3.4 Table 2 (banded SPD matrices of total
bandwidth bw, off-diagonals -1, diagonal bw), plain CG to 1e-10 as in the
paper's solver."""
import numpy as np
import pytest
import torch

import oracle
from paper_1211_1581_amd import inputs as I
from gpu_util import check_f64, spcg, to_dev

pytestmark = pytest.mark.gpu


def _table(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.txt")
    rows, cur = [], None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            cur = line.strip("[]")
            continue
        if cur == name:
            rows.append(tuple(float(v) for v in line.split()))
    return rows


TABLE1 = [(int(n), f) for n, f in _table("table1")]
TABLE2 = [(int(n), int(bw)) for _, n, bw in _table("table2")]


def test_tables_match_the_generators():
    assert TABLE1 == [(n, f) for n, f in I.TABLE1_MOD2AS]
    assert TABLE2 == list(I.TABLE2_CG)


@pytest.mark.parametrize("n,fill", TABLE1)
def test_table1_spmv(n, fill):
    A, x = I.random_fill(n, fill, seed=n)
    S = spcg()
    M = S.CsrMatrix.from_host(A)
    y = S.spmv_csr(M, to_dev(x))
    torch.cuda.synchronize()
    check_f64(y.cpu().numpy(), oracle.spmv(A, x), A, x, f"table1 n={n}")


@pytest.mark.parametrize("n,bw", TABLE2)
def test_table2_cg(n, bw):
    A = I.banded_spd(n, bw)
    b = I.rhs_from_solution(A, I.uniform_vector(n, n + bw))
    ref = oracle.pcg(A, b, tol=1e-10, maxit=2000, precond="none")
    S = spcg()
    g = S.cg_solve(S.CsrMatrix.from_host(A), to_dev(b), tol=1e-10, maxit=2000, precond="none")
    assert ref["status"] == 0 and g["status"] == 0
    assert abs(g["iters"] - ref["iters"]) <= 0.02 * ref["iters"] + 2
    assert oracle.true_relres(A, b, g["x"].cpu().numpy()) <= 1e-10

"""FP64 CPU oracle of the factorized sparse approximate inverse -- TEST
INFRASTRUCTURE ONLY.

Classical FSAI (Kolotilina and Yeremin) for M^-1 = G G^T with G lower
triangular on a prescribed pattern.  Each column of G is found on its own:
for column i let J = {j >= i : (j, i) in the pattern}, in ascending order (so
J[0] = i).  Minimising the Frobenius distance between G's column and the
corresponding column of the inverse upper Cholesky factor of A, restricted to
J, gives the small SPD system

    A[J, J] y = e_1,        G[J, i] = y / sqrt(y_1),

and the scaling makes (G^T A G)_ii = 1.  With the full lower pattern the
columns are exact and G G^T = A^-1.  The systems are solved with
numpy.linalg.solve, one column at a time.
"""
from __future__ import annotations

import numpy as np


def fsai_values(A, G) -> np.ndarray:
    """Values of G (FP64, in G's CSR order) for the pattern of the lower CSR G.

    A: CSR object (n_rows, row_ptr, col, vals), square and symmetric.
    G: CSR object of the lower pattern (its values are ignored)."""
    n = A.n_rows
    S = A.to_scipy().tocsr()
    grp = np.asarray(G.row_ptr, dtype=np.int64)
    gcol = np.asarray(G.col, dtype=np.int64)
    # row sets of the columns of G: J_i = rows j with (j, i) in the pattern
    rows = np.repeat(np.arange(n), np.diff(grp))
    order = np.lexsort((rows, gcol))          # by column, then row
    starts = np.searchsorted(gcol[order], np.arange(n + 1))
    out = np.zeros(len(gcol))
    for i in range(n):
        idx = order[starts[i]:starts[i + 1]]  # positions in G of column i's entries
        J = rows[idx]
        if len(J) == 0 or J[0] != i:
            raise ValueError(f"column {i} of the pattern lacks its diagonal")
        M = S[J][:, J].toarray()
        e = np.zeros(len(J))
        e[0] = 1.0
        y = np.linalg.solve(M, e)
        out[idx] = y / np.sqrt(y[0])
    return out

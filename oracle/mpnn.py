"""FP64 CPU oracle of the learned preconditioner -- TEST INFRASTRUCTURE ONLY.

The preconditioner is M^-1 = G G^T with G lower-triangular on A's own lower
pattern, so it is SPD for any network output and applying it is two
SpMV-shaped products (the factor and its transpose).  A message-passing
network reads the Jacobi-scaled matrix A~ = D^-1/2 A D^-1/2 and predicts the
factor; G = D^-1/2 L~ with L~_ii = exp(o_ii) and L~_ij = o_ij (j < i), so
G^T A G = L~^T A~ L~ and a zero head gives G = D^-1/2, i.e. exactly
Jacobi-PCG.

Network (hidden width H = 32, SiLU activations, 4 layers):
  node features  f_i  = [1, log a_ii - mean(log a)]               -> h_i  (2 -> H, affine)
  edge features  g_ij = [a~_ij, log max(|a~_ij|, 1e-30)], i != j  -> e_ij (2 -> H, affine)
  layer:  m_ij = W2e silu(W1e [h_i; h_j; e_ij] + c1e) + c2e        (3H -> H -> H)
          agg_i = sum over off-diagonal entries (i, j) of row i of m_ij
          h_i  += W2n silu(W1n [h_i; agg_i] + c1n) + c2n          (2H -> H -> H)
          e_ij  = m_ij
  head:   o_ij = w_e . e_ij + c_e  (j < i),   o_ii = w_n . h_i + c_n   (zero-initialised)

Probe loss over m probe vectors v (rows of V):  L = sum_v ||G^T A G v - v||^2 / (n m).
Gradients come from torch.autograd in FP64 on the CPU.
"""
from __future__ import annotations

import numpy as np
import torch

H = 32
N_LAYERS = 4


def param_spec():
    """(name, shape) of every parameter, in the order of the flat weight vector."""
    spec = [("enc_n_w", (H, 2)), ("enc_n_b", (H,)), ("enc_e_w", (H, 2)), ("enc_e_b", (H,))]
    for l in range(N_LAYERS):
        spec += [(f"l{l}_e1_w", (H, 3 * H)), (f"l{l}_e1_b", (H,)),
                 (f"l{l}_e2_w", (H, H)), (f"l{l}_e2_b", (H,)),
                 (f"l{l}_n1_w", (H, 2 * H)), (f"l{l}_n1_b", (H,)),
                 (f"l{l}_n2_w", (H, H)), (f"l{l}_n2_b", (H,))]
    spec += [("head_e_w", (H,)), ("head_e_b", (1,)), ("head_n_w", (H,)), ("head_n_b", (1,))]
    return spec


def n_params() -> int:
    return int(sum(np.prod(s) for _, s in param_spec()))


def unflatten(flat):
    flat = np.asarray(flat, dtype=np.float64)
    out, o = {}, 0
    for name, shape in param_spec():
        k = int(np.prod(shape))
        out[name] = flat[o:o + k].reshape(shape)
        o += k
    assert o == flat.size
    return out


def flatten(params) -> np.ndarray:
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel()
                           for name, _ in param_spec()])


def _silu(x):
    return x * torch.sigmoid(x)


def graph(A):
    """Edge lists of A (CSR, sorted columns): off-diagonal entries in CSR order,
    the diagonal position of every row, and the lower pattern (j <= i) in CSR
    order, which is the pattern of G."""
    rp = np.asarray(A.row_ptr, dtype=np.int64)
    col = np.asarray(A.col, dtype=np.int64)
    n = A.n_rows
    row = np.repeat(np.arange(n), np.diff(rp))
    off = row != col
    lower = col <= row
    diag_pos = np.flatnonzero(~off)
    assert diag_pos.size == n and np.all(row[diag_pos] == np.arange(n)), "one diagonal per row"
    return dict(row=row, col=col, off=off, lower=lower, diag_pos=diag_pos)


def forward(params, A, V=None, need_grad=False):
    """Returns dict(o_off, o_diag, g_vals (G on tril(A) in CSR order),
    loss (if V is given), grads (flat, if need_grad))."""
    gr = graph(A)
    n = A.n_rows
    P = {k: torch.tensor(v, dtype=torch.float64, requires_grad=need_grad)
         for k, v in params.items()}
    vals = torch.tensor(np.asarray(A.vals), dtype=torch.float64)
    row = torch.tensor(gr["row"])
    col = torch.tensor(gr["col"])
    off = torch.tensor(gr["off"])
    d = vals[torch.tensor(gr["diag_pos"])]
    s = d.rsqrt()
    logd = torch.log(d)
    f = torch.stack([torch.ones(n, dtype=torch.float64), logd - logd.mean()], dim=1)
    ei, ej = row[off], col[off]
    at = vals[off] * s[ei] * s[ej]
    g = torch.stack([at, torch.log(torch.clamp(at.abs(), min=1e-30))], dim=1)

    h = f @ P["enc_n_w"].T + P["enc_n_b"]
    e = g @ P["enc_e_w"].T + P["enc_e_b"]
    for l in range(N_LAYERS):
        x = torch.cat([h[ei], h[ej], e], dim=1)
        z = x @ P[f"l{l}_e1_w"].T + P[f"l{l}_e1_b"]
        m = _silu(z) @ P[f"l{l}_e2_w"].T + P[f"l{l}_e2_b"]
        agg = torch.zeros(n, H, dtype=torch.float64).index_add(0, ei, m)
        u = torch.cat([h, agg], dim=1) @ P[f"l{l}_n1_w"].T + P[f"l{l}_n1_b"]
        h = h + _silu(u) @ P[f"l{l}_n2_w"].T + P[f"l{l}_n2_b"]
        e = m
    o_off = e @ P["head_e_w"] + P["head_e_b"][0]
    o_diag = h @ P["head_n_w"] + P["head_n_b"][0]

    # G on the lower pattern, CSR order
    lower = torch.tensor(gr["lower"])
    lt = torch.zeros(A.nnz, dtype=torch.float64)
    lt = lt.index_put((torch.nonzero(off).flatten(),), o_off)
    lt = lt.index_put((torch.tensor(gr["diag_pos"]),), torch.exp(o_diag))
    gvals_full = lt * s[row]
    g_vals = gvals_full[lower]

    out = dict(o_off=o_off.detach().numpy().copy(), o_diag=o_diag.detach().numpy().copy(),
               g_vals=g_vals.detach().numpy().copy())
    if V is not None:
        V = torch.tensor(np.asarray(V), dtype=torch.float64)
        loss = probe_loss_torch(A, gr, gvals_full, lower, V)
        out["loss"] = float(loss.detach())
        if need_grad:
            loss.backward()
            out["grads"] = flatten({k: P[k].grad.numpy() for k in P})
    return out


def probe_loss_torch(A, gr, gvals_full, lower, V):
    """sum_v ||G^T A G v - v||^2 / (n m) with G the lower part of gvals_full."""
    n = A.n_rows
    m = V.shape[0]
    row = torch.tensor(gr["row"])
    col = torch.tensor(gr["col"])
    lw = lower
    gi, gj, gv = row[lw], col[lw], gvals_full[lw]
    av = torch.tensor(np.asarray(A.vals), dtype=torch.float64)
    total = 0.0
    for k in range(m):
        v = V[k]
        w = torch.zeros(n, dtype=torch.float64).index_add(0, gi, gv * v[gj])      # G v
        u = torch.zeros(n, dtype=torch.float64).index_add(0, row, av * w[col])    # A w
        t = torch.zeros(n, dtype=torch.float64).index_add(0, gj, gv * u[gi])      # G^T u
        total = total + ((t - v) ** 2).sum()
    return total / (n * m)


def g_csr(A, g_vals):
    """G as a CSR object (lower pattern of A, values g_vals)."""
    from types import SimpleNamespace
    gr = graph(A)
    row, col, lower = gr["row"], gr["col"], gr["lower"]
    counts = np.bincount(row[lower], minlength=A.n_rows)
    rp = np.zeros(A.n_rows + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    return SimpleNamespace(n_rows=A.n_rows, n_cols=A.n_cols, row_ptr=rp.astype(np.int32),
                           col=col[lower].astype(np.int32),
                           vals=np.asarray(g_vals, dtype=np.float64),
                           nnz=int(rp[-1]))


def probe_loss_grad_g(A, g_vals, V):
    """Loss and its gradient with respect to the G values (autograd, FP64)."""
    gr = graph(A)
    lower = torch.tensor(gr["lower"])
    gv = torch.tensor(np.asarray(g_vals, dtype=np.float64), requires_grad=True)
    full = torch.zeros(A.nnz, dtype=torch.float64).index_put((torch.nonzero(lower).flatten(),), gv)
    loss = probe_loss_torch(A, gr, full, lower, torch.tensor(np.asarray(V), dtype=torch.float64))
    loss.backward()
    return float(loss.detach()), gv.grad.numpy().copy()

"""Thin ctypes binding of libspcg.so (include/spcg.h).

Argument marshalling only: torch tensors provide device memory and the
current HIP stream; every step of SpMV and CG runs in the library's kernels.
Importing works without a GPU; calls need the built library and a device and
raise if either is missing (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspcg.so")

OK, NOT_CONVERGED, FELL_BACK = 0, 1, 2
INVALID_ARG, INVALID_CSR, HIP_ERROR, NOT_SPD, NON_FINITE, TOO_LARGE = -1, -2, -3, -4, -5, -6
STATIC_WORK_BYTES = 96 << 20  # SPCG_STATIC_WORK_BYTES
F64, F32 = 0, 1
PRECOND = {"none": 0, "jacobi": 1, "learned": 2}
PRECISION = {"f64": 0, "mixed": 1}


class SpcgError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} {last_error()}".strip())


class CgOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("delta", ctypes.c_double),
                ("G", ctypes.c_void_p), ("GT", ctypes.c_void_p),
                ("budget", ctypes.c_int32), ("small_path", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("variant", ctypes.c_int32)]


class CgResult(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("iters_fallback", ctypes.c_int32),
                ("n_updates", ctypes.c_int32), ("n_restarts", ctypes.c_int32),
                ("true_relres", ctypes.c_double), ("spmv_ms", ctypes.c_double),
                ("spmv_calls", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None


def lib():
    """Load libspcg.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1211_1581_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.spcg_status_str.argtypes = [ctypes.c_int]
        L.spcg_status_str.restype = ctypes.c_char_p
        L.spcg_last_error.argtypes = []
        L.spcg_last_error.restype = ctypes.c_char_p
        L.spcg_csr_create.argtypes = [ctypes.POINTER(P), i32, i32, i64, P, P, P, i32, P]
        L.spcg_keep_bytes.argtypes = [i64]
        L.spcg_keep_bytes.restype = i64
        L.spcg_csr_destroy.argtypes = [P]
        L.spcg_csr_info.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                    ctypes.POINTER(i64)]
        L.spcg_csr_wide_blocks.argtypes = [P, ctypes.POINTER(i64)]
        L.spmv_csr.argtypes = [P, P, P, P]
        L.spcg_row_binning.argtypes = [ctypes.c_int]
        L.spcg_row_binning.restype = ctypes.c_int
        L.spcg_csr_bin_counts.argtypes = [P, ctypes.POINTER(i64)]
        L.spcg_run_columns.argtypes = [ctypes.c_int]
        L.spcg_run_columns.restype = ctypes.c_int
        L.spcg_csr_run_info.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.spcg_column_panels.argtypes = [ctypes.c_int]
        L.spcg_column_panels.restype = ctypes.c_int
        L.spcg_csr_panel_info.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.spcg_dot_workspace_bytes.argtypes = [i64]
        L.spcg_dot_workspace_bytes.restype = sz
        L.spcg_dot.argtypes = [i64, P, P, P, P, P]
        L.spcg_cg_default_opts.argtypes = [ctypes.POINTER(CgOpts)]
        L.spcg_cg_default_opts.restype = None
        L.spcg_cg_workspace_bytes.argtypes = [P, ctypes.POINTER(CgOpts)]
        L.spcg_cg_workspace_bytes.restype = sz
        L.cg_solve.argtypes = [P, P, P, ctypes.POINTER(CgOpts), P, sz,
                               ctypes.POINTER(CgResult), P, P]
        L.cg_solve_static.argtypes = [P, P, P, ctypes.POINTER(CgOpts),
                                      ctypes.POINTER(CgResult), P, P]
        _lib = L
    return _lib


def status_str(st: int) -> str:
    return lib().spcg_status_str(st).decode()


def keep_bytes(value=None) -> int:
    """Matrix-stream load policy (spcg_keep_bytes): with value, set the limit
    in bytes and return the previous one; without, return the current one."""
    return int(lib().spcg_keep_bytes(-1 if value is None else int(value)))


BINNING = {"off": 0, "on": 1}
BINNING_NAME = {v: k for k, v in BINNING.items()}


def row_binning(mode=None):
    """Row-length binning policy of spmv_csr (spcg_row_binning): with mode
    ("off", "on"), set it and return the previous one; without, return the
    current one."""
    st = lib().spcg_row_binning(-1 if mode is None else BINNING[mode])
    if st < 0:
        raise SpcgError(st, "spcg_row_binning")
    return BINNING_NAME[st]


RUNS = {"off": 0, "on": 1}
RUNS_NAME = {v: k for k, v in RUNS.items()}


def run_columns(mode=None):
    """Run-compressed column policy of spmv_csr (spcg_run_columns): with mode
    ("off", "on"), set it and return the previous one; without, return the
    current one."""
    st = lib().spcg_run_columns(-1 if mode is None else RUNS[mode])
    if st < 0:
        raise SpcgError(st, "spcg_run_columns")
    return RUNS_NAME[st]


PANELS = {"off": 0, "on": 1, "auto": 2}
PANELS_NAME = {v: k for k, v in PANELS.items()}


def column_panels(mode=None):
    """Column-panel policy of spmv_csr (spcg_column_panels): with mode ("off",
    "on", "auto"), set it and return the previous one; without, return the
    current one."""
    st = lib().spcg_column_panels(-1 if mode is None else PANELS[mode])
    if st < 0:
        raise SpcgError(st, "spcg_column_panels")
    return PANELS_NAME[st]


def last_error() -> str:
    return lib().spcg_last_error().decode()


def _check(st, what):
    if st < 0 and st != NOT_SPD and st != NON_FINITE:
        raise SpcgError(st, what)
    return st


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _workspace(nbytes: int, device) -> torch.Tensor:
    """Device buffer of nbytes whose start is 256-byte aligned."""
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + nbytes]


class CsrMatrix:
    """A CSR matrix resident on the device and its library handle.

    row_ptr int32[n+1], col int32[nnz], vals float64 or float32[nnz], all
    device tensors that this object keeps alive for the handle's lifetime."""

    def __init__(self, row_ptr, col, vals, n_cols=None):
        self.row_ptr = row_ptr.contiguous()
        self.col = col.contiguous()
        self.vals = vals.contiguous()
        self.n_rows = self.row_ptr.numel() - 1
        self.n_cols = self.n_rows if n_cols is None else int(n_cols)
        self.nnz = self.col.numel()
        self.dtype = {torch.float64: F64, torch.float32: F32}[self.vals.dtype]
        self._h = ctypes.c_void_p(0)
        st = lib().spcg_csr_create(ctypes.byref(self._h), self.n_rows, self.n_cols, self.nnz,
                                   _ptr(self.row_ptr), _ptr(self.col), _ptr(self.vals),
                                   self.dtype, _stream())
        if st != OK:
            self._h = ctypes.c_void_p(0)
            raise SpcgError(st, "spcg_csr_create")

    @classmethod
    def from_host(cls, A, device="cuda", dtype=torch.float64):
        """From an object with n_rows, n_cols, row_ptr, col, vals (numpy)."""
        rp = torch.as_tensor(A.row_ptr, dtype=torch.int32).to(device)
        c = torch.as_tensor(A.col, dtype=torch.int32).to(device)
        v = torch.as_tensor(A.vals).to(dtype).to(device)
        return cls(rp, c, v, n_cols=A.n_cols)

    @property
    def handle(self):
        return self._h

    def info(self):
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().spcg_csr_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
               "spcg_csr_info")
        w = ctypes.c_int64()
        _check(lib().spcg_csr_wide_blocks(self._h, ctypes.byref(w)), "spcg_csr_wide_blocks")
        return dict(n_blocks=a.value, n_long=b.value, max_row_len=c.value, n_wide_blocks=w.value)

    def has_bins(self) -> bool:
        c = (ctypes.c_int64 * 8)()
        return lib().spcg_csr_bin_counts(self._h, c) == OK

    def bin_counts(self):
        """Rows per row-length bin (a list of 8), for a handle made with bins."""
        c = (ctypes.c_int64 * 8)()
        _check(lib().spcg_csr_bin_counts(self._h, c), "spcg_csr_bin_counts")
        return list(c)

    def run_info(self):
        """(chunks, run starts) of a handle made with run-compressed columns, or None."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        if lib().spcg_csr_run_info(self._h, ctypes.byref(a), ctypes.byref(b)) != OK:
            return None
        return a.value, b.value

    def panel_info(self):
        """(row ranges, column panels, entries of the panel copy with its
        padding) of a handle made with column panels, or None."""
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        if lib().spcg_csr_panel_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)) != OK:
            return None
        return a.value, b.value, c.value

    def close(self):
        if self._h and self._h.value:
            lib().spcg_csr_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def spmv_csr(A: CsrMatrix, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
    """y = A x on the current stream (asynchronous)."""
    if y is None:
        y = torch.empty(A.n_rows, dtype=A.vals.dtype, device=A.vals.device)
    assert x.dtype == A.vals.dtype and y.dtype == A.vals.dtype
    assert x.numel() == A.n_cols and y.numel() == A.n_rows and x.is_contiguous()
    _check(lib().spmv_csr(A.handle, _ptr(x), _ptr(y), _stream()), "spmv_csr")
    return y


def dot(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """Deterministic FP64 inner product, result as a 1-element device tensor."""
    assert a.dtype == torch.float64 and b.dtype == torch.float64 and a.numel() == b.numel()
    n = a.numel()
    out = torch.empty(1, dtype=torch.float64, device=a.device)
    work = _workspace(lib().spcg_dot_workspace_bytes(n), a.device)
    _check(lib().spcg_dot(n, _ptr(a), _ptr(b), _ptr(out), _ptr(work), _stream()), "spcg_dot")
    return out


VARIANT = {"standard": 0, "single_reduction": 1}


def cg_opts(tol=1e-10, maxit=20000, precond="jacobi", precision="f64", check_every=0,
            delta=0.1, G=None, GT=None, budget=None, small_path=True, timing=False,
            variant="standard") -> CgOpts:
    o = CgOpts()
    lib().spcg_cg_default_opts(ctypes.byref(o))
    o.tol = tol
    o.maxit = maxit
    o.precond = PRECOND[precond]
    o.precision = PRECISION[precision]
    o.check_every = check_every
    o.delta = delta
    o.G = G.handle.value if G is not None else None
    o.GT = GT.handle.value if GT is not None else None
    if budget is not None:
        o.budget = budget
    o.small_path = 1 if small_path else 0
    o.timing = int(timing)  # N > 0: time every N-th pass's SpMV (True = every pass)
    o.variant = VARIANT[variant]
    return o


class CgWorkspace:
    """Reusable device workspace for cg_solve with fixed options."""

    def __init__(self, A: CsrMatrix, opts: CgOpts):
        self.nbytes = lib().spcg_cg_workspace_bytes(A.handle, ctypes.byref(opts))
        self.buf = _workspace(self.nbytes, A.vals.device)


def cg_solve(A: CsrMatrix, b: torch.Tensor, x: torch.Tensor | None = None, *, opts=None,
             work: CgWorkspace | None = None, want_hist=True, **kw):
    """Solve A x = b (x: in x0, out solution; zero if None).  Returns a dict with
    status, x, iters, iters_fallback, n_updates, n_restarts, true_relres, hist."""
    if opts is None:
        opts = cg_opts(**kw)
    if x is None:
        x = torch.zeros_like(b)
    assert b.dtype == torch.float64 and x.dtype == torch.float64 and x.is_contiguous()
    if work is None:
        work = CgWorkspace(A, opts)
    res = CgResult()
    hist = (ctypes.c_double * (opts.maxit + 1))() if want_hist else None
    hp = ctypes.cast(hist, ctypes.c_void_p) if want_hist else ctypes.c_void_p(0)
    st = lib().cg_solve(A.handle, _ptr(b), _ptr(x), ctypes.byref(opts), _ptr(work.buf),
                        work.nbytes, ctypes.byref(res), hp, _stream())
    _check(st, "cg_solve")
    return _result(st, x, res, hist)


def cg_solve_static(A: CsrMatrix, b: torch.Tensor, x: torch.Tensor | None = None, *, opts=None,
                    want_hist=True, **kw):
    """cg_solve on the library's static scratch area (cg_solve_static): no
    workspace argument, no device allocation in the call.  Same result dict."""
    if opts is None:
        opts = cg_opts(**kw)
    if x is None:
        x = torch.zeros_like(b)
    assert b.dtype == torch.float64 and x.dtype == torch.float64 and x.is_contiguous()
    res = CgResult()
    hist = (ctypes.c_double * (opts.maxit + 1))() if want_hist else None
    hp = ctypes.cast(hist, ctypes.c_void_p) if want_hist else ctypes.c_void_p(0)
    st = lib().cg_solve_static(A.handle, _ptr(b), _ptr(x), ctypes.byref(opts),
                               ctypes.byref(res), hp, _stream())
    _check(st, "cg_solve_static")
    return _result(st, x, res, hist)


def _result(st, x, res, hist):
    k = res.iters + res.iters_fallback  # one history over both phases of a fallback
    out = dict(status=st, x=x, iters=res.iters, iters_fallback=res.iters_fallback,
               n_updates=res.n_updates, n_restarts=res.n_restarts,
               true_relres=res.true_relres, spmv_ms=res.spmv_ms, spmv_calls=res.spmv_calls)
    if hist is not None:
        import numpy as np
        out["hist"] = np.ctypeslib.as_array(hist)[:k + 1].copy()
    return out


# ------------------------------------------------------------ learned factor --

MPNN_PARAMS = 29442


def _mpnn_sigs(L):
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    if getattr(L, "_mpnn_ready", False):
        return L
    L.spcg_mpnn_create.argtypes = [ctypes.POINTER(P), P, i32, P]
    L.spcg_mpnn_destroy.argtypes = [P]
    L.spcg_mpnn_info.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.spcg_mpnn_factor.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P)]
    L.spcg_mpnn_factor_arrays.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P),
                                          ctypes.POINTER(P), ctypes.POINTER(P)]
    L.spcg_mpnn_workspace_bytes.argtypes = [i64, i64, i32]
    L.spcg_mpnn_workspace_bytes.restype = ctypes.c_size_t
    L.spcg_mpnn_predict.argtypes = [P, P, P, ctypes.c_size_t, P]
    L.spcg_mpnn_loss_grad.argtypes = [P, P, P, i32, P, ctypes.POINTER(ctypes.c_double), P,
                                      ctypes.c_size_t, P]
    L.spcg_adam_step.argtypes = [P, P, P, P, i64, i32, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_float, P]
    L._mpnn_ready = True
    return L


class _Borrowed:
    """A matrix handle owned by another object (no destroy)."""

    def __init__(self, h, owner):
        self._h = ctypes.c_void_p(h)
        self.owner = owner

    @property
    def handle(self):
        return self._h


class MpnnWorkspace:
    """Device workspace of the network calls (spcg_mpnn_workspace_bytes), a
    torch buffer shared by the graphs of many matrices used one at a time."""

    def __init__(self, max_rows: int, max_edges: int, train: bool = False, device="cuda"):
        L = _mpnn_sigs(lib())
        self.max_rows, self.max_edges, self.train = max_rows, max_edges, train
        self.nbytes = L.spcg_mpnn_workspace_bytes(max_rows, max_edges, 1 if train else 0)
        if self.nbytes == 0:
            raise SpcgError(INVALID_ARG, "spcg_mpnn_workspace_bytes")
        self.buf = _workspace(self.nbytes, device)


class MpnnGraph:
    """Network state for one matrix (see spcg_mpnn_create).  Without an explicit
    workspace, the graph gets one of its own size."""

    def __init__(self, A: CsrMatrix, train: bool = False, ws: "MpnnWorkspace | None" = None):
        L = _mpnn_sigs(lib())
        self.A = A
        self.train = train
        self._h = ctypes.c_void_p(0)
        st = L.spcg_mpnn_create(ctypes.byref(self._h), A.handle, 1 if train else 0, _stream())
        if st != OK:
            self._h = ctypes.c_void_p(0)
            raise SpcgError(st, "spcg_mpnn_create")
        e, g = ctypes.c_int64(), ctypes.c_int64()
        _check(L.spcg_mpnn_info(self._h, ctypes.byref(e), ctypes.byref(g)), "spcg_mpnn_info")
        self.n_edges, self.nnz_factor = e.value, g.value
        hg, hgt = ctypes.c_void_p(0), ctypes.c_void_p(0)
        _check(L.spcg_mpnn_factor(self._h, ctypes.byref(hg), ctypes.byref(hgt)), "spcg_mpnn_factor")
        self.G, self.GT = _Borrowed(hg.value, self), _Borrowed(hgt.value, self)
        self.ws = ws if ws is not None else MpnnWorkspace(A.n_rows, self.n_edges, train,
                                                          A.vals.device)

    def predict(self, w: torch.Tensor):
        assert w.dtype == torch.float32 and w.numel() == MPNN_PARAMS and w.is_contiguous()
        _check(lib().spcg_mpnn_predict(self._h, _ptr(w), _ptr(self.ws.buf), self.ws.nbytes,
                                       _stream()), "spcg_mpnn_predict")

    def loss_grad(self, w: torch.Tensor, probes: torch.Tensor, grad: torch.Tensor | None = None,
                  want_loss: bool = True):
        """Probe loss (float, or None without want_loss, which avoids a
        synchronisation); fills grad if given."""
        assert probes.dtype == torch.float32 and probes.is_contiguous()
        assert probes.shape[1] == self.A.n_rows
        m = probes.shape[0]
        loss = ctypes.c_double(0.0)
        _check(lib().spcg_mpnn_loss_grad(self._h, _ptr(w), _ptr(probes), m, _ptr(grad),
                                         ctypes.byref(loss) if want_loss else None,
                                         _ptr(self.ws.buf), self.ws.nbytes, _stream()),
               "spcg_mpnn_loss_grad")
        return loss.value if want_loss else None

    def factor_arrays(self):
        """(row_ptr, col, G values, G^T values) as host numpy arrays."""
        import numpy as np
        P = ctypes.c_void_p
        rp, c, v, vt = P(), P(), P(), P()
        _check(lib().spcg_mpnn_factor_arrays(self._h, ctypes.byref(rp), ctypes.byref(c),
                                             ctypes.byref(v), ctypes.byref(vt)),
               "spcg_mpnn_factor_arrays")
        torch.cuda.synchronize()
        n, k = self.A.n_rows, self.nnz_factor

        def grab(ptr, count, ctype, dt):
            buf = (ctype * count)()
            import ctypes as C
            hip = _hip()
            assert hip.hipMemcpy(C.cast(buf, C.c_void_p), C.c_void_p(ptr.value),
                                 C.c_size_t(count * C.sizeof(ctype)), 2) == 0
            return np.frombuffer(buf, dtype=dt).copy()

        return (grab(rp, n + 1, ctypes.c_int32, np.int32), grab(c, k, ctypes.c_int32, np.int32),
                grab(v, k, ctypes.c_float, np.float32), grab(vt, k, ctypes.c_float, np.float32))

    def close(self):
        if self._h and self._h.value:
            lib().spcg_mpnn_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_hip_lib = None


def _hip():
    global _hip_lib
    if _hip_lib is None:
        _hip_lib = ctypes.CDLL("libamdhip64.so")
        _hip_lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_int]
    return _hip_lib


def adam_step(w, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    L = _mpnn_sigs(lib())
    _check(L.spcg_adam_step(_ptr(w), _ptr(g), _ptr(m), _ptr(v), w.numel(), t, lr, beta1, beta2,
                            eps, _stream()), "spcg_adam_step")


# --------------------------------------------- factorized sparse approximate inverse --

FSAI_MAX_SET = 8


def fsai_values(A: CsrMatrix, G, GT):
    """Overwrite the FP32 values of the lower factor G and of its transpose GT
    (handles on one pattern, e.g. an MpnnGraph's G and GT) with the classical
    factorized sparse approximate inverse of A (see spcg_fsai_values)."""
    L = lib()
    if not getattr(L, "_fsai_ready", False):
        P = ctypes.c_void_p
        L.spcg_fsai_values.argtypes = [P, P, P, P]
        L._fsai_ready = True
    st = L.spcg_fsai_values(A.handle, G.handle, GT.handle, _stream())
    if st != OK:  # a local system that is not SPD is an error here, not a solver outcome
        raise SpcgError(st, "spcg_fsai_values")

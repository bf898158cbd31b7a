"""Host-side checks of the C ABI: the library loads without a GPU and exports
every function that include/spcg.h declares; struct layouts of the binding
match the header; the oracle library builds.  No compute call is made."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spcg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ["spcg_csr_create", "spcg_csr_destroy", "spmv_csr", "cg_solve",
                     "spcg_cg_workspace_bytes", "spcg_dot", "spcg_status_str"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1211_1581_amd import spcg
    if not os.path.exists(spcg.LIB_PATH):
        from paper_1211_1581_amd import build
        build.build()
    L = ctypes.CDLL(spcg.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings_and_struct_sizes():
    from paper_1211_1581_amd import spcg
    assert spcg.status_str(spcg.OK) == "OK"
    assert spcg.status_str(spcg.NOT_SPD) == "NOT_SPD"
    # spcg_cg_opts: double, 4 x int32, double, 2 pointers, 4 x int32
    assert ctypes.sizeof(spcg.CgOpts) == 8 + 16 + 8 + 16 + 16
    assert ctypes.sizeof(spcg.CgResult) == 16 + 8 + 8 + 8
    o = spcg.CgOpts()
    spcg.lib().spcg_cg_default_opts(ctypes.byref(o))
    assert o.tol == 1e-10 and o.maxit == 20000 and o.precond == 1 and o.delta == 0.1


def test_invalid_args_rejected_on_host():
    from paper_1211_1581_amd import spcg
    L = spcg.lib()
    h = ctypes.c_void_p(0)
    # negative sizes and bad dtype are rejected before any device work
    assert L.spcg_csr_create(ctypes.byref(h), -1, 3, 0, None, None, None, 0, None) == spcg.INVALID_ARG
    assert L.spcg_csr_create(ctypes.byref(h), 3, 3, 0, None, None, None, 7, None) == spcg.INVALID_ARG
    # sizes above SPCG_MAX_INDEX = 2^31 - 2^16 - 1 (32-bit indexing with headroom)
    big = 2**31 - 2**16
    fake = ctypes.c_void_p(1)  # never dereferenced: the size check comes first
    assert L.spcg_csr_create(ctypes.byref(h), 3, 3, big, fake, fake, fake, 0, None) == spcg.INVALID_ARG
    assert L.spcg_csr_create(ctypes.byref(h), big, 3, 0, fake, fake, fake, 0, None) == spcg.INVALID_ARG
    assert L.spcg_csr_create(ctypes.byref(h), 3, big, 0, fake, fake, fake, 0, None) == spcg.INVALID_ARG
    assert L.spmv_csr(None, None, None, None) == spcg.INVALID_ARG
    nb = ctypes.c_int64(-1)
    assert L.spcg_csr_wide_blocks(None, ctypes.byref(nb)) == spcg.INVALID_ARG and nb.value == -1
    res = spcg.CgResult()
    assert L.cg_solve(None, None, None, None, None, 0, ctypes.byref(res), None, None) == spcg.INVALID_ARG


def test_oracle_builds():
    import oracle
    path = oracle.build(force=False)
    assert os.path.exists(path)


def test_weight_layout_matches_oracle():
    # the library's documented flat weight order is the oracle's parameter order
    from oracle import mpnn
    from paper_1211_1581_amd import spcg, train
    assert train.param_spec() == mpnn.param_spec()
    assert spcg.MPNN_PARAMS == mpnn.n_params()
    src = open(os.path.join(ROOT, "include", "spcg.h")).read()
    assert "#define SPCG_MPNN_PARAMS 29442" in src


def test_keep_bytes_setting_round_trips():
    # process-wide load policy of the matrix streams: no device work involved
    from paper_1211_1581_amd import spcg
    d = spcg.keep_bytes()
    assert d == 192 << 20
    assert spcg.keep_bytes(0) == d and spcg.keep_bytes() == 0
    assert spcg.keep_bytes(d) == 0 and spcg.keep_bytes() == d


def test_network_workspace_sizes_on_host():
    # spcg_mpnn_workspace_bytes is host arithmetic: no device call
    from paper_1211_1581_amd import spcg
    L = spcg._mpnn_sigs(spcg.lib())
    n, E = 110592, 649728  # the 48^3 training matrices
    infer = L.spcg_mpnn_workspace_bytes(n, E, 0)
    train = L.spcg_mpnn_workspace_bytes(n, E, 1)
    assert infer % 256 == 0 and train % 256 == 0
    assert 0 < infer < train
    # two alternating BF16 layers of width 32 at least
    assert infer >= 2 * 2 * 32 * (n + E)
    assert L.spcg_mpnn_workspace_bytes(2 * n, 2 * E, 0) > infer
    assert L.spcg_mpnn_workspace_bytes(0, E, 0) == 0 and L.spcg_mpnn_workspace_bytes(n, -1, 1) == 0

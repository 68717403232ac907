"""Boundary checks that need no GPU: the built library exports every entry
point include/fc.h declares, the ctypes layouts match the C structs, the
argument checks fail before any device work, and the product path does not
reach the oracle."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fc.h")


@pytest.fixture(scope="module")
def N():
    from paper_2506_04045_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        from paper_2506_04045_amd import build
        build.build()
    _native.load()
    return _native


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("fc_create", "fc_step", "fc_solve", "fc_objective", "fc_project",
                     "fc_destroy", "fc_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(N):
    lib = ctypes.CDLL(N.LIB_PATH)
    missing = [name for name in declared_functions() if not hasattr(lib, name)]
    assert not missing, missing
    assert sorted(N.EXPORTED) == declared_functions()


def test_struct_layouts(N):
    o = N.default_options()
    assert o.struct_size == ctypes.sizeof(N.Options) == 112
    assert ctypes.sizeof(N.CSR) == 48 and ctypes.sizeof(N.Info) == 72
    assert o.eta == 2.0 and o.max_iter == 100 and o.check_every == 16
    assert o.precision == N.FC_PREC_FP32 and o.diag == N.FC_DIAG_UNIT and o.accelerate == 1
    assert o.tol_loss != o.tol_loss  # NaN disables the loss stop by default
    so = N.default_server_options()
    assert so.struct_size == ctypes.sizeof(N.ServerOpts) == 96
    assert list(so.grid_fused) == [0] * 5 and list(so.grid_spmm) == [0] * 5
    assert list(so.spmm_depth) == [0] * 5 and so.solo_max == 4


def test_server_argument_errors_before_device_work(N):
    lib = N.load()
    so = N.default_server_options()
    so.grid_spmm[3] = 65
    h = ctypes.c_void_p()
    assert lib.fc_server_create(ctypes.byref(so), None, ctypes.byref(h)) == N.FC_ERR_INVALID_ARG
    assert b"launch table" in lib.fc_last_error()
    best, rate = N.ServerOpts(), ctypes.c_double()
    assert lib.fc_server_tune(ctypes.byref(N.default_server_options()), 0, None, None, None,
                              N.FC_F32, None, ctypes.byref(best), ctypes.byref(rate),
                              None) == N.FC_ERR_INVALID_ARG


def test_argument_errors_before_device_work(N):
    lib = N.load()
    h = ctypes.c_void_p()
    opt = N.default_options()
    assert lib.fc_create(None, ctypes.byref(opt), None, N.FC_F32, None, ctypes.byref(h)) == \
        N.FC_ERR_INVALID_ARG
    assert b"NULL" in lib.fc_last_error()
    csr = N.CSR(0, 0, None, None, None, N.FC_F32)
    assert lib.fc_create(ctypes.byref(csr), ctypes.byref(opt), None, N.FC_F32, None,
                         ctypes.byref(h)) == N.FC_ERR_INVALID_ARG
    csr = N.CSR(10, 0, 1, None, None, N.FC_F32)   # fake pointer, never dereferenced
    opt.c = 0
    assert lib.fc_create(ctypes.byref(csr), ctypes.byref(opt), None, N.FC_F32, None,
                         ctypes.byref(h)) == N.FC_ERR_INVALID_ARG
    assert b"c must be" in lib.fc_last_error()
    opt.c = 65
    assert lib.fc_create(ctypes.byref(csr), ctypes.byref(opt), None, N.FC_F32, None,
                         ctypes.byref(h)) == N.FC_ERR_INVALID_ARG
    opt.c = 8
    opt.precision = N.FC_PREC_FP64       # FP64 needs FC_F64 values
    assert lib.fc_create(ctypes.byref(csr), ctypes.byref(opt), None, N.FC_F32, None,
                         ctypes.byref(h)) == N.FC_ERR_INVALID_ARG
    bad = N.Options()
    assert lib.fc_create(ctypes.byref(csr), ctypes.byref(bad), None, N.FC_F32, None,
                         ctypes.byref(h)) == N.FC_ERR_INVALID_ARG
    assert b"struct_size" in lib.fc_last_error()
    assert lib.fc_project(None, None, N.FC_F32, 4, 3, 3, None) == N.FC_ERR_INVALID_ARG
    assert lib.fc_project(1, 1, N.FC_F32, 4, 3, 2, None) == N.FC_ERR_INVALID_ARG  # ld < c
    assert lib.fc_project(1, 1, N.FC_F16, 4, 3, 3, None) == N.FC_ERR_INVALID_ARG
    assert lib.fc_spmm(ctypes.byref(csr), N.FC_DIAG_UNIT, 1, 1, N.FC_F32, 0, None) == \
        N.FC_ERR_INVALID_ARG
    f = ctypes.c_double()
    assert lib.fc_objective(ctypes.byref(csr), N.FC_DIAG_UNIT, 1, N.FC_F64, 4, None,
                            ctypes.byref(f)) == N.FC_ERR_INVALID_ARG
    assert lib.fc_gram(None, N.FC_F32, 4, 3, None, None) == N.FC_ERR_INVALID_ARG
    assert lib.fc_step(None, 1, None) == N.FC_ERR_INVALID_ARG
    assert lib.fc_solve(None, None) == N.FC_ERR_INVALID_ARG
    lib.fc_destroy(None)


def test_given_order_errors_before_device_work(N):
    """FC_REORDER_GIVEN: a missing, repeating or out-of-range order is
    rejected by fc_create's host-side checks, naming the first bad entry."""
    lib = N.load()
    h = ctypes.c_void_p()
    csr = N.CSR(10, 0, 1, None, None, N.FC_F32)   # fake pointer, never dereferenced
    opt = N.default_options()
    opt.c = 4
    opt.reorder = N.FC_REORDER_GIVEN
    assert lib.fc_create(ctypes.byref(csr), ctypes.byref(opt), None, N.FC_F32, None,
                         ctypes.byref(h)) == N.FC_ERR_INVALID_ARG
    assert b"perm" in lib.fc_last_error() and not h.value
    for perm, msg in (([0, 1, 2, 3, 4, 5, 6, 7, 8, 8], b"entry 9 repeats"),
                      ([0, 1, 2, 3, 10, 5, 6, 7, 8, 9], b"entry 4 is outside"),
                      ([0, 1, -1, 3, 4, 5, 6, 7, 8, 9], b"entry 2 is outside")):
        arr = (ctypes.c_int32 * 10)(*perm)
        opt.perm = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))
        assert lib.fc_create(ctypes.byref(csr), ctypes.byref(opt), None, N.FC_F32, None,
                             ctypes.byref(h)) == N.FC_ERR_INVALID_ARG
        assert msg in lib.fc_last_error() and not h.value
    opt.reorder = 3
    assert lib.fc_create(ctypes.byref(csr), ctypes.byref(opt), None, N.FC_F32, None,
                         ctypes.byref(h)) == N.FC_ERR_INVALID_ARG
    assert b"reorder" in lib.fc_last_error()


def test_binding_marshals_a_given_order(N):
    import numpy as np
    import torch
    import paper_2506_04045_amd as fc
    for src in ([3, 0, 2, 1], np.array([3, 0, 2, 1], dtype=np.int64), torch.tensor([3, 0, 2, 1])):
        opt = fc._options(2, reorder=src, n=4)
        assert opt.reorder == N.FC_REORDER_GIVEN
        assert [opt.perm[i] for i in range(4)] == [3, 0, 2, 1]
    for bad in ([0, 1, 2], [[0, 1], [2, 3]], [0, 1, 2, -1], [0, 1, 2, 2 ** 31]):
        with pytest.raises(ValueError):
            fc._options(2, reorder=bad, n=4)
    assert fc._options(2, reorder="degree").reorder == N.FC_REORDER_DEGREE
    assert not fc._options(2, reorder="none").perm


def test_product_code_does_not_use_the_oracle():
    pkg = os.path.join(ROOT, "paper_2506_04045_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "fcref" not in text, fn
                assert "from oracle" not in text, fn
    # and the oracle does not use the product
    for fn in os.listdir(os.path.join(ROOT, "oracle")):
        if fn.endswith((".py", ".c")):
            text = open(os.path.join(ROOT, "oracle", fn)).read()
            assert "paper_2506_04045_amd" not in text and "fc_kernels" not in text, fn


def test_binding_fails_loudly_without_the_library(tmp_path, monkeypatch):
    from paper_2506_04045_amd import _native
    monkeypatch.setattr(_native, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_native, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _native.load()


def test_tuner_and_launch_table_arguments_in_the_binding(N):
    import paper_2506_04045_amd as fc
    with pytest.raises(ValueError):
        fc.tune_server([])
    with pytest.raises(ValueError):
        fc._server_options(64, 2.0**30, 8, False, grid_fused=[1, 2, 3])
    o = fc._server_options(64, 2.0**30, 16, False, grid_fused=[1, 2, 4, 2, 1],
                           grid_spmm=[4, 8, 16, 32, 8])
    assert list(o.grid_fused) == [1, 2, 4, 2, 1] and list(o.grid_spmm) == [4, 8, 16, 32, 8]
    assert o.ticks_per_poll == 16 and o.use_graph == 0

"""The C-ABI library loads on the CPU host and exports every declared symbol."""
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def declared_functions():
    src = (ROOT / "include" / "hmle.h").read_text()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(hm_[a-zA-Z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hm_model_create", "hm_sketch_create", "hm_H_create", "hm_build", "hm_factor",
                     "hm_logdet", "hm_solve", "hm_loglik_grad", "hm_fisher", "hm_kapply"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2303_10102_amd import hmle
    if not hmle.LIBPATH.exists():
        pytest.skip("libhmle.so not built")
    L = hmle.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) == set(hmle.exported_symbols())


def test_errors_are_reported_without_a_device():
    from paper_2303_10102_amd import hmle
    if not hmle.LIBPATH.exists():
        pytest.skip("libhmle.so not built")
    import ctypes as C
    L = hmle.lib()
    out = C.c_void_p()
    # invalid arguments are rejected before any device call
    assert L.hm_model_create(0, None, 3, 16, 4, C.byref(out)) == 1
    assert b"dim" in L.hm_last_error()
    assert L.hm_model_create(0, None, 2, 15, 200, C.byref(out)) == 1   # leaf larger than half the grid
    assert L.hm_factor(None) == 1


def test_context_and_model_arguments_are_checked_without_a_device():
    from paper_2303_10102_amd import hmle
    if not hmle.LIBPATH.exists():
        pytest.skip("libhmle.so not built")
    import ctypes as C
    L = hmle.lib()
    out = C.c_void_p()
    cb = hmle._ALLOC_FN(lambda u, n: None)
    # one allocator callback without the other
    assert L.hm_ctx_create(0, None, C.cast(cb, C.c_void_p), None, None, C.byref(out)) == 1
    assert b"both" in L.hm_last_error()
    # a model needs a context
    assert L.hm_model_create_spde(None, 2, 16, 16, 1.0 / 17, 1, None, 0, 16, C.byref(out)) == 1
    # a solve needs a handle; statistics need a handle
    assert L.hm_solve(None, None, None, 0, 0) == 1
    assert L.hm_stats(None, None, 0) == 1
    assert L.hm_grad_reverse(None, None) == 1


def test_observation_selection_is_checked_without_a_device():
    from paper_2303_10102_amd import hmle
    if not hmle.LIBPATH.exists():
        pytest.skip("libhmle.so not built")
    import ctypes as C
    L = hmle.lib()
    out = C.c_void_p()
    ctx = C.c_void_p(1)          # never dereferenced: the selection is rejected first
    bad = [((C.c_int * 3)(0, 5, 5), 3, b"repeated"), ((C.c_int * 3)(0, 5, 256), 3, b"outside"),
           ((C.c_int * 3)(0, 5, -1), 3, b"outside"), ((C.c_int * 1)(0), 1, b"nobs")]
    for idx, nobs, msg in bad:
        assert L.hm_model_create_spde(ctx, 2, 16, 16, 1.0 / 17, 1, idx, nobs, 4, C.byref(out)) == 1
        assert msg in L.hm_last_error(), L.hm_last_error()
    # an index array without a count
    assert L.hm_model_create_spde(ctx, 2, 16, 16, 1.0 / 17, 1, (C.c_int * 2)(0, 1), 0, 4, C.byref(out)) == 1

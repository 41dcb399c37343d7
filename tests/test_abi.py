"""Host-side checks of the C ABI: the built library loads, exports every
function declared in include/evd.h, and validates arguments before touching
a device (validation-only context, device = -1)."""
import ctypes
import os
import re

import pytest

from paper_2511_16174_amd import evd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "evd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(evd_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(evd.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    # the binding declares prototypes for exactly the header's functions
    assert sorted(evd.PROTOTYPES) == names


def test_no_cpu_fallback_symbols():
    """The product library must not contain the oracle."""
    lib = ctypes.CDLL(evd.LIB_PATH)
    for name in ("oracle_syev", "oracle_ql", "oracle_tridiag"):
        assert not hasattr(lib, name)


@pytest.fixture()
def vctx():
    lib = evd.load_library()
    h = ctypes.c_void_p()
    assert lib.evd_create(ctypes.byref(h), -1) == evd.EVD_OK
    yield lib, h
    lib.evd_destroy(h)


def test_status_strings():
    lib = evd.load_library()
    assert lib.evd_status_string(0) == b"ok"
    assert lib.evd_status_string(1) == b"invalid argument"


def test_params(vctx):
    lib, h = vctx
    assert lib.evd_set_param(h, b"b", 32) == evd.EVD_OK
    v = ctypes.c_int64()
    assert lib.evd_get_param(h, b"b", ctypes.byref(v)) == evd.EVD_OK and v.value == 32
    assert lib.evd_set_param(h, b"nonsense", 1) == evd.EVD_ERR_INVALID_ARG
    assert lib.evd_last_invalid_arg(h) == 2
    assert lib.evd_set_param(h, b"b", -1) == evd.EVD_ERR_INVALID_ARG
    assert lib.evd_last_invalid_arg(h) == 3


@pytest.mark.parametrize("args,bad", [
    ((b"X", b"N", 0, 4, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4), 2),
    ((b"N", b"S", 0, 4, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4), 3),
    ((b"N", b"N", 0, -1, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4), 5),
    ((b"N", b"N", 0, 4, 4, 4, 1.0, 8, 3, 8, 4, 0.0, 8, 4), 10),
    ((b"N", b"N", 0, 4, 4, 4, 1.0, 8, 4, 8, 3, 0.0, 8, 4), 12),
    ((b"N", b"N", 0, 4, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 2), 15),
    ((b"S", b"N", 0, 4, 4, 5, 1.0, 8, 4, 8, 5, 0.0, 8, 4), 7),
    ((b"N", b"N", 1, 4, 5, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4), 4),
])
def test_dgemm_argument_checks(vctx, args, bad):
    lib, h = vctx
    opa, opb, low, m, n, k, al, A, lda, B, ldb, be, C, ldc = args
    st = lib.evd_dgemm(h, opa, opb, low, m, n, k, al, A, lda, B, ldb, be, C, ldc, None, 0)
    assert st == evd.EVD_ERR_INVALID_ARG
    assert lib.evd_last_invalid_arg(h) == bad


def test_dgemm_valid_args_reach_device_check(vctx):
    lib, h = vctx
    st = lib.evd_dgemm(h, b"N", b"T", 0, 4, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4, None, 0)
    assert st == evd.EVD_ERR_HIP  # validation passed; no device in this context

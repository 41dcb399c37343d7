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
    for key, good, bad in ((b"bcback_group", (0, 32, 64), (16, 48)), (b"bcback_rows", (0, 64, 128), (32, 96)),
                           (b"bcback_sub", (0, 16, 32, 64), (8, 48)), (b"bcback_rt", (0, 1, 2), (3, 4)),
                           (b"gemm_staged", (0, 1), (2, 5)), (b"bcback_lds2", (0, 1), (2, 3)),
                           (b"panel_generic", (0, 1), (2, 3))):
        for v in good:
            assert lib.evd_set_param(h, key, v) == evd.EVD_OK
        for v in bad:
            assert lib.evd_set_param(h, key, v) == evd.EVD_ERR_INVALID_ARG
            assert lib.evd_last_invalid_arg(h) == 3
        assert lib.evd_set_param(h, key, 0) == evd.EVD_OK


def test_bcback_work_size_and_argument_checks(vctx):
    """The blocked BC-back needs T-factor scratch only for b = 16, 32, 64;
    a short workspace is reported as such, before any device work."""
    lib, h = vctx
    sz = ctypes.c_size_t()
    for b, blocked in ((4, False), (8, False), (16, True), (32, True), (64, True)):
        assert lib.evd_dbcback_work_size(h, 300, b, ctypes.byref(sz)) == evd.EVD_OK
        assert (sz.value > 0) == blocked
    assert lib.evd_dbcback_work_size(h, 300, 48, ctypes.byref(sz)) == evd.EVD_ERR_INVALID_ARG
    lib.evd_dbcback_work_size(h, 300, 64, ctypes.byref(sz))
    need = sz.value
    p = ctypes.c_void_p(256)  # never dereferenced: the checks fail first, or the context has no device
    assert lib.evd_dbcback(h, b"X", 10, 300, 64, p, p, p, 10, p, need) == evd.EVD_ERR_INVALID_ARG
    assert lib.evd_last_invalid_arg(h) == 2
    assert lib.evd_dbcback(h, b"T", 10, 300, 64, p, p, p, 9, p, need) == evd.EVD_ERR_INVALID_ARG
    assert lib.evd_last_invalid_arg(h) == 9
    assert lib.evd_dbcback(h, b"N", 10, 300, 64, p, p, p, 10, None, need) == evd.EVD_ERR_INVALID_ARG
    assert lib.evd_last_invalid_arg(h) == 10
    assert lib.evd_dbcback(h, b"N", 10, 300, 64, p, p, p, 10, p, need - 8) == evd.EVD_ERR_WORKSPACE
    assert lib.evd_last_invalid_arg(h) == 11
    assert lib.evd_dbcback(h, b"N", 10, 300, 64, p, p, p, 10, p, need) == evd.EVD_ERR_HIP  # validation-only context


@pytest.mark.parametrize("args,bad", [
    ((b"X", b"N", 0, 4, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4), 2),
    ((b"N", b"S", 0, 4, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4), 3),
    ((b"N", b"N", 0, -1, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4), 5),
    ((b"N", b"N", 0, 4, 4, 4, 1.0, 8, 3, 8, 4, 0.0, 8, 4), 10),
    ((b"N", b"N", 0, 4, 4, 4, 1.0, 8, 4, 8, 3, 0.0, 8, 4), 12),
    ((b"N", b"N", 0, 4, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 2), 15),
    ((b"S", b"N", 0, 4, 4, 5, 1.0, 8, 4, 8, 5, 0.0, 8, 4), 7),
    ((b"N", b"N", 1, 4, 5, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4), 4),
    ((b"N", b"N", 2, 4, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4), 4),   # mirrored lower mode needs op(B) = B^T
    ((b"T", b"T", 2, 4, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4), 4),
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


def test_defaults_and_failure_knobs(vctx):
    """The conventional stage order is the default; the D&C iteration cap
    (failure-path knob) is a settable parameter."""
    lib, h = vctx
    v = ctypes.c_int64()
    assert lib.evd_get_param(h, b"order", ctypes.byref(v)) == evd.EVD_OK and v.value == 1
    assert lib.evd_set_param(h, b"dc_max_iter", 1) == evd.EVD_OK
    assert lib.evd_get_param(h, b"dc_max_iter", ctypes.byref(v)) == evd.EVD_OK and v.value == 1
    assert lib.evd_set_param(h, b"dc_max_iter", 0) == evd.EVD_OK
    assert lib.evd_status_string(evd.EVD_ERR_NONFINITE) == b"non-finite input"
    assert lib.evd_status_string(evd.EVD_ERR_NOT_CONVERGED) == b"not converged"


def test_device_status_word_maps_to_errors():
    evd.raise_for_info("f", 0)
    for info, status in ((evd.EVD_ERR_NONFINITE, evd.EVD_ERR_NONFINITE),
                         (evd.EVD_ERR_NOT_CONVERGED, evd.EVD_ERR_NOT_CONVERGED), (1, evd.EVD_ERR_NOT_CONVERGED)):
        with pytest.raises(evd.EvdError) as e:
            evd.raise_for_info("f", info)
        assert e.value.status == status and e.value.arg == info


def test_mixed_argument_checks(vctx):
    """max_sweeps in 0..8, target_residual not NaN, workspace size: reported
    on the host before any device work."""
    lib, h = vctx
    d = ctypes.c_double
    args = lambda sweeps, target, wb: (h, b"V", b"L", ctypes.c_int64(10), ctypes.c_void_p(256), ctypes.c_int64(10),
                                       ctypes.c_void_p(256), ctypes.c_int(sweeps), d(target), ctypes.c_void_p(256),
                                       ctypes.c_size_t(wb), ctypes.c_void_p(256), None)
    sz = ctypes.c_size_t()
    assert lib.evd_dsyevd_mixed_work_size(h, b"V", b"L", ctypes.c_int64(10), ctypes.c_int64(10),
                                          ctypes.byref(sz)) == evd.EVD_OK
    assert lib.evd_dsyevd_mixed(*args(9, 0.0, sz.value)) == evd.EVD_ERR_INVALID_ARG
    assert lib.evd_last_invalid_arg(h) == 8
    assert lib.evd_dsyevd_mixed(*args(2, float("nan"), sz.value)) == evd.EVD_ERR_INVALID_ARG
    assert lib.evd_last_invalid_arg(h) == 9
    assert lib.evd_dsyevd_mixed(*args(2, 1e-13, sz.value - 1)) == evd.EVD_ERR_WORKSPACE
    assert lib.evd_last_invalid_arg(h) == 11


def test_size_limits(vctx):
    """n and lda above EVD_MAX_N (2^21: the tile loaders keep byte offsets in
    32 bits) are rejected on the host, before any device work; the largest
    sizes that fit in 288 GB (n = 98304, eigenvalues only) are accepted."""
    lib, h = vctx
    sz = ctypes.c_size_t()
    big = (1 << 21) + 1
    assert lib.evd_dsyevd_work_size(h, b"N", b"L", big, big, ctypes.byref(sz)) == evd.EVD_ERR_INVALID_ARG
    assert lib.evd_last_invalid_arg(h) == 4
    assert lib.evd_dsyevd_work_size(h, b"N", b"L", 1000, big, ctypes.byref(sz)) == evd.EVD_ERR_INVALID_ARG
    assert lib.evd_last_invalid_arg(h) == 5
    assert lib.evd_dsyevd_work_size(h, b"N", b"L", 98304, 98304, ctypes.byref(sz)) == evd.EVD_OK
    assert sz.value < 8 * 2**30          # eigenvalues only: O(n b) scratch besides A
    assert lib.evd_dsyevd_work_size(h, b"V", b"L", 98304, 98304, ctypes.byref(sz)) == evd.EVD_OK
    assert sz.value > 288 * 10**9        # with vectors it would not fit one GPU

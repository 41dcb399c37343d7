"""ctypes binding of ``libevd.so`` (C ABI in ``include/evd.h``).

Argument marshalling only: every step of the computation runs in the HIP
library.  Entry points keep their C names.  Device buffers are passed as
torch CUDA(HIP) tensors or raw integer addresses; the stream is torch's
current stream unless one is given.  If the library is missing this module
raises ImportError-like ``RuntimeError`` -- there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libevd.so")

EVD_OK = 0
EVD_ERR_INVALID_ARG = 1
EVD_ERR_WORKSPACE = 2
EVD_ERR_HIP = 3
EVD_ERR_NONFINITE = 4
EVD_ERR_NOT_CONVERGED = 5
EVD_ERR_NOT_IMPLEMENTED = 6
EVD_ERR_TIMEOUT = 7

_i64, _i32, _sz, _d, _c, _vp = (ctypes.c_int64, ctypes.c_int, ctypes.c_size_t, ctypes.c_double,
                                 ctypes.c_char, ctypes.c_void_p)
_st = ctypes.c_int  # evd_status_t

# name -> (restype, argtypes), in the order of include/evd.h
PROTOTYPES = {
    "evd_create": (_st, [ctypes.POINTER(_vp), _i32]),
    "evd_destroy": (_st, [_vp]),
    "evd_set_stream": (_st, [_vp, _vp]),
    "evd_set_param": (_st, [_vp, ctypes.c_char_p, _i64]),
    "evd_get_param": (_st, [_vp, ctypes.c_char_p, ctypes.POINTER(_i64)]),
    "evd_last_invalid_arg": (_i32, [_vp]),
    "evd_status_string": (ctypes.c_char_p, [_st]),
    "evd_get_stage_times": (_st, [_vp, ctypes.POINTER(ctypes.c_float)]),
    "evd_dgemm": (_st, [_vp, _c, _c, _i32, _i64, _i64, _i64, _d, _vp, _i64, _vp, _i64, _d, _vp, _i64, _vp, _sz]),
    "evd_dgemm_work_size": (_st, [_vp, _i64, _i64, _i64, ctypes.POINTER(_sz)]),
    "evd_sgemm_x3": (_st, [_vp, _c, _c, _i32, _i64, _i64, _i64, ctypes.c_float, _vp, _i64, _vp, _i64,
                           ctypes.c_float, _vp, _i64, _vp, _sz]),
    "evd_sgemm_x3_work_size": (_st, [_vp, _i64, _i64, _i64, ctypes.POINTER(_sz)]),
    "evd_dsyevd_work_size": (_st, [_vp, _c, _c, _i64, _i64, ctypes.POINTER(_sz)]),
    "evd_dsyevd": (_st, [_vp, _c, _c, _i64, _vp, _i64, _vp, _vp, _sz, _vp]),
    "evd_dsyevd_noalloc": (_st, [_vp, _c, _c, _i64, _vp, _i64, _vp, _vp]),
    "evd_dsyevd_mixed_work_size": (_st, [_vp, _c, _c, _i64, _i64, ctypes.POINTER(_sz)]),
    "evd_dsyevd_mixed": (_st, [_vp, _c, _c, _i64, _vp, _i64, _vp, _i32, _d, _vp, _sz, _vp, _vp]),
    "evd_autotune_work_size": (_st, [_vp, _c, _i64, ctypes.POINTER(_sz)]),
    "evd_autotune": (_st, [_vp, _c, _i64, _vp, _i64, _vp, _sz, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_float)]),
    "evd_dsyevd_batched_work_size": (_st, [_vp, _c, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                                           ctypes.POINTER(_sz)]),
    "evd_dsyevd_batched": (_st, [_vp, _c, _c, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_vp),
                                 ctypes.POINTER(_i64), ctypes.POINTER(_vp), _vp, _sz, _vp, _vp]),
    "evd_sbr_num_panels": (_i64, [_i64, _i64]),
    "evd_dsy2sb_work_size": (_st, [_vp, _i64, _i64, ctypes.POINTER(_sz)]),
    "evd_dsy2sb": (_st, [_vp, _c, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _sz]),
    "evd_bc_num_steps": (_i64, [_i64, _i64]),
    "evd_dsb2st_work_size": (_st, [_vp, _i64, ctypes.POINTER(_sz)]),
    "evd_dsb2st": (_st, [_vp, _c, _i64, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _sz]),
    "evd_dstedc_work_size": (_st, [_vp, _c, _i64, ctypes.POINTER(_sz)]),
    "evd_dstedc": (_st, [_vp, _c, _i64, _vp, _vp, _vp, _vp, _i64, _vp, _sz, _vp]),
    "evd_dstedc_host": (_st, [_c, _i64, _vp, _vp, _vp, _vp, _i64, _i32, _vp]),
    "evd_dorgsb_work_size": (_st, [_vp, _i64, _i64, ctypes.POINTER(_sz)]),
    "evd_dorgsb": (_st, [_vp, _i64, _i64, _vp, _i64, _vp, _vp, _i64, _vp, _sz]),
    "evd_dbcback_work_size": (_st, [_vp, _i64, _i64, _vp]),
    "evd_dbcback": (_st, [_vp, _c, _i64, _i64, _i64, _vp, _vp, _vp, _i64, _vp, _sz]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load ``libevd.so`` and attach prototypes; raises if absent or incomplete."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run __graft_entry__.build())")
    # torch ships its own HIP runtime under the same soname as the system one;
    # importing torch first makes this library bind to torch's copy, so the
    # streams and device memory torch hands out belong to the same runtime
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)  # AttributeError if a declared symbol is missing
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class EvdError(RuntimeError):
    def __init__(self, func, status, arg=0):
        lib = load_library()
        msg = lib.evd_status_string(status).decode()
        super().__init__(f"{func}: {msg} (status {status}, argument {arg})")
        self.status = status
        self.arg = arg


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _ch(c: str) -> bytes:
    return c.encode()[:1]


_live_contexts = weakref.WeakSet()


class Context:
    """Owns one ``evd_ctx_t``.  The stream defaults to torch's current stream.

    Every live context is closed by an ``atexit`` hook, i.e. while the HIP
    runtime (and any profiler attached to it) is still up: a context owns
    streams, events and possibly an instantiated graph, and destroying those
    from a finaliser during interpreter teardown would call into a runtime
    that is already being torn down."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        h = _vp()
        st = self.lib.evd_create(ctypes.byref(h), device)
        if st != EVD_OK:
            raise EvdError("evd_create", st)
        self.handle = h
        self.device = device
        _live_contexts.add(self)

    def close(self):
        if self.handle:
            self.lib.evd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers
    def _check(self, name, st):
        if st != EVD_OK:
            raise EvdError(name, st, self.lib.evd_last_invalid_arg(self.handle))

    def set_stream(self, stream=None):
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(self.device).cuda_stream
        self._check("evd_set_stream", self.lib.evd_set_stream(self.handle, stream))

    def set_param(self, key: str, value: int):
        self._check("evd_set_param", self.lib.evd_set_param(self.handle, key.encode(), int(value)))

    def get_param(self, key: str) -> int:
        v = _i64()
        self._check("evd_get_param", self.lib.evd_get_param(self.handle, key.encode(), ctypes.byref(v)))
        return v.value

    def stage_times(self):
        arr = (ctypes.c_float * 8)()
        self._check("evd_get_stage_times", self.lib.evd_get_stage_times(self.handle, arr))
        return list(arr)

    # -- entry points (same names as the C ABI)
    def evd_dgemm(self, opa, opb, lower_c, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, work=None, work_bytes=0):
        self.set_stream()
        st = self.lib.evd_dgemm(self.handle, _ch(opa), _ch(opb), int(lower_c), m, n, k, alpha, _ptr(A), lda,
                                _ptr(B), ldb, beta, _ptr(C), ldc, _ptr(work), work_bytes)
        self._check("evd_dgemm", st)

    def evd_dgemm_work_size(self, m, n, k) -> int:
        b = _sz()
        self._check("evd_dgemm_work_size", self.lib.evd_dgemm_work_size(self.handle, m, n, k, ctypes.byref(b)))
        return b.value

    def evd_sgemm_x3(self, opa, opb, lower_c, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, work=None,
                     work_bytes=0):
        self.set_stream()
        st = self.lib.evd_sgemm_x3(self.handle, _ch(opa), _ch(opb), int(lower_c), m, n, k, alpha, _ptr(A), lda,
                                   _ptr(B), ldb, beta, _ptr(C), ldc, _ptr(work), work_bytes)
        self._check("evd_sgemm_x3", st)

    def evd_sgemm_x3_work_size(self, m, n, k) -> int:
        b = _sz()
        self._check("evd_sgemm_x3_work_size", self.lib.evd_sgemm_x3_work_size(self.handle, m, n, k,
                                                                              ctypes.byref(b)))
        return b.value

    def evd_dsyevd_work_size(self, jobz, uplo, n, lda) -> int:
        b = _sz()
        st = self.lib.evd_dsyevd_work_size(self.handle, _ch(jobz), _ch(uplo), n, lda, ctypes.byref(b))
        self._check("evd_dsyevd_work_size", st)
        return b.value

    def evd_dsyevd(self, jobz, uplo, n, A, lda, W, work, work_bytes, info):
        self.set_stream()
        st = self.lib.evd_dsyevd(self.handle, _ch(jobz), _ch(uplo), n, _ptr(A), lda, _ptr(W), _ptr(work),
                                 work_bytes, _ptr(info))
        self._check("evd_dsyevd", st)

    def evd_dsyevd_noalloc(self, jobz, uplo, n, A, lda, W, info):
        self.set_stream()
        st = self.lib.evd_dsyevd_noalloc(self.handle, _ch(jobz), _ch(uplo), n, _ptr(A), lda, _ptr(W), _ptr(info))
        self._check("evd_dsyevd_noalloc", st)

    def evd_dsyevd_mixed_work_size(self, jobz, uplo, n, lda) -> int:
        b = _sz()
        st = self.lib.evd_dsyevd_mixed_work_size(self.handle, _ch(jobz), _ch(uplo), n, lda, ctypes.byref(b))
        self._check("evd_dsyevd_mixed_work_size", st)
        return b.value

    def evd_dsyevd_mixed(self, jobz, uplo, n, A, lda, W, max_sweeps, target_residual, work, work_bytes, info,
                         achieved=None):
        self.set_stream()
        st = self.lib.evd_dsyevd_mixed(self.handle, _ch(jobz), _ch(uplo), n, _ptr(A), lda, _ptr(W),
                                       int(max_sweeps), float(target_residual), _ptr(work), work_bytes, _ptr(info),
                                       _ptr(achieved))
        self._check("evd_dsyevd_mixed", st)

    def evd_autotune_work_size(self, jobz, n) -> int:
        b = _sz()
        self._check("evd_autotune_work_size", self.lib.evd_autotune_work_size(self.handle, _ch(jobz), n,
                                                                              ctypes.byref(b)))
        return b.value

    def evd_autotune(self, jobz, n, A, lda, work, work_bytes):
        self.set_stream()
        bb, ms = _i64(), ctypes.c_float()
        st = self.lib.evd_autotune(self.handle, _ch(jobz), n, _ptr(A), lda, _ptr(work), work_bytes,
                                   ctypes.byref(bb), ctypes.byref(ms))
        self._check("evd_autotune", st)
        return bb.value, ms.value

    def evd_dsyevd_batched_work_size(self, jobz, ns, ldas) -> int:
        k = len(ns)
        na, la = (_i64 * max(k, 1))(*ns), (_i64 * max(k, 1))(*ldas)
        b = _sz()
        st = self.lib.evd_dsyevd_batched_work_size(self.handle, _ch(jobz), k, na, la, ctypes.byref(b))
        self._check("evd_dsyevd_batched_work_size", st)
        return b.value

    def evd_dsyevd_batched(self, jobz, uplo, ns, As, ldas, Ws, work, work_bytes, info, stamps=None):
        self.set_stream()
        k = len(ns)
        na, la = (_i64 * max(k, 1))(*ns), (_i64 * max(k, 1))(*ldas)
        ap = (_vp * max(k, 1))(*[_ptr(a) for a in As])
        wp = (_vp * max(k, 1))(*[_ptr(w) for w in Ws])
        st = self.lib.evd_dsyevd_batched(self.handle, _ch(jobz), _ch(uplo), k, na, ap, la, wp, _ptr(work),
                                         work_bytes, _ptr(info), _ptr(stamps))
        self._check("evd_dsyevd_batched", st)

    def evd_dsy2sb_work_size(self, n, b) -> int:
        s = _sz()
        self._check("evd_dsy2sb_work_size", self.lib.evd_dsy2sb_work_size(self.handle, n, b, ctypes.byref(s)))
        return s.value

    def evd_dsy2sb(self, uplo, n, b, A, lda, AB, ldab, T, work, work_bytes):
        self.set_stream()
        st = self.lib.evd_dsy2sb(self.handle, _ch(uplo), n, b, _ptr(A), lda, _ptr(AB), ldab, _ptr(T),
                                 _ptr(work), work_bytes)
        self._check("evd_dsy2sb", st)

    def evd_dsb2st_work_size(self, n) -> int:
        s = _sz()
        self._check("evd_dsb2st_work_size", self.lib.evd_dsb2st_work_size(self.handle, n, ctypes.byref(s)))
        return s.value

    def evd_dsb2st(self, jobz, n, b, AB, ldab, d, e, V, TAU, work, work_bytes):
        self.set_stream()
        st = self.lib.evd_dsb2st(self.handle, _ch(jobz), n, b, _ptr(AB), ldab, _ptr(d), _ptr(e), _ptr(V),
                                 _ptr(TAU), _ptr(work), work_bytes)
        self._check("evd_dsb2st", st)

    def evd_dstedc_work_size(self, compz, n) -> int:
        s = _sz()
        self._check("evd_dstedc_work_size", self.lib.evd_dstedc_work_size(self.handle, _ch(compz), n,
                                                                          ctypes.byref(s)))
        return s.value

    def evd_dstedc(self, compz, n, d, e, W, Z, ldz, work, work_bytes, info):
        self.set_stream()
        st = self.lib.evd_dstedc(self.handle, _ch(compz), n, _ptr(d), _ptr(e), _ptr(W), _ptr(Z), ldz,
                                 _ptr(work), work_bytes, _ptr(info))
        self._check("evd_dstedc", st)

    def evd_dorgsb_work_size(self, n, b) -> int:
        s = _sz()
        self._check("evd_dorgsb_work_size", self.lib.evd_dorgsb_work_size(self.handle, n, b, ctypes.byref(s)))
        return s.value

    def evd_dorgsb(self, n, b, A, lda, T, Q, ldq, work, work_bytes):
        self.set_stream()
        st = self.lib.evd_dorgsb(self.handle, n, b, _ptr(A), lda, _ptr(T), _ptr(Q), ldq, _ptr(work), work_bytes)
        self._check("evd_dorgsb", st)

    def evd_dbcback_work_size(self, n, b) -> int:
        s = _sz()
        self._check("evd_dbcback_work_size", self.lib.evd_dbcback_work_size(self.handle, n, b, ctypes.byref(s)))
        return s.value

    def evd_dbcback(self, trans, m_rows, n, b, V, TAU, Q, ldq, work, work_bytes):
        self.set_stream()
        st = self.lib.evd_dbcback(self.handle, trans.encode(), m_rows, n, b, _ptr(V), _ptr(TAU), _ptr(Q), ldq,
                                  _ptr(work), work_bytes)
        self._check("evd_dbcback", st)


def evd_sbr_num_panels(n: int, b: int) -> int:
    return int(load_library().evd_sbr_num_panels(n, b))


def evd_bc_num_steps(n: int, b: int) -> int:
    return int(load_library().evd_bc_num_steps(n, b))


def raise_for_info(func: str, info: int):
    """Raise EvdError for a nonzero device status word (an evd_status_t:
    EVD_ERR_NONFINITE or EVD_ERR_NOT_CONVERGED)."""
    if info != 0:
        status = info if info in (EVD_ERR_NONFINITE, EVD_ERR_NOT_CONVERGED, EVD_ERR_TIMEOUT) else EVD_ERR_NOT_CONVERGED
        raise EvdError(func, status, info)


_default_ctx = {}


@atexit.register
def close_all():
    """Destroy every live context (registered with ``atexit``)."""
    _default_ctx.clear()
    for ctx in list(_live_contexts):
        try:
            ctx.close()
        except Exception:
            pass


def context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def eigh_mixed(A, sweeps: int = 3, target: float = 0.0, uplo: str = "L", b: int = 0, ctx: Context | None = None,
               check: bool = True):
    """``evd_dsyevd_mixed`` on a float64 GPU tensor: returns (w, Q, achieved)
    -- at most ``sweeps`` refinement sweeps, stopping early once the scaled
    residual and orthogonality reach ``target`` (> 0)."""
    import torch

    n = A.shape[0]
    ctx = ctx or context(A.device.index or 0)
    ctx.set_param("b", b)  # 0 = automatic
    Acm = A.t().contiguous().t()
    Acm = Acm.clone() if Acm.data_ptr() == A.data_ptr() else Acm
    W = torch.empty(max(n, 1), dtype=torch.float64, device=A.device)
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    stats = torch.zeros(8, dtype=torch.float64, device=A.device)
    wb = ctx.evd_dsyevd_mixed_work_size("V", uplo, n, max(n, 1))
    work = torch.empty(max(wb, 256) // 8 + 32, dtype=torch.float64, device=A.device)
    ctx.evd_dsyevd_mixed("V", uplo, n, Acm, max(n, 1), W, sweeps, target, work, wb, info, stats)
    if check:
        raise_for_info("evd_dsyevd_mixed", int(info.item()))
    return W[:n], Acm, stats


def eigh(A, jobz: str = "V", uplo: str = "L", b: int = 0, ctx: Context | None = None):
    """Convenience wrapper over ``evd_dsyevd`` for a torch float64 CUDA(HIP)
    tensor A (n x n).  Buffers are allocated with torch (memory plumbing only);
    A is not modified.  Returns ``w`` or ``(w, Q)`` as torch tensors
    (Q column i pairs with w[i])."""
    import torch

    if not (isinstance(A, torch.Tensor) and A.is_cuda and A.dtype == torch.float64 and A.dim() == 2):
        raise TypeError("eigh expects a float64 GPU tensor of shape (n, n)")
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("A must be square")
    ctx = ctx or context(A.device.index or 0)
    ctx.set_param("b", b)  # 0 = automatic
    # column-major copy: the transpose of a contiguous row-major tensor
    Acm = A.t().contiguous().t() if n > 0 else A.clone()
    Acm = Acm.clone() if Acm.data_ptr() == A.data_ptr() else Acm
    W = torch.empty(max(n, 1), dtype=torch.float64, device=A.device)
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    wb = ctx.evd_dsyevd_work_size(jobz, uplo, n, max(n, 1))
    work = torch.empty(max(wb, 256) // 8 + 32, dtype=torch.float64, device=A.device)
    ctx.evd_dsyevd(jobz, uplo, n, Acm, max(n, 1), W, work, wb, info)
    raise_for_info("evd_dsyevd", int(info.item()))
    w = W[:n]
    if jobz.upper() == "V":
        return w, Acm
    return w

"""ctypes binding of libqrx.so (the C ABI declared in include/qrx.h).

Argument marshalling only: every step of the factorisation and of the
least-squares iteration runs in the HIP kernels of the library. Loading fails
loudly when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqrx.so")

QRX_OK, QRX_EINVAL, QRX_ENOMEM, QRX_EHIP = 0, -1, -2, -3
QRX_ESINGULAR, QRX_ENONFINITE, QRX_ENOCONV, QRX_ESYNC = 1, 2, 3, 4
QRX_NOALLOC_SCRATCH_BYTES = 64 << 20   # the static workspace of qrx_qr_factor_noalloc
QRX_FP32, QRX_FP16, QRX_BF16, QRX_FP16X3 = 0, 1, 2, 3
PREC = {"fp32": QRX_FP32, "fp16": QRX_FP16, "bf16": QRX_BF16, "fp16x3": QRX_FP16X3}


class qrx_qr_opts(C.Structure):
    _fields_ = [("gemm_prec", C.c_int), ("panel_width", C.c_int), ("cutoff", C.c_int),
                ("block_rows", C.c_int), ("no_col_scaling", C.c_int),
                ("panel_single_pass", C.c_int), ("panel_alg", C.c_int),
                ("node_reorth", C.c_int), ("gemm_tiles", C.c_int), ("split_target", C.c_int),
                ("q_reorth", C.c_int)]


class qrx_lls_opts(C.Structure):
    _fields_ = [("qr", qrx_qr_opts), ("method", C.c_int), ("tol", C.c_double),
                ("max_iter", C.c_int), ("use_x0", C.c_int), ("zero_start", C.c_int)]


class qrx_lls_info(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int), ("restarts", C.c_int),
                ("accepted", C.c_int), ("eta_F", C.c_double), ("resid_norm", C.c_double),
                ("normA_F", C.c_double), ("eta_start", C.c_double), ("score", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class qrx_tune_result(C.Structure):
    _fields_ = [("panel_width", C.c_int), ("cutoff", C.c_int), ("gemm_tiles", C.c_int),
                ("split_target", C.c_int), ("ms", C.c_double), ("trials", C.c_int),
                ("from_cache", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class qrx_kernel_stat(C.Structure):
    _fields_ = [("name", C.c_char * 40), ("launches", C.c_int64), ("total_ms", C.c_double),
                ("flops", C.c_double), ("bytes", C.c_double)]


_lib = None

_P = C.c_void_p
_I64 = C.c_int64
_SIGS = {
    "qrx_create": (C.c_int, [C.POINTER(_P), C.c_int]),
    "qrx_destroy": (C.c_int, [_P]),
    "qrx_status_string": (C.c_char_p, [C.c_int]),
    "qrx_qr_workspace_size": (C.c_int, [_P, _I64, _I64, C.POINTER(qrx_qr_opts), C.POINTER(C.c_size_t)]),
    "qrx_qr_factor": (C.c_int, [_P, _I64, _I64, _P, _I64, _P, _I64, _P, C.c_size_t,
                                C.POINTER(qrx_qr_opts), _P, _P]),
    "qrx_qr_factor_noalloc": (C.c_int, [_P, _I64, _I64, _P, _I64, _P, _I64,
                                        C.POINTER(qrx_qr_opts), _P, _P]),
    "qrx_qr_factor_out": (C.c_int, [_P, _I64, _I64, _P, _I64, _P, _I64, _P, _I64, _P, C.c_size_t,
                                    C.POINTER(qrx_qr_opts), _P, _P]),
    "qrx_lls_workspace_size": (C.c_int, [_P, _I64, _I64, C.POINTER(qrx_lls_opts), C.POINTER(C.c_size_t)]),
    # info is a device pointer (qrx_lls_info written by the device)
    "qrx_lls_solve": (C.c_int, [_P, _I64, _I64, _P, _I64, _P, _P, _P, C.c_size_t,
                                C.POINTER(qrx_lls_opts), _P, _P]),
    "qrx_lls_solve_with_R": (C.c_int, [_P, _I64, _I64, _P, _I64, _P, _I64, _P, _P, _P, C.c_size_t,
                                       C.POINTER(qrx_lls_opts), _P, _P]),
    # batched: a host-built plan, then device descriptor arrays
    "qrx_batch_plan_create": (C.c_int, [_P, C.c_int, _P, _P, _P, _P, C.POINTER(qrx_lls_opts),
                                        C.c_int, C.POINTER(_P)]),
    "qrx_batch_plan_workspace_size": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "qrx_batch_plan_destroy": (C.c_int, [_P]),
    "qrx_qr_factor_batched": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, C.c_size_t, _P, _P]),
    "qrx_lls_solve_batched": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, C.c_size_t, _P, _P]),
    "qrx_tune": (C.c_int, [_P, _I64, _I64, _P, _I64, C.POINTER(qrx_qr_opts), C.c_int, C.c_char_p,
                           C.POINTER(qrx_tune_result), _P]),
    "qrx_tune_batched": (C.c_int, [_P, C.c_int, _P, _P, _P, _P, C.POINTER(qrx_qr_opts), C.c_int,
                                   C.c_char_p, _P, _P, C.POINTER(qrx_tune_result), _P]),
    "qrx_tune_key": (C.c_int, [C.c_char_p, _I64, _I64, C.c_int, C.c_int, C.c_char_p, C.c_size_t]),
    "qrx_tune_cache_get": (C.c_int, [C.c_char_p, C.c_char_p, C.POINTER(qrx_tune_result)]),
    "qrx_tune_cache_put": (C.c_int, [C.c_char_p, C.c_char_p, C.POINTER(qrx_tune_result)]),
    "qrx_timing_enable": (C.c_int, [_P, C.c_int]),
    "qrx_timing_reset": (C.c_int, [_P]),
    "qrx_timing_get": (C.c_int, [_P, C.POINTER(qrx_kernel_stat), C.c_int, C.POINTER(C.c_int)]),
}


def load():
    """Load libqrx.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def __getattr__(name):
    # qrx_* names resolve to the raw C functions of the loaded library
    if name.startswith("qrx_"):
        return getattr(load(), name)
    raise AttributeError(name)


def status_string(code: int) -> str:
    return load().qrx_status_string(code).decode()


class QrxError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {status_string(code)} ({code})")
        self.code = code


def check(code, where="qrx"):
    if code != QRX_OK:
        raise QrxError(code, where)
    return code


PANEL = {"gram": 0, "tsqr": 1, "mgs": 1}


def qr_opts(prec="fp32", panel_width=0, cutoff=0, col_scaling=True, reorth=True, panel="gram",
            node_reorth=None, gemm_tiles=0, split_target=0, q_reorth=False):
    o = qrx_qr_opts()
    o.q_reorth = 1 if q_reorth else 0
    o.gemm_tiles = gemm_tiles
    o.split_target = split_target
    o.node_reorth = 0 if node_reorth is None else (1 if node_reorth else 2)
    o.panel_alg = PANEL[panel] if isinstance(panel, str) else int(panel)
    o.gemm_prec = PREC[prec] if isinstance(prec, str) else int(prec)
    o.panel_width = panel_width
    o.cutoff = cutoff
    o.block_rows = 0
    o.no_col_scaling = 0 if col_scaling else 1
    o.panel_single_pass = 0 if reorth else 1
    return o


def lls_opts(prec="fp32", method="lsqr", tol=1e-10, max_iter=200, use_x0=False, zero_start=False,
             **qr_kw):
    o = qrx_lls_opts()
    o.zero_start = 1 if zero_start else 0
    o.qr = qr_opts(prec, **qr_kw)
    o.method = {"lsqr": 0, "cgls": 1}[method] if isinstance(method, str) else int(method)
    o.tol = tol
    o.max_iter = max_iter
    o.use_x0 = 1 if use_x0 else 0
    return o


# -- tuning cache (host only) ------------------------------------------------
TUNE_KIND = {"gram": 0, "batched": 1, "tsqr": 2}


def tune_key(arch, m, n, prec="fp16", kind="gram"):
    buf = C.create_string_buffer(256)
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    k = TUNE_KIND[kind] if isinstance(kind, str) else int(kind)
    check(load().qrx_tune_key(arch.encode(), int(m), int(n), p, k, buf, 256), "qrx_tune_key")
    return buf.value.decode()


def tune_cache_get(path, key):
    """The cached entry for key as a dict, or None when absent."""
    r = qrx_tune_result()
    rc = load().qrx_tune_cache_get(os.fsencode(path), key.encode(), C.byref(r))
    if rc == 1:
        return None
    check(rc, "qrx_tune_cache_get")
    return r.as_dict()


def tune_cache_put(path, key, panel_width, cutoff, gemm_tiles=0, split_target=0, ms=0.0):
    r = qrx_tune_result(panel_width, cutoff, gemm_tiles, split_target, ms, 0, 0)
    check(load().qrx_tune_cache_put(os.fsencode(path), key.encode(), C.byref(r)), "qrx_tune_cache_put")

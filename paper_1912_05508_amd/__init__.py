"""Mixed-precision QR and least squares on AMD MI355X (gfx950).

Python front-end over libqrx.so: torch supplies device memory and the current
stream; the computation is the library's HIP kernels.

    qr(A, prec="fp16")          -> (Q, R, status)   A: (m, n) float32 cuda tensor
    lstsq(A, b, prec="fp16")    -> (x, info)        b: (m,) float64 cuda tensor

A is read as a column-major matrix (a tensor with strides (1, lda)); other
layouts are copied into one first.
"""
from __future__ import annotations

import ctypes as C
import os

from . import _lib
from ._lib import (QRX_BF16, QRX_EHIP, QRX_EINVAL, QRX_ENOCONV, QRX_ENOMEM,  # noqa: F401
                   QRX_ENONFINITE, QRX_ESINGULAR, QRX_FP16, QRX_FP32, QRX_OK, QrxError,
                   lls_opts, qr_opts, qrx_kernel_stat, qrx_lls_info, qrx_lls_opts,
                   qrx_qr_opts, status_string)

__all__ = ["Handle", "qr", "lstsq", "colmajor", "qr_opts", "lls_opts", "QrxError", "info_tensor",
           "read_info", "QrxArgumentError", "BatchPlan"]


def colmajor(t, ld=None):
    """A (m, n) tensor laid out column-major with leading dimension ld >= m."""
    import torch
    m, n = t.shape
    ld = ld or m
    if t.stride() == (1, ld) or (n == 1 and t.stride(0) == 1 and ld == m):
        return t
    buf = torch.empty((n, ld), dtype=t.dtype, device=t.device)
    out = buf.t()[:m, :]
    out.copy_(t)
    return out


def _ld(t):
    return t.stride(1) if t.shape[1] > 1 else max(t.shape[0], 1)


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class QrxArgumentError(ValueError):
    """A tensor handed to the library has the wrong dtype, device, size or layout
    (raised before any library call)."""


def _check_mat(name, t, m, n, dtype):
    """A column-major (m, n) device tensor of `dtype` (strides (1, ld), ld >= m)."""
    import torch
    if not (torch.is_tensor(t) and t.is_cuda and t.dtype == dtype):
        raise QrxArgumentError(f"{name}: expected a {dtype} cuda tensor")
    if tuple(t.shape) != (m, n):
        raise QrxArgumentError(f"{name}: expected shape {(m, n)}, got {tuple(t.shape)}")
    if n > 1 and not (t.stride(0) == 1 and t.stride(1) >= m):
        raise QrxArgumentError(f"{name}: expected a column-major layout, strides {t.stride()}")
    if n == 1 and t.stride(0) != 1:
        raise QrxArgumentError(f"{name}: expected unit row stride")


def _check_vec(name, t, length, dtype):
    """A contiguous device vector of `length` entries of `dtype`."""
    import torch
    if not (torch.is_tensor(t) and t.is_cuda and t.dtype == dtype):
        raise QrxArgumentError(f"{name}: expected a {dtype} cuda tensor")
    if t.numel() != length or not t.is_contiguous():
        raise QrxArgumentError(f"{name}: expected {length} contiguous entries, got {t.numel()}")


def info_tensor(count=1, device=None):
    """Device memory for `count` qrx_lls_info records (written by the library)."""
    import torch
    return torch.zeros(count * C.sizeof(qrx_lls_info), dtype=torch.uint8, device=device)


def read_info(t, count=1):
    """The qrx_lls_info records of a device buffer as dicts (synchronises with it)."""
    raw = bytes(t.cpu().numpy())
    sz = C.sizeof(qrx_lls_info)
    return [qrx_lls_info.from_buffer_copy(raw[i * sz:(i + 1) * sz]).as_dict()
            for i in range(count)]


class Handle:
    """Owns a qrx handle bound to the current CUDA (HIP) device."""

    def __init__(self, device=None):
        import torch
        lib = _lib.load()
        dev = torch.cuda.current_device() if device is None else device
        h = C.c_void_p()
        _lib.check(lib.qrx_create(C.byref(h), int(dev)), "qrx_create")
        self.h = h
        self.lib = lib

    def close(self):
        if self.h:
            self.lib.qrx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- QR -----------------------------------------------------------------
    def qr(self, A, prec="fp32", R=None, status=None, **kw):
        """Factor column-major A in place (A -> Q); returns (Q, R, status tensor)."""
        import torch
        m, n = A.shape
        if not (A.dtype == torch.float32 and A.is_cuda):
            raise QrxArgumentError("A: expected a float32 cuda tensor")
        A = colmajor(A)
        if R is None:
            R = torch.empty((n, n), dtype=torch.float32, device=A.device).t()
        _check_mat("R", R, n, n, torch.float32)
        if status is None:
            status = torch.zeros(1, dtype=torch.int32, device=A.device)
        _check_vec("status", status, 1, torch.int32)
        o = qr_opts(prec, **kw)
        rc = self.lib.qrx_qr_factor(self.h, m, n, C.c_void_p(A.data_ptr()), _ld(A),
                                    C.c_void_p(R.data_ptr()), _ld(R), None, 0, C.byref(o),
                                    C.c_void_p(status.data_ptr()), _stream())
        _lib.check(rc, "qrx_qr_factor")
        return A, R, status

    def qr_out(self, A, Q, R, status, prec="fp32", **kw):
        """Out-of-place QR: A (column-major, untouched) -> Q, R (preallocated)."""
        import torch
        m, n = A.shape
        _check_mat("A", A, m, n, torch.float32)
        _check_mat("Q", Q, m, n, torch.float32)
        _check_mat("R", R, n, n, torch.float32)
        _check_vec("status", status, 1, torch.int32)
        o = qr_opts(prec, **kw)
        rc = self.lib.qrx_qr_factor_out(self.h, m, n, C.c_void_p(A.data_ptr()), _ld(A),
                                        C.c_void_p(Q.data_ptr()), _ld(Q),
                                        C.c_void_p(R.data_ptr()), _ld(R), None, 0, C.byref(o),
                                        C.c_void_p(status.data_ptr()), _stream())
        _lib.check(rc, "qrx_qr_factor_out")
        return Q, R, status

    # -- least squares --------------------------------------------------------
    def lstsq_async(self, A, b, x, info, prec="fp32", R=None, with_R=False, use_x0=False,
                    **kw):
        """Enqueue x = argmin ||A x - b|| on the current stream without waiting:
        A (column-major float32, untouched), b (float64, m), x (float64, n; the
        start when use_x0), info (from info_tensor()) are device tensors the
        caller keeps alive until the stream reaches the end of the call."""
        import torch
        m, n = A.shape
        _check_mat("A", A, m, n, torch.float32)
        _check_vec("b", b, m, torch.float64)
        _check_vec("x", x, n, torch.float64)
        if not (torch.is_tensor(info) and info.is_cuda and info.dtype == torch.uint8
                and info.numel() >= C.sizeof(qrx_lls_info) and info.is_contiguous()):
            raise QrxArgumentError("info: expected a device buffer from info_tensor()")
        o = lls_opts(prec, use_x0=use_x0, **kw)
        ip = C.c_void_p(info.data_ptr())
        if with_R:
            if R is not None:
                _check_mat("R", R, n, n, torch.float32)
            rp = C.c_void_p(R.data_ptr()) if R is not None else None
            ldr = _ld(R) if R is not None else n
            rc = self.lib.qrx_lls_solve_with_R(self.h, m, n, C.c_void_p(A.data_ptr()), _ld(A),
                                               rp, ldr, C.c_void_p(b.data_ptr()),
                                               C.c_void_p(x.data_ptr()), None, 0, C.byref(o),
                                               ip, _stream())
        else:
            rc = self.lib.qrx_lls_solve(self.h, m, n, C.c_void_p(A.data_ptr()), _ld(A),
                                        C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                        None, 0, C.byref(o), ip, _stream())
        _lib.check(rc, "qrx_lls_solve")

    def lstsq(self, A, b, prec="fp32", x=None, R=None, with_R=False, **kw):
        """x = argmin ||A x - b|| (A untouched); waits for the result and returns
        (x, info dict)."""
        import torch
        m, n = A.shape
        if not (A.dtype == torch.float32 and A.is_cuda):
            raise QrxArgumentError("A: expected a float32 cuda tensor")
        A = colmajor(A)
        b = b.contiguous()
        use_x0 = x is not None
        if x is None:
            x = torch.zeros(n, dtype=torch.float64, device=A.device)
        info = info_tensor(device=A.device)
        self.lstsq_async(A, b, x, info, prec=prec, R=R, with_R=with_R, use_x0=use_x0, **kw)
        return x, read_info(info)[0]

    # -- batched ---------------------------------------------------------------
    def plan_batched(self, sizes, prec="bf16", lls=True, cutoff=None, tiles=None, **kw):
        """A plan for problems of the given (m, n) sizes: schedules, longest-first
        order and workspace size; cutoff and tiles are one value or one per problem."""
        return BatchPlan(self, sizes, prec, lls, cutoff, tiles, **kw)

    @staticmethod
    def _arrays(mats):
        m = (C.c_int64 * len(mats))(*[int(a.shape[0]) for a in mats])
        n = (C.c_int64 * len(mats))(*[int(a.shape[1]) for a in mats])
        lda = (C.c_int64 * len(mats))(*[_ld(a) for a in mats])
        return m, n, lda

    @staticmethod
    def _ptrs(ts, device):
        import torch
        return torch.tensor([t.data_ptr() for t in ts], dtype=torch.int64, device=device)

    def qr_batched_async(self, plan, A_ptrs, lda, R_ptrs, ldr, status, work=None):
        """Enqueue the batched QR of `plan` (lls = False) on the current stream:
        device int64 tensors of matrix pointers and leading dimensions, a device
        int32 status tensor; nothing is synchronised or allocated (with work)."""
        wp, wb = (C.c_void_p(work.data_ptr()), work.numel() * work.element_size()) if work is not None \
            else (None, 0)
        rc = self.lib.qrx_qr_factor_batched(self.h, plan.p, C.c_void_p(A_ptrs.data_ptr()),
                                            C.c_void_p(lda.data_ptr()), C.c_void_p(R_ptrs.data_ptr()),
                                            C.c_void_p(ldr.data_ptr()), wp, wb,
                                            C.c_void_p(status.data_ptr()), _stream())
        _lib.check(rc, "qrx_qr_factor_batched")

    def lstsq_batched_async(self, plan, A_ptrs, lda, b_ptrs, x_ptrs, info, work=None):
        """Enqueue the batched least squares of `plan` (lls = True) on the current
        stream: device int64 tensors of pointers (A, b, x) and leading dimensions,
        an info buffer from info_tensor(batch)."""
        wp, wb = (C.c_void_p(work.data_ptr()), work.numel() * work.element_size()) if work is not None \
            else (None, 0)
        rc = self.lib.qrx_lls_solve_batched(self.h, plan.p, C.c_void_p(A_ptrs.data_ptr()),
                                            C.c_void_p(lda.data_ptr()), C.c_void_p(b_ptrs.data_ptr()),
                                            C.c_void_p(x_ptrs.data_ptr()), wp, wb,
                                            C.c_void_p(info.data_ptr()), _stream())
        _lib.check(rc, "qrx_lls_solve_batched")

    def qr_batched(self, mats, prec="fp32", cutoff=None, tiles=None, **kw):
        """In-place QR of a list of column-major (m_i, n_i) float32 tensors
        (n_i <= 256): returns (list of Q = the same tensors, list of R, statuses)."""
        import torch
        mats = [colmajor(a) for a in mats]
        for i, a in enumerate(mats):
            if not (a.dtype == torch.float32 and a.is_cuda):
                raise QrxArgumentError(f"mats[{i}]: expected a float32 cuda tensor")
        dev = mats[0].device
        Rs = [torch.empty((int(a.shape[1]),) * 2, dtype=torch.float32, device=dev).t()
              for a in mats]
        plan = self.plan_batched([tuple(a.shape) for a in mats], prec=prec, lls=False,
                                 cutoff=cutoff, tiles=tiles, **kw)
        try:
            st = torch.zeros(len(mats), dtype=torch.int32, device=dev)
            lda = torch.tensor([_ld(a) for a in mats], dtype=torch.int64, device=dev)
            ldr = torch.tensor([_ld(r) for r in Rs], dtype=torch.int64, device=dev)
            self.qr_batched_async(plan, self._ptrs(mats, dev), lda, self._ptrs(Rs, dev), ldr, st)
            return mats, Rs, st.cpu().tolist()
        finally:
            plan.close()

    def lstsq_batched(self, mats, rhs, prec="bf16", cutoff=None, tiles=None, plan=None, **kw):
        """Least squares for lists of column-major (m_i, n_i) float32 tensors and
        float64 (m_i,) vectors with the persistent work-queue kernels: returns (list of x_i, list
        of info dicts)."""
        import torch
        mats = [colmajor(a) for a in mats]
        rhs = [b.contiguous() for b in rhs]
        k = len(mats)
        for i, (a, b) in enumerate(zip(mats, rhs)):
            if not (a.dtype == torch.float32 and a.is_cuda):
                raise QrxArgumentError(f"mats[{i}]: expected a float32 cuda tensor")
            _check_vec(f"rhs[{i}]", b, int(a.shape[0]), torch.float64)
        dev = mats[0].device
        ns = [int(a.shape[1]) for a in mats]
        flat = torch.zeros(sum(ns), dtype=torch.float64, device=dev)
        xs = list(torch.split(flat, ns))
        own = plan is None
        if own:
            plan = self.plan_batched([tuple(a.shape) for a in mats], prec=prec, lls=True,
                                     cutoff=cutoff, tiles=tiles, **kw)
        try:
            info = info_tensor(k, device=dev)
            lda = torch.tensor([_ld(a) for a in mats], dtype=torch.int64, device=dev)
            self.lstsq_batched_async(plan, self._ptrs(mats, dev), lda, self._ptrs(rhs, dev),
                                     self._ptrs(xs, dev), info)
            return xs, read_info(info, k)
        finally:
            if own:
                plan.close()

    # -- autotuning -------------------------------------------------------------
    def tune(self, A, prec="fp16", cache=None, reps=3, **kw):
        """Tune nb, cutoff, tile family and projection split for QR of A's size
        class (A column-major float32, not modified); returns the result dict
        (qr_opts keyword arguments panel_width, cutoff, gemm_tiles, split_target,
        plus ms, trials, from_cache)."""
        import torch
        m, n = A.shape
        assert A.dtype == torch.float32 and A.is_cuda
        A = colmajor(A)
        o = qr_opts(prec, **kw)
        r = _lib.qrx_tune_result()
        path = os.fsencode(cache) if cache is not None else None
        rc = self.lib.qrx_tune(self.h, m, n, C.c_void_p(A.data_ptr()), _ld(A), C.byref(o), int(reps),
                               path, C.byref(r), _stream())
        _lib.check(rc, "qrx_tune")
        return r.as_dict()

    def tune_batched(self, mats, prec="bf16", cache=None, reps=3, **kw):
        """Tune the batched QR per size class of this batch (matrices not modified):
        returns a dict with per-problem lists 'cutoff' and 'tiles' (for
        plan_batched) and the summary fields ms, trials, from_cache."""
        mats = [colmajor(a) for a in mats]
        k = len(mats)
        m, n, lda = self._arrays(mats)
        Ap = (C.c_void_p * k)(*[a.data_ptr() for a in mats])
        o = qr_opts(prec, **kw)
        r = _lib.qrx_tune_result()
        cut = (C.c_int * k)()
        til = (C.c_int * k)()
        path = os.fsencode(cache) if cache is not None else None
        rc = self.lib.qrx_tune_batched(self.h, k, m, n, Ap, lda, C.byref(o), int(reps), path,
                                       cut, til, C.byref(r), _stream())
        _lib.check(rc, "qrx_tune_batched")
        d = r.as_dict()
        d["cutoff"] = list(cut)
        d["tiles"] = list(til)
        return d

    # -- timing ---------------------------------------------------------------
    def timing(self, enable=True):
        _lib.check(self.lib.qrx_timing_enable(self.h, 1 if enable else 0))

    def timing_reset(self):
        _lib.check(self.lib.qrx_timing_reset(self.h))

    def timing_get(self):
        cap = 64
        arr = (qrx_kernel_stat * cap)()
        cnt = C.c_int()
        _lib.check(self.lib.qrx_timing_get(self.h, arr, cap, C.byref(cnt)))
        out = {}
        for i in range(min(cnt.value, cap)):
            s = arr[i]
            out[s.name.decode()] = dict(launches=s.launches, total_ms=s.total_ms, flops=s.flops,
                                        bytes=s.bytes)
        return out


class BatchPlan:
    """A batch plan (qrx_batch_plan): the problems' sizes, schedules and
    longest-first order, uploaded to the device once."""

    def __init__(self, handle, sizes, prec="bf16", lls=True, cutoff=None, tiles=None, **kw):
        k = len(sizes)
        self.handle = handle
        self.batch = k
        m = (C.c_int64 * k)(*[int(s[0]) for s in sizes])
        n = (C.c_int64 * k)(*[int(s[1]) for s in sizes])

        def per(v):
            if v is None:
                return None
            vals = list(v) if hasattr(v, "__len__") else [int(v)] * k
            if len(vals) != k:
                raise QrxArgumentError("per-problem values: expected one per problem")
            return (C.c_int * k)(*[int(x) for x in vals])
        o = lls_opts(prec, **kw)
        p = C.c_void_p()
        rc = handle.lib.qrx_batch_plan_create(handle.h, k, m, n, per(cutoff), per(tiles),
                                              C.byref(o), 1 if lls else 0, C.byref(p))
        _lib.check(rc, "qrx_batch_plan_create")
        self.p = p
        sz = C.c_size_t()
        _lib.check(handle.lib.qrx_batch_plan_workspace_size(p, C.byref(sz)))
        self.work_bytes = sz.value

    def close(self):
        if self.p:
            self.handle.lib.qrx_batch_plan_destroy(self.p)
            self.p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default = None


def _handle():
    global _default
    if _default is None:
        _default = Handle()
    return _default


def qr(A, prec="fp32", **kw):
    """QR of a column-major copy of A: returns (Q, R, status)."""
    import torch
    m, n = A.shape
    W = torch.empty((n, m), dtype=torch.float32, device=A.device).t()
    W.copy_(A)
    return _handle().qr(W, prec=prec, **kw)


def lstsq(A, b, prec="fp32", **kw):
    return _handle().lstsq(A, b, prec=prec, **kw)

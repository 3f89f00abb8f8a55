"""Recursive MGS QR (Alg. 2) with MGS panels (Alg. 4): an error-model emulator.

This follows the paper's algorithm step by step, in numpy:

* Alg. 4 (``mgs``): for k = 1..n: R(k,k) = ||Q(:,k)||, Q(:,k) /= R(k,k),
  R(k,k+1:n) = Q(:,k)^T Q(:,k+1:n), Q(:,k+1:n) -= Q(:,k) R(k,k+1:n).
  A column whose norm is exactly zero is left as zero with R(k,k) = 0.
* ``mgs2``: Alg. 4 applied twice (the re-orthogonalisation remedy of
  Sec. 4.1.2 applied to each panel); R = R2 R1.
* Alg. 2 (``rmgs``): split the columns [A1 | A2], factor A1 recursively,
  R12 = Q1^T A2, A2 <- A2 - Q1 R12, factor A2 recursively, assemble Q and R
  as in eq. recqr. The split is n1 = c * ceil(n / (2c)) so that every leaf
  has width at most the cutoff c (the listing assumes n = c 2^L).

``prec`` rounds the operands of the two trailing products the way a
low-precision matrix unit would see them: "fp16" or "bf16" round-to-nearest-
even of the FP32 operand ("fp16x3": its FP16 hi part plus the FP16-rounded
remainder) after an exact power-of-two column scaling (max-abs
of each A2 column brought to [2^13, 2^14), Q1 multiplied by 2^14, and each
R12 column brought to [2^13, 2^14) before the update); the products of the
rounded operands are summed in float32 (a float32 matrix product), as a
matrix unit with FP32 accumulation does, and the results rounded to the
working precision. ``prec=None`` is plain float64 arithmetic. This module calibrates error bounds for the
low-precision modes; it is not the definition of the factorisation (that is
``householder``). Parity of its FP16/BF16 rounding model is unpinned.
"""
from __future__ import annotations

import math

import numpy as np


def to_bf16(x):
    """Round float32 values to bfloat16 (RNE), returned as float32."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).reshape(np.shape(x))


def round_operand(x, prec):
    x32 = np.asarray(x, dtype=np.float32)
    if prec == "fp16":
        return x32.astype(np.float16).astype(np.float64)
    if prec == "fp16x3":
        # hi = fl16(x), lo = fl16(x - hi); the operand seen is hi + lo
        hi = x32.astype(np.float16).astype(np.float32)
        lo = (x32 - hi).astype(np.float16).astype(np.float64)
        return hi.astype(np.float64) + lo
    if prec == "bf16":
        return to_bf16(x32).astype(np.float64)
    return np.asarray(x, dtype=np.float64)


def pow2_scale(colmax, target_exp: int = 14):
    """2^(target - E) where colmax = f 2^E, f in [0.5, 1); 1 for a zero column."""
    _, E = np.frexp(np.asarray(colmax, dtype=np.float64))
    s = np.ldexp(1.0, target_exp - E)
    return np.where(np.asarray(colmax) > 0, s, 1.0)


def mgs(A):
    """Alg. 4: modified Gram-Schmidt, returns (Q, R)."""
    Q = np.array(A, dtype=np.float64, copy=True)
    n = Q.shape[1]
    R = np.zeros((n, n))
    for k in range(n):
        rkk = float(np.sqrt(Q[:, k] @ Q[:, k]))
        R[k, k] = rkk
        if rkk == 0.0:
            Q[:, k] = 0.0
            continue
        Q[:, k] /= rkk
        R[k, k + 1:] = Q[:, k] @ Q[:, k + 1:]
        Q[:, k + 1:] -= np.outer(Q[:, k], R[k, k + 1:])
    return Q, R


def mgs2(A):
    Q1, R1 = mgs(A)
    Q, R2 = mgs(Q1)
    return Q, R2 @ R1


def _mm32(X, Y):
    """Product of rounded operands with float32 summation (each operand is
    exactly representable in float32, so only the sums round)."""
    return (X.astype(np.float32) @ Y.astype(np.float32)).astype(np.float64)


def _project(Q1, A2, prec, scale, work):
    if prec is None:
        return (Q1.T @ A2).astype(work)
    if scale:
        e = pow2_scale(np.max(np.abs(A2), axis=0))
        fq = 2.0 ** 14
        acc = _mm32(round_operand(Q1 * fq, prec).T, round_operand(A2 * e, prec))
        return (acc / (fq * e)).astype(np.float32).astype(work)
    return _mm32(round_operand(Q1, prec).T, round_operand(A2, prec)).astype(np.float32).astype(work)


def _update(Q1, R12, A2, prec, scale, work):
    if prec is None:
        return (A2 - Q1 @ R12).astype(work)
    if scale:
        fq = 2.0 ** 14
        h = pow2_scale(np.max(np.abs(R12), axis=0))
        acc = _mm32(round_operand(Q1 * fq, prec), round_operand(R12 * h, prec))
        return (A2 - acc / (fq * h)).astype(np.float32).astype(work)
    acc = _mm32(round_operand(Q1, prec), round_operand(R12, prec))
    return (A2 - acc).astype(np.float32).astype(work)


def rmgs(A, cutoff: int = 32, prec=None, scale: bool = True, panel=mgs2,
         work=np.float64):
    """Alg. 2 with leaves of width <= cutoff factored by ``panel``."""
    A = np.array(A, dtype=work, copy=True)
    m, n = A.shape
    if n <= cutoff:
        Q, R = panel(A)
        return Q.astype(work), R.astype(work)
    n1 = cutoff * math.ceil(n / (2 * cutoff))
    Q1, R11 = rmgs(A[:, :n1], cutoff, prec, scale, panel, work)
    R12 = _project(Q1, A[:, n1:], prec, scale, work)
    A2 = _update(Q1, R12, A[:, n1:], prec, scale, work)
    Q2, R22 = rmgs(A2, cutoff, prec, scale, panel, work)
    Q = np.concatenate([Q1, Q2], axis=1)
    R = np.zeros((n, n), dtype=work)
    R[:n1, :n1] = R11
    R[:n1, n1:] = R12
    R[n1:, n1:] = R22
    return Q, R

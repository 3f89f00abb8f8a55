"""Least-squares solution x = argmin_x ||A x - b||_2 in FP64 (oracle).

Sec. 2.2 (eq. opt:lls) states the problem for A (m x n, m > n, full column
rank) and b in R^m (the text prints R^n; the only consistent reading is R^m).
Its unique solution is (A^T A)^{-1} A^T b. Following Alg. 1, the oracle forms
the Householder QR, x0 = R^{-1} (Q^T b) by back substitution, then applies
correction steps x <- x + R^{-1} Q^T r with r = b - A x evaluated in
np.longdouble (64-bit significand on x86) and rounded to float64. The
instance solved is the stored data: A exactly as given (FP32 upcast), b as
given (FP64).
"""
from __future__ import annotations

import numpy as np

from .householder import qr


def back_substitute(R, y):
    """Solve R x = y for upper-triangular R (row-oriented, float64)."""
    R = np.asarray(R, dtype=np.float64)
    n = R.shape[0]
    x = np.zeros(n)
    for i in range(n - 1, -1, -1):
        x[i] = (y[i] - np.dot(R[i, i + 1:], x[i + 1:])) / R[i, i]
    return x


def forward_substitute_t(R, y):
    """Solve R^T x = y for upper-triangular R (R^T is lower triangular)."""
    R = np.asarray(R, dtype=np.float64)
    n = R.shape[0]
    x = np.zeros(n)
    for i in range(n):
        x[i] = (y[i] - np.dot(R[:i, i], x[:i])) / R[i, i]
    return x


def matvec_ld(A, x, chunk: int = 256):
    """A @ x accumulated in np.longdouble (column chunks bound the memory)."""
    A = np.asarray(A)
    m, n = A.shape
    acc = np.zeros(m, dtype=np.longdouble)
    xl = np.asarray(x, dtype=np.longdouble)
    for j0 in range(0, n, chunk):
        j1 = min(n, j0 + chunk)
        acc += A[:, j0:j1].astype(np.longdouble) @ xl[j0:j1]
    return acc


def rmatvec_ld(A, y, chunk: int = 256):
    """A^T @ y accumulated in np.longdouble."""
    A = np.asarray(A)
    m, n = A.shape
    out = np.zeros(n, dtype=np.longdouble)
    yl = np.asarray(y, dtype=np.longdouble)
    for j0 in range(0, n, chunk):
        j1 = min(n, j0 + chunk)
        out[j0:j1] = A[:, j0:j1].astype(np.longdouble).T @ yl
    return out


def residual_ld(A, b, x):
    """r = b - A x in extended precision (returned as np.longdouble)."""
    return np.asarray(b, dtype=np.longdouble) - matvec_ld(A, x)


def lls_direct(A, b, refine: int = 3, QR=None):
    """Alg. 1 on the stored instance, then ``refine`` correction steps.

    Returns (x, Q, R). Pass QR=(Q, R) to reuse an existing factorisation.
    """
    A = np.asarray(A)
    b = np.asarray(b, dtype=np.float64)
    Q, R = QR if QR is not None else qr(A)
    x = back_substitute(R, Q.T @ b)
    for _ in range(refine):
        r = residual_ld(A, b, x).astype(np.float64)
        x = x + back_substitute(R, Q.T @ r)
    return x, Q, R

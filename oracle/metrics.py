"""Accuracy metrics of Sec. 3.2.1-3.2.2, computed by the oracle from outputs.

* QR backward error ||A - Q R|| / ||A|| (Sec. 3.2.1; the text uses the
  2-norm, Fig. 2 the unlabelled norm) -- Frobenius as the primary figure,
  the 2-norm by power iteration on the implicit operator A - Q R.
* Orthogonality ||I - Q^T Q||_2 (Sec. 3.2.1) and its /N form of Fig. 2.
* LLS accuracy A^T (A x - b) (Sec. 3.2.2), normalised as
  eta_F = ||A^T r|| / (||A||_F ||r||) with r = b - A x and A^T r in
  np.longdouble; eta_2 uses ||A||_2.

Inputs are the stored arrays (FP32 A exactly upcast, FP64 b and x); GPU
outputs are evaluated here, never their self-reported values.
"""
from __future__ import annotations

import numpy as np

from .lls import residual_ld, rmatvec_ld


def _f64(X):
    return np.asarray(X, dtype=np.float64)


def fro(X):
    X = _f64(X)
    return float(np.sqrt(np.sum(X * X)))


def qr_backward_error(A, Q, R, cols=None):
    """||A - QR||_F / ||A||_F, optionally restricted to column indices ``cols``."""
    A, Q, R = _f64(A), _f64(Q), _f64(R)
    if cols is not None:
        cols = np.asarray(cols)
        E = A[:, cols] - Q @ R[:, cols]
        return fro(E) / fro(A[:, cols])
    return fro(A - Q @ R) / fro(A)


def norm2_power(matvec, rmatvec, n, iters: int = 30, seed: int = 1):
    """Largest singular value of an implicit operator by power iteration."""
    g = np.random.default_rng(seed)
    v = g.standard_normal(n)
    v /= np.linalg.norm(v)
    s = 0.0
    for _ in range(iters):
        w = rmatvec(matvec(v))
        nw = float(np.linalg.norm(w))
        if nw == 0.0:
            return 0.0
        s = np.sqrt(nw)
        v = w / nw
    return float(s)


def qr_backward_error_2(A, Q, R, iters: int = 30):
    """||A - QR||_2 / ||A||_2 (both by power iteration)."""
    A, Q, R = _f64(A), _f64(Q), _f64(R)
    n = A.shape[1]
    num = norm2_power(lambda v: A @ v - Q @ (R @ v), lambda y: A.T @ y - R.T @ (Q.T @ y),
                      n, iters)
    den = norm2_power(lambda v: A @ v, lambda y: A.T @ y, n, iters)
    return num / den


def orthogonality(Q, cols=None):
    """||I - Q^T Q||_2 via a symmetric eigensolve (on a column subset if given)."""
    Q = _f64(Q)
    if cols is not None:
        Q = Q[:, np.asarray(cols)]
    G = Q.T @ Q - np.eye(Q.shape[1])
    return float(np.max(np.abs(np.linalg.eigvalsh(G))))


def upper_triangular_ok(R):
    """R exactly upper triangular with a positive finite diagonal."""
    R = np.asarray(R)
    d = np.diag(R)
    return bool(np.all(np.tril(R, -1) == 0) and np.all(np.isfinite(d)) and np.all(d > 0))


def r_relative_error(R, R_ref):
    return fro(_f64(R) - _f64(R_ref)) / fro(R_ref)


def eta(A, b, x, normA=None):
    """Normal-equation backward error ||A^T r|| / (||A|| ||r||), r in longdouble.

    normA defaults to ||A||_F. Returns (eta, ||r||).
    """
    r = residual_ld(A, b, x)
    atr = rmatvec_ld(A, r)
    nr = float(np.sqrt(np.sum(r * r)))
    if normA is None:
        normA = fro(A)
    if nr == 0.0:
        return 0.0, 0.0
    return float(np.sqrt(np.sum(atr * atr))) / (normA * nr), nr


def eta_F(A, b, x):
    return eta(A, b, x)[0]


def eta_2(A, b, x):
    A64 = _f64(A)
    n2 = norm2_power(lambda v: A64 @ v, lambda y: A64.T @ y, A64.shape[1])
    return eta(A, b, x, normA=n2)[0]


def forward_error(x, x_ref):
    x, x_ref = _f64(x), _f64(x_ref)
    return float(np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref))


def ls_forward_bound(kappa, normA2, normx, normr, tol):
    """First-order LS perturbation bound scaled by 10: the bar a solution with
    backward error ``tol`` must meet in forward error."""
    return 10.0 * (kappa + kappa * kappa * normr / (normA2 * normx)) * tol

"""Householder QR in FP64: the oracle for the thin factorisation A = QR.

Sec. 2.2 defines the target: for A (m x n, m >= n, full column rank) a thin
factorisation A = QR with Q (m x n) having orthonormal columns and R (n x n)
upper triangular. With the sign convention R_kk > 0 this factorisation is
unique, so any correct method (the paper's recursive Gram-Schmidt included)
reaches the same Q and R up to rounding. The oracle computes it with the
textbook Householder method (the xGEQRF of Alg. 1).

Reflector k: x = A[k:, k]; alpha = -sgn(x_0) ||x|| with sgn(0) = +1;
v = x - alpha e_1; H = I - beta v v^T with beta = 2 / (v^T v) (H = I when
v = 0). The blocked form accumulates nb reflectors as I - Y T Y^T
(Schreiber & Van Loan's compact WY representation, cited in Sec. 3.1.2).
"""
from __future__ import annotations

import numpy as np


def _reflector(x):
    normx = float(np.sqrt(np.dot(x, x)))
    alpha = -normx if x[0] >= 0.0 else normx
    v = x.copy()
    v[0] -= alpha
    vtv = float(np.dot(v, v))
    beta = 2.0 / vtv if vtv > 0.0 else 0.0
    return v, beta, alpha


def _sign_normalise(Q, R):
    d = np.sign(np.diag(R))
    d[d == 0.0] = 1.0
    return Q * d, R * d[:, None]


def householder_qr(A):
    """Unblocked Householder QR. Returns (Q, R) in float64 with R_kk >= 0."""
    W = np.array(A, dtype=np.float64, copy=True)
    m, n = W.shape
    if m < n:
        raise ValueError("need m >= n")
    vs, betas = [], []
    for k in range(n):
        v, beta, alpha = _reflector(W[k:, k])
        if beta != 0.0:
            W[k:, k:] -= beta * np.outer(v, v @ W[k:, k:])
        W[k, k] = alpha
        W[k + 1:, k] = 0.0
        vs.append(v)
        betas.append(beta)
    R = np.triu(W[:n, :])
    Q = np.zeros((m, n))
    Q[:n, :n] = np.eye(n)
    for k in range(n - 1, -1, -1):
        v, beta = vs[k], betas[k]
        if beta != 0.0:
            Q[k:, :] -= beta * np.outer(v, v @ Q[k:, :])
    return _sign_normalise(Q, R)


def householder_qr_blocked(A, nb: int = 64):
    """Compact-WY blocked Householder QR (same result as ``householder_qr``).

    Panel of nb columns: unblocked reflectors; T built column by column as
    T <- [[T, -beta T (Y^T v)], [0, beta]]; the trailing matrix is updated by
    (I - Y T Y^T)^T = I - Y T^T Y^T; the explicit Q applies the block
    reflectors to [I_n; 0] in reverse order.
    """
    W = np.array(A, dtype=np.float64, copy=True, order="F")
    m, n = W.shape
    if m < n:
        raise ValueError("need m >= n")
    blocks = []
    for k0 in range(0, n, nb):
        k1 = min(n, k0 + nb)
        w = k1 - k0
        Y = np.zeros((m - k0, w))
        T = np.zeros((w, w))
        for j in range(w):
            k = k0 + j
            v, beta, alpha = _reflector(W[k:, k])
            if beta != 0.0:
                W[k:, k:k1] -= beta * np.outer(v, v @ W[k:, k:k1])
            W[k, k] = alpha
            W[k + 1:, k] = 0.0
            Y[j:, j] = v
            if j > 0:
                T[:j, j] = -beta * (T[:j, :j] @ (Y[:, :j].T @ Y[:, j]))
            T[j, j] = beta
        if k1 < n:
            C = W[k0:, k1:]
            C -= Y @ (T.T @ (Y.T @ C))
        blocks.append((k0, Y, T))
    R = np.triu(W[:n, :])
    Q = np.zeros((m, n), order="F")
    Q[:n, :n] = np.eye(n)
    for k0, Y, T in reversed(blocks):
        X = Q[k0:, :]
        X -= Y @ (T @ (Y.T @ X))
    return _sign_normalise(Q, R)


def qr(A, blocked: bool | None = None, nb: int = 64):
    """Thin QR of A (upcast exactly to float64). Blocked for larger inputs."""
    A = np.asarray(A)
    if blocked is None:
        blocked = A.shape[1] > 2 * nb
    return householder_qr_blocked(A, nb) if blocked else householder_qr(A)

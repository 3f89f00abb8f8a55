"""LSQR and CGLS on the right-preconditioned operator B = A R^{-1} (FP64).

Sec. 3.2.3 runs a Krylov least-squares iteration with the low-precision R as
a right preconditioner: with y = R x the problem min ||A x - b|| becomes
min ||B y - b||, B = A R^{-1}, whose conditioning is kappa(A R^{-1}) (close
to 1 for a good R); the error contracts by (kappa-1)/(kappa+1) per step, and
an exact R gives convergence in one step.

LSQR keeps its iterate in x-space: each direction d = R^{-1} w is kept next
to w so that x += step * d; no final back-transformation is needed.

``cgls`` is conjugate gradients on the normal equations of A R^{-1}, written
from the mathematics in the preconditioned variable y = R x (see its
docstring); in exact arithmetic its iterates are those of the paper's CGLS
(Alg. 5).

``lsqr`` is Paige & Saunders' LSQR (the numerically preferred equivalent the
paper cites in Sec. 5), Golub-Kahan bidiagonalisation with Givens rotations.

Stopping: the iteration stops at the first iterate whose true normal-equation
backward error eta_F = ||A^T r|| / (||A||_F ||r||) (r = b - A x in extended
precision) is <= tol, or when ||r|| <= tol (||A||_F ||x|| + ||b||) (consistent
systems), or at maxit. ``estimate_only=True`` uses LSQR's own estimates
instead (Paige & Saunders' tests S1 and S2) and skips the true residual.
"""
from __future__ import annotations

import numpy as np

from .lls import back_substitute, forward_substitute_t, residual_ld, rmatvec_ld


class _Op:
    def __init__(self, A, R=None):
        self.A = np.asarray(A, dtype=np.float64)
        self.R = None if R is None else np.asarray(R, dtype=np.float64)

    def rinv(self, v):          # R^{-1} v
        return v.copy() if self.R is None else back_substitute(self.R, v)

    def rinv_t(self, v):        # R^{-T} v
        return v.copy() if self.R is None else forward_substitute_t(self.R, v)


def _true_eta(A, b, x, normA_F):
    r = residual_ld(A, b, x)
    atr = rmatvec_ld(A, r)
    nr = float(np.sqrt(np.sum(r * r)))
    return float(np.sqrt(np.sum(atr * atr))) / (normA_F * nr) if nr > 0 else 0.0, nr


def _converged(A, b, x, normA_F, nb, tol, compatible_test=True):
    eta, nr = _true_eta(A, b, x, normA_F)
    compatible = compatible_test and nr <= tol * (normA_F * float(np.linalg.norm(x)) + nb)
    return (eta <= tol) or compatible, eta


def lsqr(A, b, R=None, x0=None, tol=1e-10, maxit=200, estimate_only=False,
         record=False, compatible_test=True):
    """LSQR on A R^{-1}; returns (x, iterations, info dict). compatible_test=False
    stops on eta_F <= tol alone (not on the consistent-system residual test)."""
    op = _Op(A, R)
    A64 = op.A
    m, n = A64.shape
    b = np.asarray(b, dtype=np.float64)
    normA_F = float(np.sqrt(np.sum(A64 * A64)))
    nb = float(np.linalg.norm(b))
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    r0 = b - A64 @ x if x0 is not None else b.copy()
    hist = []
    beta = float(np.linalg.norm(r0))
    if beta == 0.0:
        return x, 0, dict(eta=0.0, hist=hist)
    u = r0 / beta
    v = op.rinv_t(A64.T @ u)
    alpha = float(np.linalg.norm(v))
    if alpha == 0.0:
        return x, 0, dict(eta=0.0, hist=hist)
    v = v / alpha
    d = op.rinv(v)                      # d = R^{-1} w, w_1 = v_1
    phibar, rhobar = beta, alpha
    bnorm2 = 0.0                        # running ||B||_F^2 estimate
    it = 0
    eta = np.inf
    while it < maxit:
        it += 1
        t = op.rinv(v)                  # R^{-1} v_i
        if it > 1:
            d = t - (theta / rho) * d   # d_i = R^{-1} (v_i - (theta_i/rho_{i-1}) w_{i-1})
        u = A64 @ t - alpha * u
        beta = float(np.linalg.norm(u))
        if beta > 0.0:
            u = u / beta
        bnorm2 += alpha * alpha + beta * beta
        v = op.rinv_t(A64.T @ u) - beta * v
        alpha = float(np.linalg.norm(v))
        if alpha > 0.0:
            v = v / alpha
        rho = float(np.hypot(rhobar, beta))
        c, s = rhobar / rho, beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        x = x + (phi / rho) * d
        est = phibar * alpha * abs(c)   # ||B^T r|| estimate
        if estimate_only:
            eta = est / (np.sqrt(bnorm2) * phibar) if phibar > 0 else 0.0
            if record:
                hist.append(eta)
            if eta <= tol or phibar <= tol * nb:
                break
        else:
            done, eta = _converged(A64, b, x, normA_F, nb, tol, compatible_test)
            if record:
                hist.append(eta)
            if done:
                break
        if alpha == 0.0 or beta == 0.0:
            break
    return x, it, dict(eta=eta, hist=hist)


def cgls(A, b, R=None, x0=None, tol=1e-10, maxit=200, record=False):
    """Conjugate gradients on the normal equations of B = A R^{-1} (Sec. 3.2.3).

    With y = R x the preconditioned problem min ||B y - b|| has the normal
    equations B^T B y = B^T b, a symmetric positive definite system; this is
    the textbook Hestenes-Stiefel CG for it, written in y:

        g_k     = B^T (b - B y_k)            (the normal-equation residual)
        p_0     = g_0,  p_k = g_k + (|g_k|^2 / |g_{k-1}|^2) p_{k-1}
        a_k     = |g_k|^2 / (p_k^T B^T B p_k) = |g_k|^2 / |B p_k|^2
        y_{k+1} = y_k + a_k p_k

    g_k is recomputed from the iterate every step (never updated by a
    recurrence), and x = R^{-1} y is formed by back substitution whenever the
    stopping test needs it. In exact arithmetic these are the iterates of the
    paper's CGLS (Alg. 5), which updates r = b - A x by a recurrence instead.
    """
    op = _Op(A, R)
    A64 = op.A
    m, n = A64.shape
    b = np.asarray(b, dtype=np.float64)
    normA_F = float(np.sqrt(np.sum(A64 * A64)))
    nb = float(np.linalg.norm(b))
    if x0 is None:
        y = np.zeros(n)
    else:
        x0 = np.asarray(x0, dtype=np.float64)
        y = x0.copy() if op.R is None else op.R @ x0

    def B(v):                   # B v = A (R^{-1} v)
        return A64 @ op.rinv(v)

    def Bt(w):                  # B^T w = R^{-T} (A^T w)
        return op.rinv_t(A64.T @ w)

    g = Bt(b - B(y))
    gg = float(g @ g)
    p = g.copy()
    hist = []
    it = 0
    eta = np.inf
    x = op.rinv(y)
    while it < maxit and gg > 0.0:
        it += 1
        Bp = B(p)
        pBBp = float(Bp @ Bp)
        if pBBp == 0.0:
            break
        y = y + (gg / pBBp) * p
        x = op.rinv(y)
        g = Bt(b - A64 @ x)
        gg_new = float(g @ g)
        p = g + (gg_new / gg) * p
        gg = gg_new
        done, eta = _converged(A64, b, x, normA_F, nb, tol)
        if record:
            hist.append(eta)
        if done:
            break
    return x, it, dict(eta=eta, hist=hist)

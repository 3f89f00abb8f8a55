"""Pins for the oracle's Householder QR (the thin QR of Sec. 2.2).

Each test checks the oracle against something other than itself: the
factorisation's defining properties, closed forms, a hand-derived fixture,
LAPACK through numpy, and exact rational arithmetic.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import householder as H
from oracle import metrics as M

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand(m, n, seed=0):
    return np.random.default_rng(seed).standard_normal((m, n))


@pytest.mark.parametrize("m,n", [(1, 1), (5, 1), (7, 3), (40, 17), (128, 64), (300, 130)])
@pytest.mark.parametrize("blocked", [False, True])
def test_invariants(m, n, blocked):
    A = _rand(m, n, m * 31 + n)
    Q, R = (H.householder_qr_blocked(A, nb=16) if blocked else H.householder_qr(A))
    assert Q.shape == (m, n) and R.shape == (n, n)
    assert M.qr_backward_error(A, Q, R) < 1e-14
    assert M.orthogonality(Q) < 1e-13
    assert M.upper_triangular_ok(R)


def test_matches_lapack_after_sign_normalisation():
    A = _rand(200, 60, 3)
    Q, R = H.qr(A)
    Ql, Rl = np.linalg.qr(A)
    d = np.sign(np.diag(Rl))
    Ql, Rl = Ql * d, Rl * d[:, None]
    kappa = np.linalg.cond(A)
    assert np.max(np.abs(R - Rl)) / np.max(np.abs(Rl)) < 10 * kappa * 2.2e-16
    assert np.max(np.abs(Q - Ql)) < 10 * kappa * 2.2e-16


def test_blocked_equals_unblocked():
    A = _rand(150, 70, 4)
    Q1, R1 = H.householder_qr(A)
    for nb in (1, 7, 16, 64, 100):
        Q2, R2 = H.householder_qr_blocked(A, nb=nb)
        assert np.max(np.abs(Q1 - Q2)) < 1e-13
        assert np.max(np.abs(R1 - R2)) < 1e-12


def test_closed_form_orthonormal_columns():
    # A with orthonormal columns: Q = A, R = I.
    Q0, _ = np.linalg.qr(_rand(50, 8, 5))
    Q0 = Q0 * np.sign(Q0[0])  # any signs; R = diag(+1) after normalisation
    Q, R = H.householder_qr(Q0)
    assert np.max(np.abs(R - np.eye(8))) < 1e-14
    assert np.max(np.abs(Q - Q0)) < 1e-14


def test_closed_form_triangular_on_top():
    # A = [T; 0] with T upper triangular and positive diagonal: Q = [I; 0], R = T.
    g = np.random.default_rng(6)
    T = np.triu(g.standard_normal((6, 6)))
    T[np.diag_indices(6)] = np.abs(T[np.diag_indices(6)]) + 1.0
    A = np.vstack([T, np.zeros((9, 6))])
    for f in (H.householder_qr, lambda X: H.householder_qr_blocked(X, 4)):
        Q, R = f(A)
        assert np.max(np.abs(R - T)) < 1e-14
        assert np.max(np.abs(Q[:6] - np.eye(6))) < 1e-14
        assert np.max(np.abs(Q[6:])) < 1e-14


def test_closed_form_single_column():
    a = np.array([[2.0], [-3.0], [6.0]])
    Q, R = H.householder_qr(a)
    assert R[0, 0] == pytest.approx(7.0, rel=1e-15)
    assert np.allclose(Q[:, 0], a[:, 0] / 7.0, rtol=0, atol=4e-16)


def test_gram_identity():
    # R^T R = A^T A (from A = QR and Q^T Q = I).
    A = _rand(90, 25, 7)
    _, R = H.qr(A)
    G = A.T @ A
    assert np.max(np.abs(R.T @ R - G)) / np.max(np.abs(G)) < 1e-14


@pytest.mark.parametrize("name", ["qr_lls_3x2_poly.json", "qr_lls_3x2_pythagorean.json"])
def test_golden_hand_derived(name):
    with open(os.path.join(GOLD, name)) as f:
        g = json.load(f)
    A = np.array(g["A"], dtype=np.float64)
    Q, R = H.householder_qr(A)
    assert np.max(np.abs(Q - np.array(g["Q"]))) < 1e-15
    assert np.max(np.abs(R - np.array(g["R"]))) < 4e-15


def test_exact_rational_cholesky_pin():
    # For integer A, R^T R = A^T A exactly; the rational LDL^T of A^T A gives
    # R_kk^2 = D_kk and R_kj = L_jk R_kk. Compare with the float R.
    g = np.random.default_rng(8)
    for trial in range(5):
        m, n = 6 + trial, 3
        Ai = g.integers(-5, 6, size=(m, n))
        G = [[Fraction(int(sum(Ai[r, i] * Ai[r, j] for r in range(m)))) for j in range(n)]
             for i in range(n)]
        L = [[Fraction(0)] * n for _ in range(n)]
        D = [Fraction(0)] * n
        for j in range(n):
            D[j] = G[j][j] - sum(L[j][k] ** 2 * D[k] for k in range(j))
            L[j][j] = Fraction(1)
            for i in range(j + 1, n):
                L[i][j] = (G[i][j] - sum(L[i][k] * L[j][k] * D[k] for k in range(j))) / D[j]
        _, R = H.householder_qr(Ai.astype(np.float64))
        for k in range(n):
            assert R[k, k] ** 2 == pytest.approx(float(D[k]), rel=1e-14)
            for j in range(k + 1, n):
                assert R[k, j] == pytest.approx(float(L[j][k]) * R[k, k], rel=1e-13, abs=1e-13)


def test_planted_sign_error_is_caught():
    # A plausible mistake (alpha = +sgn(x1)||x||, i.e. a wrong sign) must fail
    # the invariant checks that every other test relies on.
    A = _rand(30, 6, 9)

    def bad_reflector(x):
        normx = float(np.sqrt(x @ x))
        alpha = normx if x[0] >= 0.0 else -normx
        v = x.copy()
        v[0] -= alpha
        vtv = float(v @ v)
        return v, (2.0 / vtv if vtv > 0 else 0.0), -alpha  # wrong R_kk sign bookkeeping

    orig = H._reflector
    try:
        H._reflector = bad_reflector
        Q, R = H.householder_qr(A)
    finally:
        H._reflector = orig
    assert M.qr_backward_error(A, Q, R) > 1e-3

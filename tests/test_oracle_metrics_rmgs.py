"""Pins for the oracle metrics (Sec. 3.2.1-3.2.2) and the Alg. 2 emulator."""
import numpy as np
import pytest

import synth
from oracle import householder as H
from oracle import lls as L
from oracle import metrics as M
from oracle import rmgs as G


def test_power_iteration_matches_two_norm():
    A = np.random.default_rng(0).standard_normal((80, 20))
    s = M.norm2_power(lambda v: A @ v, lambda y: A.T @ y, 20, iters=200)
    assert s == pytest.approx(np.linalg.norm(A, 2), rel=1e-8)


def test_orthogonality_metric_closed_form():
    # Q = [e1, e1 cos t + e2 sin t]: Q^T Q - I = [[0, c], [c, 0]], ||.||_2 = |cos t|.
    t = 0.3
    Q = np.zeros((5, 2))
    Q[0, 0] = 1.0
    Q[0, 1], Q[1, 1] = np.cos(t), np.sin(t)
    assert M.orthogonality(Q) == pytest.approx(np.cos(t), rel=1e-14)


def test_backward_error_detects_perturbation():
    A = np.random.default_rng(1).standard_normal((60, 10))
    Q, R = H.qr(A)
    assert M.qr_backward_error(A, Q, R) < 1e-15
    R2 = R.copy()
    R2[0, 3] += 1e-6 * np.abs(R).max()
    assert M.qr_backward_error(A, Q, R2) > 1e-8
    assert M.qr_backward_error_2(A, Q, R2) > 1e-8


def test_eta_zero_at_solution_and_large_elsewhere():
    p = synth.scaled_config("c1", 256, 32, seed=3)
    x, _, _ = L.lls_direct(p.A, p.b)
    e = M.eta_F(p.A, p.b, x)
    assert e < 1e-9                                  # at the FP64 floor here
    assert M.eta_F(p.A, p.b, x * (1 + 1e-6)) > 1e3 * e
    assert M.eta_2(p.A, p.b, x) >= M.eta_F(p.A, p.b, x)


def test_upper_triangular_check():
    R = np.triu(np.ones((4, 4)))
    assert M.upper_triangular_ok(R)
    R[2, 1] = 1e-30
    assert not M.upper_triangular_ok(R)
    R = np.triu(np.ones((4, 4)))
    R[3, 3] = -1.0
    assert not M.upper_triangular_ok(R)


def test_mgs_is_the_qr_in_exact_mode():
    # Alg. 4 and Alg. 2 reach the unique QR (R_kk > 0) of the definition.
    A = np.random.default_rng(2).standard_normal((200, 50))
    Qh, Rh = H.qr(A)
    for f in (G.mgs, G.mgs2, lambda X: G.rmgs(X, cutoff=8), lambda X: G.rmgs(X, cutoff=13)):
        Q, R = f(A)
        assert np.max(np.abs(R - Rh)) < 1e-12
        assert np.max(np.abs(Q - Qh)) < 1e-12


def test_mgs_zero_column_reading():
    A = np.zeros((6, 3))
    A[0, 0] = 1.0             # q1 = e1 exactly
    A[0, 1] = 3.0             # dependent column -> exactly zero after projection
    A[:, 2] = np.arange(6)
    Q, R = G.mgs(A)
    assert R[1, 1] == 0.0 and np.all(Q[:, 1] == 0.0)
    assert np.max(np.abs(Q @ R - A)) < 1e-14


def test_mgs2_orthogonality_vs_mgs():
    # Sec. 3.2.1: MGS loses orthogonality in proportion to kappa; one re-
    # orthogonalisation restores it (Sec. 4.1.2 remedy).
    g = np.random.default_rng(3)
    A = synth.svd_matrix(g, 400, 40, synth.spectrum("geometric", 40, 1e6)).astype(np.float64)
    A = A.astype(np.float32)
    Q1, _ = G.mgs(A.astype(np.float32).astype(np.float64))
    Q1 = Q1.astype(np.float32)
    o1 = M.orthogonality(Q1)
    Q2, _ = G.mgs2(A.astype(np.float64))
    assert M.orthogonality(Q2) < 1e-13 < o1 or o1 > 1e-12


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7 + 2 ** -9, 3.0e38, -2.5], dtype=np.float32)
    y = G.to_bf16(x)
    assert y[0] == 1.0
    assert y[1] == 1.0                      # tie -> even
    assert y[2] == np.float32(1.0 + 2 ** -6) or y[2] == np.float32(1.0 + 2 ** -7)
    assert y[4] == -2.5


def test_pow2_scale():
    s = G.pow2_scale(np.array([1.0, 3.0, 1e-9, 0.0]))
    assert np.all(np.log2(s[:3]) == np.round(np.log2(s[:3])))
    v = np.array([1.0, 3.0, 1e-9]) * s[:3]
    assert np.all((v >= 2 ** 13) & (v < 2 ** 14))
    assert s[3] == 1.0


@pytest.mark.parametrize("prec,bound", [("fp16", 4e-3), ("bf16", 3e-2)])
def test_low_precision_emulation_backward_error(prec, bound):
    # MGS backward error stays at the working accuracy of the products for any
    # kappa (Sec. 3.2.1): bounded by ~8u of the operand precision.
    g = np.random.default_rng(4)
    A = synth.svd_matrix(g, 512, 64, synth.spectrum("geometric", 64, 1e3))
    Q, R = G.rmgs(A.astype(np.float64), cutoff=16, prec=prec)
    assert M.qr_backward_error(A, Q, R) < bound

"""Pins for the oracle's LSQR and CGLS (Sec. 3.2.3, Alg. 5)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import householder as H
from oracle import krylov as K
from oracle import lls as L
from oracle import metrics as M


def _prob(m=400, n=50, seed=0, cond=None):
    g = np.random.default_rng(seed)
    if cond is None:
        A = g.standard_normal((m, n)).astype(np.float32)
    else:
        A = synth.svd_matrix(g, m, n, synth.spectrum("geometric", n, cond))
    b = g.standard_normal(m)
    return np.asarray(A), b


@pytest.mark.parametrize("k", [1, 3, 10])
def test_lsqr_iterates_match_scipy(k):
    A, b = _prob(300, 40, 1, cond=50.0)
    x, it, _ = K.lsqr(A, b, tol=0.0, maxit=k, estimate_only=True)
    xs = spla.lsqr(A.astype(np.float64), b, atol=0, btol=0, conlim=0, iter_lim=k)[0]
    assert it == k
    assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs)


@pytest.mark.parametrize("solver", [K.lsqr, K.cgls])
def test_converges_to_oracle_solution(solver):
    A, b = _prob(500, 60, 2, cond=30.0)
    xd, _, _ = L.lls_direct(A, b)
    x, it, info = solver(A, b, tol=1e-12, maxit=500)
    assert info["eta"] <= 1e-12
    assert M.forward_error(x, xd) < 1e-9


@pytest.mark.parametrize("solver", [K.lsqr, K.cgls])
def test_exact_preconditioner_converges_immediately(solver):
    # Sec. 3.2.3: with an exact R, A R^{-1} = Q has kappa = 1 and the
    # iteration converges in one step (up to rounding: within 3).
    A, b = _prob(600, 80, 3, cond=1e5)
    _, R = H.qr(A)
    x, it, info = solver(A, b, R=R, tol=1e-10, maxit=50)
    assert it <= 3
    assert info["eta"] <= 1e-10


@pytest.mark.parametrize("solver", [K.lsqr, K.cgls])
def test_contraction_bound(solver):
    # Error in the A-norm contracts at least by 2((k-1)/(k+1))^i with
    # k = kappa(A R^{-1}) (Sec. 3.2.3, CG bound on the normal equations).
    A, b = _prob(400, 40, 4)
    A64 = A.astype(np.float64)
    _, R = H.qr(A64)
    g = np.random.default_rng(5)
    Rp = R @ (np.eye(40) + np.triu(0.05 * g.standard_normal((40, 40))))
    kap = np.linalg.cond(A64 @ np.linalg.inv(Rp))
    rate = (kap - 1) / (kap + 1)
    xd, _, _ = L.lls_direct(A, b)
    e0 = np.linalg.norm(A64 @ xd)
    for i in (1, 2, 4, 8):
        x, _, _ = solver(A, b, R=Rp, tol=0.0, maxit=i)
        ei = np.linalg.norm(A64 @ (x - xd))
        assert ei <= 2 * rate ** i * e0 * (1 + 1e-6) + 1e-12


def test_cgls_equals_lsqr_in_exact_arithmetic():
    # Both minimise ||b - A x|| over the same Krylov space: iterate i agrees.
    A, b = _prob(200, 30, 6, cond=20.0)
    for i in (1, 2, 5):
        x1, _, _ = K.lsqr(A, b, tol=0.0, maxit=i, estimate_only=True)
        x2, _, _ = K.cgls(A, b, tol=0.0, maxit=i)
        assert np.linalg.norm(x1 - x2) <= 1e-9 * np.linalg.norm(x1)


def test_consistent_system_stops_on_residual():
    A, _ = _prob(300, 30, 7)
    xs = np.random.default_rng(8).standard_normal(30)
    b = L.matvec_ld(A, xs).astype(np.float64)
    x, it, _ = K.lsqr(A, b, tol=1e-10, maxit=300)
    assert M.forward_error(x, xs) < 1e-8


def test_lsqr_estimate_tracks_true_residual():
    A, b = _prob(300, 30, 9, cond=10.0)
    _, _, info = K.lsqr(A, b, tol=1e-12, maxit=100, estimate_only=True, record=True)
    assert info["hist"][-1] <= 1e-12
    x, _, _ = K.lsqr(A, b, tol=1e-12, maxit=100, estimate_only=True)
    assert M.eta_F(A, b, x) < 1e-10


def test_planted_missing_preconditioner_transpose_is_caught():
    # Dropping R^{-T} from the starting vector (the listing's literal form)
    # breaks the iteration; the exact-preconditioner pin catches it.
    A, b = _prob(300, 40, 10, cond=1e4)
    _, R = H.qr(A)
    orig = K._Op.rinv_t
    try:
        K._Op.rinv_t = lambda self, v: v.copy()
        _, it, info = K.cgls(A, b, R=R, tol=1e-10, maxit=3)
    finally:
        K._Op.rinv_t = orig
    assert info["eta"] > 1e-10

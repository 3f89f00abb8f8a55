"""Pins for the oracle's least-squares solution (Sec. 2.2, eq. opt:lls)."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import lls as L
from oracle import metrics as M

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rational_ls(Ai, bi):
    """Exact x = (A^T A)^{-1} A^T b by rational Gauss-Jordan elimination."""
    m, n = len(Ai), len(Ai[0])
    G = [[Fraction(sum(Ai[r][i] * Ai[r][j] for r in range(m))) for j in range(n)]
         + [Fraction(sum(Ai[r][i] * bi[r] for r in range(m)))] for i in range(n)]
    for c in range(n):
        p = next(r for r in range(c, n) if G[r][c] != 0)
        G[c], G[p] = G[p], G[c]
        piv = G[c][c]
        G[c] = [v / piv for v in G[c]]
        for r in range(n):
            if r != c and G[r][c] != 0:
                f = G[r][c]
                G[r] = [a - f * b for a, b in zip(G[r], G[c])]
    return [G[i][n] for i in range(n)]


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_rational(seed):
    g = np.random.default_rng(100 + seed)
    m, n = int(g.integers(4, 9)), int(g.integers(1, 5))
    while True:
        Ai = g.integers(-6, 7, size=(m, n))
        if np.linalg.matrix_rank(Ai) == n:
            break
    bi = g.integers(-9, 10, size=m)
    xr = _rational_ls(Ai.tolist(), bi.tolist())
    x, _, _ = L.lls_direct(Ai.astype(np.float32), bi.astype(np.float64))
    xe = np.array([float(v) for v in xr])
    assert np.linalg.norm(x - xe) <= 1e-14 * max(1.0, np.linalg.norm(xe))


@pytest.mark.parametrize("name", ["qr_lls_3x2_poly.json", "qr_lls_3x2_pythagorean.json"])
def test_golden(name):
    with open(os.path.join(GOLD, name)) as f:
        g = json.load(f)
    x, _, _ = L.lls_direct(np.array(g["A"], dtype=np.float32), np.array(g["b"], dtype=np.float64))
    xe = np.array([float(Fraction(v)) for v in g["x"]])
    assert np.max(np.abs(x - xe)) < 1e-15
    r = L.residual_ld(np.array(g["A"], dtype=np.float32), g["b"], x)
    re = np.array([float(Fraction(v)) for v in g["r"]])
    assert np.max(np.abs(r.astype(np.float64) - re)) < 1e-15


def test_matches_lapack_lstsq():
    p = synth.scaled_config("c3", 600, 80, seed=1)
    x, _, _ = L.lls_direct(p.A, p.b)
    xl = np.linalg.lstsq(p.A.astype(np.float64), p.b, rcond=None)[0]
    # both solve the same stored instance; they differ by LAPACK's rounding,
    # bounded by the LS perturbation bound at u64
    kappa = np.linalg.cond(p.A.astype(np.float64))
    assert M.forward_error(x, xl) < 10 * kappa ** 2 * 2.2e-16 + 1e-12


def test_consistent_system_recovers_x_star():
    g = np.random.default_rng(2)
    A = np.asfortranarray(g.standard_normal((300, 40)).astype(np.float32))
    xs = g.standard_normal(40)
    b = L.matvec_ld(A, xs).astype(np.float64)   # b = A x* (to longdouble rounding)
    x, _, _ = L.lls_direct(A, b)
    assert M.forward_error(x, xs) < 1e-14


def test_orthogonal_perturbation_and_orthogonal_rhs():
    # b = A y + h with A^T h = 0 -> x = y; b orthogonal to range(A) -> x = 0.
    g = np.random.default_rng(3)
    A = g.standard_normal((120, 10)).astype(np.float32)
    Q, _ = np.linalg.qr(A.astype(np.float64), mode="complete")
    h = Q[:, 10:] @ g.standard_normal(110)
    y = g.standard_normal(10)
    b = L.matvec_ld(A, y).astype(np.float64) + h
    x, _, _ = L.lls_direct(A, b)
    assert M.forward_error(x, y) < 1e-13
    x0, _, _ = L.lls_direct(A, h)
    assert np.linalg.norm(x0) < 1e-13 * np.linalg.norm(h)


def test_single_column_closed_form():
    a = np.array([[1.0], [2.0], [2.0]], dtype=np.float32)
    b = np.array([3.0, -1.0, 4.0])
    x, _, _ = L.lls_direct(a, b)
    assert x[0] == pytest.approx((3 - 2 + 8) / 9.0, rel=1e-15)


def test_backward_error_at_floor():
    # The oracle's solution reaches the FP64 representability floor of the
    # normalised normal-equation error on an ill-conditioned (kappa = 1e6)
    # instance: it scores no worse than x with every entry moved by one ulp,
    # and the refinement steps improve on the unrefined Alg. 1 solution.
    p = synth.scaled_config("c3", 2048, 256, seed=0)
    x0, _, _ = L.lls_direct(p.A, p.b, refine=0)
    x, _, _ = L.lls_direct(p.A, p.b)
    e, _ = M.eta(p.A, p.b, x)
    g = np.random.default_rng(0)
    floor = min(M.eta(p.A, p.b, x * (1 + g.choice([-1, 1], size=x.size) * 2.0 ** -53))[0]
                for _ in range(3))
    assert e < floor
    assert e < M.eta(p.A, p.b, x0)[0]


def test_triangular_solvers():
    g = np.random.default_rng(4)
    R = np.triu(g.standard_normal((30, 30))) + 5 * np.eye(30)
    y = g.standard_normal(30)
    assert np.allclose(R @ L.back_substitute(R, y), y, atol=1e-12)
    assert np.allclose(R.T @ L.forward_substitute_t(R, y), y, atol=1e-12)

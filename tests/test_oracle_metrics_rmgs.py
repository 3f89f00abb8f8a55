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


def test_bf16_rounding_against_definition():
    # BF16 keeps 8 significant bits of an FP32 value, rounding to nearest with
    # ties to even (Sec. 2.1 formats): the two candidates of each value are its
    # truncation and the next value away from zero; the nearer one wins, exact
    # distances by rational arithmetic, ties to the even last bit
    from fractions import Fraction
    g = np.random.default_rng(12)
    mags = np.float32(10.0) ** g.integers(-30, 30, 3000).astype(np.float32)
    x = np.concatenate([(g.standard_normal(3000) * mags).astype(np.float32),
                        np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8),
                                  1 + 2 ** -8 + 2 ** -20, 2 ** -100], np.float32)])
    y = G.to_bf16(x)
    for xi, yi in zip(x, y):
        bits = int(np.array([xi], np.float32).view(np.uint32)[0])
        lo = bits & 0xFFFF0000
        hi = lo + 0x10000
        flo = float(np.array([lo], np.uint32).view(np.float32)[0])
        fhi = float(np.array([hi], np.uint32).view(np.float32)[0])
        dlo = abs(Fraction(float(xi)) - Fraction(flo))
        dhi = abs(Fraction(float(xi)) - Fraction(fhi))
        if dlo != dhi:
            want = lo if dlo < dhi else hi
        else:
            want = lo if ((lo >> 16) & 1) == 0 else hi
        got = int(np.array([yi], np.float32).view(np.uint32)[0])
        assert got == want, (float(xi), hex(got), hex(want))


def _half(v):
    # IEEE binary16 round-to-nearest-even by Python's own conversion
    import struct
    return struct.unpack("<e", struct.pack("<e", float(v)))[0]


def test_fp16_operand_rounding_against_python_half():
    g = np.random.default_rng(13)
    x = (g.uniform(-1, 1, 4000) * 10.0 ** g.integers(-4, 5, 4000)).astype(np.float32)
    x = np.concatenate([x, np.array([1 + 2 ** -11, 1 + 3 * 2 ** -11, 2048 + 1, 65504.0], np.float32)])
    y = G.round_operand(x, "fp16")
    for xi, yi in zip(x, y):
        assert yi == _half(xi), (float(xi), yi, _half(xi))


def test_split_fp16_operand():
    # hi = fl16(x), lo = fl16(x - hi) (the split of the split-FP16 products): the
    # operand seen is hi + lo, within half an FP16 unit of lo of x (half the
    # subnormal spacing 2^-24 once x - hi falls below the FP16 normal range), and
    # exactly x when x is an FP16 value
    g = np.random.default_rng(14)
    x = (g.uniform(-1, 1, 4000) * 10.0 ** g.integers(-2, 4, 4000)).astype(np.float32)
    y = G.round_operand(x, "fp16x3")
    for xi, yi in zip(x, y):
        hi = _half(xi)
        lo = _half(np.float32(xi) - np.float32(hi))
        assert yi == hi + lo
        assert abs(float(xi) - yi) <= max(abs(lo) * 2.0 ** -11, 2.0 ** -25)
    exact = np.array([_half(v) for v in x], np.float32)
    assert np.array_equal(G.round_operand(exact, "fp16x3"), exact.astype(np.float64))


def test_float32_sums_exact_on_small_integers():
    # the emulator's products sum in float32; integer data whose partial sums stay
    # below 2^24 must come out exact
    g = np.random.default_rng(15)
    X = g.integers(-64, 65, (40, 32)).astype(np.float64)
    Y = g.integers(-64, 65, (32, 24)).astype(np.float64)
    assert np.array_equal(G._mm32(X, Y), X @ Y)

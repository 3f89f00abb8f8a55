"""Hand-derived values for the oracle's accuracy metrics (Sec. 3.2.1-3.2.2).

Each fixture in tests/golden/metrics_*.json states a tiny instance, its
derivation by hand, and the exact value of every metric as a closed form
(rationals and square roots). The closed forms are evaluated here by a small
expression reader that knows only numbers, + - * /, parentheses and sqrt, so
the expected values never come from the code under test. A wrong norm in the
denominator (||A||_2 for ||A||_F), a dropped ||r||, r = b without A x, or
Q Q^T in place of Q^T Q changes each value by far more than the tolerance.
"""
import ast
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import metrics as M

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def closed_form(expr: str) -> float:
    """Value of an expression over numbers, + - * /, parentheses and sqrt()."""
    def ev(node):
        if isinstance(node, ast.Expression):
            return ev(node.body)
        if isinstance(node, ast.Constant) and isinstance(node.value, (int, float)):
            return float(node.value)
        if isinstance(node, ast.UnaryOp) and isinstance(node.op, (ast.USub, ast.UAdd)):
            v = ev(node.operand)
            return -v if isinstance(node.op, ast.USub) else v
        if isinstance(node, ast.BinOp):
            a, b = ev(node.left), ev(node.right)
            if isinstance(node.op, ast.Add):
                return a + b
            if isinstance(node.op, ast.Sub):
                return a - b
            if isinstance(node.op, ast.Mult):
                return a * b
            if isinstance(node.op, ast.Div):
                return a / b
        if (isinstance(node, ast.Call) and isinstance(node.func, ast.Name)
                and node.func.id == "sqrt" and len(node.args) == 1):
            return math.sqrt(ev(node.args[0]))
        raise ValueError(f"unsupported expression: {expr}")
    return ev(ast.parse(expr, mode="eval"))


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _vec(v):
    return np.array([float(Fraction(s)) for s in v])


def test_closed_form_reader():
    assert closed_form("sqrt(13)/4") == pytest.approx(0.9013878188659973, rel=1e-15)
    assert closed_form("1/sqrt(29)") == pytest.approx(29 ** -0.5, rel=1e-15)
    with pytest.raises(ValueError):
        closed_form("__import__('os')")


@pytest.mark.parametrize("name", ["metrics_eta_diag_3x2.json", "metrics_eta_line_fit_3x2.json"])
def test_eta_hand_values(name):
    g = _load(name)
    A = np.array(g["A"], dtype=np.float32)
    b = np.array(g["b"], dtype=np.float64)
    x = _vec(g["x"])
    eF, nr = M.eta(A, b, x)
    assert eF == pytest.approx(closed_form(g["eta_F"]), rel=1e-14)
    assert nr == pytest.approx(closed_form(g["resid_norm"]), rel=1e-14)
    assert M.eta_F(A, b, x) == pytest.approx(closed_form(g["eta_F"]), rel=1e-14)
    # eta_2 takes ||A||_2 from 30 power-iteration steps: converged far below 1e-10 here
    assert M.eta_2(A, b, x) == pytest.approx(closed_form(g["eta_2"]), rel=1e-10)
    if "x_solution" in g:
        assert M.eta_F(A, b, _vec(g["x_solution"])) < 1e-15


def test_qr_backward_error_hand_values():
    g = _load("metrics_qr_error_3x2.json")
    A, Q, R = (np.array(g[k], dtype=np.float64) for k in ("A", "Q", "R"))
    assert M.qr_backward_error(A, Q, R) == pytest.approx(closed_form(g["backward_error_F"]), rel=1e-14)
    assert M.qr_backward_error_2(A, Q, R) == pytest.approx(closed_form(g["backward_error_2"]),
                                                           rel=1e-10)
    assert M.qr_backward_error(A, Q, R, cols=[1]) == pytest.approx(
        closed_form(g["backward_error_F_col1"]), rel=1e-14)
    assert M.r_relative_error(R, np.array(g["R_ref"])) == pytest.approx(
        closed_form(g["r_relative_error"]), rel=1e-14)


def test_orthogonality_hand_values():
    g = _load("metrics_orthogonality_4x3.json")
    Q = np.array(g["Q"], dtype=np.float64)
    assert M.orthogonality(Q) == pytest.approx(closed_form(g["orthogonality"]), rel=1e-14)
    assert M.orthogonality(Q, cols=[0, 2]) == pytest.approx(
        closed_form(g["orthogonality_cols_0_2"]), rel=1e-13)


def test_planted_wrong_norm_is_caught():
    # the fixture separates ||A||_F from ||A||_2 and keeps ||r|| in the
    # denominator: a metric with either mistake misses the hand value
    g = _load("metrics_eta_diag_3x2.json")
    A = np.array(g["A"], dtype=np.float64)
    b = np.array(g["b"], dtype=np.float64)
    x = _vec(g["x"])
    r = b - A @ x
    want = closed_form(g["eta_F"])
    wrong_norm = np.linalg.norm(A.T @ r) / (np.linalg.norm(A, 2) * np.linalg.norm(r))
    no_r = np.linalg.norm(A.T @ r) / np.linalg.norm(A)
    assert abs(wrong_norm - want) > 0.04 and abs(no_r - want) > 0.05

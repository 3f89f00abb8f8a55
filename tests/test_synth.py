"""Generators: seeded, column-major FP32, prescribed spectra (Sec. 4.2 families)."""
import numpy as np
import pytest

import synth


def test_reproducible_and_column_major():
    p1 = synth.scaled_config("c1", 128, 16, seed=0)
    p2 = synth.scaled_config("c1", 128, 16, seed=0)
    assert p1.A.dtype == np.float32 and p1.A.flags.f_contiguous
    assert np.array_equal(p1.A, p2.A) and np.array_equal(p1.b, p2.b)
    assert p1.b.dtype == np.float64


@pytest.mark.parametrize("kind,cond", [("geometric", 1e3), ("arithmetic", 1e5), ("cluster", 1e6)])
def test_spectrum_families(kind, cond):
    g = np.random.default_rng(1)
    A = synth.svd_matrix(g, 300, 40, synth.spectrum(kind, 40, cond))
    s = np.linalg.svd(A.astype(np.float64), compute_uv=False)
    assert s[0] == pytest.approx(1.0, rel=1e-5)
    assert s[0] / s[-1] == pytest.approx(cond, rel=1e-2)


def test_loguniform_pins_condition():
    s = synth.spectrum("loguniform", 64, 1e6, np.random.default_rng(2))
    assert s[0] == 1.0 and s[-1] == pytest.approx(1e-6)
    assert np.all(np.diff(s) <= 0)


def test_batched_shapes():
    ps = synth.batched_problems(count=20, seed=0)
    for p in ps:
        m, n = p.A.shape
        assert n % 8 == 0 and 32 <= n <= 256 and m % n == 0 and 4 <= m // n <= 16


def test_paper_families():
    g = np.random.default_rng(3)
    for kind in ("uniform01", "uniform11", "normal", "geometric"):
        A = synth.paper_family(g, kind, 64, 8)
        assert A.shape == (64, 8) and A.dtype == np.float32

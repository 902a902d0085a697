"""Pins of the oracle's SARA dictionary.

* Daubechies filters: Db1 and Db2 against their closed forms (golden fixture),
  and for every N: sum sqrt(2), double-shift orthonormality, N vanishing
  moments, extremal phase (the conditions that define DbN uniquely).
* Each periodised 2-D DWT is orthonormal; the scaled concatenation is a
  Parseval frame, Psi Psi^dagger = I (Sec. 4.4); Psi^dagger Psi is a projector.
* One Haar level on a 2 x 2 image gives the textbook sums and differences.
"""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import wavelets as wv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_db1_is_haar():
    np.testing.assert_allclose(wv.daubechies_lowpass(1), [1 / math.sqrt(2)] * 2, rtol=0, atol=1e-16)


def test_db2_closed_form():
    vals = [float(s) for s in open(os.path.join(GOLDEN, "db2_closed_form.txt"))
            if s.strip() and not s.startswith("#")]
    np.testing.assert_allclose(wv.daubechies_lowpass(2), vals, rtol=0, atol=1e-15)


@pytest.mark.parametrize("N", range(1, 9))
def test_filter_algebra(N):
    h = wv.daubechies_lowpass(N)
    L = len(h)
    assert L == 2 * N
    assert h.sum() == pytest.approx(math.sqrt(2), abs=1e-15)
    for m in range(N):
        s = sum(h[k] * h[k + 2 * m] for k in range(L - 2 * m))
        assert abs(s - (1.0 if m == 0 else 0.0)) < 1e-14
    k = np.arange(L, dtype=np.float64)
    for p in range(N):
        terms = (-1.0) ** k * k ** p * h
        assert abs(terms.sum()) <= 1e-13 * np.abs(terms).sum()
    g = wv.highpass(h)
    for m in range(N):
        s = sum(h[k] * g[k + 2 * m] for k in range(L - 2 * m)) + \
            sum(g[k] * h[k + 2 * m] for k in range(L - 2 * m))
        assert abs(s) < 1e-14
    # Extremal phase in Daubechies' orientation: the reversed filter, read as a
    # polynomial in increasing powers of z, is (1 + z)^N times a factor whose
    # zeros all lie strictly inside the unit disc.
    poly = h.copy()                      # highest power first == reversed filter
    for _ in range(N):
        poly, rem = np.polydiv(poly, [1.0, 1.0])
        assert np.abs(rem).max() < 1e-11
    if N > 1:
        assert np.all(np.abs(np.roots(poly)) < 1.0 - 1e-3)


def test_haar_one_level_2x2():
    x = np.array([[1.0, 2.0], [3.0, 4.0]])
    c = wv.dwt2(x, wv.daubechies_lowpass(1), 1)
    # Rows then columns with h = [1, 1]/sqrt2, g = [1, -1]/sqrt2.
    ll = (1 + 2 + 3 + 4) / 2
    lh = ((1 - 2) + (3 - 4)) / 2
    hl = ((1 + 2) - (3 + 4)) / 2
    hh = ((1 - 2) - (3 - 4)) / 2
    np.testing.assert_allclose(c, [[ll, lh], [hl, hh]], atol=1e-15)


@pytest.mark.parametrize("N", range(1, 9))
@pytest.mark.parametrize("n,levels", [(32, 2), (64, 3), (128, 4)])
def test_each_basis_orthonormal(N, n, levels):
    g = W.rng(101, 0, N * 1000 + n)
    h = wv.daubechies_lowpass(N)
    x = W.random_complex((n, n), g)
    c = wv.dwt2(x, h, levels)
    assert np.linalg.norm(c) == pytest.approx(np.linalg.norm(x), rel=1e-13)
    np.testing.assert_allclose(wv.idwt2(c, h, levels), x, rtol=0, atol=1e-12)
    # Transpose = inverse: <W x, c2> = <x, W^T c2>.
    c2 = W.random_complex((n, n), g)
    assert np.vdot(c, c2) == pytest.approx(np.vdot(x, wv.idwt2(c2, h, levels)), rel=1e-12)


def test_orthonormal_on_tiny_band():
    """Db8 (16 taps) on a 16-sample band still gives an orthonormal transform."""
    h = wv.daubechies_lowpass(8)
    g = W.rng(101, 1)
    x = g.normal(size=(16, 16))
    c = wv.dwt2(x, h, 1)
    assert np.linalg.norm(c) == pytest.approx(np.linalg.norm(x), rel=1e-13)


@pytest.mark.parametrize("mask", [wv.FULL_MASK, 1, 1 << 8, 0b111])
def test_parseval_frame(mask):
    n, levels = 64, 3
    s = wv.Sara(n, levels, mask)
    g = W.rng(101, 2, mask)
    x = W.random_complex((n, n), g)
    a = s.psi_adj(x)
    assert a.shape == (s.q, n, n)
    np.testing.assert_allclose(s.psi(a), x, rtol=0, atol=1e-12)
    assert np.linalg.norm(a) == pytest.approx(np.linalg.norm(x), rel=1e-13)
    # Psi^dagger Psi is an orthogonal projector onto the range of Psi^dagger.
    b = W.random_complex((s.q, n, n), g)
    pb = s.psi_adj(s.psi(b))
    np.testing.assert_allclose(s.psi_adj(s.psi(pb)), pb, rtol=0, atol=1e-12)
    assert np.vdot(a, b) == pytest.approx(np.vdot(x, s.psi(b)), rel=1e-12)


def test_full_dictionary_scale_is_one_third():
    s = wv.Sara(32, 2)
    assert s.q == 9 and s.scale == pytest.approx(1 / 3, abs=1e-16)
    x = np.zeros((32, 32))
    x[3, 4] = 1.0
    np.testing.assert_allclose(s.psi_adj(x)[0], x / 3, atol=1e-16)

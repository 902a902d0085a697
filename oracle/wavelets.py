"""SARA dictionary: Dirac plus Daubechies 1-8 orthonormal wavelet bases (oracle, FP64).

The dictionary is the concatenation Psi = [Psi_1, ..., Psi_q] of q orthonormal
bases (Sec. 3.3): the Dirac basis and the Daubechies bases Db1..Db8 (Sec. 3.3,
Sec. 5).  Scaled by 1/sqrt(q) it is a Parseval frame, Psi Psi^dagger = I, which
is what makes Q = Phi^dagger Phi + 2 I in the x-update (Sec. 4.4).

Readings (the paper is silent on these):
  * DbN has N vanishing moments and 2N taps (Db1 = Haar); the filter is the
    extremal-phase factor of Daubechies' polynomial, oriented so that
    Db2 = [(1+sqrt3), (3+sqrt3), (3-sqrt3), (1-sqrt3)] / (4 sqrt2);
  * boundaries are periodic, the only extension that keeps each basis exactly
    orthonormal;
  * a level filters image rows (axis 1) and then columns (axis 0) and stores the
    four sub-bands in the Mallat layout: low-low in the top-left quarter,
    (low axis 0, high axis 1) top-right, (high axis 0, low axis 1) bottom-left,
    high-high bottom-right; the next level recurses on the low-low quarter;
  * complex images are filtered with real filters, real and imaginary parts
    independently.
"""
from __future__ import annotations

import math

import numpy as np


def daubechies_lowpass(N: int) -> np.ndarray:
    """Scaling filter h of DbN (length 2N, sum sqrt(2)) by spectral factorisation.

    |m0(xi)|^2 = cos^(2N)(xi/2) P(sin^2(xi/2)),  P(y) = sum_{k<N} C(N-1+k, k) y^k.
    With z = exp(-i xi), sin^2(xi/2) = (2 - z - 1/z)/4, so each root y_k of P
    gives the pair z, 1/z solving z^2 - (2 - 4 y_k) z + 1 = 0.  Keeping the root
    with |z| < 1 for every y_k and multiplying by (1 + z)^N gives a polynomial
    whose coefficients, in increasing powers of z, are the filter reversed.
    """
    if N < 1:
        raise ValueError("N >= 1")
    if N == 1:
        return np.array([1.0, 1.0]) / math.sqrt(2.0)
    # P(y) coefficients, highest power first for numpy.roots.
    p = [math.comb(N - 1 + k, k) for k in range(N)][::-1]
    ys = np.roots(p)
    zs = []
    for y in ys:
        # z^2 - (2 - 4y) z + 1 = 0
        b = 2.0 - 4.0 * y
        disc = np.sqrt(b * b - 4.0 + 0j)
        z1, z2 = (b + disc) / 2.0, (b - disc) / 2.0
        zs.append(z1 if abs(z1) < 1.0 else z2)
    roots = np.concatenate([np.full(N, -1.0 + 0j), np.array(zs)])
    poly = np.poly(roots)                 # highest power first
    coeffs_increasing = np.real(poly[::-1])
    h = coeffs_increasing[::-1]           # Daubechies' orientation
    return h * (math.sqrt(2.0) / h.sum())


def highpass(h: np.ndarray) -> np.ndarray:
    """Wavelet filter g[m] = (-1)^m h[L-1-m] (quadrature mirror of h)."""
    L = len(h)
    return np.array([(-1.0) ** m * h[L - 1 - m] for m in range(L)])


def analysis_1d(x: np.ndarray, h: np.ndarray, g: np.ndarray, axis: int):
    """One periodised analysis step along ``axis``.

    a_k = sum_m h[m] x[(2k + m) mod s],  d_k = sum_m g[m] x[(2k + m) mod s].
    Returns (a, d), each half as long as x along ``axis``.
    """
    x = np.moveaxis(x, axis, -1)
    s = x.shape[-1]
    idx = (2 * np.arange(s // 2)[:, None] + np.arange(len(h))[None, :]) % s
    xs = x[..., idx]                      # (..., s/2, L)
    a = xs @ h
    d = xs @ g
    return np.moveaxis(a, -1, axis), np.moveaxis(d, -1, axis)


def synthesis_1d(a: np.ndarray, d: np.ndarray, h: np.ndarray, g: np.ndarray, axis: int):
    """Transpose of :func:`analysis_1d`: x[(2k + m) mod s] += h[m] a_k + g[m] d_k."""
    a = np.moveaxis(a, axis, -1)
    d = np.moveaxis(d, axis, -1)
    half = a.shape[-1]
    s = 2 * half
    out = np.zeros(a.shape[:-1] + (s,), dtype=np.result_type(a, d, h))
    for m in range(len(h)):
        pos = (2 * np.arange(half) + m) % s
        # Positions within one m are distinct, so fancy-index accumulation is exact.
        out[..., pos] += h[m] * a + g[m] * d
    return np.moveaxis(out, -1, axis)


def dwt2(x: np.ndarray, h: np.ndarray, levels: int) -> np.ndarray:
    """L-level periodised orthonormal 2-D DWT in the Mallat layout."""
    g = highpass(h)
    out = np.array(x, dtype=np.result_type(x, np.float64), copy=True)
    s = x.shape[0]
    for _ in range(levels):
        blk = out[:s, :s]
        lo1, hi1 = analysis_1d(blk, h, g, axis=1)         # rows
        ll, hl = analysis_1d(lo1, h, g, axis=0)           # columns of the low part
        lh, hh = analysis_1d(hi1, h, g, axis=0)           # columns of the high part
        half = s // 2
        out[:half, :half] = ll
        out[:half, half:s] = lh
        out[half:s, :half] = hl
        out[half:s, half:s] = hh
        s = half
    return out


def idwt2(c: np.ndarray, h: np.ndarray, levels: int) -> np.ndarray:
    """Inverse (= transpose) of :func:`dwt2`."""
    g = highpass(h)
    out = np.array(c, dtype=np.result_type(c, np.float64), copy=True)
    n = c.shape[0]
    s = n >> (levels - 1)
    for _ in range(levels):
        half = s // 2
        ll = out[:half, :half]
        lh = out[:half, half:s]
        hl = out[half:s, :half]
        hh = out[half:s, half:s]
        lo1 = synthesis_1d(ll, hl, h, g, axis=0)
        hi1 = synthesis_1d(lh, hh, h, g, axis=0)
        out[:s, :s] = synthesis_1d(lo1, hi1, h, g, axis=1)
        s *= 2
    return out


BASES = ("dirac",) + tuple(f"db{k}" for k in range(1, 9))
FULL_MASK = (1 << len(BASES)) - 1


def selected(mask: int):
    """Indices of the bases selected by ``mask`` (bit 0 Dirac, bit k Db_k)."""
    return [b for b in range(len(BASES)) if mask >> b & 1]


class Sara:
    """Psi^dagger and Psi for a dictionary mask (Sec. 3.3; Parseval scaling)."""

    def __init__(self, n: int, levels: int, mask: int = FULL_MASK):
        if n % (1 << levels):
            raise ValueError("image side must be divisible by 2^levels")
        self.n = n
        self.levels = levels
        self.bases = selected(mask)
        if not self.bases:
            raise ValueError("empty dictionary")
        self.q = len(self.bases)
        self.scale = 1.0 / math.sqrt(self.q)
        self.filters = {b: daubechies_lowpass(b) for b in self.bases if b > 0}

    def _w(self, b: int, x: np.ndarray) -> np.ndarray:
        return x.copy() if b == 0 else dwt2(x, self.filters[b], self.levels)

    def _wt(self, b: int, c: np.ndarray) -> np.ndarray:
        return c.copy() if b == 0 else idwt2(c, self.filters[b], self.levels)

    def psi_adj(self, x: np.ndarray) -> np.ndarray:
        """alpha = Psi^dagger x, shape (q, n, n)."""
        return np.stack([self.scale * self._w(b, x) for b in self.bases])

    def psi(self, alpha: np.ndarray) -> np.ndarray:
        """x = Psi alpha = (1/sqrt q) sum_b W_b^T alpha_b."""
        out = np.zeros((self.n, self.n), dtype=np.result_type(alpha, np.float64))
        for i, b in enumerate(self.bases):
            out += self._wt(b, alpha[i])
        return self.scale * out

"""Kaiser-Bessel interpolation kernel for the gridding matrix G (oracle, FP64).

The paper's package uses a compact-support Gaussian kernel for G and says other
kernels can be used (Sec. 5, discussion of eq. opmodel).  Here G uses the
Kaiser-Bessel kernel of width J grid cells with the shape parameter rule of
Beatty, Nishimura & Pauly (2005) for oversampling alpha = 2:

    beta = pi * sqrt((J / alpha)^2 (alpha - 1/2)^2 - 0.8)

phi(t)     = I0(beta sqrt(1 - (2t/J)^2)) / I0(beta)   for |t| <= J/2, else 0
phihat(l)  = integral phi(t) exp(2 pi i t l / K) dt
           = J sinh(sqrt(beta^2 - s^2)) / (sqrt(beta^2 - s^2) I0(beta)),  s = pi J l / K

The gridding correction D is d(l) = 1 / phihat(l) (Sec. 5, "d = 1/g-hat").
I0 is the modified Bessel function of the first kind, order zero, from its
power series sum_k (z/2)^(2k) / (k!)^2 (Abramowitz & Stegun 9.6.10).
"""
from __future__ import annotations

import math

import numpy as np


def i0(z):
    """Modified Bessel I0 by its power series, summed until terms stop mattering."""
    z = np.asarray(z, dtype=np.float64)
    q = (z * 0.5) ** 2
    term = np.ones_like(z)
    total = np.ones_like(z)
    k = 0
    while True:
        k += 1
        term = term * q / (k * k)
        total = total + term
        if np.all(term <= 1e-18 * total):
            break
        if k > 400:
            raise RuntimeError("I0 series did not converge")
    return total


def beta(J: int, alpha: float = 2.0) -> float:
    """Kaiser-Bessel shape parameter for width J at oversampling alpha."""
    return math.pi * math.sqrt((J / alpha) ** 2 * (alpha - 0.5) ** 2 - 0.8)


def phi(t, J: int, b: float | None = None):
    """Kernel value at offset t (grid cells) from the visibility position."""
    if b is None:
        b = beta(J)
    t = np.asarray(t, dtype=np.float64)
    r = 1.0 - (2.0 * t / J) ** 2
    inside = r >= 0.0
    arg = b * np.sqrt(np.where(inside, r, 0.0))
    return np.where(inside, i0(arg) / i0(b), 0.0)


def phihat(l, J: int, K: int, b: float | None = None):
    """Continuous Fourier transform of phi at image offset l on a K-point grid."""
    if b is None:
        b = beta(J)
    l = np.asarray(l, dtype=np.float64)
    s = math.pi * J * l / K
    w2 = b * b - s * s
    if np.any(w2 <= 0):
        raise ValueError("image offset beyond the kernel's positive band")
    w = np.sqrt(w2)
    return J * np.sinh(w) / (w * float(i0(b)))


def window(g, J: int):
    """First grid index of the J-tap window around continuous grid coordinate g.

    The window is the J consecutive integers a with g - J/2 < a <= g + J/2, i.e.
    a = floor(g - J/2) + 1, ..., floor(g - J/2) + J.
    """
    return np.floor(np.asarray(g, dtype=np.float64) - J / 2).astype(np.int64) + 1

"""Proximity operators of the three SDMM terms (oracle, FP64; Sec. 4.4).

f1(r) = ||W r||_1 = sum_j w_j |r_j|          prox: entrywise soft threshold (eq. prox1)
f2(r) = indicator of B = {r : ||y - r|| <= eps}  prox: projection onto B (eq. prox2)
f3(r) = indicator of the positive orthant        prox: projection (eq. prox3)

Readings:
  * eq. (prox2) is printed as min(1, eps/||r||) r, the projection onto a ball
    centred at 0; the set B of Sec. 4.3 is centred at y, so the projection used
    is y + (r - y) min(1, eps / ||r - y||), and it is the identity when
    ||r - y|| <= eps (no division then);
  * complex vectors are real vectors of twice the length (Sec. 4.1), so the
    positive orthant of C^N is {Re >= 0, Im = 0} and its projection is
    max(Re r, 0) + 0i;
  * the soft threshold returns 0 when |a| <= lambda, including a = 0 (the
    printed a/|a| is undefined there).
"""
from __future__ import annotations

import numpy as np


def soft_threshold(a: np.ndarray, lam) -> np.ndarray:
    """prox of lam |.| entrywise: a/|a| (|a| - lam)^+, 0 where |a| <= lam."""
    a = np.asarray(a)
    mag = np.abs(a)
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), mag.shape)
    keep = mag > lam
    scale = np.zeros_like(mag)
    scale[keep] = 1.0 - lam[keep] / mag[keep]
    return a * scale


def project_ball(r: np.ndarray, y: np.ndarray, eps: float) -> np.ndarray:
    """Projection onto {r : ||y - r||_2 <= eps}."""
    diff = np.asarray(r) - np.asarray(y)
    nrm = float(np.linalg.norm(diff))
    if nrm <= eps:
        return np.array(r, copy=True)
    return y + diff * (eps / nrm)


def project_positive(r: np.ndarray) -> np.ndarray:
    """Projection onto the positive orthant of C^N viewed as R^(2N)."""
    r = np.asarray(r)
    return np.maximum(np.real(r), 0.0).astype(r.dtype)

"""Reweighted l1 analysis (SARA proper, RWBP, RWBPDb8): a sequence of weighted
problems of Sec. 3.3 eq. (delta), each solved by SDMM (oracle, FP64).

The paper (Sec. 3.3) replaces the l0 prior ||Psi^dagger x||_0 by a weighted l1
norm and solves a sequence of weighted problems whose weights are essentially
the inverse of the magnitudes of the previous solution's coefficients (the
reweighting of Candes, Wakin & Boyd); the non-reweighted problems are the
weighted one with W = I (Sec. 5, Sec. 6: BP, BPDb8, BPSA).

Readings (the paper defers the details to its SARA reference, which is not
available here, so this part is parity unpinned against the paper):
  * pass 0 solves the unweighted problem (W = I) from x^(0);
  * pass k >= 1 uses w_j = delta_k / (delta_k + |alpha_j|), alpha = Psi^dagger
    x_hat^(k-1): the inverse of the coefficient magnitude, regularised by
    delta_k so that zero coefficients get weight 1 and no weight exceeds 1;
  * delta_1 = delta0 if given (> 0), else the root mean square of |alpha| of
    the first solution (1 if that is 0); delta_{k+1} = max(rho delta_k,
    delta_min);
  * each pass restarts Algorithm 1 (duals zero) from the previous solution,
    with the same penalty gamma (the first pass's) and the same T and n_cg;
  * passes stop after `outer` reweightings, or earlier once
    ||x_hat^(k) - x_hat^(k-1)|| <= tol ||x_hat^(k)|| when tol > 0.
"""
from __future__ import annotations

import math

import numpy as np

from . import sdmm as _sdmm


def weights(alpha: np.ndarray, delta: float) -> np.ndarray:
    """w = delta / (delta + |alpha|), entrywise (the reweighting rule above)."""
    return delta / (delta + np.abs(alpha))


def first_delta(alpha: np.ndarray, delta0: float) -> float:
    """delta_1: delta0 if positive, else the RMS of |alpha| (1 if all zero)."""
    if delta0 > 0:
        return float(delta0)
    rms = math.sqrt(float(np.mean(np.abs(alpha) ** 2)))
    return rms if rms > 0 else 1.0


def sdmm_reweighted(y, eps, op, sara, T, n_cg=16, outer=3, gamma=None, beta=1e-3,
                    x0=None, delta0=0.0, rho=0.1, delta_min=0.0, tol=0.0, cg_tol=0.0):
    """Pass 0 (W = I) then up to `outer` reweighted passes of Algorithm 1.

    Returns (xhat, passes, info) with passes the number of SDMM runs made and
    info a list of per-pass dicts (delta, last iteration's f1 and nu, the
    relative change of x).
    """
    x, _, hist, gamma = _sdmm.sdmm(y, eps, op, sara, T, n_cg, gamma=gamma, beta=beta, x0=x0,
                                   cg_tol=cg_tol)
    info = [{"delta": None, "f1": hist[-1]["f1"] if hist else 0.0,
             "nu": hist[-1]["nu"] if hist else 0.0, "change": None}]
    alpha = sara.psi_adj(x)
    delta = first_delta(alpha, delta0)
    passes = 1
    for _ in range(outer):
        w = weights(alpha, delta)
        x_new, _, hist, _ = _sdmm.sdmm(y, eps, op, sara, T, n_cg, gamma=gamma, weights=w, x0=x,
                                       cg_tol=cg_tol)
        nx = float(np.linalg.norm(x_new))
        change = float(np.linalg.norm(x_new - x)) / nx if nx > 0 else 0.0
        info.append({"delta": delta, "f1": hist[-1]["f1"] if hist else 0.0,
                     "nu": hist[-1]["nu"] if hist else 0.0, "change": change})
        x = x_new
        passes += 1
        if tol > 0 and change <= tol:
            break
        alpha = sara.psi_adj(x)
        delta = max(rho * delta, delta_min)
    return x, passes, info


def sdmm_tv_reweighted(y, eps, op, T, n_cg=16, n_inner=20, outer=3, gamma=None, beta=1e-3, x0=None,
                       delta0=0.0, rho=0.1, delta_min=0.0, tol=0.0):
    """Reweighted TV (RWTV, Sec. 5 and Sec. 6): the same passes as
    :func:`sdmm_reweighted` with the weighted TV problem of oracle/tv.py and
    w_ij = delta / (delta + |(grad x)_ij|); delta_1 from the gradient
    magnitudes of the first solution."""
    from . import tv
    x, _, hist, gamma = tv.sdmm_tv(y, eps, op, T, n_cg, n_inner, gamma=gamma, beta=beta, x0=x0)
    info = [{"delta": None, "nu": hist[-1]["nu"] if hist else 0.0, "change": None}]
    delta = first_delta(tv.magnitude(x), delta0)
    passes = 1
    for _ in range(outer):
        w = tv.tv_weights(x, delta)
        x_new, _, hist, _ = tv.sdmm_tv(y, eps, op, T, n_cg, n_inner, gamma=gamma, weights=w, x0=x)
        nx = float(np.linalg.norm(x_new))
        change = float(np.linalg.norm(x_new - x)) / nx if nx > 0 else 0.0
        info.append({"delta": delta, "nu": hist[-1]["nu"] if hist else 0.0, "change": change, "weights": w})
        x = x_new
        passes += 1
        if tol > 0 and change <= tol:
            break
        delta = max(rho * delta, delta_min)
    return x, passes, info

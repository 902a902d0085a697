"""Weighted total-variation prior and SDMM for the TV problems (oracle, FP64).

TV (Sec. 3.3, eq. tvproblem; Sec. 6 adds positivity): minimise ||x||_TV =
||grad x||_1, the l1 norm of the image gradient magnitude, subject to
||y - Phi x|| <= eps and x >= 0.  The weighted form ||W grad x||_1 (Sec. 5)
puts a positive weight on each pixel's gradient magnitude; W = I is plain TV.

SDMM (Algorithm 1) with S = 3: f1 = gamma-scaled weighted TV with L1 = I, f2
the l2 ball with L2 = Phi, f3 the positive orthant with L3 = I, so
Q = 2 I + Phi^dagger Phi as for a Parseval dictionary.  The proximity
operator of the TV term is computed iteratively (Sec. 5 names the fast
gradient projection of Beck & Teboulle on the dual of the denoising problem).

Readings (the paper gives no formulas for these):
  * the gradient is the forward difference with the last row / column
    differences set to zero (Beck & Teboulle's discretisation):
        (grad x)_ij = (x_{i+1,j} - x_{ij}, x_{i,j+1} - x_{ij});
  * a complex image is a real vector of twice the length (Sec. 4.1): the
    gradient magnitude at a pixel is sqrt(|dx|^2 + |dy|^2) with complex moduli,
    and the dual variables are complex;
  * the prox of lam TV_w at b: minimise ||x - b||^2 / 2 + lam sum_ij w_ij
    |(grad x)_ij| by fast gradient projection on the dual, step 1/(8 lam),
    dual variables started at zero, a fixed number of iterations;
  * the penalty gamma = beta ||L1^dagger Phi^dagger y||_inf with L1 = I;
  * TV's reweighting (RWTV) uses w_ij = delta / (delta + |(grad x)_ij|).
"""
from __future__ import annotations

import math

import numpy as np

from . import prox
from .sdmm import State, conjugate_gradient, penalty


def grad(x: np.ndarray):
    """Forward differences (dx, dy), zero on the last row (dx) / column (dy)."""
    x = np.asarray(x)
    dx = np.zeros_like(x)
    dy = np.zeros_like(x)
    dx[:-1, :] = x[1:, :] - x[:-1, :]
    dy[:, :-1] = x[:, 1:] - x[:, :-1]
    return dx, dy


def grad_adj(p: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Adjoint of :func:`grad` (minus the divergence): <grad x, (p, q)> = <x, grad_adj(p, q)>."""
    out = np.zeros(np.broadcast_shapes(p.shape, q.shape), dtype=np.result_type(p, q))
    out[:-1, :] -= p[:-1, :]
    out[1:, :] += p[:-1, :]
    out[:, :-1] -= q[:, :-1]
    out[:, 1:] += q[:, :-1]
    return out


def magnitude(x: np.ndarray) -> np.ndarray:
    """|(grad x)_ij| = sqrt(|dx|^2 + |dy|^2)."""
    dx, dy = grad(x)
    return np.sqrt(np.abs(dx) ** 2 + np.abs(dy) ** 2)


def tv_norm(x: np.ndarray, weights=None) -> float:
    """||W grad x||_1 = sum_ij w_ij |(grad x)_ij|."""
    m = magnitude(x)
    return float(np.sum(m if weights is None else weights * m))


def prox_tv(b: np.ndarray, lam: float, n_iter: int, weights=None, return_dual: bool = False):
    """prox of lam ||W grad .||_1 at b by fast gradient projection on the dual.

    Dual of the denoising problem: x = b - lam grad^dagger(p, q) with
    |(p, q)_ij| <= w_ij.  Each iteration takes a gradient step of 1/(8 lam) on
    the dual objective from the extrapolated point, projects onto the
    pointwise discs, and extrapolates with the t_k sequence of the fast
    method (t_1 = 1, t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2).
    """
    b = np.asarray(b, dtype=np.complex128)
    if lam <= 0 or n_iter <= 0:
        z = np.zeros_like(b)
        return (b.copy(), z, z.copy()) if return_dual else b.copy()
    w = np.ones(b.shape) if weights is None else np.asarray(weights, dtype=np.float64)
    p = np.zeros_like(b)
    q = np.zeros_like(b)
    r, s = p.copy(), q.copy()
    t = 1.0
    for _ in range(n_iter):
        u = b - lam * grad_adj(r, s)
        gx, gy = grad(u)
        pn = r + gx / (8.0 * lam)
        qn = s + gy / (8.0 * lam)
        mag = np.sqrt(np.abs(pn) ** 2 + np.abs(qn) ** 2)
        shrink = np.maximum(1.0, mag / np.maximum(w, 1e-300))
        shrink = np.where(w > 0, shrink, np.inf)
        pn = np.where(w > 0, pn / shrink, 0)
        qn = np.where(w > 0, qn / shrink, 0)
        t_next = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        r = pn + ((t - 1.0) / t_next) * (pn - p)
        s = qn + ((t - 1.0) / t_next) * (qn - q)
        p, q, t = pn, qn, t_next
    x = b - lam * grad_adj(p, q)
    return (x, p, q) if return_dual else x


def tv_weights(x: np.ndarray, delta: float) -> np.ndarray:
    """RWTV weights w_ij = delta / (delta + |(grad x)_ij|)."""
    return delta / (delta + magnitude(x))


def sdmm_tv(y, eps, op, T, n_cg=16, n_inner=20, gamma=None, beta=1e-3, weights=None, x0=None):
    """Algorithm 1 for the (weighted) TV problem with positivity, S = 3:
    L1 = I (TV prox), L2 = Phi (l2 ball), L3 = I (positive orthant).
    Returns (xhat, state, history, gamma); history holds f1 = ||W grad x||_1,
    zeta and nu per iteration."""
    n = op.n
    if gamma is None:
        gamma = penalty(y, op.phi_adj, lambda v: v, beta)
    x0 = np.zeros((n, n), dtype=np.complex128) if x0 is None else np.asarray(x0, dtype=np.complex128)
    # Steps 1-3: r_i = L_i x0, z_i = 0, x_i = L_i^dagger r_i.
    st = State(x0.copy(), np.zeros_like(x0), np.zeros(op.M, dtype=np.complex128), np.zeros_like(x0),
               x0 + op.phi_adj(op.phi(x0)) + x0, 0.0, 0)
    hist = []

    def Q(v):
        return v + op.phi_adj(op.phi(v)) + v

    for _ in range(T):
        xhat = conjugate_gradient(Q, st.rhs, st.xhat, n_cg)
        # i = 1: weighted TV (L1 = I).
        v1 = xhat + st.z1
        r1 = prox_tv(v1, gamma, n_inner, weights)
        z1 = v1 - r1
        x1 = r1 - z1
        # i = 2: l2 ball (L2 = Phi).
        l2 = op.phi(xhat)
        v2 = l2 + st.z2
        r2 = prox.project_ball(v2, y, eps)
        z2 = v2 - r2
        x2 = op.phi_adj(r2 - z2)
        # i = 3: positive orthant (L3 = I).
        v3 = xhat + st.z3
        r3 = prox.project_positive(v3)
        z3 = v3 - r3
        x3 = r3 - z3
        f1 = tv_norm(xhat, weights)
        zeta = math.inf if st.f1_prev == 0.0 else abs(f1 - st.f1_prev) / abs(st.f1_prev)
        nu = float(np.linalg.norm(y - l2)) / eps
        st.xhat, st.z1, st.z2, st.z3, st.rhs, st.f1_prev = xhat, z1, z2, z3, x1 + x2 + x3, f1
        st.t += 1
        hist.append({"f1": f1, "zeta": zeta, "nu": nu})
    return st.xhat, st, hist, gamma

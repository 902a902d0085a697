"""SDMM for the weighted l1 analysis problem with positivity (oracle, FP64).

Problem (Sec. 3.3, eq. delta):  min ||W Psi^dagger x||_1  s.t.  ||y - Phi x||_2 <= eps,
x in the positive orthant.  SDMM form (Sec. 4.3, eq. cvx2) with S = 3:
L1 = Psi^dagger, L2 = Phi, L3 = I and f1 = ||W .||_1, f2 = i_B, f3 = i_C.

Algorithm 1 (Sec. 4.4) is followed step by step:
  init      gamma > 0, x^(0), z_i = 0, r_i = L_i x^(0), x_i = L_i^dagger r_i
  step 5    x^(t) = Q^{-1} sum_i x_i, solved by conjugate gradient (Sec. 4.4),
            Q = Phi^dagger Phi + Psi Psi^dagger + I = Phi^dagger Phi + 2 I for a
            Parseval Psi
  step 7    r_i = prox_{gamma f_i}(L_i x^(t) + z_i)
  step 8    z_i = z_i + L_i x^(t) - r_i
  step 9    x_i = L_i^dagger (r_i - z_i)
  halting   zeta = |f1(L1 x^(t)) - f1(L1 x^(t-1))| / |f1(L1 x^(t-1))| < xi and
            nu = ||y - L2 x^(t)|| / eps in [1 - tau, 1 + tau]  (Sec. 4.4)

Readings (the paper is silent):
  * x^(0) = 0 unless given; CG is warm-started from x^(t-1) and runs a fixed
    number n_cg of iterations (stopping early only on an exactly zero
    residual, where the next step would divide 0 by 0), or, when a tolerance
    tol > 0 is given, stops before iteration k once ||r_k|| <= tol ||r_0||
    (the textbook relative-residual rule; the paper fixes no stopping rule);
  * zeta is +inf while the previous f1 is 0;
  * the algorithm runs T iterations unless early stopping is requested.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import prox


def vdot(a: np.ndarray, b: np.ndarray) -> complex:
    """Complex inner product <a, b> = sum conj(a) b."""
    return np.vdot(np.ravel(a), np.ravel(b))


def conjugate_gradient(Q, b: np.ndarray, x0: np.ndarray, n_iter: int, tol: float = 0.0) -> np.ndarray:
    """Hestenes-Stiefel CG for a Hermitian positive-definite Q (Sec. 4.4, step 5)."""
    x = np.array(x0, dtype=np.complex128, copy=True)
    r = b - Q(x)
    p = r.copy()
    rr = float(np.real(vdot(r, r)))
    rr0 = rr
    for _ in range(n_iter):
        if rr == 0.0 or (tol > 0.0 and rr <= tol * tol * rr0):
            break
        Qp = Q(p)
        alpha = rr / float(np.real(vdot(p, Qp)))
        x = x + alpha * p
        r = r - alpha * Qp
        rr_new = float(np.real(vdot(r, r)))
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x


def penalty(y: np.ndarray, phi_adj, psi_adj, beta: float = 1e-3) -> float:
    """gamma = beta ||Psi^dagger Phi^dagger y||_inf (Sec. 4.4)."""
    return beta * float(np.max(np.abs(psi_adj(phi_adj(y)))))


def noise_sigma(y0: np.ndarray, isnr_db: float) -> float:
    """sigma_n from ISNR = 20 log10(||y0|| / ||n||) with E||n||^2 = M sigma_n^2 (Sec. 6)."""
    M = y0.size
    return float(np.linalg.norm(y0)) * 10.0 ** (-isnr_db / 20.0) / math.sqrt(M)


def noise_bound(M: int, sigma: float) -> float:
    """eps with eps^2 = (2M + 4 sqrt(M)) sigma^2 / 2 (Sec. 6, chi^2 bound)."""
    return math.sqrt((2.0 * M + 4.0 * math.sqrt(M)) * sigma * sigma / 2.0)


def snr_db(x: np.ndarray, xhat: np.ndarray) -> float:
    """SNR = 20 log10(||x|| / ||x - xhat||) (Sec. 6)."""
    return 20.0 * math.log10(np.linalg.norm(x) / np.linalg.norm(x - xhat))


@dataclasses.dataclass
class State:
    """Everything Algorithm 1 carries from one iteration to the next."""
    xhat: np.ndarray
    z1: np.ndarray
    z2: np.ndarray
    z3: np.ndarray
    rhs: np.ndarray        # sum_i x_i
    f1_prev: float
    t: int = 0

    def copy(self) -> "State":
        return State(self.xhat.copy(), self.z1.copy(), self.z2.copy(), self.z3.copy(),
                     self.rhs.copy(), self.f1_prev, self.t)


def f1_value(alpha: np.ndarray, weights) -> float:
    """f1(r) = sum_j w_j |r_j| (Sec. 4.4)."""
    a = np.abs(alpha)
    return float(np.sum(a if weights is None else weights * a))


def initial_state(y, phi, phi_adj, psi, psi_adj, x0=None, n=None) -> State:
    """Steps 1-3 of Algorithm 1."""
    if x0 is None:
        x0 = np.zeros((n, n), dtype=np.complex128)
    x0 = np.asarray(x0, dtype=np.complex128)
    r1, r2, r3 = psi_adj(x0), phi(x0), x0.copy()
    z1, z2, z3 = np.zeros_like(r1), np.zeros_like(r2), np.zeros_like(r3)
    rhs = psi(r1) + phi_adj(r2) + r3
    return State(x0.copy(), z1, z2, z3, rhs, 0.0, 0)


def iterate(state: State, y, eps, gamma, phi, phi_adj, psi, psi_adj, n_cg,
            weights=None, cg_tol=0.0) -> dict:
    """One iteration t of Algorithm 1 (steps 5-9); updates ``state`` in place."""
    def Q(v):
        return phi_adj(phi(v)) + 2.0 * v

    # Step 5.
    xhat = conjugate_gradient(Q, state.rhs, state.xhat, n_cg, cg_tol)
    # Steps 7-9 for i = 1 (L1 = Psi^dagger, f1 = ||W .||_1).
    l1 = psi_adj(xhat)
    v1 = l1 + state.z1
    lam = gamma if weights is None else gamma * weights
    r1 = prox.soft_threshold(v1, lam)
    z1 = v1 - r1
    x1 = psi(r1 - z1)
    # i = 2 (L2 = Phi, f2 = indicator of the l2 ball around y).
    l2 = phi(xhat)
    v2 = l2 + state.z2
    r2 = prox.project_ball(v2, y, eps)
    z2 = v2 - r2
    x2 = phi_adj(r2 - z2)
    # i = 3 (L3 = I, f3 = indicator of the positive orthant).
    v3 = xhat + state.z3
    r3 = prox.project_positive(v3)
    z3 = v3 - r3
    x3 = r3 - z3
    # Halting quantities.
    f1 = f1_value(l1, weights)
    zeta = math.inf if state.f1_prev == 0.0 else abs(f1 - state.f1_prev) / abs(state.f1_prev)
    nu = float(np.linalg.norm(y - l2)) / eps
    state.xhat, state.z1, state.z2, state.z3 = xhat, z1, z2, z3
    state.rhs = x1 + x2 + x3
    state.f1_prev = f1
    state.t += 1
    return {"f1": f1, "zeta": zeta, "nu": nu}


def sdmm(y, eps, op, sara, T, n_cg=16, gamma=None, beta=1e-3, weights=None,
         x0=None, state=None, early_stop=False, xi=1e-3, tau=0.1, cg_tol=0.0):
    """Run Algorithm 1 for up to T iterations.

    ``op`` provides phi / phi_adj (oracle.nufft.Operator), ``sara`` provides
    psi / psi_adj (oracle.wavelets.Sara).  Returns (xhat, state, history).
    """
    if gamma is None:
        gamma = penalty(y, op.phi_adj, sara.psi_adj, beta)
    if state is None:
        state = initial_state(y, op.phi, op.phi_adj, sara.psi, sara.psi_adj, x0, n=op.n)
    history = []
    for _ in range(T):
        h = iterate(state, y, eps, gamma, op.phi, op.phi_adj, sara.psi, sara.psi_adj,
                    n_cg, weights, cg_tol)
        history.append(h)
        if early_stop and h["zeta"] < xi and (1 - tau) <= h["nu"] <= (1 + tau):
            break
    return state.xhat, state, history, gamma

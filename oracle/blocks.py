"""SDMM with the data split into R blocks (oracle, FP64; Sec. 4.5).

The visibilities and the measurement operator are partitioned into R blocks
(eq. blocks): y = [y_1; ...; y_R], Phi = [Phi_1; ...; Phi_R], and every block
gets its own data constraint ||y_i - Phi_i x|| <= eps_i (eq. dbp1).  SDMM
(Algorithm 1) then runs with S = R + 2 terms (eq. dbp2):

  f1 = ||W .||_1 with L1 = Psi^dagger,
  f2 = indicator of the positive orthant with L2 = I,
  f_{i+2} = indicator of the l2 ball of radius eps_i around y_i with
            L_{i+2} = Phi_i, i = 1..R.

Q = sum_i L_i^dagger L_i = Psi Psi^dagger + I + sum_i Phi_i^dagger Phi_i, which
is 2 I + Phi^dagger Phi for a Parseval Psi; it is applied here as the sum over
the blocks, term by term, as the paper writes it.

A block is a set of visibility indices; Phi_i is the restriction of Phi to
those rows (the same G rows, the same F and D), and Phi_i^dagger its exact
adjoint (Phi^dagger of the block's values placed at their rows, zeros
elsewhere).  Readings as in oracle/sdmm.py; the halting quantity nu of a
blocked run is the largest of the blocks' ||y_i - Phi_i x|| / eps_i.
"""
from __future__ import annotations

import math

import numpy as np

from . import prox
from .sdmm import State, conjugate_gradient, f1_value, penalty


class Block:
    """Phi_i and Phi_i^dagger of the visibility indices ``idx`` of ``op``."""

    def __init__(self, op, idx):
        self.op = op
        self.idx = np.asarray(idx, dtype=np.int64)

    def phi(self, x):
        return self.op.phi(x)[self.idx]

    def phi_adj(self, w):
        full = np.zeros(self.op.M, dtype=np.complex128)
        full[self.idx] = w
        return self.op.phi_adj(full)


def initial_state(blocks, psi, psi_adj, x0, n):
    """Algorithm 1 steps 1-3 for S = R + 2: r_i = L_i x0, z_i = 0, x_i = L_i^dagger r_i."""
    x0 = np.zeros((n, n), dtype=np.complex128) if x0 is None else np.asarray(x0, dtype=np.complex128)
    r1 = psi_adj(x0)
    rhs = psi(r1) + x0
    for b in blocks:
        rhs = rhs + b.phi_adj(b.phi(x0))
    z = [np.zeros_like(r1), np.zeros_like(x0)] + [np.zeros(len(b.idx), dtype=np.complex128) for b in blocks]
    return State(x0.copy(), z[0], z[2:], z[1], rhs, 0.0, 0)


def iterate(state, ys, eps, gamma, blocks, psi, psi_adj, n_cg, weights=None):
    """One iteration (steps 5-9) with S = R + 2; updates ``state`` in place."""
    def Q(v):
        out = psi(psi_adj(v)) + v
        for b in blocks:
            out = out + b.phi_adj(b.phi(v))
        return out

    xhat = conjugate_gradient(Q, state.rhs, state.xhat, n_cg)
    # i = 1: l1 (L1 = Psi^dagger).
    l1 = psi_adj(xhat)
    v1 = l1 + state.z1
    r1 = prox.soft_threshold(v1, gamma if weights is None else gamma * weights)
    z1 = v1 - r1
    rhs = psi(r1 - z1)
    # i = 2: positivity (L2 = I).
    v2 = xhat + state.z3
    r2 = prox.project_positive(v2)
    z_pos = v2 - r2
    rhs = rhs + (r2 - z_pos)
    # i = 3 .. R + 2: one l2 ball per block (L_{i+2} = Phi_i).
    z_blocks, nus = [], []
    for b, y_i, e_i, z_i in zip(blocks, ys, eps, state.z2):
        l = b.phi(xhat)
        v = l + z_i
        r = prox.project_ball(v, y_i, e_i)
        zn = v - r
        rhs = rhs + b.phi_adj(r - zn)
        z_blocks.append(zn)
        nus.append(float(np.linalg.norm(y_i - l)) / e_i)
    f1 = f1_value(l1, weights)
    zeta = math.inf if state.f1_prev == 0.0 else abs(f1 - state.f1_prev) / abs(state.f1_prev)
    state.xhat, state.z1, state.z2, state.z3 = xhat, z1, z_blocks, z_pos
    state.rhs = rhs
    state.f1_prev = f1
    state.t += 1
    return {"f1": f1, "zeta": zeta, "nu": max(nus) if nus else 0.0, "nu_blocks": nus}


def sdmm_blocks(y, eps, block_idx, op, sara, T, n_cg=16, gamma=None, beta=1e-3, weights=None, x0=None):
    """Algorithm 1 on the blocked problem (eq. dbp2).

    y: all M visibilities; eps: one bound per block; block_idx: one index array
    per block (a partition of range(M)).  gamma defaults to beta ||Psi^dagger
    Phi^dagger y||_inf (Phi^dagger y = sum_i Phi_i^dagger y_i).
    Returns (xhat, state, history, gamma).
    """
    blocks = [Block(op, idx) for idx in block_idx]
    ys = [np.asarray(y)[b.idx] for b in blocks]
    if gamma is None:
        gamma = penalty(y, op.phi_adj, sara.psi_adj, beta)
    state = initial_state(blocks, sara.psi, sara.psi_adj, x0, op.n)
    history = [iterate(state, ys, eps, gamma, blocks, sara.psi, sara.psi_adj, n_cg, weights) for _ in range(T)]
    return state.xhat, state, history, gamma

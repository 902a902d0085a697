"""Measurement operator Phi = G F D Z B and its adjoint (oracle, FP64).

Follows Sec. 5, eq. (opmodel), with the primary beam B = I as in every
experiment of Sec. 6 and oversampling factor k = 2 per axis:

  Z  embeds the n x n image into the K x K grid, K = 2n (zero padding);
  D  multiplies by the gridding correction d(l1) d(l2), d = 1 / phihat;
  F  is the unitary 2-D DFT on the K x K grid (numpy's fft2 scaled by 1/K);
  G  is the sparse M x K^2 interpolation matrix with J x J Kaiser-Bessel taps
     per row (kernel in oracle.kaiser_bessel).

Readings of silent passages (each also listed in the design notes):
  * pixel p of an n-pixel axis sits at offset l = p - n/2 from the image centre,
    and the zero-padded image places it at grid index (p - n/2) mod K;
  * u pairs with image axis 0 (rows), v with axis 1; u, v are in radians per
    pixel and lie in [-pi, pi]; grid coordinate g = u K / (2 pi);
  * the grid is periodic, so window index a is taken mod K;
  * the forward transform carries exp(-i u.l) (sign of eq. ri1).

The exact sum that the operator approximates, A x = (1/K) sum_l x_l
exp(-i (u l1 + v l2)), is :func:`direct` (brute force, for pins only).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import kaiser_bessel as kb


def grid_side(n: int, oversample: int = 2) -> int:
    return oversample * n


def offsets(n: int) -> np.ndarray:
    """Image offsets l = p - n/2 of the n pixels along one axis."""
    return np.arange(n, dtype=np.int64) - n // 2


def deapodisation(n: int, K: int, J: int) -> np.ndarray:
    """d(l) = 1 / phihat(l) for the n offsets of one axis (operator D, Sec. 5)."""
    return 1.0 / kb.phihat(offsets(n), J, K)


def g_rows(uv: np.ndarray, K: int, J: int):
    """Nonzeros of the rows of G for visibilities uv (M x 2).

    Returns (cols, vals), each of shape (M, J*J): column index a*K + b of the
    grid cell (a, b) (both taken mod K) and weight phi(g_u - a) phi(g_v - b).
    """
    uv = np.asarray(uv, dtype=np.float64)
    g = uv * (K / (2.0 * math.pi))                      # (M, 2) grid coordinates
    a0 = kb.window(g, J)                                # (M, 2) first window index
    taps = np.arange(J, dtype=np.int64)
    a = a0[:, :, None] + taps[None, None, :]            # (M, 2, J) window indices
    w = kb.phi(g[:, :, None] - a, J)                    # (M, 2, J) 1-D weights
    am = np.mod(a, K)
    cols = am[:, 0, :, None] * K + am[:, 1, None, :]    # (M, J, J)
    vals = w[:, 0, :, None] * w[:, 1, None, :]
    return cols.reshape(len(uv), J * J), vals.reshape(len(uv), J * J)


def real_matvec(A, v: np.ndarray) -> np.ndarray:
    """A v for a real sparse A and a complex v: A applied to Re v and Im v.

    Identical values to A @ v (each output is the same sum of real weight times
    real or imaginary part); it spares scipy a complex copy of A per product."""
    v = np.asarray(v, dtype=np.complex128)
    return (A @ np.ascontiguousarray(v.real)) + 1j * (A @ np.ascontiguousarray(v.imag))


def g_matrix(uv: np.ndarray, K: int, J: int, chunk: int = 1 << 16) -> sp.csr_matrix:
    """Sparse interpolation matrix G (M x K^2, real), built chunk by chunk."""
    M = len(uv)
    indptr = np.arange(0, M * J * J + 1, J * J, dtype=np.int64)
    indices = np.empty(M * J * J, dtype=np.int64)
    data = np.empty(M * J * J, dtype=np.float64)
    for s in range(0, M, chunk):
        c, v = g_rows(uv[s:s + chunk], K, J)
        indices[s * J * J:(s + len(c)) * J * J] = c.ravel()
        data[s * J * J:(s + len(c)) * J * J] = v.ravel()
    return sp.csr_matrix((data, indices, indptr), shape=(M, K * K))


class Operator:
    """Phi and Phi^dagger for one coverage (Sec. 5, eq. opmodel; B = I)."""

    def __init__(self, n: int, uv: np.ndarray, J: int, oversample: int = 2):
        if n % 2:
            raise ValueError("image side must be even")
        self.n = n
        self.K = grid_side(n, oversample)
        self.J = J
        self.uv = np.asarray(uv, dtype=np.float64)
        self.M = len(self.uv)
        self.d = deapodisation(n, self.K, J)
        self.G = g_matrix(self.uv, self.K, J)
        self._rows = np.mod(offsets(n), self.K)         # grid index of each pixel

    # Z then D: zero-padded, corrected image on the K x K grid.
    def _pad(self, x: np.ndarray) -> np.ndarray:
        xp = np.zeros((self.K, self.K), dtype=np.complex128)
        xp[np.ix_(self._rows, self._rows)] = self.d[:, None] * self.d[None, :] * x
        return xp

    def forward_grid(self, x: np.ndarray) -> np.ndarray:
        """F D Z x: the oversampled unitary spectrum of the corrected image."""
        return np.fft.fft2(self._pad(x)) / self.K

    def phi(self, x: np.ndarray) -> np.ndarray:
        """y = G F D Z x."""
        return real_matvec(self.G, self.forward_grid(x).ravel())

    def phi_adj(self, w: np.ndarray) -> np.ndarray:
        """x = Z^T D F^dagger G^T w (exact conjugate transpose of phi)."""
        grid = real_matvec(self.G.T, w).reshape(self.K, self.K)
        xp = np.fft.ifft2(grid) * self.K                # F^dagger of the unitary F
        return self.d[:, None] * self.d[None, :] * xp[np.ix_(self._rows, self._rows)]

    def grid_adj(self, w: np.ndarray) -> np.ndarray:
        """G^T w as a K x K grid (gridding alone)."""
        return real_matvec(self.G.T, w).reshape(self.K, self.K)

    def gram(self) -> sp.csr_matrix:
        """G^T G as a sparse K^2 x K^2 matrix (the precomputed Gram operator
        proposed for the CG x-update, Sec. 4.5 and Sec. 7)."""
        return (self.G.T @ self.G).tocsr()

    def phi_adj_phi_gram(self, x: np.ndarray, H=None) -> np.ndarray:
        """Phi^dagger Phi x with G^T G applied as the stored matrix H."""
        H = self.gram() if H is None else H
        grid = real_matvec(H, self.forward_grid(x).ravel()).reshape(self.K, self.K)
        xp = np.fft.ifft2(grid) * self.K
        return self.d[:, None] * self.d[None, :] * xp[np.ix_(self._rows, self._rows)]

    def degrid(self, grid: np.ndarray) -> np.ndarray:
        """G grid (degridding alone)."""
        return real_matvec(self.G, np.asarray(grid).ravel())


def phi_sampled(x: np.ndarray, uv: np.ndarray, J: int, idx: np.ndarray,
                oversample: int = 2) -> np.ndarray:
    """Phi x at the visibilities ``idx`` only, without building all of G.

    Each visibility is one row of G applied to the full oversampled spectrum, so
    a subset of rows gives the same values as the full operator.
    """
    n = x.shape[0]
    K = grid_side(n, oversample)
    d = deapodisation(n, K, J)
    rows = np.mod(offsets(n), K)
    xp = np.zeros((K, K), dtype=np.complex128)
    xp[np.ix_(rows, rows)] = d[:, None] * d[None, :] * x
    X = (np.fft.fft2(xp) / K).ravel()
    cols, vals = g_rows(np.asarray(uv, dtype=np.float64)[idx], K, J)
    return np.sum(vals * X[cols], axis=1)


def direct(x: np.ndarray, uv: np.ndarray, oversample: int = 2) -> np.ndarray:
    """Exact sum (1/K) sum_{p,q} x[p,q] exp(-i (u (p - n/2) + v (q - n/2)))."""
    n = x.shape[0]
    K = grid_side(n, oversample)
    l = offsets(n).astype(np.float64)
    uv = np.asarray(uv, dtype=np.float64)
    e0 = np.exp(-1j * uv[:, 0:1] * l[None, :])         # (M, n)
    e1 = np.exp(-1j * uv[:, 1:2] * l[None, :])         # (M, n)
    return np.einsum("mp,pq,mq->m", e0, x.astype(np.complex128), e1) / K


def direct_adj(w: np.ndarray, uv: np.ndarray, n: int, oversample: int = 2) -> np.ndarray:
    """Conjugate transpose of :func:`direct`."""
    K = grid_side(n, oversample)
    l = offsets(n).astype(np.float64)
    uv = np.asarray(uv, dtype=np.float64)
    e0 = np.exp(1j * uv[:, 0:1] * l[None, :])
    e1 = np.exp(1j * uv[:, 1:2] * l[None, :])
    return np.einsum("m,mp,mq->pq", np.asarray(w, dtype=np.complex128), e0, e1) / K


def direct_points(pix: np.ndarray, amps: np.ndarray, uv: np.ndarray, n: int,
                  oversample: int = 2, chunk: int = 1 << 16) -> np.ndarray:
    """:func:`direct` for an image that is zero except at the pixels ``pix``
    ((k, 2) integer rows p, q) with values ``amps`` (k,): the exact measurement
    of a sky of point sources, summed over the sources only."""
    K = grid_side(n, oversample)
    pix = np.asarray(pix, dtype=np.int64)
    l0 = (pix[:, 0] - n // 2).astype(np.float64)
    l1 = (pix[:, 1] - n // 2).astype(np.float64)
    amps = np.asarray(amps, dtype=np.complex128)
    uv = np.asarray(uv, dtype=np.float64)
    out = np.empty(len(uv), dtype=np.complex128)
    for s in range(0, len(uv), chunk):
        u = uv[s:s + chunk, 0:1]
        v = uv[s:s + chunk, 1:2]
        out[s:s + chunk] = np.exp(-1j * (u * l0[None, :] + v * l1[None, :])) @ amps / K
    return out


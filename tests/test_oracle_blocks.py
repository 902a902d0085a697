"""Pins of the oracle's blocked SDMM (Sec. 4.5, eqs. blocks, dbp1, dbp2).

* sum_i Phi_i^dagger Phi_i = Phi^dagger Phi for a partition of the
  visibilities (the identity the paper states for the CG operator).
* R = 1 is plain SDMM: the same iterates.
* Every eps_i >= ||y_i||: x = 0 is feasible and optimal; SDMM stays at 0.
* The limit of a 3-block run has the optimal value of the 3-constraint
  problem eq. (dbp1) found by a library minimiser (SLSQP).
"""
import numpy as np
import pytest
import scipy.optimize

import workloads as W
from oracle import blocks, nufft, sdmm, wavelets


def _tiny(cfg=105):
    n, M, J = 8, 60, 6
    x = W.sky(n, 2, 3, W.rng(cfg, W.STREAM_SKY), sigma_range=(0.7, 1.5))
    uv = W.coverage(M, W.rng(cfg, W.STREAM_UV))
    op = nufft.Operator(n, uv, J)
    sara = wavelets.Sara(n, 1, 0b111)
    y0 = op.phi(x)
    sig = sdmm.noise_sigma(y0, 30.0)
    y = y0 + sig * W.unit_complex_noise(M, W.rng(cfg, W.STREAM_NOISE))
    return op, sara, y, sig


def _partition(M, R, cfg=105):
    lab = W.rng(cfg, 30).integers(0, R, size=M)
    return [np.flatnonzero(lab == r) for r in range(R)]


def test_block_gram_sums_to_the_full_gram():
    op, _, _, _ = _tiny()
    parts = _partition(op.M, 3)
    p = W.random_complex((op.n, op.n), W.rng(105, 31))
    total = sum(blocks.Block(op, idx).phi_adj(blocks.Block(op, idx).phi(p)) for idx in parts)
    full = op.phi_adj(op.phi(p))
    assert np.linalg.norm(total - full) <= 1e-13 * np.linalg.norm(full)


def test_one_block_is_plain_sdmm():
    op, sara, y, sig = _tiny()
    eps = sdmm.noise_bound(op.M, sig)
    xa, sa, ha, gam = sdmm.sdmm(y, eps, op, sara, T=10, n_cg=8)
    xb, sb, hb, _ = blocks.sdmm_blocks(y, [eps], [np.arange(op.M)], op, sara, T=10, n_cg=8, gamma=gam)
    assert np.linalg.norm(xb - xa) <= 1e-12 * np.linalg.norm(xa)
    for a, b in zip(ha, hb):
        assert b["f1"] == pytest.approx(a["f1"], rel=1e-12)
        assert b["nu"] == pytest.approx(a["nu"], rel=1e-12)
    assert np.linalg.norm(sb.z2[0] - sa.z2) <= 1e-12 * np.linalg.norm(sa.z2)


def test_blocks_with_loose_bounds_give_zero():
    op, sara, y, _ = _tiny()
    parts = _partition(op.M, 4)
    eps = [1.01 * np.linalg.norm(y[idx]) for idx in parts]
    xh, _, _, _ = blocks.sdmm_blocks(y, eps, parts, op, sara, T=5, n_cg=8)
    assert np.all(xh == 0)


@pytest.mark.slow
def test_blocked_limit_is_optimal():
    op, sara, y, sig = _tiny()
    parts = _partition(op.M, 3)
    eps = [sdmm.noise_bound(len(idx), sig) for idx in parts]
    n, N = op.n, op.n * op.n
    A = np.array([op.phi(e.reshape(n, n)) for e in np.eye(N, dtype=np.complex128)]).T
    Pd = np.array([sara.psi_adj(e.reshape(n, n)).ravel() for e in np.eye(N)]).T.real
    D = Pd.shape[0]

    def fid(v, idx, e):
        r = y[idx] - A[idx] @ v[:N]
        return e ** 2 - np.real(np.vdot(r, r))

    def fid_jac(v, idx):
        r = y[idx] - A[idx] @ v[:N]
        return np.concatenate([2 * np.real(A[idx].conj().T @ r), np.zeros(D)])

    cons = [{"type": "ineq", "fun": lambda v: v[N:] - Pd @ v[:N], "jac": lambda v: np.hstack([-Pd, np.eye(D)])},
            {"type": "ineq", "fun": lambda v: v[N:] + Pd @ v[:N], "jac": lambda v: np.hstack([Pd, np.eye(D)])}]
    for idx, e in zip(parts, eps):
        cons.append({"type": "ineq", "fun": lambda v, idx=idx, e=e: fid(v, idx, e),
                     "jac": lambda v, idx=idx: fid_jac(v, idx)})
    x0 = np.real(np.linalg.lstsq(A, y, rcond=None)[0]).clip(0)
    v0 = np.concatenate([x0, np.abs(Pd @ x0) + 1e-3])
    res = scipy.optimize.minimize(lambda v: v[N:].sum(), v0, jac=lambda v: np.concatenate([np.zeros(N), np.ones(D)]),
                                  method="SLSQP", bounds=[(0, None)] * (N + D), constraints=cons,
                                  options={"ftol": 1e-12, "maxiter": 2000})
    assert res.success or res.status == 8, res.message
    v = res.x
    assert all(fid(v, idx, e) >= -1e-8 * e ** 2 for idx, e in zip(parts, eps))
    fr = float(np.abs(Pd @ v[:N]).sum())
    gam = 0.05 * np.abs(sara.psi_adj(op.phi_adj(y))).max()
    xh, _, hist, _ = blocks.sdmm_blocks(y, eps, parts, op, sara, T=600, n_cg=20, gamma=gam)
    xr = np.real(xh)
    for idx, e in zip(parts, eps):
        assert np.linalg.norm(y[idx] - op.phi(xr)[idx]) <= e * (1 + 1e-3)
    assert np.abs(np.imag(xh)).max() < 1e-6 and xr.min() > -1e-6
    assert sdmm.f1_value(sara.psi_adj(xr), None) == pytest.approx(fr, rel=2e-3)

"""Pins of the oracle's CG, SDMM (Algorithm 1) and set-up quantities.

* CG on Q = Phi^dagger Phi + 2 I against a dense direct solve (library).
* The SDMM limit on a tiny problem is optimal: same objective as a
  general-purpose constrained minimiser (library SLSQP) on the same problem.
* Special case eps >= ||y||: x = 0 is feasible and optimal; SDMM stays at 0.
* eps from the chi^2 bound covers ||n|| with high probability (Monte Carlo).
* SNR of a known perturbation; splitting a run into two halves changes nothing.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.optimize

import workloads as W
from oracle import nufft, sdmm, wavelets

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tiny(n=8, M=40, J=6, levels=1, mask=0b111, cfg=103, noise=True):
    g = W.rng(cfg, W.STREAM_SKY)
    x = W.sky(n, 2, 3, g, sigma_range=(0.7, 1.5))
    uv = W.coverage(M, W.rng(cfg, W.STREAM_UV))
    op = nufft.Operator(n, uv, J)
    sara = wavelets.Sara(n, levels, mask)
    y0 = op.phi(x)
    sig = sdmm.noise_sigma(y0, 30.0)
    y = y0 + (sig * W.unit_complex_noise(M, W.rng(cfg, W.STREAM_NOISE)) if noise else 0)
    eps = sdmm.noise_bound(M, sig)
    return x, op, sara, y, eps


def _dense(op):
    n = op.n
    cols = []
    for k in range(n * n):
        e = np.zeros(n * n, dtype=np.complex128)
        e[k] = 1.0
        cols.append(op.phi(e.reshape(n, n)))
    return np.array(cols).T      # (M, N)


def test_cg_matches_direct_solve():
    _, op, _, _, _ = _tiny()
    n = op.n
    A = _dense(op)
    Qd = A.conj().T @ A + 2 * np.eye(n * n)
    g = W.rng(103, 9)
    b = W.random_complex((n, n), g)
    x0 = W.random_complex((n, n), g)
    Q = lambda v: op.phi_adj(op.phi(v)) + 2 * v
    x = sdmm.conjugate_gradient(Q, b, x0, 80)
    xs = np.linalg.solve(Qd, b.ravel())
    assert np.linalg.norm(x.ravel() - xs) <= 1e-10 * np.linalg.norm(xs)
    # Fewer iterations reduce the residual monotonically in the Q-norm error.
    errs = []
    for k in (1, 2, 4, 8):
        e = sdmm.conjugate_gradient(Q, b, x0, k).ravel() - xs
        errs.append(np.real(np.vdot(e, Qd @ e)))
    assert all(a > b for a, b in zip(errs, errs[1:]))


def test_cg_zero_rhs_stays_at_zero():
    Q = lambda v: 3.0 * v
    x = sdmm.conjugate_gradient(Q, np.zeros((4, 4)), np.zeros((4, 4)), 5)
    assert np.all(x == 0)


def test_paper_constants_are_the_defaults():
    c = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    import inspect
    sig = inspect.signature(sdmm.sdmm)
    assert sig.parameters["xi"].default == c["halting_xi"]["value"]
    assert sig.parameters["tau"].default == c["halting_tau"]["value"]
    assert sig.parameters["beta"].default == c["penalty_beta"]["value"]
    assert inspect.signature(sdmm.penalty).parameters["beta"].default == c["penalty_beta"]["value"]
    assert len(wavelets.BASES) == c["sara_bases"]["value"]


def test_noise_bound_covers_noise():
    M, sig = 200, 0.3
    g = W.rng(103, 10)
    eps = sdmm.noise_bound(M, sig)
    norms = np.array([np.linalg.norm(sig * W.unit_complex_noise(M, g)) for _ in range(4000)])
    # ||n||^2 / (sigma^2/2) is chi^2 with 2M dof, and eps^2 / (sigma^2/2) = 2M + 4 sqrt(M)
    # is its mean plus two standard deviations: coverage from the library's chi^2 CDF.
    import scipy.stats
    expect = scipy.stats.chi2.cdf(2 * M + 4 * math.sqrt(M), 2 * M)
    assert np.mean(norms <= eps) == pytest.approx(expect, abs=4 * math.sqrt(expect * (1 - expect) / 4000))
    assert np.mean(norms ** 2) == pytest.approx(M * sig ** 2, rel=0.02)


def test_noise_sigma_matches_isnr():
    g = W.rng(103, 11)
    y0 = W.random_complex(5000, g)
    sig = sdmm.noise_sigma(y0, 30.0)
    n = sig * W.unit_complex_noise(5000, g)
    isnr = 20 * math.log10(np.linalg.norm(y0) / np.linalg.norm(n))
    assert isnr == pytest.approx(30.0, abs=0.2)


def test_snr_of_known_perturbation():
    x = np.ones((4, 4))
    assert sdmm.snr_db(x, x + 0.1 * x) == pytest.approx(20.0, abs=1e-12)


def test_penalty_with_dirac_dictionary():
    _, op, _, y, _ = _tiny()
    dirac = wavelets.Sara(op.n, 1, 1)
    gam = sdmm.penalty(y, op.phi_adj, dirac.psi_adj, 1e-3)
    assert gam == pytest.approx(1e-3 * np.abs(op.phi_adj(y)).max(), rel=1e-15)


def test_large_eps_gives_zero():
    _, op, sara, y, _ = _tiny()
    eps = 1.01 * np.linalg.norm(y)
    xh, _, hist, _ = sdmm.sdmm(y, eps, op, sara, T=5, n_cg=8)
    assert np.all(xh == 0)


def test_split_run_equals_full_run():
    _, op, sara, y, eps = _tiny()
    xa, _, _, gam = sdmm.sdmm(y, eps, op, sara, T=12, n_cg=6)
    _, st, _, _ = sdmm.sdmm(y, eps, op, sara, T=5, n_cg=6, gamma=gam)
    xb, _, _, _ = sdmm.sdmm(y, eps, op, sara, T=7, n_cg=6, gamma=gam, state=st)
    np.testing.assert_array_equal(xa, xb)


def _reference_solution(op, sara, y, eps, weights):
    """Solve eq. (delta) with a general library minimiser (SLSQP), x real >= 0.

    Variables (x, t): minimise sum w t  s.t.  -t <= Psi^dagger x <= t,
    ||y - Phi x||^2 <= eps^2, x >= 0.
    """
    n = op.n
    N = n * n
    A = _dense(op)
    Pd = np.array([sara.psi_adj(e.reshape(n, n)).ravel() for e in np.eye(N)]).T.real  # (D, N)
    D = Pd.shape[0]
    w = np.ones(D) if weights is None else weights.ravel()

    def fid(v):
        r = y - A @ v[:N]
        return eps ** 2 - np.real(np.vdot(r, r))

    def fid_jac(v):
        r = y - A @ v[:N]
        gx = 2 * np.real(A.conj().T @ r)
        return np.concatenate([gx, np.zeros(D)])

    cons = [
        {"type": "ineq", "fun": lambda v: v[N:] - Pd @ v[:N],
         "jac": lambda v: np.hstack([-Pd, np.eye(D)])},
        {"type": "ineq", "fun": lambda v: v[N:] + Pd @ v[:N],
         "jac": lambda v: np.hstack([Pd, np.eye(D)])},
        {"type": "ineq", "fun": fid, "jac": fid_jac},
    ]
    x0 = np.real(np.linalg.lstsq(A, y, rcond=None)[0]).clip(0)
    v0 = np.concatenate([x0, np.abs(Pd @ x0) + 1e-3])
    bounds = [(0, None)] * N + [(0, None)] * D
    res = scipy.optimize.minimize(lambda v: w @ v[N:], v0, jac=lambda v: np.concatenate([np.zeros(N), w]),
                                  method="SLSQP", bounds=bounds, constraints=cons,
                                  options={"ftol": 1e-12, "maxiter": 2000})
    # SLSQP can stop on a stalled line search at the optimum; accept its point
    # only if it satisfies every constraint.
    v = res.x
    assert res.success or res.status == 8, res.message
    assert fid(v) >= -1e-8 * eps ** 2
    assert np.all(v[N:] - np.abs(Pd @ v[:N]) >= -1e-9) and np.all(v[:N] >= -1e-12)
    return v[:N].reshape(n, n), float(w @ np.abs(Pd @ v[:N]))


@pytest.mark.slow
@pytest.mark.parametrize("weighted", [False, True])
def test_sdmm_limit_is_optimal(weighted):
    x, op, sara, y, eps = _tiny()
    weights = None
    if weighted:
        weights = W.rng(103, 12).uniform(0.5, 2.0, size=(sara.q, op.n, op.n))
    xr, fr = _reference_solution(op, sara, y, eps, weights)
    gam = 0.05 * np.abs(sara.psi_adj(op.phi_adj(y))).max()
    xh, _, hist, _ = sdmm.sdmm(y, eps, op, sara, T=1500, n_cg=40, gamma=gam, weights=weights)
    f_sdmm = sdmm.f1_value(sara.psi_adj(np.real(xh)), weights)
    # Feasible (to SDMM's convergence) and the same optimal value.
    assert np.linalg.norm(y - op.phi(np.real(xh))) <= eps * (1 + 1e-3)
    assert np.abs(np.imag(xh)).max() < 1e-6 and np.real(xh).min() > -1e-6
    assert f_sdmm == pytest.approx(fr, rel=2e-3)

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
    xh, _, hist, _ = sdmm.sdmm(y, eps, op, sara, T=900, n_cg=24, gamma=gam, weights=weights)
    f_sdmm = sdmm.f1_value(sara.psi_adj(np.real(xh)), weights)
    # Feasible (to SDMM's convergence) and the same optimal value.
    assert np.linalg.norm(y - op.phi(np.real(xh))) <= eps * (1 + 1e-3)
    assert np.abs(np.imag(xh)).max() < 1e-6 and np.real(xh).min() > -1e-6
    assert f_sdmm == pytest.approx(fr, rel=2e-3)


# ---------------------------------------------------------------------------
# A scalar problem worked by hand through Algorithm 1 (Sec. 4.4): n = 1,
# Phi = Psi = I (q = 1, so Psi Psi^dagger = I and Q = 3 I), y = 3, eps = 1,
# gamma = 1/2, x^(0) = 0.  CG solves Q x = b exactly in one iteration.
#   t = 1: x = 0;     r1 = 0, z1 = 0;  v2 = 0, r2 = 2, z2 = -2;  rhs = 4
#          f1 = 0, zeta = inf (previous f1 = 0), nu = |3 - 0| / 1 = 3
#   t = 2: x = 4/3;   v1 = 4/3, r1 = 5/6, z1 = 1/2, x1 = 1/3
#          v2 = 4/3 - 2 = -2/3, |v2 - y| = 11/3 > 1: r2 = 2, z2 = -8/3, x2 = 14/3
#          x3 = 4/3;  rhs = 19/3;  f1 = 4/3, zeta = inf, nu = 5/3
#   t = 3: x = 19/9;  v1 = 47/18, r1 = 19/9, z1 = 1/2, x1 = 29/18
#          v2 = -5/9, r2 = 2, z2 = -23/9, x2 = 41/9;  x3 = 19/9;  rhs = 149/18
#          f1 = 19/9, zeta = (19/9 - 4/3) / (4/3) = 7/12, nu = 8/9

class _ScalarOp:
    n = 1

    @staticmethod
    def phi(x):
        return np.asarray(x, dtype=np.complex128).reshape(1).copy()

    @staticmethod
    def phi_adj(w):
        return np.asarray(w, dtype=np.complex128).reshape(1, 1).copy()


class _ScalarDict:
    q = 1

    @staticmethod
    def psi_adj(x):
        return np.asarray(x, dtype=np.complex128).reshape(1, 1).copy()

    @staticmethod
    def psi(a):
        return np.asarray(a, dtype=np.complex128).reshape(1, 1).copy()


def test_sdmm_scalar_case_worked_by_hand():
    y = np.array([3.0 + 0j])
    xh, st, hist, gam = sdmm.sdmm(y, 1.0, _ScalarOp, _ScalarDict, T=3, n_cg=1, gamma=0.5)
    assert gam == 0.5
    assert xh[0, 0] == pytest.approx(19 / 9, abs=1e-15)
    assert st.z1[0, 0] == pytest.approx(0.5, abs=1e-15)
    assert st.z2[0] == pytest.approx(-23 / 9, abs=1e-15)
    assert st.z3[0, 0] == 0
    assert st.rhs[0, 0] == pytest.approx(149 / 18, abs=1e-14)
    assert [h["f1"] for h in hist] == pytest.approx([0.0, 4 / 3, 19 / 9], abs=1e-15)
    assert math.isinf(hist[0]["zeta"]) and math.isinf(hist[1]["zeta"])
    assert hist[2]["zeta"] == pytest.approx(7 / 12, abs=1e-15)
    assert [h["nu"] for h in hist] == pytest.approx([3.0, 5 / 3, 8 / 9], abs=1e-15)


def test_early_stop_fires_at_the_halting_rule():
    """Halting (Sec. 4.4): stop at the first iteration with zeta < xi and nu in
    [1 - tau, 1 + tau].  In the hand-worked case iteration 3 has zeta = 7/12 and
    nu = 8/9: xi = 0.6, tau = 0.2 stop there; xi = 0.5 does not."""
    y = np.array([3.0 + 0j])
    full, st_full, _, _ = sdmm.sdmm(y, 1.0, _ScalarOp, _ScalarDict, T=3, n_cg=1, gamma=0.5)
    xh, st, hist, _ = sdmm.sdmm(y, 1.0, _ScalarOp, _ScalarDict, T=50, n_cg=1, gamma=0.5,
                                early_stop=True, xi=0.6, tau=0.2)
    assert len(hist) == 3 and st.t == 3
    np.testing.assert_array_equal(xh, full)
    _, _, hist2, _ = sdmm.sdmm(y, 1.0, _ScalarOp, _ScalarDict, T=4, n_cg=1, gamma=0.5,
                               early_stop=True, xi=0.5, tau=0.2)
    assert len(hist2) == 4


def test_early_stop_on_an_imaging_problem():
    """On a small imaging problem the run stops at the first iteration meeting
    the rule, and its iterate equals the fixed-length run of that many
    iterations."""
    _, op, sara, y, eps = _tiny()
    _, _, hist, gam = sdmm.sdmm(y, eps, op, sara, T=400, n_cg=8)
    ok = [h["zeta"] < 1e-3 and 0.9 <= h["nu"] <= 1.1 for h in hist]
    assert any(ok)
    first = ok.index(True) + 1
    xs, _, hs, _ = sdmm.sdmm(y, eps, op, sara, T=400, n_cg=8, gamma=gam, early_stop=True)
    assert len(hs) == first
    xf, _, _, _ = sdmm.sdmm(y, eps, op, sara, T=first, n_cg=8, gamma=gam)
    np.testing.assert_array_equal(xs, xf)


@pytest.mark.slow
def test_sdmm_from_x0_reaches_the_optimum():
    """Algorithm 1 started from a nonzero x^(0) (steps 1-3 with r_i = L_i x^(0))
    converges to the same optimal value as the library minimiser."""
    x, op, sara, y, eps = _tiny()
    xr, fr = _reference_solution(op, sara, y, eps, None)
    gam = 0.05 * np.abs(sara.psi_adj(op.phi_adj(y))).max()
    x0 = W.rng(103, 13).uniform(0.0, 1.0, size=(op.n, op.n)) + 0.3j
    st0 = sdmm.initial_state(y, op.phi, op.phi_adj, sara.psi, sara.psi_adj, x0)
    # Steps 1-3: r_i = L_i x0, x_i = L_i^dagger r_i, so rhs = (Psi Psi^dagger + Phi^dagger Phi + I) x0.
    np.testing.assert_allclose(st0.rhs, 2 * x0 + op.phi_adj(op.phi(x0)), atol=1e-12)
    xh, _, _, _ = sdmm.sdmm(y, eps, op, sara, T=1500, n_cg=40, gamma=gam, x0=x0)
    f_sdmm = sdmm.f1_value(sara.psi_adj(np.real(xh)), None)
    assert np.linalg.norm(y - op.phi(np.real(xh))) <= eps * (1 + 1e-3)
    assert np.abs(np.imag(xh)).max() < 1e-6 and np.real(xh).min() > -1e-6
    assert f_sdmm == pytest.approx(fr, rel=2e-3)


def test_cg_tolerance_stops_at_the_relative_residual():
    """With tol > 0 the oracle's CG stops before the first iteration whose
    residual satisfies ||r_k|| <= tol ||r_0||: the result equals the fixed
    k-iteration run, and k - 1 iterations do not meet the rule."""
    _, op, _, _, _ = _tiny()
    n = op.n
    g = W.rng(103, 14)
    b = W.random_complex((n, n), g)
    x0 = np.zeros((n, n), dtype=np.complex128)
    Q = lambda v: op.phi_adj(op.phi(v)) + 2 * v
    r0 = np.linalg.norm(b - Q(x0))
    tol = 1e-6
    res = lambda k: np.linalg.norm(b - Q(sdmm.conjugate_gradient(Q, b, x0, k)))
    k = next(k for k in range(1, 200) if res(k) <= tol * r0)
    assert res(k - 1) > tol * r0
    np.testing.assert_array_equal(sdmm.conjugate_gradient(Q, b, x0, 200, tol),
                                  sdmm.conjugate_gradient(Q, b, x0, k))

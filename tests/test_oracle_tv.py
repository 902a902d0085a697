"""Pins of the oracle's weighted TV prior and TV SDMM (Sec. 3.3 eq. tvproblem,
Sec. 5 weighted TV, Sec. 6 TV with positivity).

* grad_adj is the adjoint of grad.
* The prox on a two-pixel image against its closed form (1-D TV denoising of
  two samples), lam -> 0 (identity) and lam large (the constant mean image).
* The prox on a 4 x 4 image is optimal: the denoising problem's duality gap
  at the returned primal-dual pair vanishes, and a library minimiser (SLSQP)
  finds nothing lower.
* Weights: zero weights give the identity; uniform weights c scale lam.
* The TV-SDMM limit on a tiny imaging problem has the optimal value of the
  constrained TV problem found by SLSQP.
"""
import numpy as np
import pytest
import scipy.optimize

import workloads as W
from oracle import nufft, sdmm, tv


def test_grad_adjoint():
    g = W.rng(106, 1)
    x = W.random_complex((7, 9), g)
    p, q = W.random_complex((7, 9), g), W.random_complex((7, 9), g)
    dx, dy = tv.grad(x)
    lhs = np.vdot(dx, p) + np.vdot(dy, q)
    rhs = np.vdot(x, tv.grad_adj(p, q))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("a,c,lam", [(0.0, 1.0, 0.1), (0.0, 1.0, 0.6), (2.0 + 1j, -1.0, 0.5), (3.0, 3.0, 1.0)])
def test_two_pixel_closed_form(a, c, lam):
    b = np.array([[a], [c]], dtype=np.complex128)
    x = tv.prox_tv(b, lam, 2000)
    d = c - a
    if abs(d) <= 2 * lam:
        want = np.array([[(a + c) / 2], [(a + c) / 2]])
    else:
        u = d / abs(d)
        want = np.array([[a + lam * u], [c - lam * u]])
    np.testing.assert_allclose(x, want, atol=1e-9)


def test_prox_limits():
    b = W.random_complex((6, 6), W.rng(106, 2))
    np.testing.assert_array_equal(tv.prox_tv(b, 0.0, 50), b)
    x = tv.prox_tv(b, 1e3, 4000)
    np.testing.assert_allclose(x, np.full_like(b, b.mean()), atol=1e-6)


def test_prox_matches_library_minimiser():
    """Optimality of the prox on a 4 x 4 image: the duality gap of the
    denoising problem, P(x) - D(p) with D(p) = ||b||^2/2 - ||b - lam grad^dagger p||^2/2
    for any |p_ij| <= w_ij (a lower bound on the optimum), vanishes at the
    returned pair; and no point found by a library minimiser (SLSQP) is lower."""
    g = W.rng(106, 3)
    n, lam = 4, 0.3
    b = g.uniform(0, 1, size=(n, n))
    w = g.uniform(0.5, 1.5, size=(n, n))
    x, p, q = tv.prox_tv(b, lam, 20000, w, return_dual=True)
    assert np.all(np.sqrt(np.abs(p) ** 2 + np.abs(q) ** 2) <= w * (1 + 1e-12))
    primal = 0.5 * np.linalg.norm(x - b) ** 2 + lam * tv.tv_norm(x, w)
    dual = 0.5 * np.linalg.norm(b) ** 2 - 0.5 * np.linalg.norm(b - lam * tv.grad_adj(p, q)) ** 2
    assert dual <= primal + 1e-12
    assert primal - dual <= 1e-9 * primal
    N = n * n

    def obj(v):
        return 0.5 * np.sum((v[:N] - b.ravel()) ** 2) + lam * np.sum(w.ravel() * v[N:])

    def cons(v):
        m = tv.magnitude(v[:N].reshape(n, n)).ravel()
        return v[N:] ** 2 - m ** 2

    v0 = np.concatenate([b.ravel(), tv.magnitude(b).ravel() + 0.1])
    res = scipy.optimize.minimize(obj, v0, method="SLSQP", constraints=[{"type": "ineq", "fun": cons}],
                                  bounds=[(None, None)] * N + [(0, None)] * N,
                                  options={"ftol": 1e-14, "maxiter": 2000})
    assert primal <= res.fun + 1e-9


def test_weights():
    b = W.random_complex((5, 5), W.rng(106, 4))
    np.testing.assert_allclose(tv.prox_tv(b, 0.4, 100, np.zeros((5, 5))), b, atol=0)
    np.testing.assert_allclose(tv.prox_tv(b, 0.4, 300, np.full((5, 5), 2.5)), tv.prox_tv(b, 1.0, 300), atol=1e-12)
    w = tv.tv_weights(b, 0.5)
    assert np.all((w > 0) & (w <= 1))
    assert w[-1, -1] == 1.0  # no gradient at the last pixel


@pytest.mark.slow
def test_tv_sdmm_limit_is_optimal():
    n, M, J, cfg = 8, 40, 6, 107
    x_true = W.sky(n, 2, 3, W.rng(cfg, W.STREAM_SKY), sigma_range=(0.7, 1.5))
    uv = W.coverage(M, W.rng(cfg, W.STREAM_UV))
    op = nufft.Operator(n, uv, J)
    y0 = op.phi(x_true)
    sig = sdmm.noise_sigma(y0, 30.0)
    y = y0 + sig * W.unit_complex_noise(M, W.rng(cfg, W.STREAM_NOISE))
    eps = sdmm.noise_bound(M, sig)
    N = n * n
    A = np.array([op.phi(e.reshape(n, n)) for e in np.eye(N, dtype=np.complex128)]).T

    def fid(v):
        r = y - A @ v[:N]
        return eps ** 2 - np.real(np.vdot(r, r))

    def fid_jac(v):
        r = y - A @ v[:N]
        return np.concatenate([2 * np.real(A.conj().T @ r), np.zeros(N)])

    def tvc(v):  # t_ij >= |(grad x)_ij|
        return v[N:] - tv.magnitude(v[:N].reshape(n, n)).ravel()

    x0 = np.real(np.linalg.lstsq(A, y, rcond=None)[0]).clip(0)
    v0 = np.concatenate([x0, tv.magnitude(x0.reshape(n, n)).ravel() + 1e-3])
    res = scipy.optimize.minimize(lambda v: v[N:].sum(), v0, jac=lambda v: np.concatenate([np.zeros(N), np.ones(N)]),
                                  method="SLSQP",
                                  constraints=[{"type": "ineq", "fun": fid, "jac": fid_jac},
                                               {"type": "ineq", "fun": tvc}],
                                  bounds=[(0, None)] * (2 * N), options={"ftol": 1e-12, "maxiter": 5000})
    assert res.success or res.status == 8, res.message
    assert fid(res.x) >= -1e-6 * eps ** 2 and tvc(res.x).min() >= -1e-5
    fr = tv.tv_norm(res.x[:N].reshape(n, n))
    gam = 0.05 * np.abs(op.phi_adj(y)).max()
    xh, _, hist, _ = tv.sdmm_tv(y, eps, op, T=1500, n_cg=40, n_inner=100, gamma=gam)
    xr = np.real(xh)
    assert np.linalg.norm(y - op.phi(xr)) <= eps * (1 + 1e-3)
    assert np.abs(np.imag(xh)).max() < 1e-4 and xr.min() > -1e-4
    assert tv.tv_norm(xr) == pytest.approx(fr, rel=2e-3)


def test_rwtv_without_reweighting_is_tv():
    from oracle import reweight
    n, M, J, cfg = 8, 40, 6, 108
    uv = W.coverage(M, W.rng(cfg, W.STREAM_UV))
    op = nufft.Operator(n, uv, J)
    y = W.random_complex(M, W.rng(cfg, 1)) * 0.1
    xa, _, _, gam = tv.sdmm_tv(y, 0.5 * np.linalg.norm(y), op, T=6, n_cg=6, n_inner=10)
    xb, passes, _ = reweight.sdmm_tv_reweighted(y, 0.5 * np.linalg.norm(y), op, T=6, n_cg=6, n_inner=10, outer=0)
    assert passes == 1
    np.testing.assert_array_equal(xa, xb)
    # One pass: the weighted TV run from the first solution with the rule's weights.
    xc, passes, info = reweight.sdmm_tv_reweighted(y, 0.5 * np.linalg.norm(y), op, T=6, n_cg=6, n_inner=10, outer=1)
    w = tv.tv_weights(xa, reweight.first_delta(tv.magnitude(xa), 0.0))
    xd, _, _, _ = tv.sdmm_tv(y, 0.5 * np.linalg.norm(y), op, T=6, n_cg=6, n_inner=10, gamma=gam, weights=w, x0=xa)
    np.testing.assert_array_equal(xc, xd)

"""Pins of the oracle's proximity operators (Sec. 4.1 definition, Sec. 4.4 eqs. prox1-3).

Each operator is checked against its closed form on hand-computed values and
against the definition prox_f(x) = argmin_z f(z) + 1/2 ||x - z||^2 solved by a
general-purpose library minimiser, plus idempotence / non-expansiveness.
"""
import math

import numpy as np
import pytest
import scipy.optimize

import workloads as W
from oracle import prox


def test_soft_threshold_closed_form():
    a = np.array([3 + 4j, 0.0, 0.6 + 0.8j, -2.0, 1e-300j])
    out = prox.soft_threshold(a, 1.0)
    np.testing.assert_allclose(out, [2.4 + 3.2j, 0, 0, -1.0, 0], atol=1e-15)
    # Entrywise thresholds (weights).
    out = prox.soft_threshold(np.array([2.0, 2.0]), np.array([0.5, 3.0]))
    np.testing.assert_allclose(out, [1.5, 0.0])


def test_soft_threshold_is_prox_of_modulus():
    g = W.rng(102, 0)
    for _ in range(20):
        a = complex(*g.normal(size=2) * 2)
        lam = float(g.uniform(0.1, 2.0))
        res = scipy.optimize.minimize(
            lambda z: lam * math.hypot(z[0], z[1]) + 0.5 * ((z[0] - a.real) ** 2 + (z[1] - a.imag) ** 2),
            x0=[a.real, a.imag], method="Nelder-Mead",
            options={"xatol": 1e-12, "fatol": 1e-15, "maxiter": 5000})
        got = prox.soft_threshold(np.array([a]), lam)[0]
        assert abs(got - complex(*res.x)) < 1e-6


def test_project_ball_is_nearest_point_and_centred_on_y():
    g = W.rng(102, 1)
    y = W.random_complex(6, g)
    r = y + 3.0 * W.random_complex(6, g)
    eps = 0.7
    p = prox.project_ball(r, y, eps)
    assert np.linalg.norm(p - y) == pytest.approx(eps, rel=1e-14)
    # Nearest point of the ball by a constrained library minimiser on R^12.
    rv = np.concatenate([r.real, r.imag])
    yv = np.concatenate([y.real, y.imag])
    res = scipy.optimize.minimize(
        lambda z: 0.5 * np.sum((z - rv) ** 2), x0=yv, jac=lambda z: z - rv, method="SLSQP",
        constraints=[{"type": "ineq", "fun": lambda z: eps ** 2 - np.sum((z - yv) ** 2),
                      "jac": lambda z: -2 * (z - yv)}], options={"ftol": 1e-15, "maxiter": 500})
    np.testing.assert_allclose(np.concatenate([p.real, p.imag]), res.x, atol=1e-6)
    # Points already inside are unchanged; projection is idempotent.
    inside = y + 0.1 * W.random_complex(6, g) / 10
    np.testing.assert_array_equal(prox.project_ball(inside, y, eps), inside)
    np.testing.assert_allclose(prox.project_ball(p, y, eps), p, atol=1e-15)


def test_project_positive():
    r = np.array([1 + 2j, -1 + 5j, 0.0, -3j])
    np.testing.assert_array_equal(prox.project_positive(r), [1.0, 0.0, 0.0, 0.0])
    assert prox.project_positive(r).dtype == r.dtype


def test_nonexpansive():
    g = W.rng(102, 2)
    y = W.random_complex(20, g)
    for _ in range(50):
        a, b = W.random_complex(20, g) * 3, W.random_complex(20, g) * 3
        ops = [lambda v: prox.soft_threshold(v, 0.8),
               lambda v: prox.project_ball(v, y, 1.5),
               prox.project_positive]
        for op in ops:
            assert np.linalg.norm(op(a) - op(b)) <= np.linalg.norm(a - b) * (1 + 1e-14)

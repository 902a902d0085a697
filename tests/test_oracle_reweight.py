"""Pins of the oracle's reweighted l1 loop (Sec. 3.3, the sequence of weighted
problems of eq. (delta)).

* No reweighting pass is the unweighted problem solved by SDMM (BPSA, Sec. 6).
* The weight rule on hand-computed coefficients, and its invariants.
* One pass equals SDMM with those weights started from the first solution.
* Majorisation-minimisation: with delta fixed and each weighted problem solved
  to convergence, the log-sum penalty sum log(delta + |Psi^dagger x|) never
  increases from one pass to the next (each pass minimises its linear upper
  bound over a set that holds the previous solution).

The weight formula's regularisation and the delta schedule follow the reading
stated in oracle/reweight.py; the paper defers them to its SARA reference, so
parity with the paper's own choice is unpinned.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import nufft, reweight, sdmm, wavelets


def _tiny(cfg=104):
    n, M, J = 8, 40, 6
    x = W.sky(n, 2, 3, W.rng(cfg, W.STREAM_SKY), sigma_range=(0.7, 1.5))
    uv = W.coverage(M, W.rng(cfg, W.STREAM_UV))
    op = nufft.Operator(n, uv, J)
    sara = wavelets.Sara(n, 1, 0b111)
    y0 = op.phi(x)
    sig = sdmm.noise_sigma(y0, 30.0)
    y = y0 + sig * W.unit_complex_noise(M, W.rng(cfg, W.STREAM_NOISE))
    return op, sara, y, sdmm.noise_bound(M, sig)


def test_weights_on_hand_computed_coefficients():
    a = np.array([0.0, 1.0, 3 + 4j, -2.0, 0.5j])
    w = reweight.weights(a, 1.0)
    np.testing.assert_allclose(w, [1.0, 0.5, 1 / 6, 1 / 3, 2 / 3], rtol=0, atol=1e-16)
    w2 = reweight.weights(a, 0.25)
    np.testing.assert_allclose(w2, [1.0, 0.2, 0.25 / 5.25, 0.25 / 2.25, 1 / 3], rtol=0, atol=1e-16)
    g = W.rng(104, 20)
    b = W.random_complex(1000, g)
    wb = reweight.weights(b, 0.3)
    assert np.all(wb > 0) and np.all(wb <= 1)
    order = np.argsort(np.abs(b))
    assert np.all(np.diff(wb[order]) <= 0)


def test_first_delta():
    assert reweight.first_delta(np.array([3.0, 4j]), 0.0) == pytest.approx(math.sqrt(12.5), rel=1e-15)
    assert reweight.first_delta(np.zeros(5), 0.0) == 1.0
    assert reweight.first_delta(np.array([3.0]), 0.7) == 0.7


def test_no_reweighting_is_bpsa():
    op, sara, y, eps = _tiny()
    xa, _, _, _ = sdmm.sdmm(y, eps, op, sara, T=15, n_cg=6)
    xb, passes, info = reweight.sdmm_reweighted(y, eps, op, sara, T=15, n_cg=6, outer=0)
    assert passes == 1
    np.testing.assert_array_equal(xa, xb)


def test_one_pass_is_weighted_sdmm_from_the_first_solution():
    op, sara, y, eps = _tiny()
    x0, _, _, gam = sdmm.sdmm(y, eps, op, sara, T=12, n_cg=6)
    a = sara.psi_adj(x0)
    w = reweight.weights(a, reweight.first_delta(a, 0.0))
    x1, _, _, _ = sdmm.sdmm(y, eps, op, sara, T=12, n_cg=6, gamma=gam, weights=w, x0=x0)
    xr, passes, info = reweight.sdmm_reweighted(y, eps, op, sara, T=12, n_cg=6, outer=1)
    assert passes == 2 and info[1]["delta"] == pytest.approx(math.sqrt(np.mean(np.abs(a) ** 2)))
    np.testing.assert_array_equal(xr, x1)


def test_tolerance_stops_the_passes():
    op, sara, y, eps = _tiny()
    _, passes_all, info = reweight.sdmm_reweighted(y, eps, op, sara, T=10, n_cg=6, outer=4)
    changes = [i["change"] for i in info[1:]]
    tol = 0.5 * (changes[0] + changes[1]) if changes[1] < changes[0] else changes[0] * 1.01
    _, passes, info2 = reweight.sdmm_reweighted(y, eps, op, sara, T=10, n_cg=6, outer=4, tol=tol)
    first = next(k for k, c in enumerate(changes) if c <= tol) + 2
    assert passes == first and passes_all == 5


@pytest.mark.slow
def test_log_sum_penalty_decreases_across_passes():
    op, sara, y, eps = _tiny()
    gam = 0.05 * np.abs(sara.psi_adj(op.phi_adj(y))).max()
    x = None
    delta = 0.05
    prev = None
    for k in range(4):
        w = None if x is None else reweight.weights(sara.psi_adj(np.real(x)), delta)
        x, _, _, _ = sdmm.sdmm(y, eps, op, sara, T=600, n_cg=20, gamma=gam, weights=w, x0=x)
        pen = float(np.sum(np.log(delta + np.abs(sara.psi_adj(np.real(x))))))
        if prev is not None:
            assert pen <= prev + 1e-6 * abs(prev), (k, pen, prev)
        prev = pen

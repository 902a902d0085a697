"""Reweighted l1 (Sec. 3.3) on the GPU, through the C ABI, against the oracle.

The 64^2 workload (M = 2048, J = 6, SARA at 3 levels, 30 dB): one
unweighted pass and three reweighted passes of 20 SDMM iterations each; the
final iterate and the last pass's weights against oracle/reweight.py, FP64 to
1e-10 and FP32 (FP64 norms) to 1e-4.  Also a one-basis dictionary (RWBPDb8),
a given delta0, and the relative-change stop.
"""
import numpy as np
import pytest

import workloads as W
from oracle import nufft, reweight, sdmm as osdmm, wavelets
from tests.gpu_helpers import announce, device, host, rel, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _problem(prec):
    c = W.C1
    x_true, uv = W.config_inputs(c)
    if prec == "f32":
        uv = uv.astype(np.float32).astype(np.float64)
    op = nufft.Operator(c.n, uv, c.J)
    y0 = op.phi(x_true)
    sig = osdmm.noise_sigma(y0, c.isnr_db)
    y = y0 + sig * W.unit_complex_noise(c.M, W.rng(c.cfg, W.STREAM_NOISE))
    if prec == "f32":
        y = y.astype(np.complex64).astype(np.complex128)
    return c, uv, op, y, osdmm.noise_bound(c.M, sig)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_reweighted_sara_matches_oracle(prec, tol):
    device()
    announce(f"reweighted SARA 1+3 passes x 20 iterations, {prec}")
    from paper_1307_4370_amd import Plan
    c, uv, op, y, eps = _problem(prec)
    sara = wavelets.Sara(c.n, c.levels)
    xo, passes_o, info = reweight.sdmm_reweighted(y, eps, op, sara, T=20, n_cg=16, outer=3)
    plan = Plan(c.n, to_dev(uv, prec), J=c.J, levels=c.levels, prec=prec)
    xg, st, passes, wg = plan.sdmm_reweighted(to_dev(y, prec), eps, T=20, n_cg=16, outer=3)
    assert passes == passes_o == 4
    assert rel(host(xg), xo) <= tol
    # The last pass's weights: from the solution of the pass before it.
    _, _, info2 = reweight.sdmm_reweighted(y, eps, op, sara, T=20, n_cg=16, outer=2)
    x_prev, _, _ = reweight.sdmm_reweighted(y, eps, op, sara, T=20, n_cg=16, outer=2)
    w_last = reweight.weights(sara.psi_adj(x_prev), info[3]["delta"])
    assert rel(host(wg), w_last) <= tol
    assert st["nu"] == pytest.approx(info[-1]["nu"], rel=tol)


def test_rwbp_db8_with_given_delta_and_stop():
    """A one-basis dictionary (Db8, RWBPDb8 of Sec. 6), delta0 given, and the
    stop on the relative change of x, FP64."""
    device()
    announce("RWBPDb8, delta0 given, tolerance stop, f64")
    from paper_1307_4370_amd import Plan
    c, uv, op, y, eps = _problem("f64")
    mask = 1 << 8
    sara = wavelets.Sara(c.n, c.levels, mask)
    _, _, info_all = reweight.sdmm_reweighted(y, eps, op, sara, T=10, n_cg=12, outer=5, delta0=0.02, rho=0.5)
    changes = [i["change"] for i in info_all[1:]]
    tol = changes[1] * 1.0001  # stops after the second reweighted pass at the latest
    xo, passes_o, _ = reweight.sdmm_reweighted(y, eps, op, sara, T=10, n_cg=12, outer=5, delta0=0.02, rho=0.5,
                                               tol=tol)
    plan = Plan(c.n, to_dev(uv, "f64"), J=c.J, levels=c.levels, dict_mask=mask, prec="f64")
    xg, st, passes, wg = plan.sdmm_reweighted(to_dev(y, "f64"), eps, T=10, n_cg=12, outer=5, delta0=0.02,
                                              rho=0.5, tol=tol)
    assert passes == passes_o <= 3
    assert rel(host(xg), xo) <= 1e-10


def test_no_reweighting_equals_plain_sdmm():
    device()
    announce("reweighted with outer = 0 equals riop_sdmm, f64")
    from paper_1307_4370_amd import Plan
    c, uv, op, y, eps = _problem("f64")
    plan = Plan(c.n, to_dev(uv, "f64"), J=c.J, levels=c.levels, prec="f64")
    xa, sa, _, _ = plan.sdmm(to_dev(y, "f64"), eps, T=8, n_cg=10)
    xb, sb, passes, wb = plan.sdmm_reweighted(to_dev(y, "f64"), eps, T=8, n_cg=10, outer=0)
    assert passes == 1
    assert rel(host(xb), host(xa)) <= 1e-13  # gridding sums in varying order (double LDS atomics)
    assert np.all(host(wb) == 1.0)

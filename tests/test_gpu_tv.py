"""Weighted TV with positivity (Sec. 3.3 eq. tvproblem, Sec. 5, Sec. 6: TV and
RWTV) on the GPU, through the C ABI, against oracle/tv.py and
oracle/reweight.py: the 64^2 workload (M = 2048, J = 6) for 20 iterations
with 20 dual iterations per prox, FP64 to 1e-10 and FP32 (FP64 norms) to
1e-4; per-pixel weights with a given x0; RWTV (1 + 2 passes); and the
256^2 workload (M = 131072, J = 8) for 3 iterations in FP32.
"""
import numpy as np
import pytest

import workloads as W
from oracle import nufft, reweight, sdmm as osdmm, tv
from tests.gpu_helpers import announce, device, host, rel, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _problem(c, prec):
    x_true, uv = W.config_inputs(c)
    if prec == "f32":
        uv = uv.astype(np.float32).astype(np.float64)
    op = nufft.Operator(c.n, uv, c.J)
    y0 = op.phi(x_true)
    sig = osdmm.noise_sigma(y0, c.isnr_db)
    y = y0 + sig * W.unit_complex_noise(c.M, W.rng(c.cfg, W.STREAM_NOISE))
    if prec == "f32":
        y = y.astype(np.complex64).astype(np.complex128)
    return uv, op, y, osdmm.noise_bound(c.M, sig)


@pytest.mark.parametrize("c,T,prec,tol", [(W.C1, 20, "f64", 1e-10), (W.C1, 20, "f32", 1e-4),
                                          (W.C2, 3, "f32", 1e-4)])
def test_tv_sdmm_matches_oracle(c, T, prec, tol):
    device()
    announce(f"TV SDMM {c.name} T={T} {prec}")
    from paper_1307_4370_amd import Plan
    uv, op, y, eps = _problem(c, prec)
    xo, st, hist, gam = tv.sdmm_tv(y, eps, op, T=T, n_cg=c.n_cg, n_inner=20)
    plan = Plan(c.n, to_dev(uv, prec), J=c.J, levels=c.levels, prec=prec)
    xg, stats, ghist, passes, _ = plan.sdmm_tv(to_dev(y, prec), eps, T=T, n_cg=c.n_cg, n_inner=20)
    assert passes == 1 and stats["iters"] == T
    assert stats["gamma"] == pytest.approx(gam, rel=1e-12 if prec == "f64" else 1e-5)
    assert rel(host(xg), xo) <= tol
    for t in range(1, T):
        assert ghist[t][0] == pytest.approx(hist[t]["f1"], rel=tol)
        assert ghist[t][2] == pytest.approx(hist[t]["nu"], rel=tol)


def test_weighted_tv_from_x0():
    device()
    announce("weighted TV from x0, f64")
    from paper_1307_4370_amd import Plan
    c = W.C1
    uv, op, y, eps = _problem(c, "f64")
    g = W.rng(500, 1)
    w = g.uniform(0.2, 1.5, size=(c.n, c.n))
    x0 = g.uniform(0, 0.5, size=(c.n, c.n)).astype(np.complex128)
    xo, _, hist, gam = tv.sdmm_tv(y, eps, op, T=10, n_cg=c.n_cg, n_inner=15, weights=w, x0=x0)
    plan = Plan(c.n, to_dev(uv, "f64"), J=c.J, levels=c.levels, prec="f64")
    xg, stats, ghist, _, _ = plan.sdmm_tv(to_dev(y, "f64"), eps, T=10, n_cg=c.n_cg, n_inner=15,
                                          weights=to_dev(w, "f64"), x0=to_dev(x0, "f64"))
    assert rel(host(xg), xo) <= 1e-10
    assert ghist[-1][0] == pytest.approx(hist[-1]["f1"], rel=1e-10)


def test_rwtv_matches_oracle():
    device()
    announce("RWTV 1 + 2 passes x 10 iterations, f64")
    from paper_1307_4370_amd import Plan
    c = W.C1
    uv, op, y, eps = _problem(c, "f64")
    xo, passes_o, info = reweight.sdmm_tv_reweighted(y, eps, op, T=10, n_cg=c.n_cg, n_inner=15, outer=2)
    plan = Plan(c.n, to_dev(uv, "f64"), J=c.J, levels=c.levels, prec="f64")
    xg, stats, _, passes, wg = plan.sdmm_tv(to_dev(y, "f64"), eps, T=10, n_cg=c.n_cg, n_inner=15,
                                            reweight={"outer": 2})
    assert passes == passes_o == 3
    assert rel(host(xg), xo) <= 1e-10
    assert rel(host(wg), info[-1]["weights"]) <= 1e-10

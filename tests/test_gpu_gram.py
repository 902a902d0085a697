"""The precomputed Gram operator G^T G (Sec. 4.5, Sec. 7) on the GPU.

Q = Phi^dagger Phi + 2 I applied with the stored planes against the same plan
without them and against the oracle's Q, for several widths (J up to 12, whose
window exceeds one wavefront) and grid sizes, FP64 to 1e-12 and FP32 to
1e-5; SDMM with the stored operator against the oracle's SDMM (64^2,
20 iterations); CG with it; and release back to degridding and gridding.
"""
import numpy as np
import pytest

import workloads as W
from oracle import nufft, sdmm as osdmm, wavelets
from tests.gpu_helpers import TOL, announce, device, host, rel, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,M,J", [(16, 300, 6), (64, 20000, 8), (96, 9001, 8), (48, 5000, 12)])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_gram_q_matches_oracle(n, M, J, prec):
    device()
    announce(f"Gram Q n={n} M={M} J={J} {prec}")
    from paper_1307_4370_amd import Plan
    uv = W.coverage(M, W.rng(600, n + J))
    x = W.random_complex((n, n), W.rng(601, n + J))
    if prec == "f32":
        uv = uv.astype(np.float32).astype(np.float64)
        x = x.astype(np.complex64).astype(np.complex128)
    plan = Plan(n, to_dev(uv, prec), J=J, levels=1, prec=prec)
    xd = to_dev(x, prec)
    q_plain = host(plan.apply_q(xd))
    plan.gram_build()
    q_gram = host(plan.apply_q(xd))
    op = nufft.Operator(n, uv, J)
    q_or = op.phi_adj(op.phi(x)) + 2 * x
    assert rel(q_gram, q_or) <= TOL[prec]
    assert rel(q_gram, q_plain) <= (1e-6 if prec == "f32" else 1e-13)
    plan.gram_release()
    assert rel(host(plan.apply_q(xd)), q_plain) <= (1e-7 if prec == "f32" else 1e-14)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_sdmm_with_gram_matches_oracle(prec, tol):
    device()
    announce(f"SDMM with the stored Gram operator, 64^2, {prec}")
    from paper_1307_4370_amd import Plan
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
    eps = osdmm.noise_bound(c.M, sig)
    xo, _, hist, _ = osdmm.sdmm(y, eps, op, wavelets.Sara(c.n, c.levels), T=20, n_cg=c.n_cg)
    plan = Plan(c.n, to_dev(uv, prec), J=c.J, levels=c.levels, prec=prec)
    plan.gram_build()
    xg, st, ghist, _ = plan.sdmm(to_dev(y, prec), eps, T=20, n_cg=c.n_cg)
    assert rel(host(xg), xo) <= tol
    assert ghist[-1][2] == pytest.approx(hist[-1]["nu"], rel=tol)
    b = W.random_complex((c.n, c.n), W.rng(602, 1))
    xc, _ = plan.cg(to_dev(b, prec), n_iter=8)
    Q = lambda v: op.phi_adj(op.phi(v)) + 2 * v
    assert rel(host(xc), osdmm.conjugate_gradient(Q, b, np.zeros_like(b), 8)) <= (1e-10 if prec == "f64" else 2e-5)

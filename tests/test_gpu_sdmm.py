"""GPU SDMM (Algorithm 1) against the FP64 oracle, called through the C ABI.

After a fixed number of iterations the GPU iterate must match the oracle's
iterate with the same parameters: relative L2 <= 1e-10 (FP64), <= 1e-4 (FP32
bulk with FP64 norms and CG scalars).  The per-iteration halting quantities and
the dual variables are compared too.
"""
import numpy as np
import pytest

import workloads as W
from oracle import nufft, sdmm as osdmm, wavelets
from tests.gpu_helpers import announce, device, host, rel, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _problem(c: W.Config, prec: str):
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
    return x_true, uv, op, y, eps


def _plan(c, uv, prec, mask=wavelets.FULL_MASK):
    from paper_1307_4370_amd import Plan
    return Plan(c.n, to_dev(uv, prec), J=c.J, levels=c.levels, dict_mask=mask, prec=prec)


SMALL = W.Config(50, "sdmm-small", n=32, M=700, J=6, levels=2, T=6, n_gauss=4, n_points=10)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_sdmm_small_matches_oracle(prec, tol):
    device()
    announce(f"sdmm small {prec}")
    c = SMALL
    x_true, uv, op, y, eps = _problem(c, prec)
    sara = wavelets.Sara(c.n, c.levels)
    xo, st, hist, gam = osdmm.sdmm(y, eps, op, sara, T=c.T, n_cg=8)
    plan = _plan(c, uv, prec)
    xg, stats, ghist, gstate = plan.sdmm(to_dev(y, prec), eps, T=c.T, n_cg=8)
    assert stats["iters"] == c.T
    assert stats["gamma"] == pytest.approx(gam, rel=1e-12 if prec == "f64" else 1e-5)
    assert rel(host(xg), xo) <= tol
    assert rel(host(gstate["z1"]), st.z1) <= tol * 10
    assert rel(host(gstate["z2"]), st.z2) <= tol * 10
    assert rel(host(gstate["z3"]), st.z3) <= tol * 10
    assert rel(host(gstate["rhs"]), st.rhs) <= tol * 10
    for t in range(1, c.T):
        f1, zeta, nu = ghist[t][:3]
        assert f1 == pytest.approx(hist[t]["f1"], rel=tol)
        assert nu == pytest.approx(hist[t]["nu"], rel=tol)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_sdmm_config1_fixed_iterations(prec, tol):
    """64 x 64 sky, M = 2048, J = 6, SARA at 3 levels: 100 iterations."""
    device()
    c = W.C1
    announce(f"sdmm C1 {prec} T={c.T}")
    x_true, uv, op, y, eps = _problem(c, prec)
    sara = wavelets.Sara(c.n, c.levels)
    xo, _, hist, gam = osdmm.sdmm(y, eps, op, sara, T=c.T, n_cg=c.n_cg)
    plan = _plan(c, uv, prec)
    xg, stats, ghist, _ = plan.sdmm(to_dev(y, prec), eps, T=c.T, n_cg=c.n_cg)
    assert rel(host(xg), xo) <= tol
    snr_o = osdmm.snr_db(x_true, np.real(xo))
    snr_g = osdmm.snr_db(x_true, np.real(host(xg)))
    assert snr_g == pytest.approx(snr_o, abs=0.01)
    assert ghist[-1][2] == pytest.approx(hist[-1]["nu"], rel=tol)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
@pytest.mark.parametrize("T", [0, 3])
def test_sdmm_from_x0_matches_oracle(prec, tol, T):
    """Steps 1-3 from a given x0 (r_i = L_i x0, x_i = L_i^dagger r_i) and T
    iterations after them: iterate and exported state (z_i and the right-hand
    side sum_i x_i) against the oracle."""
    device()
    announce(f"sdmm from x0 {prec} T={T}")
    c = SMALL
    x_true, uv, op, y, eps = _problem(c, prec)
    sara = wavelets.Sara(c.n, c.levels)
    x0 = np.real(x_true) * 0.5 + 0.1 * W.random_complex((c.n, c.n), W.rng(c.cfg, 77))
    if prec == "f32":
        x0 = x0.astype(np.complex64).astype(np.complex128)
    xo, st, _, _ = osdmm.sdmm(y, eps, op, sara, T=T, n_cg=8, gamma=0.01, x0=x0)
    plan = _plan(c, uv, prec)
    xg, stats, _, gstate = plan.sdmm(to_dev(y, prec), eps, T=T, n_cg=8, gamma=0.01, x0=to_dev(x0, prec))
    assert stats["iters"] == T
    assert rel(host(xg), xo) <= tol
    assert rel(host(gstate["rhs"]), st.rhs) <= tol * 10
    if T:
        assert rel(host(gstate["z1"]), st.z1) <= tol * 10
        assert rel(host(gstate["z2"]), st.z2) <= tol * 10
        assert rel(host(gstate["z3"]), st.z3) <= tol * 10


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_sdmm_without_visibilities(prec, tol):
    """M = 0: the l2-ball constraint is vacuous and Q = 2 I; the iteration
    reduces to the l1 and positivity proxes (nu = 0 with eps = 1)."""
    device()
    announce(f"sdmm M=0 {prec}")
    from paper_1307_4370_amd import Plan
    n, levels = 16, 2
    op = nufft.Operator(n, np.zeros((0, 2)), 6)
    sara = wavelets.Sara(n, levels)
    x0 = W.random_complex((n, n), W.rng(5, 1))
    if prec == "f32":
        x0 = x0.astype(np.complex64).astype(np.complex128)
    y = np.zeros(0, dtype=np.complex128)
    xo, st, hist, _ = osdmm.sdmm(y, 1.0, op, sara, T=3, n_cg=4, gamma=0.05, x0=x0)
    dt = torch.float32 if prec == "f32" else torch.float64
    plan = Plan(n, torch.zeros((0, 2), dtype=dt, device=device()), J=6, levels=levels, prec=prec)
    xg, stats, ghist, gstate = plan.sdmm(to_dev(y, prec), 1.0, T=3, n_cg=4, gamma=0.05, x0=to_dev(x0, prec))
    assert stats["iters"] == 3
    assert rel(host(xg), xo) <= tol
    assert rel(host(gstate["rhs"]), st.rhs) <= tol * 10
    assert rel(host(gstate["z1"]), st.z1) <= tol * 10
    assert rel(host(gstate["z3"]), st.z3) <= tol * 10
    for t in range(3):
        assert ghist[t][2] == 0.0
        assert ghist[t][0] == pytest.approx(hist[t]["f1"], rel=tol)


def test_gamma_query_between_steps_leaves_the_run_alone():
    """riop_gamma with another beta between riop_sdmm_step calls on the same
    plan returns its own penalty and does not change the running state."""
    import ctypes
    device()
    announce("gamma query between SDMM steps")
    from paper_1307_4370_amd import _lib
    c = SMALL
    _, uv, op, y, eps = _problem(c, "f64")
    plan = _plan(c, uv, "f64")
    yd = to_dev(y, "f64")
    xa, sa, _, _ = plan.sdmm(yd, eps, T=4, n_cg=8)
    L = _lib.lib()
    prm = _lib.SdmmParams(T=4, n_cg=8, gamma=0.0, beta=1e-3, xi=1e-3, tau=0.1)
    x = torch.zeros_like(xa)
    stream = _lib._stream(None)
    assert L.riop_sdmm_init(plan._h, yd.data_ptr(), eps, ctypes.byref(prm), None, stream) == 0
    assert L.riop_sdmm_step(plan._h, 2, stream) == 0
    g = plan.gamma(yd, beta=0.5)
    assert L.riop_sdmm_step(plan._h, 2, stream) == 0
    st = _lib.SdmmStats()
    assert L.riop_sdmm_finish(plan._h, None, x.data_ptr(), ctypes.byref(st), stream) == 0
    # Gridding's double-precision LDS atomics may reorder the last bit.
    assert g == pytest.approx(500 * sa["gamma"], rel=1e-12)
    assert st.gamma == pytest.approx(sa["gamma"], rel=1e-14) and st.iters == 4
    assert rel(host(x), host(xa)) <= 1e-12


def test_sdmm_resume_equals_single_run():
    device()
    announce("sdmm resume")
    c = SMALL
    _, uv, op, y, eps = _problem(c, "f64")
    plan = _plan(c, uv, "f64")
    yd = to_dev(y, "f64")
    xa, sa, _, _ = plan.sdmm(yd, eps, T=6, n_cg=8, gamma=0.01)
    x1, s1, _, st = plan.sdmm(yd, eps, T=2, n_cg=8, gamma=0.01)
    xb, sb, _, _ = plan.sdmm(yd, eps, T=4, n_cg=8, gamma=0.01, x0=x1, state=st)
    assert rel(host(xb), host(xa)) <= 1e-14
    assert sb["f1"] == pytest.approx(sa["f1"], rel=1e-14)


@pytest.mark.parametrize("prec,op_tol,tol", [("f64", 1e-12, 1e-10), ("f32", 1e-5, 1e-4)])
def test_config2_operators_and_sdmm(prec, op_tol, tol):
    """256 x 256 sky, M = 131072 Gaussian-density visibilities, J = 8, SARA at
    4 levels (the operator-throughput workload): Phi, Phi^dagger, Psi^dagger
    and Psi in full, and 20 SDMM iterations with n_cg = 16, against the
    oracle (about a second of oracle time per iteration)."""
    device()
    c = W.C2
    announce(f"config 2 operators and SDMM {prec}")
    x_true, uv, op, y, eps = _problem(c, prec)
    sara = wavelets.Sara(c.n, c.levels)
    plan = _plan(c, uv, prec)
    g = W.rng(c.cfg, 91)
    x = W.random_complex((c.n, c.n), g)
    w = W.random_complex(c.M, g)
    if prec == "f32":
        x = x.astype(np.complex64).astype(np.complex128)
        w = w.astype(np.complex64).astype(np.complex128)
    assert rel(host(plan.phi(to_dev(x, prec))), op.phi(x)) <= op_tol
    assert rel(host(plan.phi_adj(to_dev(w, prec))), op.phi_adj(w)) <= op_tol
    alpha = sara.psi_adj(x)
    assert rel(host(plan.psi_adj(to_dev(x, prec))), alpha) <= op_tol
    assert rel(host(plan.psi(to_dev(alpha, prec))), sara.psi(alpha)) <= op_tol
    T = 20
    xo, st, hist, gam = osdmm.sdmm(y, eps, op, sara, T=T, n_cg=16)
    xg, stats, ghist, gstate = plan.sdmm(to_dev(y, prec), eps, T=T, n_cg=16)
    assert stats["gamma"] == pytest.approx(gam, rel=1e-12 if prec == "f64" else 1e-5)
    assert rel(host(xg), xo) <= tol
    assert rel(host(gstate["rhs"]), st.rhs) <= tol * 10
    for t in range(T):
        assert ghist[t][0] == pytest.approx(hist[t]["f1"], rel=tol)
        assert ghist[t][2] == pytest.approx(hist[t]["nu"], rel=tol)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_sdmm_weighted_and_subdictionary(prec, tol):
    device()
    announce(f"sdmm weighted {prec}")
    c = SMALL
    _, uv, op, y, eps = _problem(c, prec)
    mask = 0b100000011
    sara = wavelets.Sara(c.n, c.levels, mask)
    wts = W.rng(51, 0).uniform(0.5, 2.0, size=(sara.q, c.n, c.n))
    if prec == "f32":
        wts = wts.astype(np.float32).astype(np.float64)
    xo, _, _, gam = osdmm.sdmm(y, eps, op, sara, T=5, n_cg=6, weights=wts)
    plan = _plan(c, uv, prec, mask=mask)
    xg, _, _, _ = plan.sdmm(to_dev(y, prec), eps, T=5, n_cg=6, weights=to_dev(wts, prec))
    assert rel(host(xg), xo) <= tol


def test_sdmm_large_eps_gives_zero():
    device()
    announce("sdmm eps >= ||y||")
    c = SMALL
    _, uv, op, y, eps = _problem(c, "f64")
    plan = _plan(c, uv, "f64")
    xg, stats, _, _ = plan.sdmm(to_dev(y, "f64"), 1.01 * np.linalg.norm(y), T=4, n_cg=6)
    assert np.all(host(xg) == 0)


def test_sdmm_rejects_bad_arguments():
    device()
    announce("sdmm bad args")
    from paper_1307_4370_amd import RiopError
    c = SMALL
    _, uv, op, y, eps = _problem(c, "f64")
    plan = _plan(c, uv, "f64")
    for bad_eps in (0.0, -1.0, float("inf")):
        with pytest.raises(RiopError):
            plan.sdmm(to_dev(y, "f64"), bad_eps, T=1)


def test_enqueued_run_equals_sdmm():
    """riop_sdmm_init + riop_sdmm_step + riop_sdmm_finish (no host wait
    between set-up and iterations) give the iterate of riop_sdmm."""
    device()
    announce("sdmm enqueued (init/step/finish) vs riop_sdmm, f64")
    c = W.C1
    _, uv, _, y, eps = _problem(c, "f64")
    plan = _plan(c, uv, "f64")
    yd = to_dev(y, "f64")
    xa, sa, _, _ = plan.sdmm(yd, eps, T=6, n_cg=8)
    plan.sdmm_enqueue(yd, eps, T=6, n_cg=8)
    xb, sb = plan.sdmm_collect()
    assert rel(host(xb), host(xa)) <= 1e-14
    assert sb["iters"] == sa["iters"] == 6
    assert sb["nu"] == pytest.approx(sa["nu"], rel=1e-14)

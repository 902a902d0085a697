"""The C ABI's error and control behaviour, called through the binding.

* Non-finite inputs (NaN, Inf) of every operator and solver call set the
  plan's non-finite flag; synchronising calls return RIOP_ENONFINITE.
* RIOP_DEVICE_MEMORY_LIMIT makes allocations fail with RIOP_ENOMEM, and a
  failed plan creation leaks nothing.
* CG stopped on a relative-residual tolerance, alone and inside SDMM, against
  the oracle's CG with the same rule.
* SDMM's early stop (Sec. 4.4 halting rule) ends the run at the oracle's
  iteration; stats.status_iter names it; a run whose FP32 values overflow
  reports the first non-finite iteration.
* The batch graph is captured again when T grows or n_cg changes, and reused
  otherwise (against per-channel runs).
"""
import os

import numpy as np
import pytest

import workloads as W
from oracle import nufft, sdmm as osdmm, wavelets
from tests.gpu_helpers import announce, device, host, rel, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ENONFINITE, ENOMEM = -6, -3


def _plan(n, uv, prec, J=6, levels=2, mask=wavelets.FULL_MASK):
    from paper_1307_4370_amd import Plan
    return Plan(n, to_dev(uv, prec), J=J, levels=levels, dict_mask=mask, prec=prec)


def _status(fn):
    from paper_1307_4370_amd import RiopError
    try:
        fn()
    except RiopError as e:
        return e.status
    return 0


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_nonfinite_operator_inputs_are_reported(prec):
    device()
    announce(f"non-finite operator inputs {prec}")
    n, M = 32, 500
    uv = W.coverage(M, W.rng(201, 1))
    plan = _plan(n, uv, prec)
    g = W.rng(201, 2)
    x = W.random_complex((n, n), g)
    y = W.random_complex(M, g)
    a = W.random_complex((plan.q, n, n), g)
    plan.sync()  # nothing pending
    bad_x, bad_y, bad_a = x.copy(), y.copy(), a.copy()
    bad_x[3, 5] = np.nan
    bad_y[17] = np.inf + 0j
    bad_a[4, 1, 2] = complex(0, np.nan)
    calls = [("phi", lambda: plan.phi(to_dev(bad_x, prec))),
             ("phi sorted", lambda: plan.phi(to_dev(bad_x, prec), sorted=True)),
             ("phi_adj", lambda: plan.phi_adj(to_dev(bad_y, prec))),
             ("phi_adj sorted", lambda: plan.phi_adj(to_dev(bad_y, prec), sorted=True)),
             ("psi_adj", lambda: plan.psi_adj(to_dev(bad_x, prec))),
             ("psi", lambda: plan.psi(to_dev(bad_a, prec))),
             ("apply_q", lambda: plan.apply_q(to_dev(bad_x, prec)))]
    for name, call in calls:
        call()                      # asynchronous: returns OK
        assert _status(plan.sync) == ENONFINITE, name
        assert _status(plan.sync) == 0, name       # the report clears the flag
    # Finite inputs leave the flag clear.
    plan.phi_adj(plan.phi(to_dev(x, prec)))
    plan.psi(plan.psi_adj(to_dev(x, prec)))
    assert _status(plan.sync) == 0


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_nonfinite_solver_inputs_are_reported(prec):
    device()
    announce(f"non-finite solver inputs {prec}")
    n, M = 32, 500
    uv = W.coverage(M, W.rng(202, 1))
    plan = _plan(n, uv, prec)
    g = W.rng(202, 2)
    x = W.random_complex((n, n), g)
    y = W.random_complex(M, g)
    bad_x, bad_y = x.copy(), y.copy()
    bad_x[0, 0] = np.inf
    bad_y[-1] = np.nan
    assert _status(lambda: plan.cg(to_dev(bad_x, prec), n_iter=3)) == ENONFINITE
    assert _status(lambda: plan.cg(to_dev(x, prec), to_dev(bad_x, prec), n_iter=3)) == ENONFINITE
    assert _status(lambda: plan.gamma(to_dev(bad_y, prec))) == ENONFINITE
    st = {}
    assert _status(lambda: plan.sdmm(to_dev(bad_y, prec), 1.0, T=3, n_cg=4, stats_out=st)) == ENONFINITE
    assert st["iters"] == 0 and st["status_iter"] == 0
    assert _status(lambda: plan.sdmm(to_dev(y, prec), 1.0, T=3, n_cg=4, x0=to_dev(bad_x, prec))) == ENONFINITE
    w = np.ones((plan.q, n, n))
    w[2, 3, 4] = np.nan
    assert _status(lambda: plan.sdmm(to_dev(y, prec), 1.0, T=3, n_cg=4, gamma=0.1,
                                     weights=to_dev(w, prec))) == ENONFINITE
    # A clean call afterwards runs normally.
    _, st2, _, _ = plan.sdmm(to_dev(y, prec), 1.0, T=2, n_cg=4)
    assert st2["iters"] == 2 and np.isfinite(st2["f1"])


def test_overflow_in_single_precision_names_the_iteration():
    """FP32 data near the top of the single-precision range overflow inside
    the first iterations: the run returns RIOP_ENONFINITE and status_iter is
    the first iteration whose f1 or nu is not finite (the history up to it is
    finite)."""
    device()
    announce("fp32 overflow -> status_iter")
    n, M, T = 32, 600, 4
    uv = W.coverage(M, W.rng(203, 1))
    plan = _plan(n, uv, "f32")
    y = 3.0e38 * W.unit_complex_noise(M, W.rng(203, 2)) / 4.0
    y = np.clip(y.real, -3.3e38, 3.3e38) + 1j * np.clip(y.imag, -3.3e38, 3.3e38)
    assert np.all(np.isfinite(y.astype(np.complex64)))
    st = {}
    assert _status(lambda: plan.sdmm(to_dev(y, "f32"), 1.0, T=T, n_cg=3, gamma=1.0, stats_out=st)) == ENONFINITE
    assert 1 <= st["status_iter"] <= T


def test_device_memory_limit_gives_enomem():
    import gc
    gc.collect()
    device()
    announce("RIOP_DEVICE_MEMORY_LIMIT -> ENOMEM")
    from paper_1307_4370_amd import device_bytes
    uv = W.coverage(1000, W.rng(204, 1))
    before = device_bytes()
    os.environ["RIOP_DEVICE_MEMORY_LIMIT"] = str(before + (1 << 20))
    try:
        assert _status(lambda: _plan(128, uv, "f32")) == ENOMEM
        assert device_bytes() == before
    finally:
        del os.environ["RIOP_DEVICE_MEMORY_LIMIT"]
    plan = _plan(128, uv, "f32")
    assert device_bytes() > before
    held = plan.info()["device_bytes"]
    # The SDMM workspace is allocated on first use, under the same limit.
    os.environ["RIOP_DEVICE_MEMORY_LIMIT"] = str(device_bytes() + 1024)
    try:
        y = to_dev(W.random_complex(1000, W.rng(204, 2)), "f32")
        assert _status(lambda: plan.sdmm(y, 1.0, T=1, n_cg=2)) == ENOMEM
    finally:
        del os.environ["RIOP_DEVICE_MEMORY_LIMIT"]
    plan.sdmm(y, 1.0, T=1, n_cg=2)
    assert plan.info()["device_bytes"] > held
    plan.close()
    assert device_bytes() == before


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_cg_tolerance_matches_oracle(prec, tol):
    device()
    announce(f"cg tolerance {prec}")
    n, M, J = 32, 900, 6
    uv = W.coverage(M, W.rng(205, 1))
    if prec == "f32":
        uv = uv.astype(np.float32).astype(np.float64)
    op = nufft.Operator(n, uv, J)
    plan = _plan(n, uv, prec, J=J)
    g = W.rng(205, 2)
    b = W.random_complex((n, n), g)
    x0 = 0.1 * W.random_complex((n, n), g)
    Q = lambda v: op.phi_adj(op.phi(v)) + 2 * v
    rtol = 1e-4
    xg, rr, iters = plan.cg(to_dev(b, prec), to_dev(x0, prec), n_iter=100, tol=rtol, with_iters=True)
    xo = osdmm.conjugate_gradient(Q, b, x0, 100, rtol)
    k = next(k for k in range(1, 100)
             if np.array_equal(osdmm.conjugate_gradient(Q, b, x0, k), xo))
    # FP64 takes the stopping decision on the same residuals as the oracle; FP32
    # residuals may cross the threshold one iteration apart.
    assert abs(iters - k) <= (0 if prec == "f64" else 1) and iters < 100
    assert rel(host(xg), osdmm.conjugate_gradient(Q, b, x0, iters)) <= (tol if prec == "f64" else 2e-5)
    assert np.sqrt(rr) <= rtol * np.linalg.norm(b - Q(x0)) * (1 + 1e-2)


def test_sdmm_cg_tolerance_matches_oracle():
    device()
    announce("sdmm with cg_tol f64")
    c = W.Config(51, "sdmm-tol", n=32, M=900, J=6, levels=2, T=6, n_gauss=4, n_points=10)
    x_true, uv = W.config_inputs(c)
    op = nufft.Operator(c.n, uv, c.J)
    y0 = op.phi(x_true)
    sig = osdmm.noise_sigma(y0, 30.0)
    y = y0 + sig * W.unit_complex_noise(c.M, W.rng(c.cfg, W.STREAM_NOISE))
    eps = osdmm.noise_bound(c.M, sig)
    sara = wavelets.Sara(c.n, c.levels)
    xo, _, hist, gam = osdmm.sdmm(y, eps, op, sara, T=c.T, n_cg=30, cg_tol=1e-3)
    plan = _plan(c.n, uv, "f64", J=c.J, levels=c.levels)
    xg, st, ghist, _ = plan.sdmm(to_dev(y, "f64"), eps, T=c.T, n_cg=30, cg_tol=1e-3)
    assert rel(host(xg), xo) <= 1e-10
    used = [int(h[4]) for h in ghist]
    assert all(1 <= u < 30 for u in used[1:]) and st["cg_iters"] == used[-1]
    for t in range(c.T):
        assert ghist[t][2] == pytest.approx(hist[t]["nu"], rel=1e-10)


def test_sdmm_early_stop_matches_oracle():
    """The halting rule of Sec. 4.4 (xi = 1e-3, tau = 0.1) on a small problem
    whose relative change of f1 and residual ratio clear the thresholds by a
    wide margin at every iteration up to the stop."""
    device()
    announce("sdmm early stop f64")
    n, M, J = 8, 40, 6
    g = W.rng(103, W.STREAM_SKY)
    x = W.sky(n, 2, 3, g, sigma_range=(0.7, 1.5))
    uv = W.coverage(M, W.rng(103, W.STREAM_UV))
    op = nufft.Operator(n, uv, J)
    sara = wavelets.Sara(n, 1, 0b111)
    y0 = op.phi(x)
    sig = osdmm.noise_sigma(y0, 30.0)
    y = y0 + sig * W.unit_complex_noise(M, W.rng(103, W.STREAM_NOISE))
    eps = osdmm.noise_bound(M, sig)
    xo, _, hist, gam = osdmm.sdmm(y, eps, op, sara, T=400, n_cg=8, early_stop=True)
    assert len(hist) < 400
    plan = _plan(n, uv, "f64", J=J, levels=1, mask=0b111)
    xg, st, ghist, _ = plan.sdmm(to_dev(y, "f64"), eps, T=400, n_cg=8, gamma=gam, early_stop=True)
    assert st["iters"] == len(hist) and st["status_iter"] == len(hist)
    assert rel(host(xg), xo) <= 1e-10
    assert ghist[-1][1] < 1e-3 and 0.9 <= ghist[-1][2] <= 1.1


def test_batch_graph_recaptured_when_t_or_ncg_change():
    """One batch run four times with iters_per_graph = 2: T grows (history
    buffer grows), n_cg changes, then T shrinks with n_cg unchanged (the graph
    is reused).  Every run's iterates and statistics equal per-channel runs."""
    device()
    announce("batch graph re-capture")
    from paper_1307_4370_amd import Batch
    J, levels = 6, 2
    sides, uvs, ys, eps, plans = (32, 48, 64), [], [], [], []
    for k, n in enumerate(sides):
        M = 3 * n * n // 2
        uv = W.coverage(M, W.rng(206, 1, k)).astype(np.float32).astype(np.float64)
        y = W.random_complex(M, W.rng(206, 2, k)).astype(np.complex64).astype(np.complex128)
        uvs.append(uv)
        ys.append(to_dev(y, "f32"))
        eps.append(0.5 * float(np.linalg.norm(y)))
        plans.append(_plan(n, uv, "f32", J=J, levels=levels))
    batch = Batch([(n, to_dev(uv, "f32")) for n, uv in zip(sides, uvs)], J=J, levels=levels, prec="f32",
                  autotune=False)
    for T, n_cg in ((4, 4), (6, 4), (4, 6), (2, 6)):
        xs, stats = batch.sdmm(ys, eps, T=T, n_cg=n_cg, iters_per_graph=2)
        for k, plan in enumerate(plans):
            xe, se, _, _ = plan.sdmm(ys[k], eps[k], T=T, n_cg=n_cg)
            assert stats[k]["iters"] == T
            assert rel(host(xs[k]), host(xe)) <= 1e-5, (T, n_cg, k)
            assert stats[k]["f1"] == pytest.approx(se["f1"], rel=1e-5)
            assert stats[k]["nu"] == pytest.approx(se["nu"], rel=1e-5)
    batch.close()

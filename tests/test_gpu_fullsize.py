"""Parity at the benchmark's full size (1024 x 1024, M = 4194304, J = 8, 4
levels), in the plan configuration bench.py times.

The oracle cannot apply the full operators in test time, so:
* Phi: sampled outputs, each computed by the oracle from its own row of G;
* Phi^dagger: the adjoint identity <Phi x, w> = <x, Phi^dagger w> (any size);
* Psi^dagger / Psi: one Daubechies basis (Db8) against the oracle in full;
* SDMM: the FP32 iterate after a few iterations against the FP64 GPU iterate
  (the FP64 path is pinned to the oracle at small sizes) to 1e-4.
"""
import numpy as np
import pytest

import workloads as W
from oracle import nufft, wavelets
from tests.gpu_helpers import announce, device, host, rel, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

C = W.C3


@pytest.fixture(scope="module")
def inputs():
    x, uv = W.config_inputs(C)
    return x, uv


def test_phi_sampled_fullsize(inputs):
    device()
    announce("full-size Phi sampled, f32")
    from paper_1307_4370_amd import Plan
    x, uv = inputs
    uv32 = uv.astype(np.float32).astype(np.float64)
    x32 = x.astype(np.float32).astype(np.float64)
    plan = Plan(C.n, to_dev(uv32, "f32"), J=C.J, levels=C.levels, prec="f32")
    y = host(plan.phi(to_dev(x32.astype(np.complex128), "f32")))
    g = W.rng(300, 0)
    idx = np.concatenate([[0, C.M - 1], g.integers(0, C.M, size=4000)])
    ys = nufft.phi_sampled(x32, uv32, C.J, idx)
    assert rel(y[idx], ys) <= 1e-5
    # Plan order is a permutation of caller order.
    perm = host(plan.layout()[0]).real.astype(np.int64)
    yp = host(plan.phi(to_dev(x32.astype(np.complex128), "f32"), sorted=True))
    assert rel(yp, y[perm]) <= 1e-7


@pytest.mark.parametrize("prec,tol", [("f32", 2e-6), ("f64", 1e-12)])
def test_adjoint_identity_fullsize(inputs, prec, tol):
    device()
    announce(f"full-size adjoint identity {prec}")
    from paper_1307_4370_amd import Plan
    _, uv = inputs
    plan = Plan(C.n, to_dev(uv, prec), J=C.J, levels=C.levels, prec=prec)
    g = W.rng(300, 1)
    x = W.random_complex((C.n, C.n), g)
    w = W.random_complex(C.M, g)
    xd, wd = to_dev(x, prec), to_dev(w, prec)
    y = host(plan.phi(xd))
    xa = host(plan.phi_adj(wd))
    xr, wr = host(xd), host(wd)
    lhs = np.vdot(y, wr)
    rhs = np.vdot(xr.ravel(), xa.ravel())
    assert abs(lhs - rhs) <= tol * abs(lhs)


def test_db8_fullsize(inputs):
    device()
    announce("full-size Db8 analysis/synthesis f32")
    from paper_1307_4370_amd import Plan
    x, uv = inputs
    x32 = x.astype(np.float32).astype(np.complex128)
    plan = Plan(C.n, to_dev(uv[:16].astype(np.float32), "f32"), J=C.J, levels=C.levels,
                dict_mask=1 << 8, prec="f32")
    s = wavelets.Sara(C.n, C.levels, 1 << 8)
    a = host(plan.psi_adj(to_dev(x32, "f32")))
    ao = s.psi_adj(x32)
    assert rel(a, ao) <= 1e-5
    assert rel(host(plan.psi(to_dev(ao, "f32"))), s.psi(ao)) <= 1e-5


def test_sdmm_fp32_vs_fp64_fullsize(inputs):
    device()
    announce("full-size SDMM f32 vs f64, 4 iterations")
    from paper_1307_4370_amd import Plan, noise_bound
    x, uv = inputs
    out = {}
    for prec in ("f64", "f32"):
        uvp = uv.astype(np.float32).astype(np.float64)  # same coverage for both precisions
        plan = Plan(C.n, to_dev(uvp, prec), J=C.J, levels=C.levels, prec=prec)
        y0 = host(plan.phi(to_dev(x.astype(np.complex128), prec)))
        if prec == "f64":
            sigma = np.linalg.norm(y0) * 10 ** (-C.isnr_db / 20) / np.sqrt(C.M)
            y = y0 + sigma * W.unit_complex_noise(C.M, W.rng(C.cfg, W.STREAM_NOISE))
            y = y.astype(np.complex64).astype(np.complex128)
            eps = noise_bound(C.M, sigma)
            out["y"], out["eps"] = y, eps
        xg, st, hist, _ = plan.sdmm(to_dev(out["y"], prec), out["eps"], T=4, n_cg=C.n_cg)
        out[prec] = (host(xg), st, hist)
        del plan
        torch.cuda.empty_cache()
    assert rel(out["f32"][0], out["f64"][0]) <= 1e-4
    assert out["f32"][1]["gamma"] == pytest.approx(out["f64"][1]["gamma"], rel=1e-5)
    assert out["f32"][2][-1][2] == pytest.approx(out["f64"][2][-1][2], rel=1e-4)

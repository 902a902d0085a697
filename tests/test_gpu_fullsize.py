"""Parity at the benchmark's full size (1024 x 1024, M = 4194304, J = 8, 4
levels), in the plan configuration bench.py times, against the FP64 oracle.

* Phi: all M outputs of the image of 64 point sources against their exact
  measurement (the direct Fourier sum over the sources), within the NUFFT's
  error; sampled outputs of a full image against the oracle's own rows of G.
* Phi^dagger: the dirty image Phi^dagger y at 32768 sampled pixels against the
  oracle (stored by tests/golden/make_fullsize_fixture.py, which calls only
  the oracle), and the adjoint identity.
* Psi^dagger / Psi: all nine bases (Dirac, Db1..Db8) against the oracle in full.
* SDMM: T = 2 iterations with n_cg = 16 from x = 0 on the point-source data,
  FP64 and FP32 (with FP64 norms): the penalty, f1 and nu of every iteration,
  the iterate's norm and the iterate at the sampled pixels against the
  oracle's stored values; the FP32 iterate also against the FP64 one.
"""
import numpy as np
import pytest

import os

import workloads as W
from oracle import nufft, sdmm as osdmm, wavelets
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


def test_sara_all_bases_fullsize(inputs):
    device()
    announce("full-size SARA (9 bases) analysis/synthesis f32")
    from paper_1307_4370_amd import Plan
    x, uv = inputs
    x32 = x.astype(np.float32).astype(np.complex128)
    plan = Plan(C.n, to_dev(uv[:16].astype(np.float32), "f32"), J=C.J, levels=C.levels, prec="f32")
    s = wavelets.Sara(C.n, C.levels)
    a = host(plan.psi_adj(to_dev(x32, "f32")))
    ao = s.psi_adj(x32)
    assert rel(a, ao) <= 1e-5
    for b in range(9):
        assert rel(a[b], ao[b]) <= 1e-5, b
    assert rel(host(plan.psi(to_dev(ao, "f32"))), s.psi(ao)) <= 1e-5


FIXTURE = os.path.join(os.path.dirname(__file__), "golden", "fullsize_1024_sdmm.npz")


@pytest.fixture(scope="module")
def point_data():
    """Inputs of the stored oracle run (regenerated: seeded coverage, exact
    point-source visibilities, noise) and the stored expected values."""
    from tests.golden import make_fullsize_fixture as F
    announce("full-size point-source inputs (oracle direct sum, ~30 s)")
    uv, y, eps, sample = F.inputs()
    ref = dict(np.load(FIXTURE, allow_pickle=False))
    assert np.linalg.norm(y) == pytest.approx(float(ref["y_norm"]), rel=1e-12)
    assert eps == pytest.approx(float(ref["eps"]), rel=1e-15)
    return uv, y, eps, sample, ref


def _sampled_rel(full, sample, ref_sample):
    return float(np.linalg.norm(full.ravel()[sample] - ref_sample) / np.linalg.norm(ref_sample))


@pytest.mark.parametrize("prec,tol_x", [("f64", 1e-10), ("f32", 1e-4)])
def test_fullsize_sdmm_against_oracle(point_data, prec, tol_x):
    device()
    announce(f"full-size SDMM T=2 n_cg=16 vs oracle fixture, {prec}")
    from paper_1307_4370_amd import Plan
    uv, y, eps, sample, ref = point_data
    plan = Plan(C.n, to_dev(uv, prec), J=C.J, levels=C.levels, prec=prec)
    yd = to_dev(y, prec)
    tol_op = 1e-12 if prec == "f64" else 1e-5
    dirty = host(plan.phi_adj(yd))
    assert _sampled_rel(dirty, sample, ref["dirty_sample"]) <= tol_op
    assert np.linalg.norm(dirty) == pytest.approx(float(ref["dirty_norm"]), rel=tol_op)
    assert plan.gamma(yd) == pytest.approx(float(ref["gamma"]), rel=tol_op)
    T, n_cg = int(ref["T"]), int(ref["n_cg"])
    xg, st, hist, _ = plan.sdmm(yd, eps, T=T, n_cg=n_cg)
    xg = host(xg)
    assert st["iters"] == T
    assert st["gamma"] == pytest.approx(float(ref["gamma"]), rel=tol_op)
    assert _sampled_rel(xg, sample, ref["x_sample"]) <= tol_x
    assert np.linalg.norm(xg) == pytest.approx(float(ref["x_norm"]), rel=tol_x)
    for t in range(T):
        assert hist[t][0] == pytest.approx(float(ref["f1"][t]), rel=tol_x, abs=1e-300)
        assert hist[t][2] == pytest.approx(float(ref["nu"][t]), rel=tol_x)
    print(f"{prec}: sampled rel err of x^(2) vs oracle "
          f"{_sampled_rel(xg, sample, ref['x_sample']):.3e}, nu {hist[-1][2]:.6f}", flush=True)


def test_fullsize_sdmm_graph_replay_against_oracle(point_data):
    """The same FP32 run as one captured HIP graph replayed (a one-channel
    batch, the form bench.py also times) against the stored oracle values."""
    device()
    announce("full-size SDMM T=2 n_cg=16 as a replayed graph vs oracle fixture, f32")
    from paper_1307_4370_amd import Batch
    uv, y, eps, sample, ref = point_data
    T, n_cg = int(ref["T"]), int(ref["n_cg"])
    bt = Batch([(C.n, to_dev(uv, "f32"))], J=C.J, levels=C.levels, prec="f32", autotune=False)
    xs, stats = bt.sdmm([to_dev(y, "f32")], [eps], T=T, n_cg=n_cg, iters_per_graph=T)
    xg = host(xs[0])
    bt.close()
    assert stats[0]["iters"] == T
    assert stats[0]["gamma"] == pytest.approx(float(ref["gamma"]), rel=1e-5)
    assert stats[0]["nu"] == pytest.approx(float(ref["nu"][T - 1]), rel=1e-4)
    assert _sampled_rel(xg, sample, ref["x_sample"]) <= 1e-4
    assert np.linalg.norm(xg) == pytest.approx(float(ref["x_norm"]), rel=1e-4)


@pytest.mark.parametrize("prec,tol", [("f64", 5e-7), ("f32", 1e-6)])
def test_fullsize_phi_of_point_sources_is_the_exact_sum(prec, tol):
    """Every one of the M outputs of Phi against the exact measurement of the
    point-source image (the sum the NUFFT approximates, Sec. 3.1 / Sec. 5),
    within the J = 8 Kaiser-Bessel interpolation error."""
    device()
    announce(f"full-size Phi of point sources vs exact sum, {prec}")
    from paper_1307_4370_amd import Plan
    from tests.golden import make_fullsize_fixture as F
    C3 = W.C3
    uv = W.coverage(C3.M, W.rng(C3.cfg, W.STREAM_UV)).astype(np.float32).astype(np.float64)
    g = W.rng(C3.cfg, W.STREAM_SKY, 7)
    pix = g.integers(C3.n // 8, C3.n - C3.n // 8, size=(F.N_POINTS, 2))
    amps = g.uniform(0.1, 1.0, size=F.N_POINTS).astype(np.float32).astype(np.float64)
    img = np.zeros((C3.n, C3.n), dtype=np.complex128)
    np.add.at(img, (pix[:, 0], pix[:, 1]), amps)
    exact = nufft.direct_points(pix, amps, uv, C3.n)
    plan = Plan(C3.n, to_dev(uv, prec), J=C3.J, levels=C3.levels, prec=prec)
    assert rel(host(plan.phi(to_dev(img, prec))), exact) <= tol


def test_sdmm_fp32_vs_fp64_fullsize(inputs):
    device()
    announce("full-size SDMM f32 vs f64, 4 iterations")
    from paper_1307_4370_amd import Plan
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
            eps = osdmm.noise_bound(C.M, sigma)
            out["y"], out["eps"] = y, eps
        xg, st, hist, _ = plan.sdmm(to_dev(out["y"], prec), out["eps"], T=4, n_cg=C.n_cg)
        out[prec] = (host(xg), st, hist)
        del plan
        torch.cuda.empty_cache()
    assert rel(out["f32"][0], out["f64"][0]) <= 1e-4
    assert out["f32"][1]["gamma"] == pytest.approx(out["f64"][1]["gamma"], rel=1e-5)
    assert out["f32"][2][-1][2] == pytest.approx(out["f64"][2][-1][2], rel=1e-4)

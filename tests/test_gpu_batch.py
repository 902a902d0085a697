"""Batched SDMM (one replayed HIP graph over channels of uneven sizes) and the
gridding-tile autotuner, on the GPU.

Every channel's iterate must equal the same channel run alone through
riop_sdmm (eager launches), and small channels are checked against the FP64
oracle.  The graph is replayed several times with a remainder outside the
graph, and the batch is run twice in a row (graph reuse, eager work between).
"""
import numpy as np
import pytest

import workloads as W
from oracle import nufft, sdmm as osdmm, wavelets
from tests.gpu_helpers import announce, device, host, rel, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _channels(prec, sides=(32, 48, 64, 96), levels=2, J=6, cfg=60):
    chans = []
    for c, n in enumerate(sides):
        g = W.rng(cfg, W.STREAM_UV, c)
        M = int(g.uniform(1.0, 4.0) * n * n) // 4
        uv = W.coverage(M, g, scale=float(g.uniform(1.0, 2.0)))
        x = W.sky(n, 3, 8, W.rng(cfg, W.STREAM_SKY, c))
        if prec == "f32":
            uv = uv.astype(np.float32).astype(np.float64)
        op = nufft.Operator(n, uv, J)
        y0 = op.phi(x)
        sig = osdmm.noise_sigma(y0, 30.0)
        y = y0 + sig * W.unit_complex_noise(M, W.rng(cfg, W.STREAM_NOISE, c))
        if prec == "f32":
            y = y.astype(np.complex64).astype(np.complex128)
        chans.append(dict(n=n, M=M, uv=uv, op=op, y=y, eps=osdmm.noise_bound(M, sig)))
    return chans


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
@pytest.mark.parametrize("T,ipg", [(6, 2), (7, 3)])
def test_batch_matches_single_runs_and_oracle(prec, tol, T, ipg):
    device()
    announce(f"batch sdmm {prec} T={T} ipg={ipg}")
    from paper_1307_4370_amd import Batch, Plan
    J, levels = 6, 2
    chans = _channels(prec, J=J, levels=levels)
    batch = Batch([(c["n"], to_dev(c["uv"], prec)) for c in chans], J=J, levels=levels, prec=prec,
                  autotune=True)
    ys = [to_dev(c["y"], prec) for c in chans]
    eps = [c["eps"] for c in chans]
    xs, stats = batch.sdmm(ys, eps, T=T, n_cg=6, iters_per_graph=ipg)
    # Second call: graph reused, eager work in between.
    torch.cuda.synchronize()
    _ = ys[0] * 2
    xs2, stats2 = batch.sdmm(ys, eps, T=T, n_cg=6, iters_per_graph=ipg)
    for k, c in enumerate(chans):
        assert stats[k]["iters"] == T and stats2[k]["iters"] == T
        plan = Plan(c["n"], to_dev(c["uv"], prec), J=J, levels=levels, prec=prec)
        xe, se, _, _ = plan.sdmm(ys[k], c["eps"], T=T, n_cg=6)
        single_tol = 1e-12 if prec == "f64" else 1e-5
        assert rel(host(xs[k]), host(xe)) <= single_tol
        assert rel(host(xs2[k]), host(xe)) <= single_tol
        assert stats[k]["nu"] == pytest.approx(se["nu"], rel=single_tol)
        if k < 2:
            sara = wavelets.Sara(c["n"], levels)
            xo, _, _, _ = osdmm.sdmm(c["y"], c["eps"], c["op"], sara, T=T, n_cg=6)
            assert rel(host(xs[k]), xo) <= tol


def test_batch_of_32_uneven_channels():
    """The batched workload at its real shape: 32 channels, image sides over
    {128, ..., 512}, M = 1-4 times the pixel count, (u, v) scaled by 1-2,
    FP32, autotuned tiles, 2 iterations captured in one graph.  Every
    channel's iterate equals its own per-channel run; the first 128 x 128
    channel also matches the oracle on the same data."""
    import math
    device()
    announce("batch of 32 uneven channels")
    from paper_1307_4370_amd import Batch, Plan
    cfg, J, levels, T, n_cg = 4, 8, 4, 2, 4
    chans = W.batch_channels(32, cfg)
    uvs, ys, eps, plans, ys_host = [], [], [], [], []
    for k, (n, M, f) in enumerate(chans):
        uv = W.coverage(M, W.rng(cfg, W.STREAM_UV, k), scale=f).astype(np.float32).astype(np.float64)
        x = W.sky(n, 4, 20, W.rng(cfg, W.STREAM_SKY, k))
        plan = Plan(n, to_dev(uv, "f32"), J=J, levels=levels, prec="f32")
        y0 = host(plan.phi(to_dev(x.astype(np.complex128), "f32")))
        sigma = float(np.linalg.norm(y0)) * 10 ** (-30.0 / 20) / math.sqrt(M)
        y = (y0 + sigma * W.unit_complex_noise(M, W.rng(cfg, W.STREAM_NOISE, k))).astype(np.complex64)
        uvs.append(uv)
        ys.append(to_dev(y.astype(np.complex128), "f32"))
        ys_host.append(y.astype(np.complex128))
        eps.append(osdmm.noise_bound(M, sigma))
        plans.append(plan)
    batch = Batch([(n, to_dev(uv, "f32")) for (n, _, _), uv in zip(chans, uvs)], J=J, levels=levels,
                  prec="f32", autotune=True)
    xs, stats = batch.sdmm(ys, eps, T=T, n_cg=n_cg, iters_per_graph=T)
    for k, plan in enumerate(plans):
        assert stats[k]["iters"] == T
        xe, _, _, _ = plan.sdmm(ys[k], eps[k], T=T, n_cg=n_cg)
        assert rel(host(xs[k]), host(xe)) <= 1e-5, k
    k = next(i for i, (n, _, _) in enumerate(chans) if n == 128)
    n = chans[k][0]
    op = nufft.Operator(n, uvs[k], J)
    xo, _, _, _ = osdmm.sdmm(ys_host[k], eps[k], op, wavelets.Sara(n, levels), T=T, n_cg=n_cg)
    assert rel(host(xs[k]), xo) <= 1e-4
    batch.close()


def test_autotuner_reports_all_admissible_tiles():
    device()
    announce("autotune")
    from paper_1307_4370_amd import autotune_tile
    n, M = 128, 40000
    uv = to_dev(W.coverage(M, W.rng(61, 0)), "f32")
    best, ms = autotune_tile(n, uv, J=8, prec="f32", reps=2)
    tried = [t for t, m in zip((8, 16, 32, 64), ms) if m > 0]
    assert best in tried and len(tried) == 4
    assert ms[(8, 16, 32, 64).index(best)] == min(m for m in ms if m > 0)

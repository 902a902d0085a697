"""GPU parity of the operators against the FP64 oracle (called through the C ABI).

Inputs are seeded and synthetic; for FP32 plans both sides see the same
float32-rounded inputs, so the difference measured is the GPU's arithmetic.
Tolerances: relative L2 <= 1e-5 (FP32), <= 1e-12 (FP64).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import kaiser_bessel as kb
from oracle import nufft, sdmm as osdmm, wavelets
from tests.gpu_helpers import TOL, announce, device, host, rel, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _inputs(n, M, prec, seed, uv=None):
    g = W.rng(200, seed, n * 7 + M)
    if uv is None:
        uv = W.coverage(M, g)
    x = W.random_complex((n, n), g)
    w = W.random_complex(M, g)
    if prec == "f32":
        uv = uv.astype(np.float32).astype(np.float64)
        x = x.astype(np.complex64).astype(np.complex128)
        w = w.astype(np.complex64).astype(np.complex128)
    return uv, x, w


def _plan(n, uv, J, prec, levels=1, mask=wavelets.FULL_MASK, tile=0):
    from paper_1307_4370_amd import Plan
    return Plan(n, to_dev(uv, prec), J=J, levels=levels, dict_mask=mask, prec=prec, tile=tile)


SIZES = [(16, 100, 6), (32, 1000, 8), (64, 2048, 6), (96, 3001, 8), (128, 5000, 8), (192, 4097, 8)]


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("n,M,J", SIZES)
def test_phi_and_adjoint_parity(prec, n, M, J):
    device()
    announce(f"phi parity n={n} M={M} J={J} {prec}")
    uv, x, w = _inputs(n, M, prec, 1)
    op = nufft.Operator(n, uv, J)
    plan = _plan(n, uv, J, prec)
    y = host(plan.phi(to_dev(x, prec)))
    assert rel(y, op.phi(x)) <= TOL[prec]
    xa = host(plan.phi_adj(to_dev(w, prec)))
    assert rel(xa, op.phi_adj(w)) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("J", [10, 12, 14, 16])
def test_wide_kernels(prec, J):
    """Kernel widths above 8 (two window cells per lane and axis), both orders."""
    n, M = 48, 2500
    device()
    announce(f"wide kernel J={J} {prec}")
    uv, x, w = _inputs(n, M, prec, 12)
    op = nufft.Operator(n, uv, J)
    plan = _plan(n, uv, J, prec)
    assert rel(host(plan.phi(to_dev(x, prec))), op.phi(x)) <= TOL[prec]
    assert rel(host(plan.phi_adj(to_dev(w, prec))), op.phi_adj(w)) <= TOL[prec]
    perm = host(plan.layout()[0]).real.astype(np.int64)
    assert rel(host(plan.phi_adj(to_dev(w[perm], prec), sorted=True)), op.phi_adj(w)) <= TOL[prec]


@pytest.mark.parametrize("J,tile", [(2, 8), (4, 8), (4, 32), (6, 64)])
def test_narrow_kernels_double(J, tile):
    """Kernel widths 2 and 4 on the double-precision matrix path (single
    precision needs J >= 6), and J = 6 with the 64-wide tile (two wavefronts
    per workgroup), both orders."""
    n, M, prec = 64, 2500, "f64"
    device()
    announce(f"narrow kernel J={J} tile={tile} {prec}")
    uv, x, w = _inputs(n, M, prec, 15)
    op = nufft.Operator(n, uv, J)
    plan = _plan(n, uv, J, prec, tile=tile)
    assert rel(host(plan.phi(to_dev(x, prec))), op.phi(x)) <= TOL[prec]
    assert rel(host(plan.phi_adj(to_dev(w, prec))), op.phi_adj(w)) <= TOL[prec]
    perm = host(plan.layout()[0]).real.astype(np.int64)
    assert rel(host(plan.phi_adj(to_dev(w[perm], prec), sorted=True)), op.phi_adj(w)) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("tile", [8, 16, 32, 64])
def test_tile_shapes_agree(prec, tile):
    """Every gridding tile size gives the oracle's result (gridding races would show here)."""
    n, M, J = 64, 6000, 8
    device()
    announce(f"tile {tile} {prec}")
    uv, x, w = _inputs(n, M, prec, 2)
    op = nufft.Operator(n, uv, J)
    plan = _plan(n, uv, J, prec, tile=tile)
    assert plan.info()["tile"] == tile
    assert rel(host(plan.phi(to_dev(x, prec))), op.phi(x)) <= TOL[prec]
    assert rel(host(plan.phi_adj(to_dev(w, prec))), op.phi_adj(w)) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_sorted_variants_follow_layout(prec):
    n, M, J = 64, 3000, 8
    device()
    announce(f"sorted variants {prec}")
    uv, x, w = _inputs(n, M, prec, 3)
    op = nufft.Operator(n, uv, J)
    plan = _plan(n, uv, J, prec)
    perm = host(plan.layout()[0]).real.astype(np.int64)
    ys = host(plan.phi(to_dev(x, prec), sorted=True))
    assert rel(ys, op.phi(x)[perm]) <= TOL[prec]
    ws = w[perm]
    assert rel(host(plan.phi_adj(to_dev(ws, prec), sorted=True)), op.phi_adj(w)) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("tile", [8, 32])
def test_layout_is_stable_counting_sort(prec, tile):
    """Plan binning is integer work: bit-exact against the window rule and a stable sort
    by (tile, cell inside the tile in row-major order, caller index)."""
    n, M, J = 64, 7777, 8
    device()
    announce(f"layout tile={tile} {prec}")
    uv, _, _ = _inputs(n, M, prec, 4)
    K = 2 * n
    plan = _plan(n, uv, J, prec, tile=tile)
    perm, cell, ts = (host(t).real.astype(np.int64) for t in plan.layout())
    g = uv * (K / (2 * math.pi))
    a0 = np.mod(kb.window(g, J), K)                     # (M, 2)
    tiles_per_side = K // tile
    tid = (a0[:, 0] // tile) * tiles_per_side + a0[:, 1] // tile
    key = tid * tile * tile + (a0[:, 0] % tile) * tile + a0[:, 1] % tile
    order = np.argsort(key, kind="stable")
    np.testing.assert_array_equal(perm, order)
    np.testing.assert_array_equal(cell & 0xFFFF, a0[order, 0])
    np.testing.assert_array_equal(cell >> 16, a0[order, 1])
    counts = np.bincount(tid, minlength=tiles_per_side ** 2)
    np.testing.assert_array_equal(ts, np.concatenate([[0], np.cumsum(counts)]))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_clustered_coverage_layout_and_operators(prec):
    """A coverage with half of its visibilities in 4 grid cells (50 000 per
    cell, e.g. tracks crossing near the origin): plan creation stays O(M)
    (bit-exact stable order), and Phi, Phi^dagger match the oracle."""
    import time
    n, J, M = 256, 8, 400000
    K = 2 * n
    device()
    announce(f"clustered coverage {prec}")
    g = W.rng(207, 1)
    base = W.coverage(M // 2, g)
    # Grid coordinates a + 1/4 plus up to half a cell: all points of a cluster
    # share one window.
    centres = (np.array([[3, -5], [60, 50], [-180, 110], [250, -255]]) + 0.25) * (2 * math.pi / K)
    jitter = g.uniform(0, 0.5 * 2 * math.pi / K, size=(M // 2, 2))
    clustered = centres[np.arange(M // 2) % 4] + jitter
    uv = np.concatenate([clustered, base])[g.permutation(M)]
    uv, x, w = _inputs(n, M, prec, 14, uv=uv)
    t0 = time.perf_counter()
    plan = _plan(n, uv, J, prec)
    print(f"plan creation {time.perf_counter() - t0:.3f} s", flush=True)
    perm, cell, ts = (host(t).real.astype(np.int64) for t in plan.layout())
    tile = plan.info()["tile"]
    a0 = np.mod(kb.window(uv * (K / (2 * math.pi)), J), K)
    tid = (a0[:, 0] // tile) * (K // tile) + a0[:, 1] // tile
    key = tid * tile * tile + (a0[:, 0] % tile) * tile + a0[:, 1] % tile
    assert np.sort(np.bincount(key))[-4:].min() >= M // 8 - 1000
    np.testing.assert_array_equal(perm, np.argsort(key, kind="stable"))
    op = nufft.Operator(n, uv, J)
    assert rel(host(plan.phi(to_dev(x, prec))), op.phi(x)) <= TOL[prec]
    assert rel(host(plan.phi_adj(to_dev(w, prec))), op.phi_adj(w)) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_adjoint_identity_on_gpu(prec):
    n, M, J = 128, 20000, 8
    device()
    announce(f"adjoint identity {prec}")
    uv, x, w = _inputs(n, M, prec, 5)
    plan = _plan(n, uv, J, prec)
    y = host(plan.phi(to_dev(x, prec)))
    xa = host(plan.phi_adj(to_dev(w, prec)))
    lhs, rhs = np.vdot(y, w), np.vdot(x.ravel(), xa.ravel())
    assert abs(lhs - rhs) <= (1e-6 if prec == "f32" else 1e-13) * abs(lhs)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_edge_points_and_grid_nodes(prec):
    """Coverage edges (+-pi), points exactly on grid nodes, and the centre."""
    n, J = 32, 8
    K = 2 * n
    device()
    announce(f"edge points {prec}")
    pts = [[-math.pi, -math.pi], [math.pi, math.pi], [-math.pi, math.pi], [0.0, 0.0],
           [2 * math.pi * 3 / K, -2 * math.pi * 5 / K], [math.pi - 1e-7, -math.pi + 1e-7]]
    g = W.rng(200, 6)
    uv = np.concatenate([np.array(pts), g.uniform(-math.pi, math.pi, size=(500, 2))])
    uv, x, w = _inputs(n, len(uv), prec, 6, uv=uv)
    op = nufft.Operator(n, uv, J)
    plan = _plan(n, uv, J, prec)
    assert rel(host(plan.phi(to_dev(x, prec))), op.phi(x)) <= TOL[prec]
    assert rel(host(plan.phi_adj(to_dev(w, prec))), op.phi_adj(w)) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_empty_and_single_visibility(prec):
    n, J = 32, 6
    device()
    announce(f"M=0 and M=1 {prec}")
    from paper_1307_4370_amd import Plan
    dt = torch.float32 if prec == "f32" else torch.float64
    plan = Plan(n, torch.zeros((0, 2), dtype=dt, device=device()), J=J, levels=1, prec=prec)
    x = to_dev(W.random_complex((n, n), W.rng(200, 7)), prec)
    assert plan.phi(x).numel() == 0
    xa = host(plan.phi_adj(torch.zeros(0, dtype=x.dtype, device=x.device)))
    assert np.all(xa == 0)
    uv, xx, w = _inputs(n, 1, prec, 8)
    op = nufft.Operator(n, uv, J)
    plan1 = _plan(n, uv, J, prec)
    assert rel(host(plan1.phi(to_dev(xx, prec))), op.phi(xx)) <= TOL[prec]
    assert rel(host(plan1.phi_adj(to_dev(w, prec))), op.phi_adj(w)) <= TOL[prec]


def test_invalid_coverage_is_rejected():
    device()
    announce("invalid uv")
    from paper_1307_4370_amd import Plan, RiopError
    for bad in ([4.0, 0.0], [float("nan"), 0.0], [0.0, -3.2]):
        uv = torch.tensor([[0.1, 0.2], bad], dtype=torch.float64, device=device())
        with pytest.raises(RiopError) as e:
            Plan(32, uv, J=6, levels=1, prec="f64")
        assert e.value.status == -1


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("n,levels,mask", [(32, 2, wavelets.FULL_MASK), (64, 3, wavelets.FULL_MASK),
                                           (64, 1, 1), (64, 3, 1 << 8), (192, 4, wavelets.FULL_MASK),
                                           (128, 4, 0b110)])
def test_sara_parity(prec, n, levels, mask):
    device()
    announce(f"sara n={n} L={levels} mask={mask} {prec}")
    uv, x, _ = _inputs(n, 10, prec, 9)
    s = wavelets.Sara(n, levels, mask)
    plan = _plan(n, uv, 6, prec, levels=levels, mask=mask)
    a = host(plan.psi_adj(to_dev(x, prec)))
    assert rel(a, s.psi_adj(x)) <= TOL[prec]
    g = W.rng(200, 10, n + mask)
    alpha = W.random_complex((s.q, n, n), g)
    if prec == "f32":
        alpha = alpha.astype(np.complex64).astype(np.complex128)
    assert rel(host(plan.psi(to_dev(alpha, prec))), s.psi(alpha)) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("n,M,J,tile", [(32, 5, 6, 8), (48, 700, 6, 16), (64, 4000, 6, 32), (96, 3001, 8, 64),
                                        (128, 5000, 8, 32), (72, 2500, 8, 16)])
def test_gram_matches_degrid_then_grid(prec, n, M, J, tile):
    """Q x through the CG operator path (G^T G without the caller-order
    permutation) against Phi then Phi^dagger in plan order plus 2 x, element
    by element, and against the oracle.  Sizes span several tiles, empty tiles
    (M = 5) and tiles whose region needs the two-wavefront layout (64 x 64)."""
    device()
    announce(f"gram n={n} M={M} J={J} tile={tile} {prec}")
    uv, x, _ = _inputs(n, M, prec, 12)
    plan = _plan(n, uv, J, prec, tile=tile)
    xd = to_dev(x, prec)
    q = host(plan.apply_q(xd))
    split = host(plan.phi_adj(plan.phi(xd, sorted=True), sorted=True) + 2 * xd)
    scale = max(float(np.abs(split).max()), 1e-300)
    assert float(np.abs(q - split).max()) <= (1e-6 if prec == "f32" else 1e-14) * scale
    op = nufft.Operator(n, uv, J)
    assert rel(q, op.phi_adj(op.phi(x)) + 2 * x) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_apply_q_cg_and_gamma(prec):
    n, M, J, levels = 64, 4000, 8, 3
    device()
    announce(f"Q, CG, gamma {prec}")
    uv, x, w = _inputs(n, M, prec, 11)
    op = nufft.Operator(n, uv, J)
    s = wavelets.Sara(n, levels)
    plan = _plan(n, uv, J, prec, levels=levels)
    Q = lambda v: op.phi_adj(op.phi(v)) + 2 * v
    assert rel(host(plan.apply_q(to_dev(x, prec))), Q(x)) <= TOL[prec]
    b = Q(x)
    x0 = np.zeros_like(x)
    for iters in (0, 1, 5, 12):
        xg, rr = plan.cg(to_dev(b, prec), to_dev(x0, prec), n_iter=iters)
        xo = osdmm.conjugate_gradient(Q, b, x0, iters)
        tol = 1e-10 if prec == "f64" else 2e-5
        if iters:
            assert rel(host(xg), xo) <= tol, iters
    gam = plan.gamma(to_dev(w, prec))
    assert gam == pytest.approx(osdmm.penalty(w, op.phi_adj, s.psi_adj), rel=TOL[prec] * 10)

"""Phi as a differentiable torch operation (backward = Phi^dagger), on the GPU.

* The gradient of ||Phi x - y||^2 for a real image is 2 Re Phi^dagger (Phi x - y):
  checked against the FP64 oracle (<= 1e-12 FP64, <= 1e-5 FP32).
* Central finite differences with step 1e-3 in FP64 along 32 random unit
  directions: the loss is quadratic, so they are exact up to rounding (<= 1e-8).
* Adjoint dot-product test through autograd (vector-Jacobian product).
* Batch workload: 16 images of 256 x 256, M = 65536 each, independent coverages.
"""
import numpy as np
import pytest

import workloads as W
from oracle import nufft
from tests.gpu_helpers import announce, device, host, rel, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _batch(B, n, M, J, prec, cfg=3):
    from paper_1307_4370_amd import Plan
    xs, uvs, ys, plans = [], [], [], []
    for b in range(B):
        x = W.sky(n, 10, 40, W.rng(cfg, W.STREAM_SKY, b))
        uv = W.coverage(M, W.rng(cfg, W.STREAM_UV, b))
        g = W.rng(cfg, W.STREAM_VALUES, b)
        y = W.random_complex(M, g) * 0.01
        if prec == "f32":
            uv = uv.astype(np.float32).astype(np.float64)
            x = x.astype(np.float32).astype(np.float64)
            y = y.astype(np.complex64).astype(np.complex128)
        xs.append(x)
        uvs.append(uv)
        ys.append(y)
        plans.append(Plan(n, to_dev(uv, prec), J=J, levels=2, prec=prec))
    return np.stack(xs), uvs, np.stack(ys), plans


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_gradient_matches_oracle(prec, tol):
    device()
    announce(f"autograd gradient {prec}")
    from paper_1307_4370_amd.autograd import phi
    B, n, M, J = 3, 64, 4096, 8
    xs, uvs, ys, plans = _batch(B, n, M, J, prec)
    x = to_dev(xs, prec).requires_grad_(True)
    yd = to_dev(ys, prec)
    loss = (phi(x, plans) - yd).abs().pow(2).sum()
    loss.backward()
    g = host(x.grad)
    for b in range(B):
        op = nufft.Operator(n, uvs[b], J)
        expect = 2 * np.real(op.phi_adj(op.phi(xs[b]) - ys[b]))
        assert rel(g[b], expect) <= tol


def test_finite_differences_fp64():
    device()
    announce("autograd finite differences")
    from paper_1307_4370_amd.autograd import phi
    B, n, M, J = 2, 64, 4096, 8
    xs, _, ys, plans = _batch(B, n, M, J, "f64", cfg=30)
    x = to_dev(xs, "f64").requires_grad_(True)
    yd = to_dev(ys, "f64")

    def loss_fn(v):
        return (phi(v, plans) - yd).abs().pow(2).sum()

    loss_fn(x).backward()
    grad = x.grad.detach()
    g = W.rng(31, W.STREAM_DIRECTIONS)
    h = 1e-3
    with torch.no_grad():
        for _ in range(32):
            d = torch.tensor(g.normal(size=xs.shape), device=x.device)
            d /= torch.linalg.norm(d)
            fd = (loss_fn(x + h * d) - loss_fn(x - h * d)).item() / (2 * h)
            an = float((grad * d).sum())
            assert abs(fd - an) <= 1e-8 * max(abs(an), 1e-300) + 1e-12 * float(loss_fn(x))


def test_vjp_is_adjoint():
    device()
    announce("autograd vjp adjoint")
    from paper_1307_4370_amd.autograd import phi
    B, n, M, J = 2, 64, 3000, 6
    _, _, _, plans = _batch(B, n, M, J, "f64", cfg=32)
    g = W.rng(33, 0)
    xc = to_dev(W.random_complex((B, n, n), g), "f64").requires_grad_(True)
    w = to_dev(W.random_complex((B, M), g), "f64")
    y = phi(xc, plans)
    (gx,) = torch.autograd.grad(y, xc, grad_outputs=w)
    lhs = torch.vdot(y.detach().flatten(), w.flatten()).item()
    rhs = torch.vdot(xc.detach().flatten(), gx.flatten()).item()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_batch_of_16_at_256():
    """16 x 256^2 images, M = 65536 each: forward and backward run; two items vs the oracle."""
    device()
    announce("autograd batch 16 x 256^2")
    from paper_1307_4370_amd.autograd import phi
    c = W.C4
    B = 16
    xs, uvs, ys, plans = _batch(B, c.n, c.M, c.J, "f32", cfg=c.cfg)
    x = to_dev(xs, "f32").requires_grad_(True)
    yd = to_dev(ys, "f32")
    loss = (phi(x, plans) - yd).abs().pow(2).sum()
    loss.backward()
    g = host(x.grad)
    for b in (0, B - 1):
        op = nufft.Operator(c.n, uvs[b], c.J)
        expect = 2 * np.real(op.phi_adj(op.phi(xs[b]) - ys[b]))
        assert rel(g[b], expect) <= 1e-5

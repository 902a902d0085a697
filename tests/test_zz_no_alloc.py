"""riop_cg_noalloc, the allocation-free CG entry point, against riop_cg.

Called through the C ABI with pre-allocated tensors, twice in a row (the
second call on a smaller plan), with results compared to riop_cg on the same
inputs; neither the library nor torch allocates device memory during the
calls, and a plan whose workspace exceeds the static scratch is refused.
"""
import ctypes

import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import announce, device, host, rel, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ENOTSUP = -5


def _call(fn, plan, b, x, n_iter, tol):
    from paper_1307_4370_amd._lib import _stream
    rr, it = ctypes.c_double(), ctypes.c_int32()
    st = fn(plan._h, b.data_ptr(), x.data_ptr(), n_iter, tol, ctypes.byref(rr), ctypes.byref(it), _stream(None))
    return st, rr.value, it.value


@pytest.mark.parametrize("order", ["large-then-small"])
def test_cg_noalloc_matches_cg(order):
    device()
    from paper_1307_4370_amd import Plan, device_bytes, lib
    cases = [(64, 4000, 8, "f64", 12, 0.0, 1e-13), (32, 900, 6, "f32", 20, 1e-4, 1e-6)]
    for n, M, J, prec, n_iter, tol, bar in cases:
        announce(f"cg_noalloc n={n} M={M} {prec} n_iter={n_iter} tol={tol}")
        uv = W.coverage(M, W.rng(208, 1, n))
        plan = Plan(n, to_dev(uv, prec), J=J, levels=2, prec=prec)
        g = W.rng(208, 2, n)
        b = to_dev(W.random_complex((n, n), g), prec)
        x0 = to_dev(0.1 * W.random_complex((n, n), g), prec)
        x_ref, x_na = x0.clone(), x0.clone()
        torch.cuda.synchronize()
        held = device_bytes()
        plan_bytes = plan.info()["device_bytes"]
        torch_bytes = torch.cuda.memory_allocated()
        st, rr_na, it_na = _call(lib().riop_cg_noalloc, plan, b, x_na, n_iter, tol)
        torch.cuda.synchronize()
        assert st == 0, lib().riop_last_error()
        # Nothing allocated: not by the library (its SDMM workspace included), not by torch.
        assert device_bytes() == held
        assert plan.info()["device_bytes"] == plan_bytes
        assert torch.cuda.memory_allocated() == torch_bytes
        st, rr_ref, it_ref = _call(lib().riop_cg, plan, b, x_ref, n_iter, tol)
        assert st == 0
        assert it_na == it_ref
        assert rel(host(x_na), host(x_ref)) <= bar
        assert rr_na == pytest.approx(rr_ref, rel=bar * 10, abs=1e-300)


def test_cg_noalloc_refuses_plans_beyond_the_scratch():
    device()
    announce("cg_noalloc refuses a 1536^2 FP64 plan")
    from paper_1307_4370_amd import Plan, lib
    n = 1536
    plan = Plan(n, torch.zeros((0, 2), dtype=torch.float64, device="cuda"), J=8, levels=2, prec="f64")
    b = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    x = torch.zeros_like(b)
    st, _, _ = _call(lib().riop_cg_noalloc, plan, b, x, 2, 0.0)
    assert st == ENOTSUP
    assert "static scratch" in lib().riop_last_error().decode()

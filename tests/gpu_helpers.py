"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def announce(msg: str):
    """Name the case on stdout before the GPU step runs (flushed)."""
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def rel(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def to_dev(a, prec: str):
    dev = device()
    a = np.asarray(a)
    if np.iscomplexobj(a):
        dt = torch.complex64 if prec == "f32" else torch.complex128
    else:
        dt = torch.float32 if prec == "f32" else torch.float64
    return torch.tensor(a, device=dev).to(dt)


def host(t) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)


# Tolerances (relative L2 over the whole output): FP32 operators within 1e-5 of the
# FP64 oracle; FP64 within a few hundred ulps of accumulated rounding.
TOL = {"f32": 1e-5, "f64": 1e-12}

"""Write the oracle's expected values for the full-size parity test.

Workload: the benchmark's 1024 x 1024 image, M = 4194304 Gaussian-density
(u, v) points, oversampling 2, J = 8, SARA at 4 levels.  The data are the
exact visibilities (direct Fourier sum, Sec. 3.1 eq. ri1 discretised) of 64
point sources plus complex Gaussian noise at 30 dB ISNR; every input is
rounded to single precision, so that the FP32 and FP64 library paths and the
oracle all take the same values.

Stored (FP64, from oracle/ only): the penalty gamma, the per-iteration f1,
zeta and nu of T = 2 SDMM iterations with n_cg = 16 from x = 0 (Algorithm 1),
and, at a seeded sample of pixels, the dirty image Phi^dagger y and the
iterate x^(2), with the full-vector norms of both.

Run from the repository root:  python tests/golden/make_fullsize_fixture.py
(about 5 CPU-minutes and 10 GB of memory).
"""
from __future__ import annotations

import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "fullsize_1024_sdmm.npz")
N_SAMPLE = 32768
T, N_CG, N_POINTS, ISNR = 2, 16, 64, 30.0


def inputs():
    """(uv, y, eps, sample): single-precision-exact (u, v) and y, the noise
    bound and the sampled pixel indices (flat, sorted)."""
    from oracle import nufft, sdmm
    C = W.C3
    uv = W.coverage(C.M, W.rng(C.cfg, W.STREAM_UV)).astype(np.float32).astype(np.float64)
    g = W.rng(C.cfg, W.STREAM_SKY, 7)
    pix = g.integers(C.n // 8, C.n - C.n // 8, size=(N_POINTS, 2))
    amps = g.uniform(0.1, 1.0, size=N_POINTS).astype(np.float32).astype(np.float64)
    y0 = nufft.direct_points(pix, amps, uv, C.n)
    sig = sdmm.noise_sigma(y0, ISNR)
    y = (y0 + sig * W.unit_complex_noise(C.M, W.rng(C.cfg, W.STREAM_NOISE, 7))).astype(np.complex64)
    y = y.astype(np.complex128)
    eps = sdmm.noise_bound(C.M, sig)
    sample = np.sort(W.rng(C.cfg, W.STREAM_DIRECTIONS, 7).choice(C.n * C.n, N_SAMPLE, replace=False))
    return uv, y, eps, sample


def main():
    from oracle import nufft, sdmm, wavelets
    C = W.C3
    t0 = time.time()
    uv, y, eps, sample = inputs()
    print(f"inputs {time.time() - t0:.0f} s", flush=True)
    op = nufft.Operator(C.n, uv, C.J)
    print(f"G built {time.time() - t0:.0f} s", flush=True)
    sara = wavelets.Sara(C.n, C.levels)
    dirty = op.phi_adj(y)
    gamma = sdmm.penalty(y, op.phi_adj, sara.psi_adj)
    print(f"gamma {gamma:.6e} ({time.time() - t0:.0f} s)", flush=True)
    xh, st, hist, gam = sdmm.sdmm(y, eps, op, sara, T=T, n_cg=N_CG, gamma=gamma)
    print(f"sdmm done {time.time() - t0:.0f} s: {hist}", flush=True)
    np.savez_compressed(
        OUT, T=T, n_cg=N_CG, eps=eps, gamma=gamma, y_norm=float(np.linalg.norm(y)),
        f1=np.array([h["f1"] for h in hist]), zeta=np.array([h["zeta"] for h in hist]),
        nu=np.array([h["nu"] for h in hist]),
        dirty_sample=dirty.ravel()[sample], dirty_norm=float(np.linalg.norm(dirty)),
        x_sample=xh.ravel()[sample], x_norm=float(np.linalg.norm(xh)),
        z2_norm=float(np.linalg.norm(st.z2)))
    print(f"wrote {OUT} ({os.path.getsize(OUT)} bytes)")


if __name__ == "__main__":
    main()

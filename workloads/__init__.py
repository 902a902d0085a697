"""Seeded synthetic inputs shared by the oracle-side tests and the product-side runs.

This module only draws random numbers and lays out shapes.  It holds none of the
imaging method's arithmetic (no measurement operator, no wavelet, no prox, no
noise bound): noise is drawn here at unit scale and the caller scales it.

Stand-ins for the paper's data (Sec. 6): the M31 / 30Dor test images and the
variable-density and AMI coverages are not available, so skies are sums of
elliptical Gaussians plus point sources ("compact and extended structures",
Sec. 6), and coverages are 2-D Gaussian variable-density draws of continuous
(u, v) in radians per pixel, denser at low spatial frequency (Sec. 6).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ROOT_SEED = (1307, 4370)

# Named streams inside one configuration seed.
STREAM_SKY = 0
STREAM_UV = 1
STREAM_NOISE = 2
STREAM_DIRECTIONS = 3
STREAM_VALUES = 4


def rng(cfg: int, stream: int, extra: int = 0) -> np.random.Generator:
    """Independent generator for (configuration, stream, extra index)."""
    return np.random.default_rng(np.random.SeedSequence([*ROOT_SEED, cfg, stream, extra]))


def sky(n: int, n_gauss: int, n_points: int, gen: np.random.Generator,
        sigma_range=(1.0, 6.0)) -> np.ndarray:
    """Non-negative n x n sky, peak-normalised to 1 (float64).

    Elliptical Gaussians: centre uniform over the image, axis widths uniform in
    ``sigma_range`` pixels, orientation uniform in [0, pi), amplitude uniform in
    (0, 1).  Point sources: single pixels at uniform positions with amplitude
    uniform in (0, 1).  Row index p is axis 0, column index q is axis 1.
    """
    img = np.zeros((n, n), dtype=np.float64)
    p = np.arange(n, dtype=np.float64)[:, None]
    q = np.arange(n, dtype=np.float64)[None, :]
    for _ in range(n_gauss):
        c0, c1 = gen.uniform(0, n, size=2)
        s0, s1 = gen.uniform(*sigma_range, size=2)
        th = gen.uniform(0, math.pi)
        amp = gen.uniform(0, 1)
        # Gaussian blobs are only evaluated on a window around the centre.
        r = int(math.ceil(5 * max(s0, s1))) + 1
        lo0, hi0 = max(0, int(c0) - r), min(n, int(c0) + r + 1)
        lo1, hi1 = max(0, int(c1) - r), min(n, int(c1) + r + 1)
        d0 = p[lo0:hi0] - c0
        d1 = q[:, lo1:hi1] - c1
        ct, st = math.cos(th), math.sin(th)
        a = (ct * d0 + st * d1) / s0
        b = (-st * d0 + ct * d1) / s1
        img[lo0:hi0, lo1:hi1] += amp * np.exp(-0.5 * (a * a + b * b))
    if n_points:
        idx = gen.integers(0, n, size=(n_points, 2))
        amps = gen.uniform(0, 1, size=n_points)
        np.add.at(img, (idx[:, 0], idx[:, 1]), amps)
    peak = img.max()
    if peak > 0:
        img /= peak
    return img


def coverage(M: int, gen: np.random.Generator, sigma: float = math.pi / 4,
             scale: float = 1.0) -> np.ndarray:
    """(M, 2) float64 continuous (u, v) in radians/pixel, inside [-pi, pi).

    u and v are independent N(0, sigma^2) draws multiplied by ``scale``; a draw
    that falls outside [-pi, pi) is drawn again.
    """
    out = np.empty((M, 2), dtype=np.float64)
    filled = 0
    while filled < M:
        need = M - filled
        cand = gen.normal(0.0, sigma, size=(int(need * 1.2) + 16, 2)) * scale
        ok = np.all((cand >= -math.pi) & (cand < math.pi), axis=1)
        cand = cand[ok][:need]
        out[filled:filled + len(cand)] = cand
        filled += len(cand)
    return out


def unit_complex_noise(M: int, gen: np.random.Generator) -> np.ndarray:
    """Complex Gaussian draws with E|n_m|^2 = 1 (real and imaginary variance 1/2)."""
    return (gen.normal(size=M) + 1j * gen.normal(size=M)) * math.sqrt(0.5)


def random_complex(shape, gen: np.random.Generator) -> np.ndarray:
    """Complex array with independent standard normal real and imaginary parts."""
    return gen.normal(size=shape) + 1j * gen.normal(size=shape)


@dataclasses.dataclass(frozen=True)
class Config:
    """One workload: image side n, visibilities M, KB width J, wavelet levels,
    SDMM iterations T, sky recipe and coverage width."""
    cfg: int
    name: str
    n: int
    M: int
    J: int
    levels: int
    T: int
    n_gauss: int
    n_points: int
    isnr_db: float = 30.0
    uv_sigma: float = math.pi / 4
    n_cg: int = 16


# Workload configurations.  cfg numbers index the seed streams.
C1 = Config(0, "plain-sdmm-64", n=64, M=2048, J=6, levels=3, T=100, n_gauss=20, n_points=50)
C2 = Config(1, "operator-256", n=256, M=131072, J=8, levels=4, T=300, n_gauss=80, n_points=400)
C3 = Config(2, "large-1024", n=1024, M=4194304, J=8, levels=4, T=200, n_gauss=200, n_points=2000)
C4 = Config(3, "autograd-256x16", n=256, M=65536, J=8, levels=4, T=0, n_gauss=80, n_points=400)
CONFIGS = {c.name: c for c in (C1, C2, C3, C4)}

# Batched channels: image sides and visibility multipliers of the uneven batch.
BATCH_SIDES = (128, 192, 256, 384, 512)


def batch_channels(n_channels: int = 32, cfg: int = 4):
    """Uneven channel list for the batched workload.

    Each entry: (n, M, freq_scale).  Image sides uniform over BATCH_SIDES,
    M uniform in [1, 4] times the pixel count, frequency scale uniform in [1, 2].
    """
    g = rng(cfg, STREAM_UV, 10_000)
    out = []
    for _ in range(n_channels):
        n = int(g.choice(BATCH_SIDES))
        M = int(round(g.uniform(1.0, 4.0) * n * n))
        f = float(g.uniform(1.0, 2.0))
        out.append((n, M, f))
    return out


def config_inputs(c: Config, dtype=np.float64):
    """(sky, uv) for a configuration, drawn from their own streams."""
    x = sky(c.n, c.n_gauss, c.n_points, rng(c.cfg, STREAM_SKY))
    uv = coverage(c.M, rng(c.cfg, STREAM_UV), sigma=c.uv_sigma)
    return x.astype(dtype), uv.astype(dtype)

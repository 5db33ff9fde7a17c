"""Seeded synthetic inputs for the discrete LCT / fractional transform.

This module holds input recipes only: random parameters and test functions
sampled on a grid that the caller passes in.  It contains none of the
transform's arithmetic (no nodes, chirps, DFTs or quadrature weights) and is
shared by the tests, the smoke check and the benchmark, for both the GPU path
and the CPU oracle.

Recipes (0-based, numpy ``default_rng`` streams):

* ``hermite_sum``       f = sum_{n<8} c_n psi_n(x), c_n ~ N(0,1) + i N(0,1)
                        (single-signal FP64 case, N = 128).
* ``sl2_params``        a, d ~ U(-2, 2), b = +-U(0.1, 2), c = (ad - 1)/b.
* ``chirped_gaussians`` exp(-(x - mu)^2/(2 sigma^2) + i kappa x^2),
                        mu ~ U(-3, 3), sigma ~ U(0.3, 2), kappa ~ U(-1, 1).
* ``frft_orders``       z = r e^{-i theta}, r ~ U(0.5, 1), theta ~ U(0, 2 pi).
* ``ragged_sizes``      N log-uniform on [256, 65536] snapped (in log) to the
                        nearest of {2^k, 3 2^k, 5 2^k}.
* ``white_noise``       complex Gaussian noise, std ``sigma`` per component.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 1379


def rng(config_index: int, stream: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE + config_index, stream])


def hermite_functions(nmax: int, x: np.ndarray) -> np.ndarray:
    """psi_n(x) = (2^n n! sqrt(pi))^(-1/2) H_n(x) exp(-x^2/2) for n < nmax.

    Evaluated with the three-term recurrence of the normalised functions
    (stable for moderate n), returns an array (nmax, len(x))."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty((nmax, x.size), dtype=np.float64)
    p0 = np.pi ** -0.25 * np.exp(-0.5 * x * x)
    out[0] = p0
    if nmax > 1:
        p1 = math.sqrt(2.0) * x * p0
        out[1] = p1
        for n in range(1, nmax - 1):
            p2 = math.sqrt(2.0 / (n + 1)) * x * out[n] - math.sqrt(n / (n + 1.0)) * out[n - 1]
            out[n + 1] = p2
    return out


def hermite_sum(x: np.ndarray, seed_stream: int = 0, nterms: int = 8):
    """Returns (f, coeffs): f = sum_{n<nterms} c_n psi_n(x)."""
    g = rng(0, seed_stream)
    c = g.standard_normal(nterms) + 1j * g.standard_normal(nterms)
    psi = hermite_functions(nterms, x)
    return (c[:, None] * psi).sum(axis=0), c


def sl2_params(batch: int, g: np.random.Generator) -> np.ndarray:
    """Per-signal (a, b, c, d) with ad - bc = 1: a, d ~ U(-2,2), b = +-U(0.1,2)."""
    a = g.uniform(-2.0, 2.0, batch)
    d = g.uniform(-2.0, 2.0, batch)
    b = g.uniform(0.1, 2.0, batch) * np.where(g.random(batch) < 0.5, -1.0, 1.0)
    c = (a * d - 1.0) / b
    return np.stack([a, b, c, d], axis=1)


def gaussian_params(batch: int, g: np.random.Generator) -> np.ndarray:
    """(mu, sigma, kappa) per signal."""
    mu = g.uniform(-3.0, 3.0, batch)
    sigma = g.uniform(0.3, 2.0, batch)
    kappa = g.uniform(-1.0, 1.0, batch)
    return np.stack([mu, sigma, kappa], axis=1)


def chirped_gaussians(x: np.ndarray, gp: np.ndarray) -> np.ndarray:
    """exp(-(x - mu)^2/(2 sigma^2) + i kappa x^2), one row per (mu, sigma, kappa)."""
    x = np.asarray(x, dtype=np.float64)[None, :]
    mu, sigma, kappa = gp[:, 0:1], gp[:, 1:2], gp[:, 2:3]
    return np.exp(-(x - mu) ** 2 / (2.0 * sigma ** 2) + 1j * kappa * x * x)


def frft_orders(batch: int, g: np.random.Generator) -> np.ndarray:
    r = g.uniform(0.5, 1.0, batch)
    th = g.uniform(0.0, 2.0 * np.pi, batch)
    return r * np.exp(-1j * th)


def smooth_sizes(lo: int = 256, hi: int = 65536) -> np.ndarray:
    s = set()
    for m in (1, 3, 5):
        k = 0
        while m * 2 ** k <= hi:
            if m * 2 ** k >= lo:
                s.add(m * 2 ** k)
            k += 1
    return np.array(sorted(s), dtype=np.int64)


def ragged_sizes(count: int, g: np.random.Generator, lo: int = 256, hi: int = 65536) -> np.ndarray:
    sizes = smooth_sizes(lo, hi)
    u = g.uniform(math.log(lo), math.log(hi), count)
    idx = np.abs(u[:, None] - np.log(sizes)[None, :]).argmin(axis=1)
    return sizes[idx]


def white_noise(shape, g: np.random.Generator, sigma: float = 1e-3) -> np.ndarray:
    return sigma * (g.standard_normal(shape) + 1j * g.standard_normal(shape))

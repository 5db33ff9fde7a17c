"""Pins of the oracle's aliasing-aware LCT (trigonometric interpolation of the
samples onto a grid p times finer, then the Riemann sum of the integral of §1
there, at the Algorithm's output nodes y_j = 4 b x_j / pi).

Checked against: exact reproduction of trigonometric polynomials (phases
reduced exactly in integers), the interpolation written out as an explicit
sum over samples and frequencies (no FFT), O1 itself for p = 1 and b = 0, and
the textbook Gaussian integral for chirped Gaussians whose pre-chirp aliases
on the original grid (there O1 is far from the continuum; the oversampled sum
is not).
"""
import numpy as np
import pytest

import oracle
import workloads


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def gaussian_lct(y, al, be, ga, a, b, d):
    """LCT of exp(-(al x^2 + 2 be x + ga)) (Re al > 0) by the Gaussian integral."""
    A = al - 1j * a / (2 * b)
    B = be + 1j * y / (2 * b)
    return np.sqrt(np.pi / A) / np.sqrt(2j * np.pi * b) * np.exp(1j * d * y * y / (2 * b) - ga + B * B / A)


@pytest.mark.parametrize("N,p", [(15, 3), (16, 2), (16, 3), (64, 4), (1000, 2), (1000, 5), (1001, 3)])
def test_trig_interp_reproduces_trigonometric_polynomials(N, p):
    """f = exp(2 pi i n (x - x_0) / (N h)) for |n| < N/2 is its own interpolant: the fine
    samples are exp(2 pi i n (m - (p-1)/2) / (p N)), phases reduced exactly."""
    k = np.arange(N)
    m = np.arange(p * N)
    for n in sorted({-((N - 1) // 2), -7, 0, 1, 5, (N - 1) // 2}):
        f = np.exp(2j * np.pi * ((n * k) % N) / N)
        g = oracle.trig_interp(f, p)
        num = (n * (2 * m - (p - 1))) % (2 * p * N)  # 2 pi i n (m - (p-1)/2)/(pN) = pi i num / (pN)
        ref = np.exp(1j * np.pi * num / (p * N))
        assert np.abs(g - ref).max() < 1e-12, (N, p, n)


@pytest.mark.parametrize("N,p", [(12, 3), (13, 3), (10, 2), (9, 5)])
def test_trig_interp_matches_explicit_sum(N, p):
    """The interpolant written out: g_m = sum_k f_k (1/N) sum_n w_n exp(2 pi i n ((m - (p-1)/2)/(pN) - k/N)),
    n over -N/2..N/2 with w = 1/2 at n = +-N/2 (even N), else 1; plain loops, no FFT."""
    f = np.random.default_rng(N + p).standard_normal(N) + 1j * np.random.default_rng(p).standard_normal(N)
    half = N // 2
    if N % 2 == 0:
        freqs = [(n, 0.5 if abs(n) == half else 1.0) for n in range(-half, half + 1)]
    else:
        freqs = [(n, 1.0) for n in range(-half, half + 1)]
    g_ref = np.zeros(p * N, dtype=complex)
    for mm in range(p * N):
        s = 0j
        for kk in range(N):
            ker = sum(w * np.exp(2j * np.pi * n * ((mm - (p - 1) / 2) / (p * N) - kk / N)) for n, w in freqs)
            s += f[kk] * ker / N
        g_ref[mm] = s
    assert np.abs(oracle.trig_interp(f, p) - g_ref).max() < 1e-12


def test_oversampled_p1_and_b0_are_O1():
    N = 256
    f = workloads.chirped_gaussians(oracle.nodes(N), workloads.gaussian_params(1, np.random.default_rng(2)))[0]
    for M in [(0.5, 1.0, -0.5, 1.0), (2.0, -0.3, (2.0 * 0.7 - 1) / -0.3, 0.7)]:
        assert np.array_equal(oracle.lct_oversampled(f, *M, 1), oracle.lct(f, *M))
    M = (2.0, 0.0, 0.7, 0.5)
    assert np.array_equal(oracle.lct_oversampled(f, *M, 4), oracle.lct(f, *M))


@pytest.mark.parametrize("N,M,gp,p", [
    # a/b = 20: the pre-chirp's frequency 20 x reaches 70 where f lives, beyond the
    # original grid's Nyquist sqrt(2N) = 45 at N = 1024
    (1024, (2.0, 0.1, (2.0 * 0.3 - 1) / 0.1, 0.3), (0.5, 0.5, 0.3), 2),
    (1024, (2.0, 0.1, (2.0 * 0.3 - 1) / 0.1, 0.3), (0.5, 0.5, 0.3), 8),
    (1024, (-1.5, -0.06, (-1.5 * -0.4 - 1) / -0.06, -0.4), (-0.3, 0.6, -0.5), 4),
    # a C1-range draw (a, d in (-2, 2), |b| >= 0.1) centred at x = 2.5: 19 x + 2 kappa x = 52 > 0.6 Nyquist
    (4096, (1.9, 0.1, (1.9 * 1.5 - 1) / 0.1, 1.5), (2.5, 0.5, 0.8), 2),
    (1000, (1.2, 0.06, (1.2 * 1.1 - 1) / 0.06, 1.1), (0.2, 0.4, 0.0), 3),
])
def test_oversampled_reaches_continuum_where_O1_aliases(N, M, gp, p):
    """Chirped Gaussians whose pre-chirp aliases on eq. asymcer's grid: O1 misses the
    Gaussian integral by far more than 1e-6; the sum on the grid p times finer meets it."""
    a, b, c, d = M
    mu, sigma, kappa = gp
    x = oracle.nodes(N)
    f = workloads.chirped_gaussians(x, np.array([gp]))[0]
    al = 1 / (2 * sigma ** 2) - 1j * kappa
    be = -mu / (2 * sigma ** 2)
    ga = mu ** 2 / (2 * sigma ** 2)
    y = oracle.output_nodes(N, b)
    ref = gaussian_lct(y, al, be, ga, a, b, d)
    e1 = relerr(oracle.lct(f, *M), ref)
    e5 = relerr(oracle.lct_oversampled(f, *M, p), ref)
    assert e1 > 1e-6, e1
    assert e5 < 1e-12, e5


def test_oversampled_rows_and_parity_of_p():
    """Row selection equals the full result; (p - 1) N odd is rejected."""
    N = 300
    f = workloads.chirped_gaussians(oracle.nodes(N), workloads.gaussian_params(1, np.random.default_rng(4)))[0]
    M = (1.0, 0.2, 0.0, 1.0)
    full = oracle.lct_oversampled(f, *M, 3)
    rows = np.array([0, 7, 150, 299])
    assert np.allclose(oracle.lct_oversampled(f, *M, 3, rows=rows), full[rows], rtol=0, atol=1e-15)
    with pytest.raises(ValueError):
        oracle.lct_oversampled(f[:299], *M, 2)

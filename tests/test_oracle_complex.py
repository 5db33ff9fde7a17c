"""Pins of the oracle's LCT for complex matrices at the Algorithm's complex
output nodes y_j = 4 b x_j / pi (O6): O1 itself for real matrices, the
bilateral Laplace transform of a Gaussian in closed form (the case
(a, b, d) = (0, i, 0) of §1), the complex Gaussian integral, and mpmath."""
import mpmath as mp
import numpy as np
import pytest

import oracle
import workloads


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def gaussian_lct(y, al, be, ga, a, b, d):
    """LCT of exp(-(al x^2 + 2 be x + ga)) for complex (a, b, d) at complex y, by the
    Gaussian integral (Re A > 0): sqrt(pi/A) (2 pi i b)^(-1/2) exp(i d y^2/(2b) - ga + B^2/A)."""
    A = al - 1j * a / (2 * b)
    B = be + 1j * y / (2 * b)
    return np.sqrt(np.pi / A) / np.sqrt(2j * np.pi * b) * np.exp(1j * d * y * y / (2 * b) - ga + B * B / A)


@pytest.mark.parametrize("M", [(0.5, 1.0, -0.5, 1.0), (2.0, -0.3, (2.0 * 0.7 - 1) / -0.3, 0.7), (0.0, 1.0, -1.0, 0.0)])
def test_real_matrices_are_O1(M):
    N = 256
    f = workloads.chirped_gaussians(oracle.nodes(N), workloads.gaussian_params(1, np.random.default_rng(3)))[0]
    a, b, c, d = M
    assert relerr(oracle.lct_complex(f, a, b, d), oracle.lct(f, *M)) < 1e-14


@pytest.mark.parametrize("N", [64, 256, 1024])
def test_bilateral_laplace_of_a_gaussian(N):
    """(0, i, 0): G(y) = (2 pi i * i)^(-1/2) int e^{-x y} e^{-x^2/2} dx = -i e^{y^2/2}, at y = 4 i x_j / pi."""
    x = oracle.nodes(N)
    f = np.exp(-x * x / 2) + 0j
    y = oracle.complex_output_nodes(N, 1j)
    ref = -1j * np.exp(y * y / 2)
    assert relerr(oracle.lct_complex(f, 0.0, 1j, 0.0), ref) < 1e-13


@pytest.mark.parametrize("M", [(0.9 + 0.1j, 0.6 - 0.2j, 1.1 + 0.5j), (0.0, 1j, 0.0), (-0.4 + 0.5j, 1.2 - 0.1j, 0.2 + 0.05j),
                               (1.5, -0.8 - 0.1j, -0.4 - 0.2j)])
def test_complex_gaussian_closed_form(M):
    """Chirped Gaussians at complex matrices with bounded chirps (Im(a/b) >= 0, Im(b d) >= 0)."""
    a, b, d = M
    assert np.imag(a / b) >= 0 and np.imag(b * d) >= 0
    N = 1024
    gp = workloads.gaussian_params(1, np.random.default_rng(7))[0]
    mu, sigma, kappa = gp
    f = workloads.chirped_gaussians(oracle.nodes(N), np.array([gp]))[0]
    al = 1 / (2 * sigma ** 2) - 1j * kappa
    be = -mu / (2 * sigma ** 2)
    ga = mu ** 2 / (2 * sigma ** 2)
    y = oracle.complex_output_nodes(N, b)
    ref = gaussian_lct(y, al, be, ga, a, b, d)
    assert relerr(oracle.lct_complex(f, a, b, d), ref) < 1e-10


def test_mpmath_brute_force():
    mp.mp.dps = 40
    N = 12
    a, b, d = mp.mpc(0.7, 0.2), mp.mpc(0.5, 0.4), mp.mpc(-0.3, 0.6)
    g = np.random.default_rng(12)
    f = g.standard_normal(N) + 1j * g.standard_normal(N)
    h = mp.pi / mp.sqrt(2 * N)
    xs = [(2 * k - N + 1) * mp.pi / (2 * mp.sqrt(2 * N)) for k in range(N)]
    amp = h / mp.sqrt(2j * mp.pi * b)
    ref = []
    for j in range(N):
        yj = 4 * b * xs[j] / mp.pi
        s = mp.mpc(0)
        for k in range(N):
            s += mp.exp(1j * (a * xs[k] ** 2 - 2 * xs[k] * yj + d * yj ** 2) / (2 * b)) * mp.mpc(f[k].real, f[k].imag)
        ref.append(complex(amp * s))
    got = oracle.lct_complex(f, complex(a), complex(b), complex(d))
    assert relerr(got, np.array(ref)) < 1e-15

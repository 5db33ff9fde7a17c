"""Pins of the oracle's same-grid discrete fractional transform: the Riemann sum
of eqs. (fasy), (primcuad) with y_j = x_j (eq. cuadtrfor), |z| <= 1."""
import mpmath as mp
import numpy as np
import pytest

import oracle
import workloads


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.mark.parametrize("z", [0.6 * np.exp(-1.1j), 0.9 * np.exp(2.5j), -0.7, 0.3j, 0.55,
                               0.95 * np.exp(-0.4j), np.exp(0.8j)])
def test_continuum_eigen_identity(z):
    """Mehler's formula: the continuous transform of eq. (eqifft) maps psi_n to
    sqrt(2 pi) z^n psi_n; the Riemann sum at N = 256 reproduces that."""
    N = 256
    x = oracle.nodes(N)
    psi = workloads.hermite_functions(8, x)
    for n in range(8):
        g = oracle.frft(psi[n].astype(np.complex128), z)
        ref = np.sqrt(2 * np.pi) * z ** n * psi[n]
        assert relerr(g, ref) < 1e-12, (n, z)


@pytest.mark.parametrize("s", [1, -1])
def test_z_pm_i_is_fourier_kernel(s):
    """z = +-i: eq. (fasy) reduces to exp(+-i x_j x_k) dx, eq. (fftuno)."""
    N = 100
    x = oracle.nodes(N)
    h = np.pi / np.sqrt(2 * N)
    g = np.random.default_rng(1)
    f = g.standard_normal(N) + 1j * g.standard_normal(N)
    G = oracle.frft(f, s * 1j)
    ref = h * np.exp(s * 1j * np.outer(x, x)) @ f
    assert relerr(G, ref) < 1e-13


def test_z_pm_one_limits():
    N = 33
    g = np.random.default_rng(2)
    f = g.standard_normal(N) + 1j * g.standard_normal(N)
    assert np.allclose(oracle.frft(f, 1.0), np.sqrt(2 * np.pi) * f, rtol=0, atol=1e-15)
    assert np.allclose(oracle.frft(f, -1.0), np.sqrt(2 * np.pi) * f[::-1], rtol=0, atol=1e-15)


def gaussian_frft(y, z, s):
    """Gaussian integral: eq. (eqifft) applied to exp(-s x^2)."""
    A = (1 + z * z) / (2 * (1 - z * z)) + s
    B = y * z / (1 - z * z)
    return np.sqrt(2 / (1 - z * z)) * np.sqrt(np.pi / A) * np.exp(B * B / A - (1 + z * z) * y * y / (2 * (1 - z * z)))


@pytest.mark.parametrize("z,tol", [(0.5, 1e-13), (0.98, 1e-13), (0.95 * np.exp(0.3j), 1e-13),
                                   (-0.98, 1e-13), (0.8 * np.exp(2.2j), 1e-13)])
def test_gaussian_closed_form_near_pm_one(z, tol):
    """Close to z = +-1 the kernel's Gaussian in (x_j -+ x_k) narrows; while the grid
    still resolves it the Riemann sum matches the continuous transform."""
    N = 512
    x = oracle.nodes(N)
    fs = np.exp(-x * x / 4).astype(np.complex128)
    assert relerr(oracle.frft(fs, z), gaussian_frft(x, z, 0.25)) < tol


def test_quadrature_degrades_next_to_one():
    """At N = 512 the kernel stops being resolved between z = 0.98 and 0.995: the
    discrete transform is a quadrature, not the continuum limit, next to z = 1."""
    N = 512
    x = oracle.nodes(N)
    fs = np.exp(-x * x / 4).astype(np.complex128)
    assert relerr(oracle.frft(fs, 0.995), gaussian_frft(x, 0.995, 0.25)) > 1e-6


def test_outside_unit_disc_rejected():
    with pytest.raises(ValueError):
        oracle.frft(np.ones(8, dtype=np.complex128), 1.01)


@pytest.mark.parametrize("N,z", [(7, 0.4 - 0.2j), (12, -0.5 + 0.6j), (16, np.exp(2.0j)), (9, 0.99)])
def test_mpmath_brute_force(N, z):
    g = np.random.default_rng(N)
    f = g.standard_normal(N) + 1j * g.standard_normal(N)
    G = oracle.frft(f, z)
    with mp.workdps(40):
        Z = mp.mpc(z.real, z.imag) if isinstance(z, complex) else mp.mpc(z)
        h = mp.pi / mp.sqrt(2 * N)
        xs = [(2 * k - N + 1) * mp.pi / (2 * mp.sqrt(2 * N)) for k in range(N)]
        pref = mp.sqrt(2 / (1 - Z * Z))
        for j in range(N):
            acc = mp.mpc(0)
            for k in range(N):
                e = -((1 + Z * Z) * (xs[j] ** 2 + xs[k] ** 2) - 4 * xs[j] * xs[k] * Z) / (2 * (1 - Z * Z))
                acc += mp.exp(e) * mp.mpc(f[k].real, f[k].imag) * h
            ref = complex(pref * acc)
            assert abs(G[j] - ref) <= 1e-14 * max(1.0, abs(ref))


def test_unit_circle_matches_lct():
    """On |z| = 1, z = e^{-i theta}, the kernel of eq. (fasy) is the LCT kernel of the
    rotation (cos t, sin t, -sin t, cos t) times sqrt(2 pi / z), both evaluated on the
    same nodes when the LCT's output grid is mapped back (4 b / pi = 1 needs
    b = pi/4), so compare continuum values via Hermite functions instead."""
    N = 256
    x = oracle.nodes(N)
    psi = workloads.hermite_functions(6, x)
    theta = 0.9
    z = np.exp(-1j * theta)
    a, b = np.cos(theta), np.sin(theta)
    for n in range(6):
        g = oracle.frft(psi[n].astype(np.complex128), z)
        # LCT of psi_n under the rotation: e^{-i(n+1/2) theta} psi_n(y) (Hermite-Gauss),
        # times sqrt(2 pi / z) (principal) is sqrt(2 pi) e^{-i n theta} psi_n = sqrt(2 pi) z^n psi_n
        lct_val = np.exp(-1j * (n + 0.5) * theta) * psi[n]
        assert relerr(g, np.sqrt(2 * np.pi / z) * lct_val) < 1e-12
        del a, b
        a, b = np.cos(theta), np.sin(theta)

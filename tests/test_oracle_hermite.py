"""Pins of the oracle's exact Hermite-zero quadrature (§2): the eigenvalues of
the symmetric tridiagonal H, the eigenvectors of eq. (ortvec) and the exact
discrete fractional transform F_z of eq. (tmat)."""
import json
import math
import os

import numpy as np
import pytest
from numpy.polynomial.hermite import hermgauss
from scipy.special import eval_hermite

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_closed_form_zeros(N):
    forms = json.load(open(os.path.join(GOLD, "hermite_zeros_small.json")))[str(N)]
    ref = np.array([eval(s, {"sqrt": math.sqrt}) for s in forms])
    assert np.allclose(oracle.hermite_zeros(N), ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("N", [5, 17, 64, 128, 150])
def test_zeros_and_weights_match_hermgauss(N):
    xg, wg = hermgauss(N)
    x = oracle.hermite_zeros(N)
    assert np.abs(x - xg).max() < 1e-13 * max(1.0, np.abs(xg).max())
    U = oracle.hermite_vectors(N, x)
    w = np.sqrt(np.pi) * U[0, :] ** 2
    assert np.abs(w - wg).max() < 1e-13 * wg.max() + 1e-300
    # where the weights are not tiny, relative agreement too
    big = wg > 1e-200
    assert np.abs(w[big] / wg[big] - 1).max() < 1e-10


@pytest.mark.parametrize("N", [6, 50, 257, 1024])
def test_eigenvectors_orthonormal_and_last_component(N):
    """U^T U = I and (u_k)_N = (-1)^(N+k) / sqrt(N) (eq. ortvec at n = N, paper's 1-based k)."""
    U = oracle.hermite_vectors(N)
    assert np.abs(U.T @ U - np.eye(N)).max() < 1e-12
    k1 = np.arange(1, N + 1)
    assert np.allclose(U[N - 1, :], (-1.0) ** (N + k1) / np.sqrt(N), rtol=0, atol=1e-13)


def test_eigen_relation_H():
    """H u_k = x_k u_k for the symmetric H of §2 (off-diagonal sqrt(n/2))."""
    N = 300
    x = oracle.hermite_zeros(N)
    U = oracle.hermite_vectors(N, x)
    e = np.sqrt(np.arange(1, N) / 2.0)
    H = np.diag(e, 1) + np.diag(e, -1)
    assert np.abs(H @ U - U * x[None, :]).max() < 1e-11


@pytest.mark.parametrize("N", [3, 8, 12])
def test_Fz_matches_eq_tmat(N):
    """eq. (tmat) written with scipy's Hermite polynomials at the zeros."""
    z = 0.7 * np.exp(0.9j)
    x = oracle.hermite_zeros(N)
    F = oracle.Fz_exact(N, z)
    j1 = np.arange(1, N + 1)
    HN1 = eval_hermite(N - 1, x)
    pref = np.sqrt(2 * np.pi) * 2.0 ** (N - 1) * math.factorial(N - 1) / N
    S = np.zeros((N, N), dtype=np.complex128)
    for n in range(N):
        Hn = eval_hermite(n, x)
        S += z ** n / (2.0 ** n * math.factorial(n)) * np.outer(Hn, Hn)
    ref = pref * np.outer((-1.0) ** j1 / HN1, (-1.0) ** j1 / HN1) * S
    assert np.abs(F - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("z", [0.6 * np.exp(-1.1j), np.exp(0.4j), -0.3, 1.0])
def test_Fz_eigen_identity(z):
    """Discrete Hermite vectors (rows of U) are eigenvectors of F_z with eigenvalue
    sqrt(2 pi) z^n; on |z| = 1 F_z / sqrt(2 pi) is unitary; F_1 = sqrt(2 pi) I."""
    N = 96
    U = oracle.hermite_vectors(N)
    F = oracle.Fz_exact(N, z, U)
    for n in [0, 1, 5, 40, 95]:
        v = U[n, :]
        assert np.abs(F @ v - np.sqrt(2 * np.pi) * z ** n * v).max() < 1e-12
    if abs(abs(z) - 1) < 1e-15:
        Q = F / np.sqrt(2 * np.pi)
        assert np.abs(Q.conj().T @ Q - np.eye(N)).max() < 1e-12
    if z == 1.0:
        assert np.abs(F - np.sqrt(2 * np.pi) * np.eye(N)).max() < 1e-12


def test_asymptotic_nodes_approach_true_zeros():
    """eq. (asymcer): the equispaced nodes approach the zeros of H_N near the centre
    as N grows (the error of the central nodes falls with N)."""
    errs = []
    for N in [64, 256, 1024]:
        xt = oracle.hermite_zeros(N)
        xa = oracle.nodes(N)
        mid = slice(N // 2 - 4, N // 2 + 4)
        errs.append(np.abs(xt[mid] - xa[mid]).max() / (np.pi / np.sqrt(2 * N)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-3


def test_exact_kernel_approaches_asymptotic_kernel():
    """The derivation after eq. (asymhnt): at large N the exact (F_z)_jk approaches eq.
    (fasy) evaluated at the true zeros, with the local zero spacing as weight, for
    nodes near the centre."""
    N = 400
    z = 0.5 * np.exp(0.7j)
    x = oracle.hermite_zeros(N)
    F = oracle.Fz_exact(N, z)
    mid = np.arange(N // 2 - 10, N // 2 + 10)
    dx = np.gradient(x)
    errs = []
    for j in mid:
        for k in mid:
            asy = np.sqrt(2 / (1 - z * z)) * np.exp(
                -((1 + z * z) * (x[j] ** 2 + x[k] ** 2) - 4 * x[j] * x[k] * z) / (2 * (1 - z * z))) * dx[k]
            errs.append(abs(F[j, k] - asy) / abs(asy))
    assert max(errs) < 5e-3


@pytest.mark.parametrize("N", [1, 5, 64, 200])
def test_xft_apply_matches_eq_tmat_matrix(N):
    """The batched apply sqrt(2 pi) U^T D(z) U f equals the matrix of eq. (tmat) times f."""
    g = np.random.default_rng(N)
    f = g.standard_normal((3, N)) + 1j * g.standard_normal((3, N))
    for z in [0.7 * np.exp(0.9j), -0.4 + 0.1j, 1j, 1.0]:
        F = oracle.Fz_exact(N, z)
        got = oracle.xft(f, z)
        ref = (F @ f.T).T
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
        assert np.allclose(oracle.xft(f[1], z), got[1], rtol=0, atol=1e-14 * np.abs(ref).max())


@pytest.mark.parametrize("N", [512, 1024])
def test_xft_discrete_eigen_identity(N):
    """Rows of U are eigenvectors: xft(U[n], z) = sqrt(2 pi) z^n U[n]; |z| = 1 keeps the norm."""
    U = oracle.hermite_vectors(N)
    rows = [0, 1, 7, N // 2, N - 1]
    z = np.exp(0.37j)
    got = oracle.xft(U[rows].astype(np.complex128), z, U)
    for i, n in enumerate(rows):
        assert np.abs(got[i] - np.sqrt(2 * np.pi) * z ** n * U[n]).max() < 1e-12
    f = np.random.default_rng(1).standard_normal(N) + 0j
    assert abs(np.linalg.norm(oracle.xft(f, z, U)) - np.sqrt(2 * np.pi) * np.linalg.norm(f)) < 1e-11 * np.linalg.norm(f)


def test_xft_approaches_continuum_eigen_identity():
    """The continuum transform maps the Hermite function psi_n to sqrt(2 pi) z^n psi_n
    (Mehler's formula); the exact-node discretisation reproduces it on sampled psi_n with
    an error that falls like 1/N (the O(1/N) convergence of the quadrature), and exactly
    for z = -1 (parity)."""
    errs = []
    z = 0.7 * np.exp(0.9j)
    for N in (64, 256, 1024):
        x = oracle.hermite_zeros(N)
        psi = eval_hermite(3, x) * np.exp(-x * x / 2) / np.sqrt(2 ** 3 * math.factorial(3) * np.sqrt(np.pi))
        ref = np.sqrt(2 * np.pi) * z ** 3 * psi
        errs.append(np.linalg.norm(oracle.xft(psi, z) - ref) / np.linalg.norm(ref))
        refm = -np.sqrt(2 * np.pi) * psi
        assert np.linalg.norm(oracle.xft(psi, -1.0) - refm) < 1e-13 * np.linalg.norm(refm)
    assert errs[2] < 1e-3
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0

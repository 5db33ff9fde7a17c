"""Pins of the oracle's discrete LCT (Riemann sum of the integral of §1 on the
nodes of eq. (asymcer), output nodes y_j = 4 b x_j / pi of the Algorithm).

Each test checks the oracle against something other than itself: the paper's
closed form eq. (exa1), the textbook Gaussian integral, the Hermite-Gauss
eigen-structure of the LCT, exact unitarity of the chirp-DFT-chirp matrix
(§3 and §5), numpy's FFT for the Fourier case, the composition law, finite
differences, and mpmath brute force.
"""
import json
import os

import mpmath as mp
import numpy as np
import pytest

import oracle
import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def exa1(y, al, be, ga, a, b, c, d):
    """eq. (exa1) as printed, for f(x) = exp(-(alpha x^2 + 2 beta x + gamma))."""
    D = 4 * b * b * al * al + a * a
    pre = np.sqrt(np.pi) / (np.sqrt(2j * np.pi * b) * (al * al + a * a / (4 * b * b)) ** 0.25)
    e1 = np.exp(al * (be * be - al * ga) / (al * al + a * a / (4 * b * b)))
    e2 = np.exp(0.5j * np.arctan(a / (2 * al * b)))
    e3 = np.exp(-(al * y * y + 2 * be * a * y + a * a * ga) / D)
    e4 = np.exp(1j * a * c * y * y / (2 * D))
    e5 = np.exp(1j * 2 * b * (al * al * d * y * y + 2 * be * al * y + be * be * a) / D)
    return pre * e1 * e2 * e3 * e4 * e5


def gaussian_lct(y, al, be, ga, a, b, d):
    """Textbook Gaussian integral: LCT of exp(-(al x^2 + 2 be x + ga)), complex al with
    Re(al) > 0: sqrt(pi/A) (2 pi i b)^(-1/2) exp(i d y^2/(2b) - ga + B^2/A),
    A = al - i a/(2b), B = be + i y/(2b)."""
    A = al - 1j * a / (2 * b)
    B = be + 1j * y / (2 * b)
    return np.sqrt(np.pi / A) / np.sqrt(2j * np.pi * b) * np.exp(1j * d * y * y / (2 * b) - ga + B * B / A)


@pytest.mark.parametrize("key,tol", [("fig1", 1e-13), ("fig2", 1e-12)])
def test_paper_example_closed_form(key, tol):
    """§4, Figures 1 and 2: the discrete LCT reproduces eq. (exa1)."""
    p = json.load(open(os.path.join(GOLD, "paper_examples.json")))[key]
    N = p["N"]
    x = oracle.nodes(N)
    f = np.exp(-(p["alpha"] * x * x + 2 * p["beta"] * x + p["gamma"])).astype(np.complex128)
    G = oracle.lct(f, p["a"], p["b"], p["c"], p["d"])
    y = oracle.output_nodes(N, p["b"])
    ref = exa1(y, p["alpha"], p["beta"], p["gamma"], p["a"], p["b"], p["c"], p["d"])
    assert relerr(G, ref) < tol


def test_exa1_matches_gaussian_integral():
    """eq. (exa1) agrees with the general Gaussian integral (checks the test's own closed forms)."""
    y = np.linspace(-5, 5, 41)
    for (al, be, ga, a, b, c, d) in [(1, 2, 3, 1, 2, 0.5, 2), (2, 1, 3, 1, 100, 0, 1), (0.7, -0.3, 0.1, -1.5, 0.4, 0.0, 0.0)]:
        d = d if b == 0 else d
        if (a, b, c, d) == (-1.5, 0.4, 0.0, 0.0):
            d = 1.3
            c = (a * d - 1) / b
        assert relerr(exa1(y, al, be, ga, a, b, c, d), gaussian_lct(y, al, be, ga, a, b, d)) < 1e-13


def test_chirped_gaussians_closed_form():
    """Chirped Gaussians (complex alpha) at random SL(2,R) parameters, N = 4096."""
    N = 4096
    x = oracle.nodes(N)
    g = np.random.default_rng(11)
    M = workloads.sl2_params(4, g)
    gp = workloads.gaussian_params(4, g)
    F = workloads.chirped_gaussians(x, gp)
    for i in range(4):
        a, b, c, d = M[i]
        mu, sigma, kappa = gp[i]
        al = 1 / (2 * sigma ** 2) - 1j * kappa
        be = -mu / (2 * sigma ** 2)
        ga = mu ** 2 / (2 * sigma ** 2)
        rows = np.arange(0, N, 7)
        G = oracle.lct(F[i], a, b, c, d, rows=rows)
        y = oracle.output_nodes(N, b)[rows]
        ref = gaussian_lct(y, al, be, ga, a, b, d)
        # the Riemann sum is spectrally accurate unless the chirp aliases
        # (|a/b| x_max beyond the grid's Nyquist); those draws are excluded
        nyq = np.pi / (np.pi / np.sqrt(2 * N))
        if abs(a / b + 2 * kappa) * x.max() < 0.8 * nyq:
            assert relerr(G, ref) < 1e-10, (i, M[i], gp[i])


def test_long_rows_match_closed_form_at_2_20():
    """N = 2^20: rows of 2^20-term sums (compensated) near the transform's peak against the
    Gaussian integral.  A resolved Gaussian makes the Riemann sum spectrally accurate, so
    what is left is the summation's own rounding over a million terms."""
    N = 1 << 20
    x = oracle.nodes(N)
    a, b, d = 0.8, 1.3, 0.9
    c = (a * d - 1) / b
    mu, sigma, kappa = 0.7, 1.1, 0.3
    al = 1 / (2 * sigma ** 2) - 1j * kappa
    be = -mu / (2 * sigma ** 2)
    ga = mu ** 2 / (2 * sigma ** 2)
    f = np.exp(-(al * x * x + 2 * be * x + ga))
    y = oracle.output_nodes(N, b)
    A = al - 1j * a / (2 * b)
    peak = int(np.argmax(np.real((be + 1j * y / (2 * b)) ** 2 / A)))
    rows = np.arange(peak - 24, peak + 24, 3)
    G = oracle.lct(f, a, b, c, d, rows=rows)
    ref = gaussian_lct(y[rows], al, be, ga, a, b, d)
    assert relerr(G, ref) < 1e-13


def hermite_gauss_lct(n, y, a, b, c, d):
    """Textbook identity: LCT of psi_n is rho^(-1/2) e^(-i(n+1/2)phi) psi_n(y/rho)
    e^(i(ac+bd) y^2 / (2 rho^2)) with a + i b = rho e^(i phi)."""
    z = complex(a, b)
    rho, phi = abs(z), np.angle(z)
    psi = workloads.hermite_functions(n + 1, y / rho)[n]
    return rho ** -0.5 * np.exp(-1j * (n + 0.5) * phi) * psi * np.exp(1j * (a * c + b * d) * y * y / (2 * rho ** 2))


@pytest.mark.parametrize("M,N", [((0.5, 1.0, -0.5, 1.0), 128), ((0.0, 1.0, -1.0, 0.0), 128),
                                 ((np.cos(0.7), np.sin(0.7), -np.sin(0.7), np.cos(0.7)), 128),
                                 # |a/b| = 1.9: the pre-chirp widens the band; at N = 128 the
                                 # Riemann sum still carries 1e-8 discretisation error for
                                 # psi_7, at N = 256 it is at rounding level
                                 ((1.3, -0.7, 0.2, (1 + (-0.7) * 0.2) / 1.3), 256)])
def test_hermite_gauss_eigen_structure(M, N):
    """psi_n for n < 8: the LCT maps Hermite functions to scaled Hermite functions."""
    a, b, c, d = M
    x = oracle.nodes(N)
    y = oracle.output_nodes(N, b)
    psi = workloads.hermite_functions(8, x)
    for n in range(8):
        G = oracle.lct(psi[n].astype(np.complex128), a, b, c, d)
        assert relerr(G, hermite_gauss_lct(n, y, a, b, c, d)) < 1e-13


@pytest.mark.parametrize("N,M", [(64, (0.5, 1.0, -0.5, 1.0)), (96, (1.7, -0.4, 0.3, (1 - 0.4 * 0.3) / 1.7)),
                                 (160, (-2.0, 3.0, 1.0, 2.0))])
def test_unitarity(N, M):
    """§5: the discrete LCT is unitary up to the factor sqrt(4|b|/pi): (4|b|/pi) L^H L = I."""
    a, b, c, d = M
    L = oracle.lct_matrix(N, a, b, c, d)
    E = (4 * abs(b) / np.pi) * (L.conj().T @ L) - np.eye(N)
    assert np.abs(E).max() < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3, 64, 75, 128])
def test_fourier_case_matches_numpy_fft(N):
    """a = d = 0, b = 1: the Riemann sum equals a chirp-free, index-phased FFT (eq. dislctn
    with the integral's sign), evaluated here with numpy's FFT."""
    g = np.random.default_rng(5)
    f = g.standard_normal(N) + 1j * g.standard_normal(N)
    G = oracle.lct(f, 0.0, 1.0, -1.0, 0.0)
    h = np.pi / np.sqrt(2 * N)
    k = np.arange(N)
    ph = np.exp(1j * np.pi * (N - 1) * k / N)
    ref = h / np.sqrt(2j * np.pi) * np.exp(-1j * np.pi * (N - 1) ** 2 / (2 * N)) * ph * np.fft.fft(ph * f)
    assert relerr(G, ref) < 1e-13


def test_b_zero_definition():
    """b = 0 (§1): G(y) = sqrt(d) e^(i c d y^2/2) f(d y), at y_j = x_j/d, checked against the
    continuous Gaussian evaluated at d y_j, for d > 0 and d < 0."""
    N = 200
    x = oracle.nodes(N)
    for (a, c) in [(2.0, 0.7), (-0.5, 1.2)]:
        d = 1.0 / a
        y = x / d
        fx = lambda t: np.exp(-(0.6 * t * t + 0.4 * t + 0.1)).astype(np.complex128)
        G = oracle.lct(fx(x), a, 0.0, c, d)
        ref = np.sqrt(complex(d)) * np.exp(1j * c * d * y * y / 2) * fx(d * y)
        assert relerr(G, ref) < 1e-14


def test_composition_law():
    """L_{M1} after L_{M2} equals +-sqrt(1/sigma) L_{M1 S M2} (S = diag(1/sigma, sigma),
    sigma = 4 b2 / pi: the second transform reads the first one's output grid as
    samples on x_k scaled by sigma); grids match when (M1 S M2)_12 = b1."""
    N = 512
    x = oracle.nodes(N)
    f = np.exp(-(x - 0.5) ** 2 / 1.5 + 0.3j * x * x)
    a2, b2, d2 = 0.6, 0.9, 1.1
    c2 = (a2 * d2 - 1) / b2
    sig = 4 * b2 / np.pi
    b1, d1 = 1.4, -0.8
    a1 = 4 * b1 * (1 - sig * d2) / np.pi
    c1 = (a1 * d1 - 1) / b1
    M1 = np.array([[a1, b1], [c1, d1]])
    M2 = np.array([[a2, b2], [c2, d2]])
    S = np.diag([1 / sig, sig])
    M3 = M1 @ S @ M2
    assert abs(M3[0, 1] - b1) < 1e-14
    G12 = oracle.lct(oracle.lct(f, a2, b2, c2, d2), a1, b1, c1, d1)
    G3 = oracle.lct(f, M3[0, 0], M3[0, 1], M3[1, 0], M3[1, 1]) / np.sqrt(sig)
    e = min(relerr(G12, G3), relerr(G12, -G3))
    assert e < 1e-12


SCALED_CASES = [(0.45, (0.7, 1.3, 0.4)), (0.45, (1.9, 0.25, -0.8)), (2.2, (0.7, 1.3, 0.4)),
                (2.2, (-1.2, -0.6, 1.5)), (1.37, (-0.3, 0.8, 2.1))]


@pytest.mark.parametrize("s,M", SCALED_CASES)
def test_scaled_grid_gaussian_closed_form(s, M):
    """Input grid s x_k (the scaling step of the scaling-chirp-DFT-chirp-scaling form, §1 and §3):
    samples of a complex Gaussian on s x_k, outputs at y_j = 4 b x_j / (pi s), checked against
    the textbook Gaussian integral of the LCT.  A dropped s in the pre-chirp, post-chirp,
    quadrature weight or output nodes gives O(1) errors here."""
    a, b, d = M
    c = (a * d - 1) / b
    N = 1024
    xi = s * oracle.nodes(N)
    al, be, ga = 0.5 + 0.3j, 0.4 - 0.2j, 0.1
    G = oracle.lct(np.exp(-(al * xi * xi + 2 * be * xi + ga)), a, b, c, d, scale=s)
    y = oracle.output_nodes(N, b, d, scale=s)
    assert np.allclose(y, 4 * b * oracle.nodes(N) / (np.pi * s), rtol=1e-15, atol=0)
    assert relerr(G, gaussian_lct(y, al, be, ga, a, b, d)) < 1e-13


@pytest.mark.parametrize("s", [0.6, 1.8])
def test_scaled_grid_b_zero(s):
    """b = 0 on the grid s x_k: G(y_j) = sqrt(d) e^(i c d y_j^2/2) f(d y_j) at y_j = s x_j / d."""
    N = 300
    xi = s * oracle.nodes(N)
    fx = lambda t: np.exp(-(0.6 * t * t + 0.4 * t + 0.1)).astype(np.complex128)
    for (a, c) in [(2.0, 0.7), (-0.5, 1.2)]:
        d = 1.0 / a
        y = oracle.output_nodes(N, 0.0, d, scale=s)
        G = oracle.lct(fx(xi), a, 0.0, c, d, scale=s)
        ref = np.sqrt(complex(d)) * np.exp(1j * c * d * y * y / 2) * fx(d * y)
        assert relerr(G, ref) < 1e-14


@pytest.mark.parametrize("M1,M2", [((0.7, 1.3, 0.4), (0.6, 0.9, 1.1)), ((-1.2, -0.6, 1.5), (1.1, 0.5, 0.2)),
                                   ((0.3, 2.0, 0.9), (0.8, -0.7, -0.4))])
def test_scaled_chain_matches_product_closed_form(M1, M2):
    """Two transforms in a row without resampling: the first one's outputs lie on
    (4 b2 / pi) x_j, i.e. on the grid sigma x_k with sigma = 4 |b2| / pi (reversed when b2 < 0,
    since x_{N-1-j} = -x_j); the second one takes them at scale sigma.  The result is the LCT of
    the product M1 M2 (the composition law) at y_j = 4 b1 x_j / (pi sigma), checked against the
    closed form of that product."""
    N = 1024
    x = oracle.nodes(N)
    al, be, ga = 0.5 + 0.3j, 0.4 - 0.2j, 0.1
    f = np.exp(-(al * x * x + 2 * be * x + ga))
    (a1, b1, d1), (a2, b2, d2) = M1, M2
    c1, c2 = (a1 * d1 - 1) / b1, (a2 * d2 - 1) / b2
    sig = 4 * abs(b2) / np.pi
    G1 = oracle.lct(f, a2, b2, c2, d2)
    if b2 < 0:
        G1 = G1[::-1]
    G = oracle.lct(G1, a1, b1, c1, d1, scale=sig)
    P = np.array([[a1, b1], [c1, d1]]) @ np.array([[a2, b2], [c2, d2]])
    y = oracle.output_nodes(N, b1, d1, scale=sig)
    ref = gaussian_lct(y, al, be, ga, P[0, 0], P[0, 1], P[1, 1])
    assert relerr(G, ref) < 1e-13


def test_scale_one_is_the_algorithm_grid():
    """scale = 1 reproduces the unscaled transform bit for bit."""
    g = np.random.default_rng(5)
    f = g.standard_normal(96) + 1j * g.standard_normal(96)
    M = (1.7, -0.4, 0.3, (1 - 0.4 * 0.3) / 1.7)
    assert np.array_equal(oracle.lct(f, *M), oracle.lct(f, *M, scale=1.0))


def test_scale_rejects_nonpositive():
    f = np.ones(8, dtype=np.complex128)
    for s in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(ValueError):
            oracle.lct(f, 0.5, 1.0, -0.5, 1.0, scale=s)


@pytest.mark.parametrize("N,M", [(8, (0.5, 1.0, -0.5, 1.0)), (15, (1.9, -0.3, 2.0, (1 - 0.6) / 1.9)),
                                 (32, (-1.2, 1.7, 0.4, (1 + 1.7 * 0.4) / -1.2))])
def test_mpmath_brute_force(N, M):
    """40-digit evaluation of the Riemann sum exactly as the definition reads
    (no phase substitution, no integer reduction)."""
    a, b, c, d = M
    g = np.random.default_rng(N)
    f = g.standard_normal(N) + 1j * g.standard_normal(N)
    G = oracle.lct(f, a, b, c, d)
    with mp.workdps(40):
        A, B, D = mp.mpf(a), mp.mpf(b), mp.mpf(d)
        h = mp.pi / mp.sqrt(2 * N)
        xs = [(2 * k - N + 1) * mp.pi / (2 * mp.sqrt(2 * N)) for k in range(N)]
        amp = h / mp.sqrt(2j * mp.pi * B)
        for j in range(N):
            yj = 4 * B * xs[j] / mp.pi
            acc = mp.mpc(0)
            for k in range(N):
                acc += mp.exp(1j * (A * xs[k] ** 2 - 2 * xs[k] * yj + D * yj ** 2) / (2 * B)) * mp.mpc(f[k].real, f[k].imag)
            ref = complex(amp * acc)
            assert abs(G[j] - ref) <= 1e-14 * max(1.0, abs(ref))


def test_mpmath_spot_rows_large_N():
    """Spot rows at N = 4096 with phases up to ~5e4 rad (a/b = 20)."""
    N = 4096
    a, b = 2.0, 0.1
    d = 1.5
    c = (a * d - 1) / b
    x = oracle.nodes(N)
    f = np.exp(-(x - 0.7) ** 2 / 8 + 0.2j * x * x)
    rows = np.array([0, 1500, 4095])
    G = oracle.lct(f, a, b, c, d, rows=rows)
    with mp.workdps(40):
        A, B, D = mp.mpf(a), mp.mpf(b), mp.mpf(d)
        h = mp.pi / mp.sqrt(2 * N)
        xs = [(2 * k - N + 1) * mp.pi / (2 * mp.sqrt(2 * N)) for k in range(N)]
        fk = [mp.exp(-(xv - mp.mpf(0.7)) ** 2 / 8 + mp.mpf(0.2) * 1j * xv * xv) for xv in xs]
        amp = h / mp.sqrt(2j * mp.pi * B)
        for r, j in enumerate(rows):
            yj = 4 * B * xs[j] / mp.pi
            acc = mp.fsum(mp.exp(1j * (A * xs[k] ** 2 - 2 * xs[k] * yj + D * yj ** 2) / (2 * B)) * fk[k]
                          for k in range(N))
            ref = complex(amp * acc)
            # f is rounded to FP64 before the oracle sees it: allow that input error
            assert abs(G[r] - ref) <= 1e-12 * max(1e-3, abs(ref))


def test_adjoint_inner_product():
    N = 200
    a, b, c, d = 0.8, -1.3, 0.5, (1 + 1.3 * 0.5) / 0.8
    g = np.random.default_rng(3)
    f = g.standard_normal(N) + 1j * g.standard_normal(N)
    u = g.standard_normal(N) + 1j * g.standard_normal(N)
    lhs = np.vdot(u, oracle.lct(f, a, b, c, d))
    rhs = np.vdot(oracle.lct_adjoint(u, a, b, c, d), f)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # unitarity: L^H L f = (pi / (4|b|)) f
    back = oracle.lct_adjoint(oracle.lct(f, a, b, c, d), a, b, c, d)
    assert relerr(back * 4 * abs(b) / np.pi, f) < 1e-12


def test_param_grad_finite_differences():
    """Dense-matrix parameter gradient vs central differences of the forward oracle for
    the intensity loss l = sum(|G|^2 - I)^2 (grad_G = 4 (|G|^2 - I) G)."""
    N = 64
    x = oracle.nodes(N)
    f = np.exp(-(x + 0.4) ** 2 / 2.0 + 0.3j * x * x)
    g = np.random.default_rng(9)
    I = g.uniform(0.0, 0.2, N)
    a, b, d = 0.7, 1.3, -0.4
    c = (a * d - 1) / b

    def loss(a_, b_, c_, d_):
        G = oracle.lct(f, a_, b_, c_, d_)
        return float(np.sum((np.abs(G) ** 2 - I) ** 2))

    G = oracle.lct(f, a, b, c, d)
    gG = 4 * (np.abs(G) ** 2 - I) * G
    grad = oracle.lct_param_grad(f, gG, a, b, c, d)
    eps = 1e-6
    p = [a, b, c, d]
    for i in range(4):
        pp = list(p)
        pm = list(p)
        pp[i] += eps
        pm[i] -= eps
        fd = (loss(*pp) - loss(*pm)) / (2 * eps)
        assert abs(grad[i] - fd) <= 1e-7 * max(1e-3, abs(fd)) + 1e-9, (i, grad[i], fd)
    assert grad[2] == 0.0


@pytest.mark.parametrize("c,d", [(0.7, 0.5), (1.2, -2.0)])
def test_param_grad_b_zero_finite_differences(c, d):
    """b = 0: the gradient of the diagonal of §1 (c and d enter, a and b do not) vs central
    differences of the forward oracle, for the loss l = sum |G - T|^2 (grad_G = 2 (G - T)),
    whose phase dependence makes dl/dc nonzero; d < 0 takes the principal root."""
    N = 64
    x = oracle.nodes(N)
    f = np.exp(-(x - 0.3) ** 2 / 2.0 + 0.2j * x * x)
    g = np.random.default_rng(19)
    T = g.standard_normal(N) + 1j * g.standard_normal(N)
    a = 1.0 / d

    def loss(c_, d_):
        G = oracle.lct(f, a, 0.0, c_, d_)
        return float(np.sum(np.abs(G - T) ** 2))

    G = oracle.lct(f, a, 0.0, c, d)
    grad = oracle.lct_param_grad(f, 2 * (G - T), a, 0.0, c, d)
    eps = 1e-6
    fd_c = (loss(c + eps, d) - loss(c - eps, d)) / (2 * eps)
    fd_d = (loss(c, d + eps) - loss(c, d - eps)) / (2 * eps)
    assert abs(grad[2] - fd_c) <= 1e-7 * max(1.0, abs(fd_c)), (grad, fd_c)
    assert abs(grad[3] - fd_d) <= 1e-7 * max(1.0, abs(fd_d)), (grad, fd_d)
    assert abs(fd_c) > 1e-2 and abs(fd_d) > 1e-2
    assert grad[0] == 0.0 and grad[1] == 0.0


def test_nodes_spacing_and_symmetry():
    """eq. (asymcer) and eq. (deltk): symmetric, equispaced with spacing pi/sqrt(2N)."""
    for N in [1, 2, 7, 128, 4096]:
        x = oracle.nodes(N)
        assert np.allclose(x, -x[::-1], atol=1e-15 * max(1, N))
        if N > 1:
            assert np.allclose(np.diff(x), np.pi / np.sqrt(2 * N), rtol=1e-13)


# --- same-grid LCT for complex matrices (O4) -----------------------------------
@pytest.mark.parametrize("z", [0.6 * np.exp(-1.1j), -0.7 + 0.2j, 0.9 * np.exp(2.5j), 0.5, 0.3j])
def test_same_grid_equal_corners_is_the_fractional_transform(z):
    """a = d = (z + 1/z)/2, b = i (z - 1/z)/2 turns the LCT kernel into the fractional kernel
    of eq. (fasy) times (2 pi / z)^(-1/2): against the separately pinned fractional oracle."""
    N = 200
    x = oracle.nodes(N)
    f = np.exp(-(x - 0.3) ** 2 / 1.2 + 0.2j * x * x)
    a = d = (z + 1 / z) / 2
    b = 1j * (z - 1 / z) / 2
    g = oracle.lct_same_grid(f, a, b, d) * np.sqrt(2 * np.pi / z)
    assert relerr(g, oracle.frft(f, z)) < 1e-13


@pytest.mark.parametrize("a,d", [(0.7, 1.3), (-1.4, 0.2), (1.9, -0.6)])
def test_same_grid_is_O1_where_the_grids_coincide(a, d):
    """For a real matrix with b = pi/4 the Algorithm's output nodes 4 b x_j / pi are the input
    nodes, so the same-grid sum and O1 are the same Riemann sum."""
    N = 300
    b = np.pi / 4
    g = np.random.default_rng(3)
    f = g.standard_normal(N) + 1j * g.standard_normal(N)
    ref = oracle.lct(f, a, b, (a * d - 1) / b, d)
    assert relerr(oracle.lct_same_grid(f, a, b, d), ref) < 1e-12


@pytest.mark.parametrize("M", [(0.5 + 0.3j, 1.0 + 0.2j, 0.8 + 0.4j), (1.2 + 0.5j, 0.7 + 0.1j, 0.3 + 0.6j),
                               (-0.4 - 0.3j, -0.9 + 0.3j, -0.5 - 0.4j), (0.9 + 0.1j, 0.6 - 0.2j, 1.1 + 0.05j)])
def test_same_grid_complex_gaussian_closed_form(M):
    """Complex (damped) matrices: the sum reproduces the Gaussian integral of the LCT with complex
    parameters on the grid y_j = x_j (the kernel times the Gaussian input decays in x and y for
    these matrices; the last three also split into bounded Toeplitz or Hankel factors)."""
    a, b, d = M
    N = 512
    x = oracle.nodes(N)
    al, be, ga = 0.5 + 0.3j, 0.4 - 0.2j, 0.1
    G = oracle.lct_same_grid(np.exp(-(al * x * x + 2 * be * x + ga)), a, b, d)
    assert relerr(G, gaussian_lct(x, al, be, ga, a, b, d)) < 1e-12


def test_same_grid_mpmath_brute_force():
    N = 7
    a, b, d = 0.4 + 0.2j, -0.9 + 0.3j, -0.2 + 0.5j
    g = np.random.default_rng(7)
    f = g.standard_normal(N) + 1j * g.standard_normal(N)
    G = oracle.lct_same_grid(f, a, b, d)
    with mp.workdps(40):
        A, B, D = mp.mpc(a.real, a.imag), mp.mpc(b.real, b.imag), mp.mpc(d.real, d.imag)
        xs = [(2 * k - N + 1) * mp.pi / (2 * mp.sqrt(2 * N)) for k in range(N)]
        amp = (mp.pi / mp.sqrt(2 * N)) / mp.sqrt(2j * mp.pi * B)
        for j in range(N):
            acc = mp.mpc(0)
            for k in range(N):
                acc += mp.exp(1j * (A * xs[k] ** 2 - 2 * xs[k] * xs[j] + D * xs[j] ** 2) / (2 * B)) * \
                    mp.mpc(f[k].real, f[k].imag)
            ref = complex(amp * acc)
            assert abs(G[j] - ref) <= 1e-14 * max(1.0, abs(ref))

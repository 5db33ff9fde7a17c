"""GPU parity of the LCT for complex matrices at the Algorithm's complex output
nodes y_j = 4 b x_j / pi (lct_complex_exec): the HIP path through the C ABI
against the oracle's Riemann sum (O6), element by element, FP32
(rel-L2 <= 2e-5) and FP64 (<= 1e-12); the bilateral Laplace transform
(a, b, d) = (0, i, 0) of a Gaussian against its closed form; real matrices
against the plain transform."""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_0912_1379_amd as lct

pytestmark = pytest.mark.gpu

TOL = {torch.complex64: 2e-5, torch.complex128: 1e-12}

MATRICES = [
    (0.0, 1j, 0.0),                                # bilateral Laplace
    (0.9 + 0.1j, 0.6 - 0.2j, 1.1 + 0.5j),          # both diagonals damped
    (-0.4 + 0.5j, 1.2 - 0.1j, 0.2 + 0.05j),
    (1.5, -0.8 - 0.1j, -0.4 - 0.2j),               # real a, b in the lower half-plane
    (0.5, 1.0, -0.5),                              # real matrix
    (0.0, 0.6 - 0.2j, 1.1 + 0.5j),                 # pre-diagonal a pure phase, post damped
    (0.9 + 0.1j, 0.6 - 0.2j, 0.0),                 # pre damped, post-diagonal a pure phase
]


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda").to(dtype)


def gaussian_logmag(gp, a, b, d, y):
    """log |LCT| of exp(-(al x^2 + 2 be x + ga)) at the complex nodes y, from the Gaussian
    integral (used only to choose rows where the output has its energy)."""
    mu, sigma, kappa = gp
    al = 1 / (2 * sigma ** 2) - 1j * kappa
    be = -mu / (2 * sigma ** 2)
    A = al - 1j * a / (2 * b)
    B = be + 1j * y / (2 * b)
    return np.real(B * B / A + 1j * d * y * y / (2 * b))


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("N", [1, 2, 3, 64, 1000, 3072, 4096, 5120, 6144])
@pytest.mark.parametrize("M", MATRICES)
def test_complex_nodes_match_oracle(dtype, N, M):
    a, b, d = M
    g = np.random.default_rng(N + 17)
    x = dev(workloads.chirped_gaussians(oracle.nodes(N), workloads.gaussian_params(3, g)), dtype)
    fin = x.cpu().numpy().astype(np.complex128)
    y = lct.lct_complex_exec(x, a, b, d).cpu().numpy().astype(np.complex128)
    for s in (range(3) if N <= 1000 else (0, 2)):  # dense oracle sums: two signals at the large sizes
        e = rel(y[s], oracle.lct_complex(fin[s], a, b, d))
        assert e <= TOL[dtype], (N, M, s, e)


@pytest.mark.parametrize("dtype,N", [(torch.complex64, 16384), (torch.complex128, 8192)])
@pytest.mark.parametrize("M", MATRICES[:3])
def test_complex_nodes_longest_single_pass(dtype, N, M):
    """The longest single-pass length, 128 rows: 64 where the output has its energy, 64 random."""
    a, b, d = M
    gp = workloads.gaussian_params(2, np.random.default_rng(5))
    x = dev(workloads.chirped_gaussians(oracle.nodes(N), gp), dtype)
    fin = x.cpu().numpy().astype(np.complex128)
    y = lct.lct_complex_exec(x, a, b, d).cpu().numpy().astype(np.complex128)
    nodes = oracle.complex_output_nodes(N, b)
    top = np.argsort(-gaussian_logmag(gp[1], a, b, d, nodes))[:64]
    rows = np.unique(np.concatenate([top, np.random.default_rng(N).choice(N, 64, replace=False)]))
    ref = oracle.lct_complex(fin[1], a, b, d, rows=rows)
    e = rel(y[1, rows], ref)
    assert e <= TOL[dtype], (N, M, e)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("N", [64, 1024, 4096])
def test_bilateral_laplace_of_a_gaussian(dtype, N):
    """(0, i, 0) maps e^{-x^2/2} to -i e^{y^2/2} at y = 4 i x_j / pi (the Riemann sum is
    exact to rounding here, the sampled Gaussian being far below rounding at the ends)."""
    xk = oracle.nodes(N)
    x = dev(np.exp(-xk * xk / 2).astype(np.complex128)[None, :], dtype)
    y = lct.lct_complex_exec(x, 0.0, 1j, 0.0).cpu().numpy().astype(np.complex128)[0]
    nodes = lct.lct_complex_nodes(N, 1j)
    assert np.allclose(nodes, oracle.complex_output_nodes(N, 1j), rtol=1e-14, atol=1e-14)
    e = rel(y, -1j * np.exp(nodes * nodes / 2))
    assert e <= TOL[dtype], (N, e)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_real_matrix_equals_plain_transform(dtype):
    N, B = 4096, 8
    M = (0.5, 1.0, -0.5, 1.0)
    prec = lct.LCT_FP64 if dtype == torch.complex128 else lct.LCT_FP32
    x = dev(workloads.chirped_gaussians(oracle.nodes(N), workloads.gaussian_params(B, np.random.default_rng(2))),
            dtype)
    y = lct.lct_complex_exec(x, M[0], M[1], M[3]).cpu().numpy().astype(np.complex128)
    plan = lct.lct_plan_create(N, *M, precision=prec)
    try:
        z = lct.lct_exec(plan, x).cpu().numpy().astype(np.complex128)
    finally:
        lct.lct_plan_destroy(plan)
    assert rel(y, z) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_ragged_batch_and_in_place(dtype):
    """Several signals per work-group with a partial last group, and in == out."""
    N, B = 64, 37
    a, b, d = MATRICES[1]
    x = dev(workloads.chirped_gaussians(oracle.nodes(N), workloads.gaussian_params(B, np.random.default_rng(9))),
            dtype)
    fin = x.cpu().numpy().astype(np.complex128)
    y = lct.lct_complex_exec(x, a, b, d).cpu().numpy().astype(np.complex128)
    for s in (0, 17, B - 1):
        assert rel(y[s], oracle.lct_complex(fin[s], a, b, d)) <= TOL[dtype]
    lct.lct_complex_exec(x, a, b, d, out=x)
    torch.cuda.synchronize()
    assert rel(x.cpu().numpy().astype(np.complex128), y) == 0.0


def test_empty_batch_and_domain_error():
    x = torch.empty(0, 64, dtype=torch.complex64, device="cuda")
    assert lct.lct_complex_exec(x, 0.0, 1j, 0.0).shape == (0, 64)
    x = torch.zeros(2, 64, dtype=torch.complex64, device="cuda")
    with pytest.raises(Exception):
        lct.lct_complex_exec(x, 0.9 - 0.6j, 0.6 - 0.2j, 1.1 + 0.5j)  # Im(a/b) < 0

"""GPU parity of the same-grid LCT for complex matrices (lct_same_grid_exec):
the HIP path through the C ABI against the oracle's Riemann sum (O4), element
by element, FP32 (rel-L2 <= 2e-5) and FP64 (<= 1e-12), one and two passes."""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_0912_1379_amd as lct

pytestmark = pytest.mark.gpu

TOL = {torch.complex64: 2e-5, torch.complex128: 1e-12}

MATRICES = [
    (0.9 + 0.1j, 0.6 - 0.2j, 1.1 + 0.05j),    # damped, Toeplitz form
    (1.2 + 0.5j, 0.7 + 0.1j, 0.3 + 0.6j),     # damped, Hankel form
    (-0.4 - 0.3j, -0.9 + 0.3j, -0.5 - 0.4j),  # damped, Hankel form, b in the left half-plane
    (0.7, np.pi / 4, 1.3),                    # real: the Algorithm's grid (b = pi/4)
    (1.5, -0.8, 0.4),                         # real, unit-modulus chirps
]


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def peak_rows(gp, a, b, d, N, nrow, seed):
    """Rows where the same-grid LCT of a chirped Gaussian has its energy (from the
    Gaussian integral's modulus, used only to choose rows: with f = exp(-al x^2 - 2 be x + .)
    the integral is sqrt(pi/A) exp(B^2/A) with A = al - i a/(2b), B = be + i y/(2b), times
    the output chirp exp(i d y^2/(2b))), plus random rows."""
    mu, sigma, kappa = gp
    al = 1 / (2 * sigma ** 2) - 1j * kappa
    be = -mu / (2 * sigma ** 2)
    y = oracle.nodes(N)
    A = al - 1j * a / (2 * b)
    B = be + 1j * y / (2 * b)
    logmag = np.real(B * B / A + 1j * d * y * y / (2 * b))
    top = np.argsort(-logmag)[: nrow // 2]
    rnd = np.random.default_rng(seed).choice(N, nrow - nrow // 2, replace=False)
    return np.unique(np.concatenate([top, rnd]))


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda").to(dtype)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("N", [1, 2, 3, 64, 1000, 4096, 6144])
@pytest.mark.parametrize("M", MATRICES)
def test_same_grid_matches_oracle(dtype, N, M):
    a, b, d = M
    g = np.random.default_rng(N)
    x = dev(workloads.chirped_gaussians(oracle.nodes(N), workloads.gaussian_params(3, g)), dtype)
    fin = x.cpu().numpy().astype(np.complex128)
    y = lct.lct_same_grid_exec(x, a, b, d).cpu().numpy().astype(np.complex128)
    for s in range(3 if N <= 1000 else 1):  # dense oracle sums: one signal at the large sizes
        e = rel(y[s], oracle.lct_same_grid(fin[s], a, b, d))
        assert e <= TOL[dtype], (N, M, s, e)


@pytest.mark.parametrize("dtype,N", [(torch.complex64, 16384), (torch.complex128, 8192)])
def test_same_grid_two_pass(dtype, N):
    """Lengths whose convolution (2N) exceeds the single-pass limit: sampled rows."""
    a, b, d = MATRICES[1]
    g = np.random.default_rng(5)
    gp = workloads.gaussian_params(2, g)
    x = dev(workloads.chirped_gaussians(oracle.nodes(N), gp), dtype)
    fin = x.cpu().numpy().astype(np.complex128)
    y = lct.lct_same_grid_exec(x, a, b, d).cpu().numpy().astype(np.complex128)
    ref0 = oracle.lct_same_grid(fin[0], a, b, d)  # every output: the energy is where it is
    assert rel(y[0], ref0) <= TOL[dtype]
    rows = peak_rows(gp[1], a, b, d, N, 96, 9)
    assert rel(y[1][rows], oracle.lct_same_grid(fin[1], a, b, d, rows=rows)) <= TOL[dtype]


@pytest.mark.parametrize("z", [0.6 * np.exp(-1.1j), -0.7 + 0.2j, 0.3j])
def test_same_grid_equal_corners_is_frft(z):
    """a = d = (z + 1/z)/2, b = i (z - 1/z)/2: the GPU's same-grid LCT times sqrt(2 pi / z) is the
    GPU's fractional transform (different constants, same kernels)."""
    N = 1024
    x = dev(workloads.chirped_gaussians(oracle.nodes(N), workloads.gaussian_params(4, np.random.default_rng(1))),
            torch.complex128)
    a = d = (z + 1 / z) / 2
    b = 1j * (z - 1 / z) / 2
    y = lct.lct_same_grid_exec(x, a, b, d).cpu().numpy() * np.sqrt(2 * np.pi / z)
    w = lct.frft(x, z).cpu().numpy()
    assert rel(y, w) <= 1e-12


def test_same_grid_shared_spectrum_and_errors():
    """With the workspace the kernel's spectrum is computed once for the batch; without it each
    signal transforms the kernel: same results to rounding.  Errors: no bounded form, b = 0."""
    N, B = 2048, 6
    a, b, d = MATRICES[0]
    x = dev(workloads.chirped_gaussians(oracle.nodes(N), workloads.gaussian_params(B, np.random.default_rng(3))),
            torch.complex64)
    y1 = lct.lct_same_grid_exec(x, a, b, d).cpu().numpy()
    y0 = torch.empty_like(x)
    rc = lct._lib.load().lct_same_grid_exec(N, lct.LCT_FP32, a.real, a.imag, b.real, b.imag, d.real, d.imag,
                                           x.data_ptr(), y0.data_ptr(), B, None, 0,
                                           torch.cuda.current_stream().cuda_stream)
    assert rc == lct.LCT_OK
    assert rel(y0.cpu().numpy(), y1) <= 1e-6
    with pytest.raises(lct.LctError):
        lct.lct_same_grid_exec(x, 0.5 - 0.3j, 1.0 + 0.2j, 0.8 + 0.4j)
    with pytest.raises(lct.LctError):
        lct.lct_same_grid_exec(x, 1.0, 0.0, 1.0)

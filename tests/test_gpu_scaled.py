"""GPU parity of plans on a scaled input grid s x_k (lct_plan_create_scaled):
the HIP path through the C ABI against the oracle's Riemann sum on the same
grid, element by element, FP32 (rel-L2 <= 2e-5) and FP64 (<= 1e-12)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_0912_1379_amd as lct

pytestmark = pytest.mark.gpu

TOL = {torch.complex64: 2e-5, torch.complex128: 1e-12}
PREC = {torch.complex64: lct.LCT_FP32, torch.complex128: lct.LCT_FP64}


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def inputs(N, s, seed):
    g = np.random.default_rng(seed)
    M = workloads.sl2_params(2, g)
    gp = workloads.gaussian_params(2, g)
    f = workloads.chirped_gaussians(s * oracle.nodes(N), gp)
    return M, gp, f


def peak_rows(M, gp, N, s, nrow, seed):
    """Rows where a chirped Gaussian's LCT has its energy (modulus of the Gaussian integral
    at the scaled output nodes, used only to choose rows) plus random rows."""
    a, b, c, d = M
    mu, sigma, kappa = gp
    A = 1 / (2 * sigma ** 2) - 1j * kappa - 1j * a / (2 * b)
    B = -mu / (2 * sigma ** 2) + 1j * oracle.output_nodes(N, b, d, scale=s) / (2 * b)
    top = np.argsort(-np.real(B * B / A))[: nrow // 2]
    rnd = np.random.default_rng(seed).choice(N, nrow - nrow // 2, replace=False)
    return np.unique(np.concatenate([top, rnd]))


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda").to(dtype)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("N", [1, 64, 1000, 4096, 6144, 65536])
@pytest.mark.parametrize("s", [0.45, 2.2])
def test_scaled_plan_matches_oracle(dtype, N, s):
    M, gp, f = inputs(N, s, 7000 + N)
    for i in range(2):
        rows = None if N <= 6144 else peak_rows(M[i], gp[i], N, s, 96, N + i)
        plan = lct.lct_plan_create(N, *M[i], precision=PREC[dtype], scale=s)
        x = dev(f[i], dtype)
        y = lct.lct_exec(plan, x).cpu().numpy().astype(np.complex128)
        fin = x.cpu().numpy().astype(np.complex128)
        ref = oracle.lct(fin, *M[i], rows=rows, scale=s)
        got = y if rows is None else y[rows]
        assert rel(got, ref) <= TOL[dtype], (N, s, M[i], rel(got, ref))


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_scaled_plan_b_zero(dtype):
    N, s = 1000, 1.7
    g = np.random.default_rng(3)
    f = g.standard_normal(N) + 1j * g.standard_normal(N)
    for (a, c) in [(2.0, 0.7), (-0.5, 1.2)]:
        M = (a, 0.0, c, 1.0 / a)
        plan = lct.lct_plan_create(N, *M, precision=PREC[dtype], scale=s)
        x = dev(f, dtype)
        y = lct.lct_exec(plan, x).cpu().numpy().astype(np.complex128)
        ref = oracle.lct(x.cpu().numpy().astype(np.complex128), *M, scale=s)
        assert rel(y, ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("N", [256, 4096])
def test_scaled_adjoint_inner_product(dtype, N):
    """<L_s f, g> (oracle forward on the scaled grid) equals <f, L_s^H g> (GPU adjoint)."""
    g = np.random.default_rng(N)
    f = g.standard_normal(N) + 1j * g.standard_normal(N)
    gg = g.standard_normal(N) + 1j * g.standard_normal(N)
    M = (0.8, -1.3, (0.8 * 0.4 - 1) / -1.3, 0.4)
    s = 1.9
    plan = lct.lct_plan_create(N, *M, precision=PREC[dtype], scale=s)
    fd, gd = dev(f, dtype), dev(gg, dtype)
    fin = fd.cpu().numpy().astype(np.complex128)
    gin = gd.cpu().numpy().astype(np.complex128)
    adj = lct.lct_exec_adjoint(plan, gd).cpu().numpy().astype(np.complex128)
    lhs = np.vdot(gin, oracle.lct(fin, *M, scale=s))
    rhs = np.vdot(adj, fin)
    assert abs(lhs - rhs) <= TOL[dtype] * np.linalg.norm(fin) * np.linalg.norm(adj) * 4


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("M1,M2", [((0.7, 1.3, 0.4), (0.6, 0.9, 1.1)), ((0.3, 2.0, 0.9), (0.8, -0.7, -0.4))])
def test_chain_without_resampling(dtype, M1, M2):
    """A transform reads the previous one's output as samples on s = 4 |b2| / pi (reversed when
    b2 < 0); the GPU chain matches the oracle's chain element by element."""
    N = 4096
    (a1, b1, d1), (a2, b2, d2) = M1, M2
    M1 = (a1, b1, (a1 * d1 - 1) / b1, d1)
    M2 = (a2, b2, (a2 * d2 - 1) / b2, d2)
    x = oracle.nodes(N)
    f = np.exp(-((0.5 + 0.3j) * x * x + 2 * (0.4 - 0.2j) * x + 0.1))
    sig = 4 * abs(b2) / np.pi
    p2 = lct.lct_plan_create(N, *M2, precision=PREC[dtype])
    p1 = lct.lct_plan_create(N, *M1, precision=PREC[dtype], scale=sig)
    fd = dev(f, dtype)
    G1 = lct.lct_exec(p2, fd)
    if b2 < 0:
        G1 = G1.flip(-1).contiguous()
    G = lct.lct_exec(p1, G1).cpu().numpy().astype(np.complex128)
    R1 = oracle.lct(fd.cpu().numpy().astype(np.complex128), *M2)
    if b2 < 0:
        R1 = R1[::-1]
    ref = oracle.lct(R1, *M1, scale=sig)
    assert rel(G, ref) <= 2 * TOL[dtype]
    _, y = lct.lct_nodes(N, b1, d1, scale=sig)
    assert np.allclose(y, oracle.output_nodes(N, b1, d1, scale=sig), rtol=1e-15, atol=1e-13)


def test_scaled_two_pass_2_20():
    N, s = 1 << 20, 0.8
    M, gp, f = inputs(N, s, 99)
    rows = peak_rows(M[0], gp[0], N, s, 48, 5)
    plan = lct.lct_plan_create(N, *M[0], precision=lct.LCT_FP32, scale=s)
    x = dev(f[0], torch.complex64)
    y = lct.lct_exec(plan, x).cpu().numpy().astype(np.complex128)
    ref = oracle.lct(x.cpu().numpy().astype(np.complex128), *M[0], rows=rows, scale=s)
    assert rel(y[rows], ref) <= 2e-5


def test_scaled_plan_rejects_frft():
    plan = lct.lct_plan_create(64, 1.0, 2.0, 0.5, 2.0, scale=2.0)
    x = torch.zeros(64, dtype=torch.complex64, device="cuda")
    with pytest.raises(lct.LctError):
        lct.frft_exec(plan, 0.5 + 0.2j, x)

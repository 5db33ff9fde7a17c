"""GPU parity of the exact-node discrete fractional transform of eq. (tmat):
xft_exec (two matrix-core passes through the C ABI) against the oracle's
sqrt(2 pi) U^T D(z) U f, element by element on the same seeded inputs sampled
at the zeros of H_N.

Bounds: relative L2 error per signal <= 1e-12 for FP64 and <= 2e-5 for FP32
(the bounds of the method's FP64 / FP32 variants); the FP32 path rounds U to
FP32 and accumulates N products in FP32, about 1e-6 here.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_0912_1379_amd as lct

pytestmark = pytest.mark.gpu

TOL = {torch.complex64: 2e-5, torch.complex128: 1e-12}
PREC = {torch.complex64: lct.LCT_FP32, torch.complex128: lct.LCT_FP64}
ZS = [0.7 * np.exp(0.9j), 1j, -1.0, 1.0, 0.3, -0.55 + 0.3j]


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel_rows(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda").to(dtype)


def inputs(N, batch, seed):
    g = np.random.default_rng(seed)
    gp = workloads.gaussian_params(batch, g)
    return workloads.chirped_gaussians(oracle.hermite_zeros(N), gp)


_PLANS = {}


def plan_of(N, dtype):
    key = (N, dtype)
    if key not in _PLANS:
        _PLANS[key] = lct.xft_plan_create(N, PREC[dtype])
    return _PLANS[key]


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("N,batch", [(1, 3), (2, 1), (3, 5), (17, 70), (100, 64), (128, 65), (257, 9),
                                     (1000, 33)])
def test_xft_matches_oracle(dtype, N, batch):
    print(f"[xft] N={N} batch={batch} {dtype}", flush=True)
    f = inputs(N, batch, 900 + N)
    x = dev(f, dtype)
    fin = x.cpu().numpy().astype(np.complex128)
    U = oracle.hermite_vectors(N)
    p = plan_of(N, dtype)
    for z in ZS:
        y = lct.xft_exec(p, z, x).cpu().numpy().astype(np.complex128)
        ref = oracle.xft(fin, z, U)
        e = rel_rows(y, ref)
        assert e.max() <= TOL[dtype], (N, batch, z, e.max())


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_xft_full_size_rows(dtype):
    """N = 4096 (the batched configuration's length), 96 signals, every output."""
    N, batch = 4096, 96
    print(f"[xft] N={N} batch={batch} {dtype}", flush=True)
    x = dev(inputs(N, batch, 77), dtype)
    fin = x.cpu().numpy().astype(np.complex128)
    U = oracle.hermite_vectors(N)
    p = plan_of(N, dtype)
    z = 0.8 * np.exp(-0.6j)
    y = lct.xft_exec(p, z, x).cpu().numpy().astype(np.complex128)
    e = rel_rows(y, oracle.xft(fin, z, U))
    assert e.max() <= TOL[dtype], e.max()


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_xft_eigenvectors(dtype):
    """Rows of U are eigenvectors: F_z U[n] = sqrt(2 pi) z^n U[n] (U from the oracle)."""
    N = 300
    U = oracle.hermite_vectors(N)
    rows = [0, 1, 2, 50, 151, 299]
    x = dev(U[rows].astype(np.complex128), dtype)
    z = np.exp(0.41j)
    y = lct.xft_exec(plan_of(N, dtype), z, x).cpu().numpy().astype(np.complex128)
    ref = np.stack([np.sqrt(2 * np.pi) * z ** n * U[n] for n in rows])
    assert rel_rows(y, ref).max() <= 4 * TOL[dtype]


@pytest.mark.parametrize("N,batch", [(1, 3), (3, 5), (17, 70), (100, 64), (257, 9), (1000, 33), (4096, 40)])
def test_xft_splitbf16_matches_oracle(N, batch):
    """Split-BF16 products (x = hi + lo, three BF16 matrix-core products, FP32 accumulation):
    the bound of the split-BF16 variant, 2e-4."""
    print(f"[xft-sb] N={N} batch={batch}", flush=True)
    x = dev(inputs(N, batch, 400 + N), torch.complex64)
    fin = x.cpu().numpy().astype(np.complex128)
    U = oracle.hermite_vectors(N)
    key = (N, "sb")
    if key not in _PLANS:
        _PLANS[key] = lct.xft_plan_create(N, lct.LCT_FP32_SPLITBF16)
    for z in [0.7 * np.exp(0.9j), -1.0, 0.3]:
        y = lct.xft_exec(_PLANS[key], z, x).cpu().numpy().astype(np.complex128)
        e = rel_rows(y, oracle.xft(fin, z, U))
        assert e.max() <= 2e-4, (N, batch, z, e.max())


@pytest.mark.parametrize("prec,tol", [(lct.LCT_FP32, 2e-5), (lct.LCT_FP32_SPLITBF16, 2e-4)])
def test_xft_large_eigenvectors(prec, tol):
    """N = 8192: rows of U (the library's host computation, itself pinned against the
    oracle at smaller N) are eigenvectors, F_z U[n] = sqrt(2 pi) z^n U[n]."""
    N = 8192
    print(f"[xft] N={N} prec={prec}", flush=True)
    U = lct.xft_vectors(N)
    rows = [0, 1, 2, 1000, 4095, 8191]
    x = dev(U[rows].astype(np.complex128), torch.complex64)
    z = np.exp(0.3j)  # |z| = 1: every eigenvalue has modulus sqrt(2 pi)
    p = lct.xft_plan_create(N, prec)
    y = lct.xft_exec(p, z, x).cpu().numpy().astype(np.complex128)
    ref = np.stack([np.sqrt(2 * np.pi) * z ** n * U[n] for n in rows])
    assert rel_rows(y, ref).max() <= tol
    p.destroy()


def test_xft_maximum_size_identities():
    """N = 16384, the largest plan: F_1 = sqrt(2 pi) I and, since the zeros are symmetric
    and phi_n has parity (-1)^n, F_{-1} f = sqrt(2 pi) f reversed."""
    N, B = 16384, 3
    print(f"[xft] N={N}", flush=True)
    x = dev(inputs(N, B, 11), torch.complex64)
    fin = x.cpu().numpy().astype(np.complex128)
    p = lct.xft_plan_create(N, lct.LCT_FP32)
    y1 = lct.xft_exec(p, 1.0, x).cpu().numpy().astype(np.complex128)
    ym = lct.xft_exec(p, -1.0, x).cpu().numpy().astype(np.complex128)
    s2 = np.sqrt(2 * np.pi)
    assert rel_rows(y1, s2 * fin).max() <= 2e-5
    assert rel_rows(ym, s2 * fin[:, ::-1]).max() <= 2e-5
    p.destroy()


def test_xft_in_place_and_errors():
    N, batch = 200, 7
    x = dev(inputs(N, batch, 5), torch.complex128)
    p = plan_of(N, torch.complex128)
    y = lct.xft_exec(p, 0.6j, x)
    x2 = x.clone()
    lct.xft_exec(p, 0.6j, x2, out=x2)
    assert torch.equal(x2, y)
    with pytest.raises(lct.LctError):
        lct.xft_exec(p, 1.2, x)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(lct.LctError):
        lct.xft_exec(p, 0.5, x, ws=small)
    with pytest.raises(TypeError):
        lct.xft_exec(p, 0.5, x.to(torch.complex64))
    empty = torch.empty(0, N, dtype=torch.complex128, device="cuda")
    assert lct.xft_exec(p, 0.5, empty).shape == (0, N)


def test_graph_capture_replays_match_eager():
    """xft_exec (weights kernel + two GEMM launches), the shared-order fractional
    transform (spectrum launch + main launch) and a scaled-grid LCT plan enqueue
    kernels only, with caller-owned workspaces: recorded into a HIP graph, every
    replay (with unrelated eager work and synchronisations in between) matches
    the eager result."""
    N, B = 1024, 9
    x = dev(inputs(N, B, 61), torch.complex64)
    px = plan_of(N, torch.complex64)
    wsx = torch.empty(lct.xft_workspace_size(N, lct.LCT_FP32, B), dtype=torch.uint8, device="cuda")
    pf = lct.lct_plan_create(N, 1.0, 0.0, 0.0, 1.0, precision=lct.LCT_FP32)
    wsf = torch.empty(lct.frft_workspace_size(N, lct.LCT_FP32, B), dtype=torch.uint8, device="cuda")
    ps = lct.lct_plan_create(N, 0.7, 1.3, (0.7 * 0.4 - 1) / 1.3, 0.4, precision=lct.LCT_FP32, scale=1.6)
    z = 0.8 * np.exp(-0.6j)
    eager = [lct.xft_exec(px, z, x, ws=wsx).clone(), lct.frft_exec(pf, z, x, ws=wsf).clone(),
             lct.lct_exec(ps, x).clone()]
    outs = [torch.empty_like(x) for _ in range(3)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up on the capture stream
        lct.xft_exec(px, z, x, out=outs[0], ws=wsx)
        lct.frft_exec(pf, z, x, out=outs[1], ws=wsf)
        lct.lct_exec(ps, x, out=outs[2])
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        lct.xft_exec(px, z, x, out=outs[0], ws=wsx)
        lct.frft_exec(pf, z, x, out=outs[1], ws=wsf)
        lct.lct_exec(ps, x, out=outs[2])
    for r in range(4):
        for o in outs:
            o.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()
        graph.replay()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        for o, e in zip(outs, eager):
            assert torch.equal(o, e), r

"""frft_exec_noalloc (the fractional transform of eqs. fasy, primcuad, cuadtrfor
with its workspace in the library's static device array) through the C ABI,
against frft_exec_ws with a caller workspace: two calls in a row, the second
with a smaller input, single-pass and two-pass lengths, FP32 and FP64."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_0912_1379_amd as lct

pytestmark = pytest.mark.gpu

TOL = {torch.complex64: 2e-5, torch.complex128: 1e-12}
SCRATCH = 64 << 20


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def inputs(N, B, seed, dtype):
    gp = workloads.gaussian_params(B, np.random.default_rng(seed))
    f = workloads.chirped_gaussians(oracle.nodes(N), gp)
    return torch.from_numpy(f).to("cuda").to(dtype)


def noalloc(plan, z, x):
    y = torch.full_like(x, float("nan"))
    rc = lct._lib.load().frft_exec_noalloc(plan.handle, float(np.real(z)), float(np.imag(z)), x.data_ptr(),
                                           y.data_ptr(), x.shape[0], torch.cuda.current_stream().cuda_stream)
    assert rc == lct.LCT_OK, lct.lct_strerror(rc)
    return y


def with_ws(plan, z, x, prec):
    ws = torch.full((lct.frft_workspace_size(x.shape[1], prec, x.shape[0]),), 255, dtype=torch.uint8,
                    device="cuda")
    return lct.frft_exec(plan, z, x, ws=ws)


@pytest.mark.parametrize("dtype,N1,B1,N2,B2", [
    (torch.complex64, 4096, 8, 1000, 3),      # single pass: the shared spectrum in the array
    (torch.complex64, 16384, 4, 16384, 2),    # two passes: data and kernel spectra per signal
    (torch.complex64, 65536, 3, 24576, 2),
    (torch.complex128, 8192, 4, 5120, 2),     # FP64 two passes
    (torch.complex128, 2048, 6, 64, 1),
])
def test_noalloc_matches_workspace_entry(dtype, N1, B1, N2, B2):
    prec = lct.LCT_FP64 if dtype == torch.complex128 else lct.LCT_FP32
    for k, (N, B, z) in enumerate(((N1, B1, 0.7 * np.exp(-0.9j)), (N2, B2, -0.6 + 0.35j))):
        print(f"[noalloc] call {k}: N={N} batch={B} {dtype} z={z}", flush=True)
        x = inputs(N, B, 100 * k + N, dtype)
        p = lct.lct_plan_create(N, 1.0, 1.0, 0.0, 1.0, precision=prec)
        got = noalloc(p, z, x).cpu().numpy().astype(np.complex128)
        ref = with_ws(p, z, x, prec).cpu().numpy().astype(np.complex128)
        for s in range(B):
            assert rel(got[s], ref[s]) <= TOL[dtype], (N, B, s)


def test_noalloc_rejects_batches_beyond_the_array():
    N = 65536
    p = lct.lct_plan_create(N, 1.0, 1.0, 0.0, 1.0)
    per = lct.frft_workspace_size(N, lct.LCT_FP32, 1)
    too_many = SCRATCH // per + 1
    lib = lct._lib.load()
    rc = lib.frft_exec_noalloc(p.handle, 0.5, 0.1, 8, 16, too_many, None)
    assert rc == lct.LCT_ERR_WORKSPACE
    rc = lib.frft_exec_noalloc(p.handle, 1.5, 0.1, 8, 16, 1, None)
    assert rc == lct.LCT_ERR_DOMAIN

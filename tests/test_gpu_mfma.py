"""Split-BF16 matrix-core variant (LCT_FP32_SPLITBF16): the radix-16 stages
as complex 16 x 16 DFT products on MFMA with x = hi + lo BF16 operands.
Parity against the FP64 oracle within the variant's bound of 2e-4 relative
L2 per signal (the bound stated for it at N = 4096, applied at every size).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_0912_1379_amd as lct
from test_gpu_lct import dev, peak_rows, rel_rows

pytestmark = pytest.mark.gpu

SPLIT_TOL = 2e-4
SPLIT = lct.LCT_FP32_SPLITBF16


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _case(N, batch, seed):
    g = np.random.default_rng(seed)
    M = workloads.sl2_params(batch, g)
    gp = workloads.gaussian_params(batch, g)
    f = workloads.chirped_gaussians(oracle.nodes(N), gp)
    return M, gp, f


@pytest.mark.parametrize("N", [256, 512, 1024, 2048, 4096, 8192, 16384, 1 << 15, 1 << 17, 1 << 20])
def test_split_bf16_matches_oracle(N):
    batch = 3 if N <= 1 << 17 else 2
    M, gp, f = _case(N, batch, 300 + N)
    x = dev(f, torch.complex64)
    M4 = dev(M, torch.float64)
    y = lct.lct_exec_many(x, M4, precision=SPLIT).cpu().numpy().astype(np.complex128)
    y32 = lct.lct_exec_many(x, M4).cpu().numpy().astype(np.complex128)
    fin = x.cpu().numpy().astype(np.complex128)
    for s in range(batch):
        rows = None if N <= 8192 else peak_rows(M[s], gp[s], N, 96, s)
        ref = oracle.lct(fin[s], *M[s], rows=rows)
        got = y[s] if rows is None else y[s][rows]
        e = rel_rows(got, ref)[0]
        assert e <= SPLIT_TOL, (N, s, e)
        # the matrix-core arithmetic is really a different one from the FP32 path
        other = y32[s] if rows is None else y32[s][rows]
        assert rel_rows(got, other)[0] > 1e-8, (N, s)


@pytest.mark.parametrize("N", [1024, 4096, 1 << 16])
def test_split_bf16_adjoint_and_plan(N):
    M, gp, f = _case(N, 2, 500 + N)
    x = dev(f, torch.complex64)
    M4 = dev(M, torch.float64)
    g32 = lct.lct_exec_many_adjoint(x, M4).cpu().numpy()
    gsp = lct.lct_exec_many_adjoint(x, M4, precision=SPLIT).cpu().numpy()
    assert rel_rows(gsp, g32).max() <= SPLIT_TOL
    plan = lct.Plan(N, *M[0], precision=SPLIT)
    yp = lct.lct_exec(plan, x[:1]).cpu().numpy()
    ym = lct.lct_exec_many(x[:1], M4[:1], precision=SPLIT).cpu().numpy()
    assert np.array_equal(yp, ym)  # same kernels, same arithmetic


def test_split_bf16_unsupported_requests():
    x = torch.zeros(2, 3000, dtype=torch.complex64, device="cuda")
    M4 = torch.tensor([[1.0, 1.0, 0.0, 1.0]] * 2, dtype=torch.float64, device="cuda")
    for n in (3000, 128):
        with pytest.raises(lct.LctError) as ei:
            lct.lct_exec_many(x[:, :n].contiguous(), M4, precision=SPLIT)
        assert ei.value.code == lct.LCT_ERR_UNSUPPORTED
    plan = lct.Plan(1024, 1.0, 1.0, 0.0, 1.0, precision=SPLIT)
    with pytest.raises(lct.LctError) as ei:
        lct.frft_exec(plan, 0.5, torch.zeros(1, 1024, dtype=torch.complex64, device="cuda"))
    assert ei.value.code == lct.LCT_ERR_UNSUPPORTED
    with pytest.raises(TypeError):
        lct.lct_exec_many(x.to(torch.complex128)[:, :1024].contiguous(), M4, precision=SPLIT)

"""Autotuner on the GPU: every candidate geometry the tuner can choose gives
the oracle's result to the precision's bound, and a tuned table entry is the
one the entry points then use.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_0912_1379_amd as lct
from test_gpu_lct import TOL, dev, frft_peak_rows, peak_rows, rel_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _clean_table():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lct.lct_tune_clear()
    yield
    lct.lct_tune_clear()


def _lct_case(N, dtype, batch=3):
    g = np.random.default_rng(700 + N)
    M = workloads.sl2_params(batch, g)
    gp = workloads.gaussian_params(batch, g)
    f = workloads.chirped_gaussians(oracle.nodes(N), gp)
    x = dev(f, dtype)
    M4 = dev(M, torch.float64)
    fin = x.cpu().numpy().astype(np.complex128)
    # beyond 8192 points: rows where the output has its energy plus random
    # rows (random rows alone can all fall in the tails, where the relative
    # error of a few rows measures only the floor of the arithmetic)
    rows = [None if N <= 8192 else peak_rows(M[s], gp[s], N, 96, s) for s in range(batch)]
    refs = [oracle.lct(fin[s], *M[s], rows=rows[s]) for s in range(batch)]
    return x, M4, rows, refs


def _frft_case(N, dtype, batch=2):
    g = np.random.default_rng(900 + N)
    gp = workloads.gaussian_params(batch, g)
    z = workloads.frft_orders(batch, g)
    f = workloads.chirped_gaussians(oracle.nodes(N), gp)
    x = dev(f, dtype)
    Z2 = dev(np.stack([z.real, z.imag], axis=1), torch.float64)
    fin = x.cpu().numpy().astype(np.complex128)
    rows = [None if N <= 4096 else frft_peak_rows(gp[s], z[s], N, 64, s) for s in range(batch)]
    refs = [oracle.frft(fin[s], z[s], rows=rows[s]) for s in range(batch)]
    return x, Z2, rows, refs


def _errors_lct(x, M4, rows, refs):
    y = lct.lct_exec_many(x, M4).cpu().numpy().astype(np.complex128)
    return [rel_rows(y[s] if rows[s] is None else y[s][rows[s]], refs[s])[0] for s in range(len(refs))]


def _errors_frft(x, Z2, rows, refs):
    y = lct.frft_exec_many(x, Z2).cpu().numpy().astype(np.complex128)
    return [rel_rows(y[s] if rows[s] is None else y[s][rows[s]], refs[s])[0] for s in range(len(refs))]


CASES = [
    (256, "lct", torch.complex64), (1024, "lct", torch.complex64), (4096, "lct", torch.complex64),
    (6000, "lct", torch.complex64), (4096, "lct", torch.complex128), (65536, "lct", torch.complex64),
    (3 * 2 ** 15, "lct", torch.complex128), (2048, "frft", torch.complex64), (12288, "frft", torch.complex64),
    (2048, "frft", torch.complex128),
]


@pytest.mark.parametrize("N,kind,dtype", CASES)
def test_every_candidate_matches_oracle(N, kind, dtype):
    prec = lct.LCT_FP64 if dtype == torch.complex128 else lct.LCT_FP32
    case = _lct_case(N, dtype) if kind == "lct" else _frft_case(N, dtype)
    run = _errors_lct if kind == "lct" else _errors_frft
    cands = lct.lct_tune_candidates(N, prec, kind)
    assert len(cands) >= 2
    bad = []
    for line in cands:
        lct.lct_tune_set(line)
        assert lct.lct_tune_get(N, prec, kind) == line
        err = max(run(*case))
        if not err <= TOL[dtype]:
            bad.append((line, err))
    assert not bad, bad


@pytest.mark.parametrize("N,kind,dtype", [(4096, "lct", torch.complex64), (1536, "frft", torch.complex64),
                                          (2 ** 17, "lct", torch.complex64)])
def test_autotune_records_a_candidate_and_keeps_parity(N, kind, dtype):
    prec = lct.LCT_FP64 if dtype == torch.complex128 else lct.LCT_FP32
    res = lct.lct_autotune(N, prec, kind, batch=64)
    print(res)
    assert res["config"] in lct.lct_tune_candidates(N, prec, kind)
    assert res["candidates"] == len(lct.lct_tune_candidates(N, prec, kind))
    assert res["best_us"] > 0 and res["default_us"] > 0 and res["best_us"] <= res["default_us"] * 1.000001
    assert lct.lct_tune_get(N, prec, kind) == res["config"]
    case = _lct_case(N, dtype) if kind == "lct" else _frft_case(N, dtype)
    errs = (_errors_lct if kind == "lct" else _errors_frft)(*case)
    assert max(errs) <= TOL[dtype], errs


def test_autotune_env_flags_tune_at_plan_creation_and_write_the_cache(tmp_path, monkeypatch):
    """LCT_AUTOTUNE=1: plan creation tunes both transforms of its length and
    precision; LCT_TUNE_CACHE: the table is written there and a cleared table
    reads it back; the tuned plan still matches the oracle."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("LCT_AUTOTUNE", "1")
    monkeypatch.setenv("LCT_TUNE_CACHE", str(cache))
    N = 2048
    plan = lct.lct_plan_create(N, 0.5, 1.0, -0.5, 1.0)
    try:
        text = cache.read_text()
        lines = [ln for ln in text.splitlines() if ln and not ln.startswith("#")]
        assert any(ln.startswith(f"lct N={N} prec=fp32 ") for ln in lines), text
        assert any(ln.startswith(f"frft N={N} prec=fp32 ") for ln in lines), text
        tuned = lct.lct_tune_get(N, lct.LCT_FP32, "lct")
        assert tuned in lines
        x = dev(workloads.chirped_gaussians(oracle.nodes(N), workloads.gaussian_params(1, np.random.default_rng(4))),
                torch.complex64)
        y = lct.lct_exec(plan, x).cpu().numpy().astype(np.complex128)
        ref = oracle.lct(x.cpu().numpy().astype(np.complex128)[0], 0.5, 1.0, -0.5, 1.0)
        assert rel_rows(y[0], ref)[0] <= TOL[torch.complex64]
    finally:
        lct.lct_plan_destroy(plan)
    # a second plan of the same length finds the entries and does not tune again
    mtime = cache.stat().st_mtime_ns
    lct.lct_plan_destroy(lct.lct_plan_create(N, 0.0, 1.0, -1.0, 0.0))
    assert cache.stat().st_mtime_ns == mtime
    monkeypatch.delenv("LCT_AUTOTUNE")
    lct.lct_tune_clear()
    monkeypatch.setenv("LCT_TUNE_CACHE", str(tmp_path / "other.txt"))  # missing file: heuristics
    heur = lct.lct_tune_get(N, lct.LCT_FP32, "lct")
    monkeypatch.setenv("LCT_TUNE_CACHE", str(cache))
    assert lct.lct_tune_get(N, lct.LCT_FP32, "lct") == tuned
    assert heur == lct.lct_tune_candidates(N, lct.LCT_FP32, "lct")[0]

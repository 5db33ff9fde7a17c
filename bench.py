"""Benchmark of the batched discrete LCT on one MI355X.

Workload (one step): 4096 signals x N = 4096 complex64 samples, one SL(2,R)
matrix per signal (a, d ~ U(-2,2), b = +-U(0.1,2), c = (ad-1)/b), inputs
chirped Gaussians exp(-(x-mu)^2/(2 sigma^2) + i kappa x^2) sampled on the
nodes x_k; one step is one lct_exec_many call over the whole batch (pre-chirp,
DFT and post-chirp in one kernel).  Inputs are resident in HBM before timing.

Prints one JSON line: throughput in complex samples/s, the HBM roofline of the
kernel (algorithmic bytes 16 B per sample over the kernel's average time from
HIP events), the FP64 path on the same workload, the relative L2 error against
the CPU oracle on sampled signals, and the oracle's own throughput on the
host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
METRIC = "complex samples/s, FP32 batched LCT N=4096 vs FP64 path; % HBM peak; rel-L2 err"
KERNEL_SOURCES = ["paper_0912_1379_amd/csrc/fft_core.hpp", "paper_0912_1379_amd/csrc/kernels_impl.hpp",
                  "paper_0912_1379_amd/csrc/lct_params.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lct_fp32_n4096_b4096_traffic.json")


def code_text(src: str) -> str:
    """C++ source without comments and whitespace (string and character
    literals kept): edits to comments or layout leave it unchanged."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
        elif c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            if not c.isspace():
                out.append(c)
            i += 1
    return "".join(out)


def kernel_hash() -> str:
    """Hash of the headline kernel's code (its three headers, comments and
    whitespace removed), recorded beside the traffic counters taken for it."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def mfma_flops(B: int, N: int) -> float:
    """Matrix-core flops of one split-BF16 launch: every radix-16 stage runs
    N / 256 groups of 16 butterflies per signal, six 16x16x32 MFMAs (2 x 16 x
    16 x 32 flops each) per group."""
    stages16 = 0
    n = N
    while n % 16 == 0 and n > 1:
        stages16 += 1
        n //= 16
    return float(B) * stages16 * (N // 256) * 6 * 2 * 16 * 16 * 32


def time_cold(fn, reps: int, flush_bytes: int = 1 << 30):
    """Launch time with a cold last-level cache: before each launch a
    reduction reads `flush_bytes` (default 1 GiB, four times the 256 MB
    memory-side cache), so no line of the inputs is left cached.  The touch
    reads rather than writes so that the cache holds clean lines: a written
    flush would leave dirty lines whose write-back the timed launch would pay.
    Event pair around the launch only.  Returns (mean ms, median ms)."""
    import torch

    flush = torch.ones(flush_bytes // 4, dtype=torch.float32, device="cuda")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    fn()
    for a, b in ev:
        flush.sum()
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in ev])
    del flush
    return float(t.mean()), float(np.median(t))


def make_inputs(B: int, N: int, seed_index: int = 1):
    import workloads
    import paper_0912_1379_amd as lct

    x_nodes, _ = lct.lct_nodes(N, 1.0)
    g = workloads.rng(seed_index)
    M = workloads.sl2_params(B, g)
    gp = workloads.gaussian_params(B, g)
    f = workloads.chirped_gaussians(x_nodes, gp)
    return M, f


def time_launches(fn, steps: int, warmup: int):
    """Times `steps` calls on the current stream (the stream the library
    launches on) between two HIP events, with nothing else in the timed
    region.  Returns (ms per step, the same figure as the average duration of
    the step's launches -- a step is one library call, whose kernels run back
    to back on that stream --, wall seconds of the timed region)."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop) / steps
    return ms, ms, wall


def time_event_pairs(fn, steps: int) -> float:
    """Mean ms of an event pair recorded around each of `steps` calls (a second
    view of the launch duration; the events themselves add a little)."""
    import torch

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in ev) / steps


def cpu_baseline(xh: np.ndarray, M: np.ndarray, outs: dict, budget_s: float):
    """Oracle on a bounded sample of the same workload: whole signals (dense
    O(N^2) Riemann sums), as many as fit the time budget (at least 2).  Also
    returns, per signal of the sample, the relative L2 error of every GPU
    result in `outs` (name -> complex128 array of the batch's outputs)."""
    import oracle

    N = xh.shape[1]
    done = 0
    errs = {k: [] for k in outs}
    t0 = time.perf_counter()
    while done < xh.shape[0] and (done < 2 or time.perf_counter() - t0 < budget_s):
        ref = oracle.lct(xh[done].astype(np.complex128), *M[done])
        for k, y in outs.items():
            if done < len(y):  # a result may hold only the batch's first rows
                errs[k].append(float(np.linalg.norm(y[done] - ref) / np.linalg.norm(ref)))
        done += 1
    el = time.perf_counter() - t0
    return {
        "value": done * N / el,
        "unit": "complex samples/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{done} of the {xh.shape[0]} signals (N={N}, full dense Riemann sums), {el:.1f} s",
        "single_thread": oracle_single_thread(lambda: oracle.lct(xh[0].astype(np.complex128), *M[0]), N,
                                              f"signal 0 (N={N}, full dense Riemann sum)"),
    }, errs


def oracle_single_thread(fn, samples: int, what: str) -> dict:
    """The same oracle call on one thread: complex samples/s and what was timed."""
    import oracle

    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        fn()
        el = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(threads)
    return {"value": samples / el, "unit": "complex samples/s", "cores": 1, "sample": f"{what}, {el:.1f} s"}


def lct_energy_rows(M, gp, N, nrow, seed):
    """Rows where a chirped Gaussian's LCT has its energy (from the Gaussian
    integral's modulus; it only picks rows) plus random rows."""
    a, b, c, d = M
    mu, sigma, kappa = gp
    al = 1 / (2 * sigma ** 2) - 1j * kappa
    be = -mu / (2 * sigma ** 2)
    if b == 0.0:
        return np.random.default_rng(seed).choice(N, min(N, nrow), replace=False)
    yn = 4.0 * b * oracle_nodes(N) / np.pi
    logmag = np.real((be + 1j * yn / (2 * b)) ** 2 / (al - 1j * a / (2 * b)))
    top = np.argsort(-logmag)[: nrow // 2]
    rnd = np.random.default_rng(seed).choice(N, nrow - nrow // 2, replace=False)
    return np.unique(np.concatenate([top, rnd]))


def frft_energy_rows(gp, z, N, nrow, seed):
    """Rows where a chirped Gaussian's same-grid fractional transform has its
    energy (Gaussian integral of eq. fasy's kernel) plus random rows."""
    mu, sigma, kappa = gp
    al = 1 / (2 * sigma ** 2) - 1j * kappa
    be = -mu / (2 * sigma ** 2)
    y = oracle_nodes(N)
    if abs(1 - z * z) < 1e-12:
        logmag = np.real(-(al * y * y + 2 * be * y))
    else:
        A = (1 + z * z) / (2 * (1 - z * z)) + al
        B = y * z / (1 - z * z) - be
        logmag = np.real(B * B / A - (1 + z * z) * y * y / (2 * (1 - z * z)))
    top = np.argsort(-logmag)[: nrow // 2]
    rnd = np.random.default_rng(seed).choice(N, nrow - nrow // 2, replace=False)
    return np.unique(np.concatenate([top, rnd]))


def oracle_nodes(N):
    import oracle

    return oracle.nodes(N)


def bench_ragged(args):
    """Uneven batch in one persistent launch: 10,000 signals, N log-uniform on
    [256, 65536] snapped to {2^k, 3 2^k, 5 2^k}, half LCTs (one matrix each),
    half fractional transforms (one order each), FP32."""
    import torch
    import workloads
    import paper_0912_1379_amd as lct

    count = args.signals if args.signals != 4096 else 10000
    g = workloads.rng(2)
    N = workloads.ragged_sizes(count, g)
    kinds = np.where(np.arange(count) % 2 == 0, lct.LCT_KIND_LCT, lct.LCT_KIND_FRFT)
    M = workloads.sl2_params(count, g)
    z = workloads.frft_orders(count, g)
    gp = workloads.gaussian_params(count, g)
    params = np.where(kinds[:, None] == lct.LCT_KIND_LCT, M, np.stack([z.real, z.imag, 0 * z.real, 0 * z.real], 1))
    if args.ragged_subset != "all":
        # one part of the same batch (per-kind timings and counters): the long signals are those
        # beyond one work-group's registers (LCT N > 6144, fractional 2N > 6144)
        is_lct = kinds == lct.LCT_KIND_LCT
        big = np.where(is_lct, N > 6144, 2 * N > 6144)
        sel = {"lct": is_lct, "frft": ~is_lct, "lct_big": is_lct & big, "frft_big": ~is_lct & big,
               "small": ~big}[args.ragged_subset]
        N, kinds, params, gp = N[sel], kinds[sel], params[sel], gp[sel]
        count = int(sel.sum())
    desc = lct.make_descriptors(N, kinds, params)
    parts = []
    for i, n in enumerate(N):
        xn, _ = lct.lct_nodes(int(n), 1.0)
        parts.append(workloads.chirped_gaussians(xn, gp[i:i + 1])[0].astype(np.complex64))
    x = torch.from_numpy(np.concatenate(parts)).to("cuda")
    plan = lct.RaggedPlan(desc)
    y = torch.empty_like(x)
    ms, ms_kernel, wall = time_launches(lambda: lct.lct_exec_ragged(plan, x, out=y), args.steps, args.warmup)
    samples = int(N.sum())
    gbps = 16.0 * samples / (ms_kernel * 1e-3) / 1e9
    errors = None if args.no_cpu_baseline else ragged_errors(x, y, desc, kinds, N, params, gp, lct)
    out = {
        "metric": "complex samples/s, ragged batch in one persistent launch",
        "value": samples / (ms * 1e-3), "unit": "complex samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"ragged: {count} signals, N in [256, 65536] (2^k, 3 2^k, 5 2^k), half LCT half "
                               "fractional transform, one persistent launch", "signals": count, "samples": samples,
                   "items": plan.items, "grid": plan.grid, "subset": args.ragged_subset},
        "roofline": {"bound": "hbm", "achieved": gbps, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": gbps / PEAK_HBM_GBPS, "traffic": None, "kernel": "k_ragged", "kernel_ms": ms_kernel,
                     "algorithmic_bytes_per_launch": 16.0 * samples},
        "wall_s_timed": wall,
    }
    if errors is not None:
        out["rel_l2"], out["cpu_baseline"] = errors
    return out


def ragged_errors(x, y, desc, kinds, N, params, gp, lct):
    """Relative L2 error of the ragged launch against the oracle on a seeded
    sample: two signals per (kind, length band), short (in LDS), middle and long
    (four-step inside one work-group); every output up to N = 4096, else 128
    rows (energy rows plus random rows).  Also the oracle's rate on them."""
    import oracle

    xh = x.cpu().numpy()
    yh = y.cpu().numpy()
    gs = np.random.default_rng(1379)
    pick = []
    for kind in (lct.LCT_KIND_LCT, lct.LCT_KIND_FRFT):
        for lo, hi in ((256, 2048), (2049, 16384), (16385, 65536)):
            cand = np.flatnonzero((kinds == kind) & (N >= lo) & (N <= hi))
            if cand.size:
                pick.extend(int(i) for i in gs.choice(cand, min(2, cand.size), replace=False))
    errs = {"lct": [], "frft": []}
    worst = {"lct": None, "frft": None}
    done = 0
    t0 = time.perf_counter()
    for i in pick:
        n, o = int(N[i]), int(desc["offset"][i])
        fin = xh[o:o + n].astype(np.complex128)
        got = yh[o:o + n].astype(np.complex128)
        name = "lct" if kinds[i] == lct.LCT_KIND_LCT else "frft"
        if name == "lct":
            rows = None if n <= 4096 else lct_energy_rows(params[i], gp[i], n, 128, i)
            ref = oracle.lct(fin, *params[i], rows=rows)
        else:
            z = complex(params[i][0], params[i][1])
            rows = None if n <= 4096 else frft_energy_rows(gp[i], z, n, 128, i)
            ref = oracle.frft(fin, z, rows=rows)
        g = got if rows is None else got[rows]
        e = float(np.linalg.norm(g - ref) / np.linalg.norm(ref))
        errs[name].append(e)
        if worst[name] is None or e > worst[name][0]:
            worst[name] = (e, n)
        done += n * (n if rows is None else len(rows))
    el = time.perf_counter() - t0
    rel = {k: {"max": max(v), "median": float(np.median(v)), "signals": len(v), "worst_N": worst[k][1]}
           for k, v in errs.items() if v}
    rel["rows"] = "every output up to N = 4096, else 128 rows (64 where the output has its energy, 64 random)"
    # the oracle's rate on the whole batch, from its measured multiply-add rate:
    # a dense transform of length n costs n^2 of them
    mac_rate = done / el
    whole = float(np.sum(N.astype(np.float64) ** 2)) / mac_rate
    cb = {"value": float(N.sum()) / whole, "unit": "complex samples/s", "cores": oracle.num_threads(),
          "kind": "oracle",
          "sample": f"{len(pick)} signals of the batch (2 per kind and length band; {done:.3g} multiply-adds "
                    f"in {el:.1f} s), scaled to the whole batch's sum of N^2 ({whole:.0f} s)"}
    return rel, cb


def bench_large(args):
    """16 signals x N = 2^20: FP32 and FP64 two-pass paths, chirped Gaussians
    plus white complex noise (std 1e-3)."""
    import torch
    import workloads
    import paper_0912_1379_amd as lct

    B, N = 16, 1 << 20
    g = workloads.rng(3)
    M = workloads.sl2_params(B, g)
    gp = workloads.gaussian_params(B, g)
    xn, _ = lct.lct_nodes(N, 1.0)
    f = workloads.chirped_gaussians(xn, gp) + workloads.white_noise((B, N), g)
    x32 = torch.from_numpy(f).to("cuda").to(torch.complex64)
    x64 = x32.to(torch.complex128)
    M4 = torch.from_numpy(M).to("cuda")
    y32, y64 = torch.empty_like(x32), torch.empty_like(x64)
    tuning = None
    if not args.no_tune:
        tuning = {"fp32": lct.lct_autotune(N, lct.LCT_FP32, "lct", batch=B),
                  "fp64": lct.lct_autotune(N, lct.LCT_FP64, "lct", batch=B)}
        print(f"[bench] tuned: {tuning}", file=sys.stderr, flush=True)
    ms, ms_kernel, wall = time_launches(lambda: lct.lct_exec_many(x32, M4, out=y32), args.steps, args.warmup)
    ms64, ms64_kernel, _ = time_launches(lambda: lct.lct_exec_many(x64, M4, out=y64), max(5, args.steps // 2), 2)
    ysp = torch.empty_like(x32)
    mss, mss_kernel, _ = time_launches(lambda: lct.lct_exec_many(x32, M4, out=ysp, precision=lct.LCT_FP32_SPLITBF16),
                                       max(5, args.steps // 2), 2)
    samples = B * N
    gbps = 16.0 * samples / (ms_kernel * 1e-3) / 1e9
    out = {
        "metric": "complex samples/s, batched LCT N=2^20 (two-pass)",
        "value": samples / (ms * 1e-3), "unit": "complex samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "16 signals x N=2^20, chirped Gaussians + 1e-3 white noise, one matrix per signal",
                   "signals": B, "N": N},
        "roofline": {"bound": "hbm", "achieved": gbps, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": gbps / PEAK_HBM_GBPS, "traffic": None, "kernel": "k_fs1+k_fs2",
                     "kernel_ms": ms_kernel, "algorithmic_bytes_per_launch": 16.0 * samples,
                     "actual_bytes_per_launch_two_pass": 32.0 * samples},
        "wall_s_timed": wall,
        "fp64_path": {"ms_per_step": ms64, "kernel_ms": ms64_kernel, "fp32_speedup": ms64 / ms},
        "splitbf16_path": {"ms_per_step": mss, "kernel_ms": mss_kernel},
        "tuning": tuning,
        "geometry": {"fp32": lct.lct_tune_get(N, lct.LCT_FP32, "lct"), "fp64": lct.lct_tune_get(N, lct.LCT_FP64, "lct")},
    }
    if not args.no_cpu_baseline:
        import oracle

        def energy_rows(s, nrow=64):
            return lct_energy_rows(M[s], gp[s], N, nrow, 4 + s)
        errs32, errs64, errsp = [], [], []
        t0 = time.perf_counter()
        for s in range(2):
            rows = energy_rows(s)
            fin = x32[s].cpu().numpy().astype(np.complex128)
            ref = oracle.lct(fin, *M[s], rows=rows)
            errs32.append(float(np.linalg.norm(y32[s].cpu().numpy()[rows] - ref) / np.linalg.norm(ref)))
            errsp.append(float(np.linalg.norm(ysp[s].cpu().numpy()[rows] - ref) / np.linalg.norm(ref)))
            ref64 = oracle.lct(x64[s].cpu().numpy(), *M[s], rows=rows)
            errs64.append(float(np.linalg.norm(y64[s].cpu().numpy()[rows] - ref64) / np.linalg.norm(ref64)))
        el = time.perf_counter() - t0
        out["rel_l2_sampled"] = {"fp32_max": max(errs32), "fp64_max": max(errs64), "splitbf16_max": max(errsp),
                                 "rows": "64 per signal (32 where the output has its energy, 32 random)",
                                 "signals": 2}
        out["cpu_baseline"] = {"value": 2 * 2 * 64 / el, "unit": "output samples/s (dense rows of 2^20 terms)",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"2 signals x 64 rows, FP32 and FP64 inputs, {el:.1f} s"}
    return out


def bench_frft(args):
    """Batched same-grid fractional transform: 4096 signals x N = 4096
    complex64, one order z = r e^{-i theta} per signal (r ~ U(0.5, 1)),
    chirped-Gaussian inputs; one step = one frft_exec_many call (length-8192
    convolution in LDS per signal)."""
    import torch
    import workloads
    import paper_0912_1379_amd as lct

    B, N = args.signals, args.N
    g = workloads.rng(2, 1)
    z = workloads.frft_orders(B, g)
    gp = workloads.gaussian_params(B, g)
    xn, _ = lct.lct_nodes(N, 1.0)
    x = torch.from_numpy(workloads.chirped_gaussians(xn, gp)).to("cuda").to(torch.complex64)
    Z2 = torch.from_numpy(np.stack([z.real, z.imag], axis=1)).to("cuda")
    y = torch.empty_like(x)
    tuning = None if args.no_tune else lct.lct_autotune(N, lct.LCT_FP32, "frft", batch=B)
    ms, ms_kernel, wall = time_launches(lambda: lct.frft_exec_many(x, Z2, out=y), args.steps, args.warmup)
    samples = B * N
    gbps = 16.0 * samples / (ms_kernel * 1e-3) / 1e9
    out = {
        "metric": "complex samples/s, batched same-grid fractional transform",
        "value": samples / (ms * 1e-3), "unit": "complex samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"fractional transform, {B} signals x N={N} complex64, one order per signal",
                   "signals": B, "N": N, "geometry": lct.lct_tune_get(N, lct.LCT_FP32, "frft")},
        "roofline": {"bound": "hbm", "achieved": gbps, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": gbps / PEAK_HBM_GBPS, "traffic": None, "kernel": "k_frft (FP32)",
                     "kernel_ms": ms_kernel, "algorithmic_bytes_per_launch": 16.0 * samples},
        "wall_s_timed": wall, "tuning": tuning,
    }
    # one order for the whole batch (plan path): the kernel's spectrum is
    # computed once per call and shared, two length-2N FFTs per signal
    if args.no_shared:
        if not args.no_cpu_baseline:
            frft_errors(out, x, y, None, z, N, gp)
        return out
    z0 = complex(z[0])
    plan = lct.lct_plan_create(N, 1.0, 0.0, 0.0, 1.0, precision=lct.LCT_FP32)
    ws = torch.empty(lct.frft_workspace_size(N, lct.LCT_FP32, B), dtype=torch.uint8, device="cuda")
    ysh = torch.empty_like(x)
    ms_sh, ms_sh_kernel, _ = time_launches(lambda: lct.frft_exec(plan, z0, x, out=ysh, ws=ws), args.steps,
                                           args.warmup)
    out["shared_order"] = {"ms_per_step": ms_sh, "value": samples / (ms_sh * 1e-3), "kernel_ms": ms_sh_kernel,
                           "achieved_GBps": 16.0 * samples / (ms_sh_kernel * 1e-3) / 1e9,
                           "speedup_vs_per_signal_order": ms / ms_sh,
                           "what": "frft_exec with one order for all signals: spectrum launch + main launch"}
    print(f"[bench] frft per-signal order {ms * 1e3:.1f} us, shared order {ms_sh * 1e3:.1f} us",
          file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        frft_errors(out, x, y, ysh, z, N, gp)
    return out


def frft_errors(out, x, y, ysh, z, N, gp):
    """Relative L2 errors against the oracle (3 signals of the per-signal-order
    output, 2 of the shared-order one) and the oracle's own rate.  Up to
    N = 8192 every output of those signals; beyond, 128 rows each (64 where the
    output has its energy, 64 random), so that the dense sums stay within
    seconds."""
    import oracle

    def rows_of(s, zz):
        return None if N <= 8192 else frft_energy_rows(gp[s], zz, N, 128, s)

    errs = []
    done = 0
    t0 = time.perf_counter()
    for s in range(3):
        fin = x[s].cpu().numpy().astype(np.complex128)
        rows = rows_of(s, complex(z[s]))
        ref = oracle.frft(fin, complex(z[s]), rows=rows)
        got = y[s].cpu().numpy()
        got = got if rows is None else got[rows]
        errs.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
        done += N if rows is None else len(rows)
    el = time.perf_counter() - t0
    out["rel_l2"] = {"max": max(errs), "signals": 3}
    if N <= 8192:
        out["cpu_baseline"] = {"value": 3 * N / el, "unit": "complex samples/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"3 whole signals (dense N={N} sums), {el:.1f} s"}
    else:
        out["rel_l2"]["rows"] = "128 per signal (64 where the output has its energy, 64 random)"
        out["cpu_baseline"] = {"value": done / el, "unit": f"output samples/s (dense rows of {N} terms)",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"3 signals x 128 rows, {el:.1f} s"}
    if ysh is not None:
        esh = []
        for s in range(2):
            rows = rows_of(s, complex(z[0]))
            ref = oracle.frft(x[s].cpu().numpy().astype(np.complex128), complex(z[0]), rows=rows)
            got = ysh[s].cpu().numpy()
            got = got if rows is None else got[rows]
            esh.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
        out["shared_order"]["rel_l2_max"] = max(esh)


def bench_next(args):
    """The widened entry points on 4096 signals x N = 4096 chirped Gaussians, FP32 steps with FP64
    legs: the same-grid LCT of a damped complex matrix (lct_same_grid_exec, one length-2N
    convolution per signal with the kernel's spectrum computed once), the LCT at the Algorithm's
    complex output nodes (lct_complex_exec) for the bilateral Laplace matrix (0, i, 0), and the
    aliasing-aware LCT (lct_exec_oversampled: interpolation onto the P times finer grid, the
    transform there, the middle block; P = 4 in FP32, 2 in FP64), and the LCT of samples on the scaled
    input grid s x_k (lct_plan_create_scaled, s = 1/2).  The step is the complex-node LCT; each leg
    reports its time, rate, the relative L2 error of 2 signals against the oracle and the oracle's
    time on them."""
    import torch
    import workloads
    import paper_0912_1379_amd as lct
    import oracle

    B, N = args.signals, args.N
    g = workloads.rng(6)
    gp = workloads.gaussian_params(B, g)
    xn, _ = lct.lct_nodes(N, 1.0)
    f = workloads.chirped_gaussians(xn, gp)
    samples = B * N
    legs = {}
    cpu = {"seconds": 0.0, "samples": 0}

    def leg(name, dt, run, ref_fn, nref=2, data=None):
        x = torch.from_numpy(f if data is None else data).to("cuda").to(dt)
        y = torch.empty_like(x)
        steps = args.steps if dt == torch.complex64 else max(3, args.steps // 2)
        ms, ms_kernel, wall = time_launches(lambda: run(x, y), steps, args.warmup)
        out = {"ms_per_step": ms, "kernel_ms": ms_kernel, "value": samples / (ms * 1e-3),
               "achieved_GBps": (16.0 if dt == torch.complex64 else 32.0) * samples / (ms_kernel * 1e-3) / 1e9}
        if not args.no_cpu_baseline:
            errs = []
            t0 = time.perf_counter()
            for s in range(nref):
                fin = x[s].cpu().numpy().astype(np.complex128)
                ref = ref_fn(fin)
                errs.append(float(np.linalg.norm(y[s].cpu().numpy() - ref) / np.linalg.norm(ref)))
            el = time.perf_counter() - t0
            cpu["seconds"] += el
            cpu["samples"] += nref * N
            out["rel_l2"] = {"max": max(errs), "signals": nref}
        print(f"[bench] {name}: {ms * 1e3:.1f} us/step", file=sys.stderr, flush=True)
        legs[name] = out
        return out

    # complex output nodes, bilateral Laplace (0, i, 0)
    for name, dt in (("complex_nodes_f32", torch.complex64), ("complex_nodes_f64", torch.complex128)):
        if dt == torch.complex128 and args.no_fp64:
            continue
        leg(name, dt, lambda x, y: lct.lct_complex_exec(x, 0.0, 1j, 0.0, out=y),
            lambda fin: oracle.lct_complex(fin, 0.0, 1j, 0.0))
    # same grid, a damped matrix (Toeplitz form)
    a, b, d = 0.9 + 0.1j, 0.6 - 0.2j, 1.1 + 0.05j
    for name, dt in (("same_grid_f32", torch.complex64), ("same_grid_f64", torch.complex128)):
        if dt == torch.complex128 and args.no_fp64:
            continue
        prec = lct.LCT_FP64 if dt == torch.complex128 else lct.LCT_FP32
        ws = torch.empty(lct.frft_workspace_size(N, prec, B), dtype=torch.uint8, device="cuda")
        leg(name, dt, lambda x, y: lct.lct_same_grid_exec(x, a, b, d, out=y, ws=ws),
            lambda fin: oracle.lct_same_grid(fin, a, b, d))
    # aliasing-aware mode on a matrix whose pre-chirp aliases on the plain grid (a/b = 16): P = 4 in
    # FP32 (16384-point fine grid), P = 2 in FP64 (8192, the longest FP64 single pass)
    M = (8.0, 0.5, (8.0 * 0.3 - 1.0) / 0.5, 0.3)
    for name, dt, p in (("oversampled_f32", torch.complex64, 4), ("oversampled_f64", torch.complex128, 2)):
        if dt == torch.complex128 and args.no_fp64:
            continue
        prec = lct.LCT_FP64 if dt == torch.complex128 else lct.LCT_FP32
        plan = lct.lct_plan_create(N, *M, precision=prec)
        ws = torch.empty(lct.lct_oversampled_workspace_size(N, p, prec, B), dtype=torch.uint8, device="cuda")
        leg(name, dt, lambda x, y: lct.lct_exec_oversampled(plan, p, x, out=y, ws=ws),
            lambda fin: oracle.lct_oversampled(fin, *M, p))
        legs[name]["P"] = p
    # scaled input grid: samples on s x_k, outputs at 4 b x_j / (pi s)
    sc = 0.5
    Ms = (0.6, 0.8, (0.6 * 1.1 - 1.0) / 0.8, 1.1)
    fs = workloads.chirped_gaussians(sc * xn, gp)
    for name, dt in (("scaled_f32", torch.complex64), ("scaled_f64", torch.complex128)):
        if dt == torch.complex128 and args.no_fp64:
            continue
        prec = lct.LCT_FP64 if dt == torch.complex128 else lct.LCT_FP32
        plan = lct.lct_plan_create_scaled(N, *Ms, sc, precision=prec)
        leg(name, dt, lambda x, y: lct.lct_exec(plan, x, out=y), lambda fin: oracle.lct(fin, *Ms, scale=sc),
            data=fs)
        legs[name]["s"] = sc
    head = legs["complex_nodes_f32"]
    out = {
        "metric": "complex samples/s, LCT of a complex matrix at the Algorithm's complex output nodes",
        "value": head["value"], "unit": "complex samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"complex-matrix, same-grid, oversampled and scaled-grid LCTs, {B} signals x N={N}",
                   "signals": B, "N": N, "complex_matrix": "(0, i, 0): bilateral Laplace",
                   "same_grid_matrix": [str(a), str(b), str(d)],
                   "oversampled": {"M": list(M), "P": {"f32": 4, "f64": 2}},
                   "scaled": {"M": list(Ms), "s": sc}},
        "roofline": {"bound": "hbm", "achieved": head["achieved_GBps"], "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": head["achieved_GBps"] / PEAK_HBM_GBPS, "traffic": None, "kernel": "k_lct_cx (FP32)",
                     "kernel_ms": head["kernel_ms"], "algorithmic_bytes_per_launch": 16.0 * samples},
        "legs": legs,
    }
    if not args.no_cpu_baseline:
        out["rel_l2"] = head["rel_l2"]
        out["cpu_baseline"] = {"value": cpu["samples"] / cpu["seconds"], "unit": "complex samples/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"2 whole signals per leg (dense N={N} sums; the oversampled legs on the "
                                         f"finer grid), {cpu['seconds']:.1f} s in all"}
    return out


PEAK_MFMA_TFLOPS = {"f32": 157.3, "f64": 78.6}


def bench_xft(args):
    """Exact-node discrete fractional transform of eq. (tmat) on the matrix
    cores: 4096 signals x N = 4096 sampled at the zeros of H_N, one order z
    for the batch; FP32 (the step) and FP64 legs.  One call = a weights
    kernel and two GEMM passes, 8 B N^2 flops."""
    import torch
    import workloads
    import paper_0912_1379_amd as lct

    B, N = args.signals, args.N
    g = workloads.rng(5)
    gp = workloads.gaussian_params(B, g)
    xe = lct.xft_nodes(N)
    f = workloads.chirped_gaussians(xe, gp)
    z = 0.8 * np.exp(-0.6j)
    flops = 8.0 * B * N * N
    legs = {}
    outs = {}
    for name, prec, dt in [("f32", lct.LCT_FP32, torch.complex64), ("f64", lct.LCT_FP64, torch.complex128),
                           ("splitbf16", lct.LCT_FP32_SPLITBF16, torch.complex64)]:
        if (name == "f64" and args.no_fp64) or (name == "splitbf16" and args.no_split):
            continue
        plan = lct.xft_plan_create(N, prec)
        x = torch.from_numpy(f).to("cuda").to(dt)
        y = torch.empty_like(x)
        ws = torch.empty(lct.xft_workspace_size(N, prec, B), dtype=torch.uint8, device="cuda")
        steps = args.steps if name == "f32" else max(3, args.steps // 2)
        ms, ms_kernel, wall = time_launches(lambda: lct.xft_exec(plan, z, x, out=y, ws=ws), steps, args.warmup)
        tf = flops / (ms_kernel * 1e-3) / 1e12
        legs[name] = {"ms_per_step": ms, "kernel_ms": ms_kernel, "TFLOPs": tf, "steps": steps, "wall_s_timed": wall}
        if name in PEAK_MFMA_TFLOPS:
            legs[name]["frac"] = tf / PEAK_MFMA_TFLOPS[name]
        else:
            # three BF16 products per term: matrix-core rate against the 2.5 PFLOP/s BF16 peak
            legs[name]["bf16_TFLOPs"] = 3 * tf
            legs[name]["frac_of_bf16_peak"] = 3 * tf / 2500.0
        outs[name] = (x, y)
        print(f"[bench] xft {name}: {ms:.3f} ms/step, {tf:.1f} TFLOP/s", file=sys.stderr, flush=True)
    main = legs["f32"]
    out = {
        "metric": "complex samples/s, exact-node discrete fractional transform (eq. tmat) on the matrix cores",
        "value": B * N / (main["ms_per_step"] * 1e-3), "unit": "complex samples/s", "n_gpus": 1,
        "steps": main["steps"], "warmup": args.warmup, "ms_per_step": main["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"exact-node transform, {B} signals x N={N} complex64 at the zeros of H_N, "
                               "one order z for the batch", "signals": B, "N": N},
        "roofline": {"bound": "mfma", "achieved": main["TFLOPs"], "peak": PEAK_MFMA_TFLOPS["f32"], "unit": "TFLOP/s",
                     "frac": main["frac"], "traffic": None,
                     "kernel": "k_xft_gemm<float> x 2 (+ k_xft_weights)", "kernel_ms": main["kernel_ms"],
                     "algorithmic_flops_per_call": flops},
        "wall_s_timed": main["wall_s_timed"], "fp64_path": legs.get("f64"), "splitbf16_path": legs.get("splitbf16"),
    }
    if not args.no_cpu_baseline:
        import oracle

        t0 = time.perf_counter()
        U = oracle.hermite_vectors(N)
        nb = 64
        ref = oracle.xft(f[:nb], z, U)
        el = time.perf_counter() - t0
        errs = {}
        for name, (x, y) in outs.items():
            fin = x[:nb].cpu().numpy().astype(np.complex128)
            r = oracle.xft(fin, z, U)
            got = y[:nb].cpu().numpy().astype(np.complex128)
            errs[name] = float((np.linalg.norm(got - r, axis=1) / np.linalg.norm(r, axis=1)).max())
        out["rel_l2"] = errs
        out["cpu_baseline"] = {"value": nb * N / el, "unit": "complex samples/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"{nb} of the {B} signals (U of eq. ortvec in long "
                                                           f"double, then numpy products), {el:.1f} s"}
        del ref
    return out


def bench_fit(args):
    """Differentiable LCT fit: 256 signals x N = 2048 complex64, loss
    ||abs(LCT_M(f))^2 - I_target||^2 with I_target from a hidden matrix; one
    step = forward + backward (input and parameter gradients)."""
    import torch
    import workloads
    import paper_0912_1379_amd as lct

    B, N = 256, 2048
    g = workloads.rng(4)
    Mstar = workloads.sl2_params(B, g)
    gp = workloads.gaussian_params(B, g)
    xn, _ = lct.lct_nodes(N, 1.0)
    f = torch.from_numpy(workloads.chirped_gaussians(xn, gp)).to("cuda").to(torch.complex64)
    with torch.no_grad():
        target = lct.lct(f, torch.from_numpy(Mstar).to("cuda")).abs() ** 2
    M0 = Mstar + 0.01 * g.standard_normal(Mstar.shape)
    M0[:, 2] = (M0[:, 0] * M0[:, 3] - 1) / M0[:, 1]
    Mp = torch.from_numpy(M0).to("cuda").requires_grad_(True)
    fp = f.clone().requires_grad_(True)

    def step():
        y = lct.lct(fp, Mp)
        loss = ((y.abs() ** 2 - target) ** 2).sum()
        loss.backward()

    ms, ms_kernel, wall = time_launches(step, args.steps, args.warmup)
    out = {
        "metric": "steps/s, differentiable LCT fit (forward + backward)",
        "value": 1e3 / ms, "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fit: 256 signals x N=2048, intensity loss, grads w.r.t. f and (a,b,c,d)",
                   "signals": B, "N": N},
        "roofline": None, "wall_s_timed": wall,
    }
    if not args.no_cpu_baseline:
        import oracle

        # one step's three products on sampled signals, against the oracle: the
        # forward transform, the input gradient (adjoint of the output gradient)
        # and the parameter gradient, with the output gradient of this loss,
        # g = 4 (|y|^2 - I) y, formed from the GPU forward (an input to both sides)
        with torch.no_grad():
            y = lct.lct(fp, Mp)
            gy = (4 * (y.abs() ** 2 - target) * y).contiguous()
            gf = lct.lct_exec_many_adjoint(gy, Mp.detach())
            gM = lct.lct_param_grad_many(fp.detach(), gy, Mp.detach())
        fh, yh, gyh = fp.detach().cpu().numpy(), y.cpu().numpy(), gy.cpu().numpy()
        gfh, gMh, Mh = gf.cpu().numpy(), gM.cpu().numpy(), Mp.detach().cpu().numpy()
        ef, eg, ep = [], [], []
        t0 = time.perf_counter()
        nsig = 0
        while nsig < B and (nsig < 2 or time.perf_counter() - t0 < args.cpu_budget):
            s = nsig
            fin, gin = fh[s].astype(np.complex128), gyh[s].astype(np.complex128)
            ref = oracle.lct(fin, *Mh[s])
            ef.append(float(np.linalg.norm(yh[s] - ref) / np.linalg.norm(ref)))
            refg = oracle.lct_adjoint(gin, *Mh[s])
            eg.append(float(np.linalg.norm(gfh[s] - refg) / np.linalg.norm(refg)))
            refp = oracle.lct_param_grad(fin, gin, *Mh[s])
            ep.append(float(np.abs(gMh[s] - refp).max() / np.abs(refp).max()))
            nsig += 1
        el = time.perf_counter() - t0
        out["rel_l2"] = {"forward_max": max(ef), "input_grad_max": max(eg), "param_grad_max_rel": max(ep),
                         "signals": nsig}
        out["cpu_baseline"] = {"value": nsig / el / B, "unit": "steps/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"{nsig} of the {B} signals (forward, adjoint and parameter gradient, "
                                         f"dense N={N} sums), {el:.1f} s, scaled to the {B}-signal step"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--signals", type=int, default=4096)
    ap.add_argument("--N", type=int, default=4096)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-split", action="store_true", help="skip the split-BF16 matrix-core variant")
    ap.add_argument("--no-copy", action="store_true", help="skip the device-to-device copy reference")
    ap.add_argument("--no-cold", action="store_true", help="skip the cold-cache (flushed) launch timing")
    ap.add_argument("--no-shared", action="store_true",
                    help="frft workload: skip the shared-order (precomputed kernel spectrum) leg")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the built-in geometry heuristic instead of autotuning first")
    ap.add_argument("--ragged-subset", default="all", choices=["all", "lct", "frft", "lct_big", "frft_big", "small"],
                    help="ragged workload: time one part of the batch only")
    ap.add_argument("--workload", choices=["batched", "ragged", "large", "fit", "frft", "xft", "next"],
                    default="batched",
                    help="batched: 4096 x N=4096 (default); ragged: 10,000 uneven signals in one launch; "
                         "large: 16 x 2^20; fit: autograd step at 256 x 2048; frft: 4096 x N=4096 fractional; "
                         "xft: 4096 x N=4096 exact-node transform on the matrix cores; next: complex-matrix, "
                         "same-grid and oversampled LCTs at 4096 x N=4096")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(signals are independent: a multi-GPU run would shard the batch with no communication)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload != "batched":
        fn = {"ragged": bench_ragged, "large": bench_large, "fit": bench_fit, "frft": bench_frft,
              "xft": bench_xft, "next": bench_next}[args.workload]
        print(json.dumps(fn(args)), flush=True)
        return

    import torch
    import paper_0912_1379_amd as lct

    B, N = args.signals, args.N
    print(f"[bench] inputs: {B} signals x N={N}", file=sys.stderr, flush=True)
    M, f = make_inputs(B, N)
    dev = torch.device("cuda:0")
    x32 = torch.from_numpy(f).to(dev).to(torch.complex64)
    M4 = torch.from_numpy(M).to(dev)
    y32 = torch.empty_like(x32)

    tuning = None
    if not args.no_tune:
        # launch geometry picked by the library's autotuner on this device
        tuning = {"fp32": lct.lct_autotune(N, lct.LCT_FP32, "lct", batch=B)}
        if not args.no_fp64:
            tuning["fp64"] = lct.lct_autotune(N, lct.LCT_FP64, "lct", batch=B)
        print(f"[bench] tuned: {tuning}", file=sys.stderr, flush=True)
    geometry = lct.lct_tune_get(N, lct.LCT_FP32, "lct")

    def step32():
        lct.lct_exec_many(x32, M4, out=y32)

    ms, ms_kernel, wall = time_launches(step32, args.steps, args.warmup)
    ms_pairs = time_event_pairs(step32, args.steps)
    samples = B * N
    value = samples / (ms * 1e-3)
    algo_bytes = 16.0 * samples
    achieved_gbps = algo_bytes / (ms_kernel * 1e-3) / 1e9
    print(f"[bench] fp32: {ms * 1e3:.1f} us/step, kernel {ms_kernel * 1e3:.1f} us, {achieved_gbps:.0f} GB/s",
          file=sys.stderr, flush=True)

    # the same launch with the last-level cache flushed before each one (the
    # 268 MB working set is slightly above the 256 MB memory-side cache, so the
    # warm figure above may still find part of the input cached)
    cold = None
    if not args.no_cold:
        cold_ms, cold_med = time_cold(step32, 20)
        cold = {"kernel_ms": cold_ms, "kernel_ms_median": cold_med,
                "achieved_GBps": algo_bytes / (cold_ms * 1e-3) / 1e9,
                "frac": algo_bytes / (cold_ms * 1e-3) / 1e9 / PEAK_HBM_GBPS,
                "flush_bytes": 1 << 30, "launches": 20}
        print(f"[bench] fp32 cold: kernel {cold_ms * 1e3:.1f} us, {cold['achieved_GBps']:.0f} GB/s",
              file=sys.stderr, flush=True)

    fp64 = None
    y64_head = None
    if not args.no_fp64:
        x64 = x32.to(torch.complex128)
        y64 = torch.empty_like(x64)
        ms64, ms64_kernel, _ = time_launches(lambda: lct.lct_exec_many(x64, M4, out=y64),
                                              max(5, args.steps // 2), 3)
        fp64 = {"ms_per_step": ms64, "value": samples / (ms64 * 1e-3),
                "kernel_ms": ms64_kernel, "achieved_GBps": 32.0 * samples / (ms64_kernel * 1e-3) / 1e9,
                "fp32_speedup": ms64 / ms}
        print(f"[bench] fp64: {ms64 * 1e3:.1f} us/step", file=sys.stderr, flush=True)
        y64_head = y64[:256].cpu().numpy()  # rows the error check below may reach
        del x64, y64

    split = None
    ysp = None
    if not args.no_split:
        ysp = torch.empty_like(x32)
        mss, mss_kernel, _ = time_launches(
            lambda: lct.lct_exec_many(x32, M4, out=ysp, precision=lct.LCT_FP32_SPLITBF16), max(5, args.steps // 2), 3)
        split = {"ms_per_step": mss, "value": samples / (mss * 1e-3), "kernel_ms": mss_kernel,
                 "achieved_GBps": 16.0 * samples / (mss_kernel * 1e-3) / 1e9,
                 "mfma_flops_per_launch": mfma_flops(B, N),
                 "mfma_TFLOPs": mfma_flops(B, N) / (mss_kernel * 1e-3) / 1e12,
                 "kernel": "k_lct (FP32 data, radix-16 stages as split-BF16 MFMA)"}
        print(f"[bench] split-bf16: {mss * 1e3:.1f} us/step", file=sys.stderr, flush=True)

    # device-to-device copy of the same bytes (128 MiB read + 128 MiB written):
    # the practical streaming rate of this part, beside the 8 TB/s peak
    hbm_copy = None
    if not args.no_copy:
        copy_ms, copy_kernel_ms, _ = time_launches(lambda: y32.copy_(x32), 20, 3)
        hbm_copy = {"GBps": algo_bytes / (copy_kernel_ms * 1e-3) / 1e9, "bytes_per_launch": algo_bytes,
                    "kernel_ms": copy_kernel_ms, "what": "torch copy_ of the 4096 x 4096 complex64 input"}
        print(f"[bench] copy: {copy_kernel_ms * 1e3:.1f} us, {hbm_copy['GBps']:.0f} GB/s", file=sys.stderr,
              flush=True)
        lct.lct_exec_many(x32, M4, out=y32)  # restore the output the error check reads

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        rec = json.load(open(TRAFFIC_FILE))
        if (rec.get("kernel_hash") == kernel_hash() and rec.get("signals") == B and rec.get("N") == N
                and rec.get("geometry") == geometry):
            traffic = rec.get("bytes_per_launch")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "complex samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched LCT, {B} signals x N={N} complex64, one (a,b,c,d) per signal, "
                               "chirped-Gaussian inputs", "signals": B, "N": N, "precision": "fp32",
                   "parallelism": "single GPU", "geometry": geometry},
        "roofline": {"bound": "hbm", "achieved": achieved_gbps, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": achieved_gbps / PEAK_HBM_GBPS, "traffic": traffic,
                     "kernel": "k_lct (FP32, forward)", "kernel_ms": ms_kernel,
                     "kernel_ms_event_pairs": ms_pairs,
                     "algorithmic_bytes_per_launch": algo_bytes},
        "wall_s_timed": wall,
        "cold_cache": cold,
        "fp64_path": fp64,
        "splitbf16_path": split,
        "hbm_copy": hbm_copy,
        "tuning": tuning,
    }

    if not args.no_cpu_baseline:
        torch.cuda.synchronize()
        xh = x32.cpu().numpy()
        outs = {"fp32": y32.cpu().numpy().astype(np.complex128)}
        if ysp is not None:
            outs["splitbf16"] = ysp.cpu().numpy().astype(np.complex128)
        if y64_head is not None:
            outs["fp64"] = y64_head
        cb, errs = cpu_baseline(xh, M, outs, args.cpu_budget)
        out["cpu_baseline"] = cb
        e32 = errs["fp32"]
        out["rel_l2"] = {"max": max(e32), "median": float(np.median(e32)), "signals": len(e32)}
        if split is not None:
            es = errs["splitbf16"]
            split["rel_l2"] = {"max": max(es), "median": float(np.median(es)), "signals": len(es)}
        if fp64 is not None:
            e64 = errs["fp64"]
            fp64["rel_l2"] = {"max": max(e64), "median": float(np.median(e64)), "signals": len(e64)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

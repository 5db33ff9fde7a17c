"""MI355X (gfx950) fast discrete linear canonical transform.

Implements the scaling-chirp-DFT-chirp-scaling factorisation of R. G. Campos
and J. Figueroa, "A fast algorithm for the linear canonical transform"
(arXiv:0912.1379): the Algorithm of §3 (eq. algfxft1) for batches of signals
with one or many matrices M = (a b; c d), ad - bc = 1, and the same-grid
fractional Fourier transform of §2 (eqs. fasy, primcuad, cuadtrfor) for complex
orders |z| <= 1.  All arithmetic runs in the HIP library behind the C ABI of
``include/lct.h``; this package marshals torch tensors (device memory and the
current stream) into those calls.

The functions named like the C entry points take and return torch tensors:

    plan = lct_plan_create(N, a, b, c, d, precision=LCT_FP32)
    y = lct_exec(plan, x)                 # x: (..., N) complex64 / complex128 on cuda
    y = lct_exec_many(x, M4)              # M4: (batch, 4) float64 on cuda
    g = lct_exec_adjoint(plan, y)         # L^H y
    g = lct_exec_many_adjoint(y, M4)
    d = lct_param_grad_many(x, gy, M4)    # (batch, 4) float64: dl/d(a, b, c, d)
    y = frft_exec(plan, z, x)             # same-grid fractional transform
    y = frft_exec_many(x, Z2)             # Z2: (batch, 2) float64 (re z, im z)
    x, y = lct_nodes(N, b, d)             # input / output nodes (numpy)
    plan = lct_plan_create(N, a, b, c, d, scale=s)   # samples on s x_k
    x, y = lct_nodes(N, b, d, scale=s)

``lct(x, M)`` and ``frft(x, z)`` are conveniences; ``LCTFunction`` is the
autograd function whose backward is the adjoint transform plus the
parameter-gradient kernel.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (LCT_ERR_ARG, LCT_ERR_DOMAIN, LCT_ERR_HIP, LCT_ERR_NOT_UNIMODULAR,  # noqa: F401
                   LCT_ERR_UNSUPPORTED, LCT_ERR_UNSUPPORTED_N, LCT_ERR_WORKSPACE, LCT_FP32, LCT_FP64,
                   LCT_FP32_SPLITBF16, LCT_OK, LCT_TUNE_FRFT, LCT_TUNE_LCT, LctError)

__all__ = [
    "Plan", "lct_plan_create", "lct_plan_create_ex", "lct_plan_create_scaled", "lct_plan_destroy", "lct_exec", "lct_exec_many",
    "lct_exec_adjoint", "lct_exec_many_adjoint", "lct_param_grad_many", "frft_exec", "frft_exec_many",
    "frft_workspace_size", "lct_same_grid_exec", "RaggedPlan", "make_descriptors", "lct_ragged_plan_create", "lct_exec_ragged",
    "LCT_KIND_LCT", "LCT_KIND_FRFT",
    "lct_autotune", "lct_tune_candidates", "lct_tune_get", "lct_tune_set", "lct_tune_load", "lct_tune_save",
    "lct_tune_clear", "LCT_TUNE_LCT", "LCT_TUNE_FRFT",
    "lct_nodes", "lct_strerror", "lct_max_single_pass", "lct", "frft", "LCTFunction", "LctError",
    "XftPlan", "xft_plan_create", "xft_plan_destroy", "xft_exec", "xft_workspace_size", "xft_nodes", "xft_vectors",
    "LCT_FP32", "LCT_FP64", "LCT_FP32_SPLITBF16",
]


def _stream_handle(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _prec_of(t: torch.Tensor) -> int:
    if t.dtype == torch.complex64:
        return LCT_FP32
    if t.dtype == torch.complex128:
        return LCT_FP64
    raise TypeError(f"expected complex64 or complex128, got {t.dtype}")


def _dtype_of(prec: int) -> torch.dtype:
    return torch.complex128 if prec == LCT_FP64 else torch.complex64


def _check_data(t: torch.Tensor, name: str) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a GPU (the library has no CPU path)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _batch_of(t: torch.Tensor, N: int) -> int:
    if t.dim() == 0 or t.shape[-1] != N:
        raise ValueError(f"last dimension must be N = {N}, got shape {tuple(t.shape)}")
    return t.numel() // N


def _out_like(x: torch.Tensor, out):
    if out is None:
        return torch.empty_like(x)
    _check_data(out, "out")
    if out.shape != x.shape or out.dtype != x.dtype or out.device != x.device:
        raise ValueError("out must match the input's shape, dtype and device")
    return out


class Plan:
    """Owns an ``lct_plan`` handle (one size, one matrix, one precision)."""

    def __init__(self, N: int, a: float, b: float, c: float, d: float, precision: int = LCT_FP32,
                 scale: float = 1.0):
        lib = _lib.load()
        h = ctypes.c_void_p()
        _lib.check(lib.lct_plan_create_scaled(ctypes.byref(h), int(N), float(a), float(b), float(c), float(d),
                                              float(scale), int(precision)), "lct_plan_create_scaled")
        self._h = h
        self.N = int(N)
        self.M = (float(a), float(b), float(c), float(d))
        self.precision = int(precision)
        self.scale = float(scale)

    @property
    def handle(self):
        return self._h

    def destroy(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().lct_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def lct_plan_create(N, a, b, c, d, precision: int = LCT_FP32, scale: float = 1.0) -> Plan:
    """Plan for samples on the input grid scale * x_k (scale 1: the Algorithm's x_k)."""
    return Plan(N, a, b, c, d, precision, scale)


lct_plan_create_ex = lct_plan_create


def lct_plan_create_scaled(N, a, b, c, d, s: float, precision: int = LCT_FP32) -> Plan:
    return Plan(N, a, b, c, d, precision, s)


def lct_plan_destroy(plan: Plan) -> None:
    plan.destroy()


def _plan_io(plan: Plan, x: torch.Tensor, out):
    _check_data(x, "x")
    if _dtype_of(plan.precision) != x.dtype:
        raise TypeError("input dtype does not match the plan's precision")
    batch = _batch_of(x, plan.N)
    return batch, _out_like(x, out)


def lct_exec(plan: Plan, x: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    batch, out = _plan_io(plan, x, out)
    rc = _lib.load().lct_exec(plan.handle, x.data_ptr(), out.data_ptr(), batch, _stream_handle(stream))
    _lib.check(rc, "lct_exec")
    return out


def lct_exec_adjoint(plan: Plan, g: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    batch, out = _plan_io(plan, g, out)
    rc = _lib.load().lct_exec_adjoint(plan.handle, g.data_ptr(), out.data_ptr(), batch, _stream_handle(stream))
    _lib.check(rc, "lct_exec_adjoint")
    return out


def _check_params(P: torch.Tensor, batch: int, width: int, name: str) -> None:
    _check_data(P, name)
    if P.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if P.numel() != batch * width:
        raise ValueError(f"{name} must hold {batch} x {width} values")


def _prec_for(x: torch.Tensor, precision) -> int:
    """The data type fixes FP32 or FP64; complex64 data may also ask for
    LCT_FP32_SPLITBF16 (radix-16 stages on the matrix cores)."""
    prec = _prec_of(x)
    if precision is None or precision == prec:
        return prec
    if precision == LCT_FP32_SPLITBF16 and prec == LCT_FP32:
        return LCT_FP32_SPLITBF16
    raise TypeError(f"precision {precision} does not match data of dtype {x.dtype}")


def lct_exec_many(x: torch.Tensor, M4: torch.Tensor, out=None, stream=None, precision=None) -> torch.Tensor:
    _check_data(x, "x")
    prec = _prec_for(x, precision)
    N = x.shape[-1]
    batch = _batch_of(x, N)
    _check_params(M4, batch, 4, "M4")
    out = _out_like(x, out)
    rc = _lib.load().lct_exec_many(N, prec, M4.data_ptr(), x.data_ptr(), out.data_ptr(), batch,
                                   _stream_handle(stream))
    _lib.check(rc, "lct_exec_many")
    return out


def lct_exec_many_adjoint(g: torch.Tensor, M4: torch.Tensor, out=None, stream=None,
                          precision=None) -> torch.Tensor:
    _check_data(g, "g")
    prec = _prec_for(g, precision)
    N = g.shape[-1]
    batch = _batch_of(g, N)
    _check_params(M4, batch, 4, "M4")
    out = _out_like(g, out)
    rc = _lib.load().lct_exec_many_adjoint(N, prec, M4.data_ptr(), g.data_ptr(), out.data_ptr(), batch,
                                           _stream_handle(stream))
    _lib.check(rc, "lct_exec_many_adjoint")
    return out


def lct_param_grad_many(f: torch.Tensor, g: torch.Tensor, M4: torch.Tensor, grad4=None,
                        stream=None) -> torch.Tensor:
    _check_data(f, "f")
    _check_data(g, "g")
    prec = _prec_of(f)
    if g.dtype != f.dtype or g.shape != f.shape:
        raise ValueError("f and g must have the same shape and dtype")
    N = f.shape[-1]
    batch = _batch_of(f, N)
    _check_params(M4, batch, 4, "M4")
    if grad4 is None:
        grad4 = torch.empty((batch, 4), dtype=torch.float64, device=f.device)
    else:
        _check_params(grad4, batch, 4, "grad4")
    rc = _lib.load().lct_param_grad_many(N, prec, M4.data_ptr(), f.data_ptr(), g.data_ptr(), grad4.data_ptr(),
                                         batch, _stream_handle(stream))
    _lib.check(rc, "lct_param_grad_many")
    return grad4


def lct_complex_exec(x: torch.Tensor, a: complex, b: complex, d: complex, out=None, stream=None) -> torch.Tensor:
    """LCT of a complex matrix at the Algorithm's complex output nodes 4 b x_j / pi
    ((0, i, 0): the bilateral Laplace transform on the imaginary axis)."""
    _check_data(x, "x")
    N = x.shape[-1]
    batch = _batch_of(x, N)
    out = _out_like(x, out)
    a, b, d = complex(a), complex(b), complex(d)
    rc = _lib.load().lct_complex_exec(N, _prec_of(x), a.real, a.imag, b.real, b.imag, d.real, d.imag, x.data_ptr(),
                                      out.data_ptr(), batch, _stream_handle(stream))
    _lib.check(rc, "lct_complex_exec")
    return out


def lct_complex_nodes(N: int, b: complex) -> np.ndarray:
    """Output nodes 4 b x_j / pi (complex) of lct_complex_exec."""
    y = np.empty(2 * int(N), dtype=np.float64)
    b = complex(b)
    _lib.check(_lib.load().lct_complex_nodes(int(N), b.real, b.imag, y.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "lct_complex_nodes")
    return y.view(np.complex128)


def lct_oversampled_workspace_size(N: int, P: int, precision: int, batch: int) -> int:
    return int(_lib.load().lct_oversampled_workspace_size(int(N), int(P), int(precision), int(batch)))


def lct_exec_oversampled(plan: Plan, P: int, x: torch.Tensor, out=None, ws=None, stream=None) -> torch.Tensor:
    """Aliasing-aware LCT: the samples interpolated onto the grid P times finer,
    the Riemann sum taken there, returned at the Algorithm's output nodes."""
    batch, out = _plan_io(plan, x, out)
    need = lct_oversampled_workspace_size(plan.N, P, plan.precision, batch)
    if ws is None:
        ws = _workspace(need, x.device)
    rc = _lib.load().lct_exec_oversampled(plan.handle, int(P), x.data_ptr(), out.data_ptr(), batch,
                                          None if ws is None else ws.data_ptr(), 0 if ws is None else ws.numel(),
                                          _stream_handle(stream))
    _lib.check(rc, "lct_exec_oversampled")
    return out


def frft_workspace_size(N: int, precision: int, batch: int) -> int:
    return int(_lib.load().frft_workspace_size(int(N), int(precision), int(batch)))


def _workspace(nbytes: int, device) -> torch.Tensor | None:
    if nbytes == 0:
        return None
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def frft_exec(plan: Plan, z: complex, x: torch.Tensor, out=None, stream=None, ws=None) -> torch.Tensor:
    """Fractional transform with the plan's size and precision.  A workspace is
    allocated (torch) when the size needs one and `ws` is not given."""
    batch, out = _plan_io(plan, x, out)
    z = complex(z)
    need = frft_workspace_size(plan.N, plan.precision, batch)
    if ws is None:
        ws = _workspace(need, x.device)
    rc = _lib.load().frft_exec_ws(plan.handle, z.real, z.imag, x.data_ptr(), out.data_ptr(), batch,
                                  0 if ws is None else ws.data_ptr(), 0 if ws is None else ws.numel(),
                                  _stream_handle(stream))
    _lib.check(rc, "frft_exec_ws")
    return out


def frft_exec_many(x: torch.Tensor, Z2: torch.Tensor, out=None, stream=None, ws=None) -> torch.Tensor:
    _check_data(x, "x")
    prec = _prec_of(x)
    N = x.shape[-1]
    batch = _batch_of(x, N)
    _check_params(Z2, batch, 2, "Z2")
    out = _out_like(x, out)
    # one order per signal: only the two-pass sizes use a workspace
    need = frft_workspace_size(N, prec, batch) if 2 * N > lct_max_single_pass(prec) else 0
    if ws is None:
        ws = _workspace(need, x.device)
    rc = _lib.load().frft_exec_many_ws(N, prec, Z2.data_ptr(), x.data_ptr(), out.data_ptr(), batch,
                                       0 if ws is None else ws.data_ptr(), 0 if ws is None else ws.numel(),
                                       _stream_handle(stream))
    _lib.check(rc, "frft_exec_many_ws")
    return out


# ---------------------------------------------------------------------------
# Ragged batches: one persistent launch over signals of different lengths.
# ---------------------------------------------------------------------------
DESC_DTYPE = np.dtype([("offset", "<i8"), ("N", "<i4"), ("kind", "<i4"), ("prec", "<i4"), ("pad", "<i4"),
                       ("p", "<f8", (4,))])
LCT_KIND_LCT = 0
LCT_KIND_FRFT = 1


def make_descriptors(sizes, kinds, params, precision: int = LCT_FP32) -> np.ndarray:
    """Descriptor array (C layout lct_desc) for signals stored back to back:
    sizes[i] samples, kinds[i] in {LCT_KIND_LCT, LCT_KIND_FRFT}, params[i] =
    (a, b, c, d) or (re z, im z, 0, 0)."""
    sizes = np.asarray(sizes, dtype=np.int64)
    d = np.zeros(sizes.shape[0], dtype=DESC_DTYPE)
    d["offset"] = np.concatenate([[0], np.cumsum(sizes)[:-1]]) if sizes.size else []
    d["N"] = sizes
    d["kind"] = np.asarray(kinds, dtype=np.int32)
    d["prec"] = int(precision)
    d["p"] = np.asarray(params, dtype=np.float64).reshape(-1, 4)
    return d


def lct_workspace_size(desc: np.ndarray) -> int:
    """Workspace bytes of lct_exec_ragged for these (host) descriptors."""
    desc = np.ascontiguousarray(desc, dtype=DESC_DTYPE)
    n = ctypes.c_size_t()
    _lib.check(_lib.load().lct_workspace_size(desc.ctypes.data if desc.size else None, desc.shape[0],
                                              ctypes.byref(n)), "lct_workspace_size")
    return int(n.value)


def lct_check_params(P: torch.Tensor, kind: int = None, status=None, stream=None) -> torch.Tensor:
    """Device-side check of per-signal parameters: P is a (batch, 4) float64 tensor
    of matrices (kind LCT_KIND_LCT) or (batch, 2) of orders (LCT_KIND_FRFT).
    Returns a device int64 tensor {number of invalid rows, first invalid row or -1}."""
    if P.dtype != torch.float64 or not P.is_contiguous() or P.dim() != 2 or P.shape[1] not in (2, 4):
        raise ValueError("P must be a contiguous (batch, 4) or (batch, 2) float64 tensor")
    if kind is None:
        kind = LCT_KIND_LCT if P.shape[1] == 4 else LCT_KIND_FRFT
    if P.shape[1] != (4 if kind == LCT_KIND_LCT else 2):
        raise ValueError("row width does not match the kind")
    if status is None:
        status = torch.empty(2, dtype=torch.int64, device=P.device)
    rc = _lib.load().lct_check_params(int(kind), P.data_ptr(), P.shape[0], status.data_ptr(), _stream_handle(stream))
    _lib.check(rc, "lct_check_params")
    return status


def lct_check_desc(d_desc: torch.Tensor, nsig: int, status=None, stream=None) -> torch.Tensor:
    """Device-side check of ragged descriptors held on the device (uint8 tensor of
    nsig lct_desc records).  Returns {number of invalid descriptors, first or -1}."""
    if d_desc.dtype != torch.uint8 or d_desc.numel() != nsig * DESC_DTYPE.itemsize:
        raise ValueError("d_desc must hold nsig lct_desc records as uint8")
    if status is None:
        status = torch.empty(2, dtype=torch.int64, device=d_desc.device)
    rc = _lib.load().lct_check_desc(d_desc.data_ptr(), int(nsig), status.data_ptr(), _stream_handle(stream))
    _lib.check(rc, "lct_check_desc")
    return status


class RaggedPlan:
    """Owns an ``lct_ragged_plan`` and a device copy of the descriptors."""

    def __init__(self, desc: np.ndarray, precision: int = LCT_FP32, device="cuda"):
        desc = np.ascontiguousarray(desc, dtype=DESC_DTYPE)
        lib = _lib.load()
        h = ctypes.c_void_p()
        _lib.check(lib.lct_ragged_plan_create(ctypes.byref(h), desc.ctypes.data, desc.shape[0], int(precision)),
                   "lct_ragged_plan_create")
        self._h = h
        self.desc = desc
        self.total = int((desc["offset"] + desc["N"]).max()) if desc.size else 0
        self.d_desc = torch.from_numpy(desc.view(np.uint8).copy()).to(device)
        self.ws_bytes = int(lib.lct_ragged_workspace_size(h))
        ni, gr, ld = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
        lib.lct_ragged_info(h, ctypes.byref(ni), ctypes.byref(gr), ctypes.byref(ld))
        self.items, self.grid, self.lds = ni.value, gr.value, ld.value
        self.ws = None

    def set_params(self, params) -> None:
        """New per-signal parameters (same sizes, kinds and offsets)."""
        self.desc["p"] = np.asarray(params, dtype=np.float64).reshape(-1, 4)
        self.d_desc.copy_(torch.from_numpy(self.desc.view(np.uint8).copy()))

    def destroy(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().lct_ragged_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def lct_ragged_plan_create(desc: np.ndarray, precision: int = LCT_FP32) -> RaggedPlan:
    return RaggedPlan(desc, precision)


def lct_exec_ragged(plan: RaggedPlan, x: torch.Tensor, out=None, ws=None, stream=None) -> torch.Tensor:
    """x: 1-D complex64 tensor holding every signal at its descriptor offset."""
    _check_data(x, "x")
    if x.dtype != torch.complex64 or x.dim() != 1 or x.numel() < plan.total:
        raise ValueError("x must be a 1-D complex64 tensor covering every descriptor")
    out = _out_like(x, out)
    if ws is None:
        if plan.ws is None or plan.ws.numel() < plan.ws_bytes:
            plan.ws = torch.empty(plan.ws_bytes + 256, dtype=torch.uint8, device=x.device)
        ws = plan.ws
    base = ws.data_ptr()
    aligned = (base + 255) // 256 * 256
    rc = _lib.load().lct_exec_ragged(plan._h, plan.d_desc.data_ptr(), x.data_ptr(), out.data_ptr(), aligned,
                                     ws.numel() - (aligned - base), _stream_handle(stream))
    _lib.check(rc, "lct_exec_ragged")
    return out


def _tune_kind(kind) -> int:
    if kind in ("lct", LCT_TUNE_LCT):
        return LCT_TUNE_LCT
    if kind in ("frft", LCT_TUNE_FRFT):
        return LCT_TUNE_FRFT
    raise ValueError(f"unknown transform kind {kind!r}")


def lct_autotune(N: int, precision: int = LCT_FP32, kind="lct", batch: int = 0, stream=None) -> dict:
    """Times every candidate launch geometry for (kind, N, precision) on the
    current device, records the fastest in the library's table and returns
    what was measured (synchronises the stream)."""
    res = _lib.TuneResult()
    rc = _lib.load().lct_autotune(int(N), int(precision), _tune_kind(kind), int(batch), _stream_handle(stream),
                                  ctypes.byref(res))
    _lib.check(rc, "lct_autotune")
    return {"config": res.config.decode(), "candidates": res.candidates, "best_us": res.best_us,
            "default_us": res.default_us, "batch": res.batch}


def lct_tune_candidates(N: int, precision: int = LCT_FP32, kind="lct") -> list:
    """The candidate geometries (entry lines) the autotuner would time."""
    lib = _lib.load()
    n = ctypes.c_int(0)
    buf = ctypes.create_string_buffer(1 << 16)
    _lib.check(lib.lct_tune_candidates(int(N), int(precision), _tune_kind(kind), buf, len(buf), ctypes.byref(n)),
               "lct_tune_candidates")
    lines = [ln for ln in buf.value.decode().split("\n") if ln]
    assert len(lines) == n.value
    return lines


def lct_tune_get(N: int, precision: int = LCT_FP32, kind="lct") -> str:
    """The geometry line the entry points use for (kind, N, precision)."""
    buf = ctypes.create_string_buffer(512)
    _lib.check(_lib.load().lct_tune_get(int(N), int(precision), _tune_kind(kind), buf, len(buf)), "lct_tune_get")
    return buf.value.decode()


def lct_tune_set(line: str) -> None:
    _lib.check(_lib.load().lct_tune_set(line.encode()), "lct_tune_set")


def lct_tune_load(path: str) -> None:
    _lib.check(_lib.load().lct_tune_load(str(path).encode()), "lct_tune_load")


def lct_tune_save(path: str) -> None:
    _lib.check(_lib.load().lct_tune_save(str(path).encode()), "lct_tune_save")


def lct_tune_clear() -> None:
    _lib.load().lct_tune_clear()


def lct_nodes(N: int, b: float, d: float = 1.0, scale: float = 1.0):
    """Input nodes (scale * x_k, eq. asymcer) and output nodes y_j (numpy float64)."""
    x = np.empty(N, dtype=np.float64)
    y = np.empty(N, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    if scale == 1.0:
        rc = _lib.load().lct_nodes(int(N), float(b), float(d), x.ctypes.data_as(dp), y.ctypes.data_as(dp))
        _lib.check(rc, "lct_nodes")
    else:
        rc = _lib.load().lct_nodes_scaled(int(N), float(b), float(d), float(scale), x.ctypes.data_as(dp),
                                          y.ctypes.data_as(dp))
        _lib.check(rc, "lct_nodes_scaled")
    return x, y


def lct_same_grid_exec(x: torch.Tensor, a: complex, b: complex, d: complex, out=None, stream=None,
                       ws=None) -> torch.Tensor:
    """LCT of a complex matrix (a, b, d) with the output on the input grid (the
    nodes of lct_nodes(N, ...)[0]); one matrix for every signal of x."""
    _check_data(x, "x")
    prec = _prec_of(x)
    N = x.shape[-1]
    batch = _batch_of(x, N)
    out = _out_like(x, out)
    a, b, d = complex(a), complex(b), complex(d)
    if ws is None:
        ws = _workspace(frft_workspace_size(N, prec, batch), x.device)
    rc = _lib.load().lct_same_grid_exec(N, prec, a.real, a.imag, b.real, b.imag, d.real, d.imag, x.data_ptr(),
                                        out.data_ptr(), batch, 0 if ws is None else ws.data_ptr(),
                                        0 if ws is None else ws.numel(), _stream_handle(stream))
    _lib.check(rc, "lct_same_grid_exec")
    return out


# ---------------------------------------------------------------------------
# Exact-node discrete fractional transform (eq. tmat)
# ---------------------------------------------------------------------------
class XftPlan:
    """Plan of the exact-node transform F_z = sqrt(2 pi) U^T D(z) U for length N:
    U and U^T live on the device for the plan's lifetime."""

    def __init__(self, N: int, precision: int = LCT_FP32):
        h = ctypes.c_void_p()
        _lib.check(_lib.load().xft_plan_create(ctypes.byref(h), int(N), int(precision)), "xft_plan_create")
        self._h = h
        self.N = int(N)
        self.precision = int(precision)

    @property
    def handle(self):
        return self._h

    def destroy(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().xft_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def xft_plan_create(N: int, precision: int = LCT_FP32) -> XftPlan:
    return XftPlan(N, precision)


def xft_plan_destroy(plan: XftPlan) -> None:
    plan.destroy()


def xft_workspace_size(N: int, precision: int, batch: int) -> int:
    return int(_lib.load().xft_workspace_size(int(N), int(precision), int(batch)))


def xft_exec(plan: XftPlan, z: complex, x: torch.Tensor, out=None, stream=None, ws=None) -> torch.Tensor:
    """F_z applied to every length-N signal of x (sampled at the zeros of H_N,
    xft_nodes(N)).  A workspace is allocated (torch) when `ws` is not given."""
    batch, out = _plan_io(plan, x, out)
    z = complex(z)
    if ws is None:
        ws = _workspace(xft_workspace_size(plan.N, plan.precision, batch), x.device)
    rc = _lib.load().xft_exec(plan.handle, z.real, z.imag, x.data_ptr(), out.data_ptr(), batch,
                              0 if ws is None else ws.data_ptr(), 0 if ws is None else ws.numel(),
                              _stream_handle(stream))
    _lib.check(rc, "xft_exec")
    return out


def xft_nodes(N: int) -> np.ndarray:
    """The zeros of H_N, ascending (host computation of the library)."""
    x = np.empty(N, dtype=np.float64)
    _lib.check(_lib.load().xft_nodes(int(N), x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "xft_nodes")
    return x


def xft_vectors(N: int) -> np.ndarray:
    """U of eq. (ortvec), U[n, k] = (u_k)_n (host computation of the library)."""
    U = np.empty((N, N), dtype=np.float64)
    _lib.check(_lib.load().xft_vectors(int(N), U.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "xft_vectors")
    return U


def lct_strerror(code: int) -> str:
    return _lib.load().lct_strerror(int(code)).decode()


def lct_max_single_pass(precision: int = LCT_FP32) -> int:
    return int(_lib.load().lct_max_single_pass(int(precision)))


def _as_M4(M, batch: int, device) -> torch.Tensor:
    if isinstance(M, torch.Tensor):
        M4 = M.to(device=device, dtype=torch.float64)
    else:
        M4 = torch.as_tensor(np.asarray(M, dtype=np.float64), device=device)
    if M4.dim() == 1:
        M4 = M4.reshape(1, 4).expand(batch, 4)
    return M4.reshape(batch, 4).contiguous()


class LCTFunction(torch.autograd.Function):
    """y = L_M f per signal; backward gives L^H grad_y and dl/d(a, b, c, d)."""

    @staticmethod
    def forward(ctx, f: torch.Tensor, M4: torch.Tensor):
        f = f.contiguous()
        M4 = M4.contiguous()
        y = lct_exec_many(f, M4)
        ctx.save_for_backward(f, M4)
        return y

    @staticmethod
    def backward(ctx, gy: torch.Tensor):
        f, M4 = ctx.saved_tensors
        gy = gy.contiguous()
        gf = lct_exec_many_adjoint(gy, M4) if ctx.needs_input_grad[0] else None
        gM = lct_param_grad_many(f, gy, M4).reshape(M4.shape) if ctx.needs_input_grad[1] else None
        return gf, gM


def lct(x: torch.Tensor, M) -> torch.Tensor:
    """Discrete LCT of every length-N signal of x (last dimension) for one matrix
    M = (a, b, c, d) or one matrix per signal (a (batch, 4) float64 tensor)."""
    N = x.shape[-1]
    batch = _batch_of(x, N)
    M4 = _as_M4(M, batch, x.device)
    return LCTFunction.apply(x, M4)


def frft(x: torch.Tensor, z) -> torch.Tensor:
    """Same-grid discrete fractional transform of every signal of x for one
    complex order z or one order per signal (a (batch,) complex tensor)."""
    _check_data(x, "x")
    N = x.shape[-1]
    batch = _batch_of(x, N)
    if isinstance(z, torch.Tensor):
        zc = z.to(torch.complex128).reshape(batch)
        Z2 = torch.view_as_real(zc).to(device=x.device).contiguous()
        return frft_exec_many(x, Z2)
    # one order for every signal: the plan path shares the kernel's spectrum
    return frft_exec(_frft_plan(N, _prec_of(x)), complex(z), x)


_FRFT_PLANS: dict = {}


def _frft_plan(N: int, precision: int) -> Plan:
    """A plan of size N (the fractional transform uses only its size and precision)."""
    key = (int(N), int(precision))
    if key not in _FRFT_PLANS:
        _FRFT_PLANS[key] = Plan(N, 1.0, 0.0, 0.0, 1.0, precision)
    return _FRFT_PLANS[key]

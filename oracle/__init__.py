"""Oracle for the fast discrete linear canonical transform (arXiv:0912.1379).

TEST INFRASTRUCTURE ONLY.  A plain, slow, obviously correct CPU evaluation of
what the paper defines (FP64 in and out, long-double arithmetic inside).  Only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
``paper_0912_1379_amd``; neither imports the other.

Functions and what pins them (the pins live in ``tests/test_oracle_*.py``):

``nodes(N)``                eq. (asymcer); pinned against the true Hermite
                            zeros' spacing and symmetry.
``lct(f, a, b, c, d)``      Riemann sum of the LCT integral of §1 on the
                            Algorithm's nodes (b != 0) or the b = 0 formula of
                            §1; pinned by eq. (exa1) at the two parameter sets
                            of §4, the Hermite-Gauss closed form, unitarity,
                            numpy's FFT for a=d=0, b=1, the composition law
                            and mpmath brute force.  ``scale=s`` takes the
                            samples on s x_k (outputs on 4 b x_j / (pi s));
                            pinned by the Gaussian closed form on scaled grids
                            and by chains of two transforms.
``lct_same_grid(f, a, b, d)`` LCT of §1 for complex a, b, d as a Riemann sum
                            with output on the input grid; pinned by the
                            fractional transform (a = d), O1 at b = pi/4 for
                            real matrices, the complex Gaussian closed form
                            and mpmath brute force.
``trig_interp(f, p)``       trigonometric interpolation of the samples onto the
                            grid of step h / p; pinned by exact reproduction of
                            trigonometric polynomials and by the explicit
                            periodic-interpolation sum.
``lct_oversampled(f, a, b, c, d, p)``  aliasing-aware LCT: O1 on that finer
                            grid at the Algorithm's output nodes; pinned by
                            p = 1 (O1), the chirped-Gaussian closed form where
                            O1 aliases, and the explicit interpolation sum.
``lct_complex(f, a, b, d)`` LCT of §1 for a complex matrix at the Algorithm's
                            complex output nodes 4 b x_j / pi (O6; the bilateral
                            Laplace transform for (0, i, 0)); pinned by O1 for
                            real matrices, the complex Gaussian integral, the
                            Laplace transform of a Gaussian and mpmath.
``lct_adjoint``             conjugate transpose of the same matrix; pinned by
                            the inner-product identity and unitarity.
``lct_param_grad``          derivative of the dense matrix w.r.t. (a,b,c,d)
                            (for b = 0, of the diagonal of §1: c and d
                            enter, a and b do not); pinned by central finite
                            differences of ``lct``.
``frft(f, z)``              same-grid Riemann sum of eqs. (fasy), (primcuad),
                            (cuadtrfor); pinned by the continuum eigen-identity
                            on Hermite functions, the z=+-i Fourier kernel of
                            eq. (fftuno) and mpmath brute force.
``hermite_zeros(N)``        eigenvalues of the symmetric tridiagonal H of §2;
                            pinned by numpy hermgauss and closed-form zeros.
``hermite_vectors``         eq. (ortvec); pinned by orthogonality, the
                            |u_N| = 1/sqrt(N) identity and Gauss-Hermite weights.
``Fz_exact(N, z)``          eq. (tmat); pinned by its eigen-identity and
                            unitarity on |z| = 1.
``xft(f, z)``               F_z of eq. (tmat) applied to signals sampled at
                            the zeros of H_N, as sqrt(2 pi) U^T (z^n (U f))
                            with numpy matmuls; pinned by Fz_exact @ f, the
                            discrete eigen-identity on the rows of U, and the
                            O(1/N) approach to the continuum eigen-identity
                            on sampled Hermite functions.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liblct_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("LCT_ORACLE_LIBRARY")  # e.g. the sanitized build of build.py --sanitize
    if not path:
        path = _LIBPATH
        if not os.path.exists(path) or (
                os.path.getmtime(path) < os.path.getmtime(os.path.join(_HERE, "lct_oracle.c"))):
            from . import build as _b
            _b.build()
    lib = ctypes.CDLL(path)
    i64, d = ctypes.c_int64, ctypes.c_double
    lib.oracle_nodes.argtypes = [i64, _dp]
    lib.oracle_lct_rows.argtypes = [i64, d, d, d, d, _dp, _i64p, i64, _dp]
    lib.oracle_lct_rows.restype = ctypes.c_int
    lib.oracle_lct_rows_scaled.argtypes = [i64, d, d, d, d, d, _dp, _i64p, i64, _dp]
    lib.oracle_lct_rows_scaled.restype = ctypes.c_int
    lib.oracle_lct_same_rows.argtypes = [i64, d, d, d, d, d, d, _dp, _i64p, i64, _dp]
    lib.oracle_lct_complex_rows.argtypes = [i64, d, d, d, d, d, d, _dp, _i64p, i64, _dp]
    lib.oracle_lct_complex_rows.restype = ctypes.c_int
    lib.oracle_lct_same_rows.restype = ctypes.c_int
    lib.oracle_lct_adjoint.argtypes = [i64, d, d, d, d, _dp, _dp]
    lib.oracle_lct_adjoint.restype = ctypes.c_int
    lib.oracle_lct_param_grad.argtypes = [i64, d, d, d, d, _dp, _dp, _dp]
    lib.oracle_lct_param_grad.restype = ctypes.c_int
    lib.oracle_frft_rows.argtypes = [i64, d, d, _dp, _i64p, i64, _dp]
    lib.oracle_frft_rows.restype = ctypes.c_int
    lib.oracle_hermite_zeros.argtypes = [i64, _dp]
    lib.oracle_hermite_vectors.argtypes = [i64, _dp, _dp]
    lib.oracle_Fz_exact.argtypes = [i64, _dp, d, d, _dp]
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_num_threads.restype = None
    _lib = lib
    return lib


def _cplx_in(f) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(f, dtype=np.complex128))
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads of later oracle calls (for timing the oracle on one core)."""
    _load().oracle_set_num_threads(int(n))


def nodes(N: int) -> np.ndarray:
    """x_k of eq. (asymcer), 0-based: (2k - N + 1) pi / (2 sqrt(2N))."""
    x = np.empty(N, dtype=np.float64)
    _load().oracle_nodes(N, _ptr(x))
    return x


def output_nodes(N: int, b: float, d: float = 1.0, scale: float = 1.0) -> np.ndarray:
    """Output nodes for samples on the input grid scale * x_k:
    y_j = 4 b x_j / (pi scale) for b != 0 (the Algorithm's y_j at scale 1),
    scale * x_j / d for b = 0."""
    x = nodes(N)
    if b == 0.0:
        return scale * x / d
    return 4.0 * b * x / (np.pi * scale)


def lct(f, a: float, b: float, c: float, d: float, rows=None, scale: float = 1.0) -> np.ndarray:
    """Discrete LCT (O1) of the length-N sample vector f (complex), sampled on
    the input grid scale * x_k.

    ``f`` may be 1-D (one signal) or 2-D (signals x N, all with the same M).
    ``rows`` selects output indices (default: all N)."""
    f = _cplx_in(f)
    if f.ndim == 2:
        return np.stack([lct(fi, a, b, c, d, rows, scale) for fi in f])
    N = f.shape[0]
    if rows is None:
        r = None
        nr = N
    else:
        r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        nr = r.shape[0]
    out = np.empty(nr, dtype=np.complex128)
    rc = _load().oracle_lct_rows_scaled(N, a, b, c, d, float(scale), _ptr(f.view(np.float64)),
                                        None if r is None else r.ctypes.data_as(_i64p), nr,
                                        _ptr(out.view(np.float64)))
    if rc != 0:
        raise ValueError(f"oracle_lct_rows failed ({rc})")
    return out


def trig_interp(f, p: int) -> np.ndarray:
    """Trigonometric interpolation of the samples f_k = f(x_k) (eq. asymcer's
    grid, step h, period N h) onto the grid of step h / p over the same span,
    xi_m = (h / p)(m - (p N - 1) / 2), m < p N:
        f(x) = sum_n c_n exp(2 pi i n (x - x_0) / (N h)),  c_n = (1/N) sum_k f_k e^{-2 pi i n k / N},
    n over -N/2 .. N/2 (for even N the coefficient of n = +-N/2 split in two
    halves).  At xi_m, (xi_m - x_0) / (N h) = (m - (p - 1)/2) / (p N), so the fine
    samples are a length-pN inverse DFT of the twisted coefficients.  numpy's
    FFT serves as the DFT."""
    f = _cplx_in(f)
    N = f.shape[0]
    p = int(p)
    if p < 1:
        raise ValueError("p >= 1")
    if p == 1:
        return f.copy()
    M = p * N
    c = np.fft.fft(f) / N
    n = np.arange(N)
    n = np.where(n < (N + 1) // 2, n, n - N)  # -floor(N/2) .. ceil(N/2) - 1
    twist = lambda k: np.exp(-1j * np.pi * k * (p - 1) / M)
    dpad = np.zeros(M, dtype=np.complex128)
    if N % 2 == 0:
        nyq = N // 2
        half = c[nyq] / 2  # c at n = -N/2 (index N/2 of the DFT)
        keep = n != -nyq
        dpad[n[keep] % M] = c[keep] * twist(n[keep])
        dpad[(-nyq) % M] += half * twist(-nyq)
        dpad[nyq % M] += half * twist(nyq)
    else:
        dpad[n % M] = c * twist(n)
    return np.fft.ifft(dpad) * M


def lct_oversampled(f, a: float, b: float, c: float, d: float, p: int, rows=None) -> np.ndarray:
    """Aliasing-aware discrete LCT: the samples f_k on x_k are interpolated
    trigonometrically onto the grid of step h / p (trig_interp), and the
    Riemann sum of the integral of §1 is taken there (weight h / p), at the
    Algorithm's output nodes y_j = 4 b x_j / pi.  That fine grid is the scaled
    grid s x'_m of p N points with s = 1 / sqrt(p) (x'_m eq. asymcer's nodes
    for p N), whose output nodes 4 b x'_m / (pi s) hold the y_j as the middle
    block m = j + (p - 1) N / 2; so this is O1 on the scaled grid (lct with
    scale = s) at those rows.  For b = 0 (a diagonal, no aliasing) it is O1
    itself; p = 1 is O1."""
    f = _cplx_in(f)
    N = f.shape[0]
    if b == 0.0 or int(p) == 1:
        return lct(f, a, b, c, d, rows=rows)
    p = int(p)
    if ((p - 1) * N) % 2:
        raise ValueError("(p - 1) N must be even (the y_j then sit on the fine output grid)")
    g = trig_interp(f, p)
    off = (p - 1) * N // 2
    r = np.arange(N) if rows is None else np.asarray(rows, dtype=np.int64)
    return lct(g, a, b, c, d, rows=r + off, scale=1.0 / np.sqrt(p))


def lct_same_grid(f, a: complex, b: complex, d: complex, rows=None) -> np.ndarray:
    """LCT of §1 for a complex matrix, output on the input grid (O4); 1-D f."""
    f = _cplx_in(f)
    N = f.shape[0]
    if rows is None:
        r = None
        nr = N
    else:
        r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        nr = r.shape[0]
    a, b, d = complex(a), complex(b), complex(d)
    out = np.empty(nr, dtype=np.complex128)
    rc = _load().oracle_lct_same_rows(N, a.real, a.imag, b.real, b.imag, d.real, d.imag, _ptr(f.view(np.float64)),
                                      None if r is None else r.ctypes.data_as(_i64p), nr,
                                      _ptr(out.view(np.float64)))
    if rc != 0:
        raise ValueError(f"oracle_lct_same_rows failed ({rc})")
    return out


def complex_output_nodes(N: int, b: complex) -> np.ndarray:
    """The Algorithm's output nodes y_j = 4 b x_j / pi for a complex b."""
    return 4.0 * complex(b) * nodes(N) / np.pi


def lct_complex(f, a: complex, b: complex, d: complex, rows=None) -> np.ndarray:
    """LCT of §1 for a complex matrix (O6): the Riemann sum on the input nodes
    x_k at the complex output nodes y_j = 4 b x_j / pi; 1-D f.  (0, i, 0) is
    the bilateral Laplace transform (times (-2 pi)^(-1/2)) on the imaginary
    axis."""
    f = _cplx_in(f)
    N = f.shape[0]
    if rows is None:
        r = None
        nr = N
    else:
        r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        nr = r.shape[0]
    a, b, d = complex(a), complex(b), complex(d)
    out = np.empty(nr, dtype=np.complex128)
    rc = _load().oracle_lct_complex_rows(N, a.real, a.imag, b.real, b.imag, d.real, d.imag,
                                         _ptr(f.view(np.float64)), None if r is None else r.ctypes.data_as(_i64p),
                                         nr, _ptr(out.view(np.float64)))
    if rc != 0:
        raise ValueError(f"oracle_lct_complex_rows failed ({rc})")
    return out


def lct_adjoint(g, a: float, b: float, c: float, d: float) -> np.ndarray:
    """L^H g for the b != 0 discrete LCT matrix."""
    g = _cplx_in(g)
    N = g.shape[0]
    out = np.empty(N, dtype=np.complex128)
    rc = _load().oracle_lct_adjoint(N, a, b, c, d, _ptr(g.view(np.float64)),
                                    _ptr(out.view(np.float64)))
    if rc != 0:
        raise ValueError(f"oracle_lct_adjoint failed ({rc})")
    return out


def lct_param_grad(f, g, a: float, b: float, c: float, d: float) -> np.ndarray:
    """(dl/da, dl/db, dl/dc, dl/dd) = Re sum_j conj(g_j) dG_j/dtheta; for b = 0 the
    derivative of the diagonal of §1 (dl/da = dl/db = 0)."""
    f = _cplx_in(f)
    g = _cplx_in(g)
    N = f.shape[0]
    out = np.empty(4, dtype=np.float64)
    rc = _load().oracle_lct_param_grad(N, a, b, c, d, _ptr(f.view(np.float64)),
                                       _ptr(g.view(np.float64)), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_lct_param_grad failed ({rc})")
    return out


def frft(f, z: complex, rows=None) -> np.ndarray:
    """Same-grid discrete fractional transform (O3) of f for complex |z| <= 1."""
    f = _cplx_in(f)
    if f.ndim == 2:
        return np.stack([frft(fi, z, rows) for fi in f])
    N = f.shape[0]
    z = complex(z)
    if rows is None:
        r = None
        nr = N
    else:
        r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        nr = r.shape[0]
    out = np.empty(nr, dtype=np.complex128)
    rc = _load().oracle_frft_rows(N, z.real, z.imag, _ptr(f.view(np.float64)),
                                  None if r is None else r.ctypes.data_as(_i64p), nr,
                                  _ptr(out.view(np.float64)))
    if rc == -2:
        raise ValueError("|z| > 1")
    if rc != 0:
        raise ValueError(f"oracle_frft_rows failed ({rc})")
    return out


def hermite_zeros(N: int) -> np.ndarray:
    """Eigenvalues of the symmetric tridiagonal H of §2 (zeros of H_N)."""
    x = np.empty(N, dtype=np.float64)
    _load().oracle_hermite_zeros(N, _ptr(x))
    return x


def hermite_vectors(N: int, x=None) -> np.ndarray:
    """U with U[n, k] = (u_k)_n of eq. (ortvec) (0-based n, k)."""
    if x is None:
        x = hermite_zeros(N)
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    U = np.empty((N, N), dtype=np.float64)
    _load().oracle_hermite_vectors(N, _ptr(x), _ptr(U))
    return U


def Fz_exact(N: int, z: complex, U=None) -> np.ndarray:
    """F_z = sqrt(2 pi) U^T D(z) U of eq. (tmat)."""
    if U is None:
        U = hermite_vectors(N)
    U = np.ascontiguousarray(np.asarray(U, dtype=np.float64))
    z = complex(z)
    F = np.empty((N, N), dtype=np.complex128)
    _load().oracle_Fz_exact(N, _ptr(U), z.real, z.imag, _ptr(F.view(np.float64)))
    return F


def xft(f, z: complex, U=None) -> np.ndarray:
    """Exact-node discrete fractional transform of eq. (tmat) applied to
    signals f (shape (N,) or (batch, N)) sampled at the zeros of H_N:
    g = sqrt(2 pi) U^T D(z) U f, D(z) = diag(1, z, ..., z^(N-1)); the powers
    of z by repeated multiplication in extended precision."""
    f = np.asarray(f, dtype=np.complex128)
    one = f.ndim == 1
    F = f[None, :] if one else f
    N = F.shape[-1]
    if U is None:
        U = hermite_vectors(N)
    steps = np.full(N, complex(z), dtype=np.clongdouble)
    steps[0] = 1.0
    zp = np.cumprod(steps).astype(np.complex128)
    V = U @ F.T                                   # (N, batch): U f
    G = np.sqrt(2.0 * np.pi) * (U.T @ (zp[:, None] * V))
    G = np.ascontiguousarray(G.T)
    return G[0] if one else G


def lct_matrix(N: int, a: float, b: float, c: float, d: float) -> np.ndarray:
    """Dense matrix of the discrete LCT, column k = lct(e_k)."""
    cols = [lct(np.eye(N, dtype=np.complex128)[k], a, b, c, d) for k in range(N)]
    return np.stack(cols, axis=1)

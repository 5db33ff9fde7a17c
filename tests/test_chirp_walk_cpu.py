"""Host check of the FP64 kernels' chirp walk (ChirpSeq<double> in
kernels_impl.hpp): the values c_e = cis(2 pi (A + e B + e^2 C)) of one thread,
e = 0, 1, ..., formed by products c_{e+1} = c_e d_e, d_{e+1} = d_e cis(4 pi C)
from three direct evaluations, against the same values with the phase summed
in extended precision.  The walk's error grows like e^2 rounding units and
stays below that of evaluating the phase polynomial directly in FP64 (whose
sum reaches e^2 |C| turns), for every width a thread can hold (up to 30
values): 1e-13 at most, inside the FP64 path's 1e-12 bound.  Emulated in numpy
complex128."""
import numpy as np
import pytest


def cis_turns(t):
    t = t - np.rint(t)
    return np.exp(2j * np.pi * t)


@pytest.mark.skipif(np.finfo(np.longdouble).nmant < 60, reason="needs an extended long double")
def test_walk_error_grows_like_e_squared():
    g = np.random.default_rng(1)
    A, B, C = (g.uniform(-0.5, 0.5, 20000) for _ in range(3))
    Al, Bl, Cl = (v.astype(np.longdouble) for v in (A, B, C))
    c = cis_turns(A)
    d = cis_turns(B + C)
    r = cis_turns(2.0 * C)
    u = 2.0 ** -53
    for e in range(31):
        t = Al + np.longdouble(e) * Bl + np.longdouble(e * e) * Cl
        ref = np.exp(2j * np.pi * (t - np.rint(t)).astype(np.float64))
        walk = np.abs(c - ref).max()
        direct = np.abs(cis_turns(A + e * B + e * e * C) - ref).max()
        assert walk <= (8 + 2.5 * e * e) * u, (e, walk / u)
        if e >= 4:
            assert walk < direct, (e, walk / u, direct / u)
        c = c * d
        d = d * r
    assert walk < 2e-13

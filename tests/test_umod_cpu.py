"""Host check of the bound behind the kernels' stride remainder (umod24 in
fft_core.hpp): for 0 <= a < 2^24 and a divisor m >= 3 that is not a power of
two, the FP32 estimate trunc(a * rcp(m)) is within one of floor(a / m) even
when the reciprocal is one unit in the last place off (the accuracy of the
hardware reciprocal), so the integer corrections made after it (up to two
each way) always land on a mod m.  The estimate is emulated in numpy FP32 with
the reciprocal rounded correctly and moved one ulp either way."""
import numpy as np


def smooth_non_pow2(limit):
    out = []
    p2 = 1
    while p2 < limit:
        p3 = 1
        while p2 * p3 < limit:
            p5 = 1
            while p2 * p3 * p5 < limit:
                m = p2 * p3 * p5
                if m >= 3 and (m & (m - 1)) != 0:
                    out.append(m)
                p5 *= 5
            p3 *= 3
        p2 *= 2
    return sorted(out)


def corrected(a, m, q):
    r = a - q * m
    r = np.where(r < 0, r + m, r)
    r = np.where(r < 0, r + m, r)
    r = np.where(r >= m, r - m, r)
    r = np.where(r >= m, r - m, r)
    return r


def test_quotient_estimate_within_one():
    g = np.random.default_rng(0)
    ms = smooth_non_pow2(1 << 24)
    assert len(ms) > 300
    for m in ms:
        # edges (0, the top of the domain, multiples of m and their neighbours) and random values
        k = np.arange(0, (1 << 24) // m + 1, max(1, ((1 << 24) // m) // 64), dtype=np.int64)
        a = np.concatenate([k * m - 1, k * m, k * m + 1, [0, (1 << 24) - 1],
                            g.integers(0, 1 << 24, 2000)])
        a = a[(a >= 0) & (a < (1 << 24))]
        exact_q = a // m
        rc = np.float32(1.0) / np.float32(m)
        for rcp in (np.nextafter(rc, np.float32(0)), rc, np.nextafter(rc, np.float32(1))):
            q = np.trunc(a.astype(np.float32) * rcp).astype(np.int64)
            assert np.abs(q - exact_q).max() <= 1, m
            assert np.array_equal(corrected(a, m, q), a % m), m

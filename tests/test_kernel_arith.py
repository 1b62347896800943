"""Host checks of the arithmetic claims the kernels rely on (no GPU): each emulates, step by
step in the same precision, a device helper whose correctness rests on a numerical
argument, and checks it over the whole range the kernels use it on."""
import numpy as np


def _divmod_small(n, d, rcp):
    """The index decoding of the small matrices: q = trunc(float(n) * rcp(d)) in FP32, then
    one correction each way (la::divmod_small)."""
    f = n.astype(np.float32) * np.float32(rcp)
    q = np.trunc(f).astype(np.int64)
    r = n - q * d
    up = r >= d
    q[up] += 1
    r[up] -= d
    dn = r < 0
    q[dn] -= 1
    r[dn] += d
    return q, r


def test_divmod_small_is_exact_for_matrix_indices():
    """Exact quotient and remainder for every n < 2^20 (strided sample plus the ends) and
    divisor d <= 2^12, with the hardware reciprocal anywhere within one ulp of 1/d."""
    n = np.concatenate([np.arange(0, 1 << 20, 5, dtype=np.int64),
                        np.arange((1 << 20) - 64, 1 << 20, dtype=np.int64)])
    for d in list(range(1, 260)) + [511, 512, 1000, 2047, 4095, 4096]:
        r0 = np.float32(1.0) / np.float32(d)
        for rcp in (r0, np.nextafter(r0, np.float32(0.0)), np.nextafter(r0, np.float32(np.inf))):
            q, r = _divmod_small(n, d, rcp)
            assert np.array_equal(q, n // d), (d, rcp)
            assert np.array_equal(r, n % d), (d, rcp)


def test_divmod_small_needs_the_correction():
    """Without the correction the truncated quotient is wrong for some n (so the test above
    exercises it): n = q d exactly, with a reciprocal one ulp low."""
    d = 3
    rcp = np.nextafter(np.float32(1.0) / np.float32(d), np.float32(0.0))
    n = np.arange(0, 1 << 16, dtype=np.int64)
    f = n.astype(np.float32) * rcp
    assert np.any(np.trunc(f).astype(np.int64) != n // d)

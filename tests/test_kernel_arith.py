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


def _pivot_key(n2, c):
    """The zip-up's pivot key: the bit pattern of the squared norm n2 >= 0 with its low byte
    replaced by 255 - c (column c < 128); the argmax over keys is the pivot."""
    bits = np.asarray(n2, dtype=np.float64).view(np.uint64)
    return (bits & ~np.uint64(0xFF)) | (np.uint64(255) - np.asarray(c, dtype=np.uint64))


def _key_col(key):
    return 255 - int(key & np.uint64(0xFF))


def test_pivot_key_orders_by_norm_with_ties_to_the_smaller_column():
    """On random norms (including zeros, a subnormal and exact ties) the largest key is a
    column whose norm is within 2^-44 relative of the largest when that is a normal number
    (the exact argmax whenever the norms differ by more), ties go to the smaller column, no
    key is 0 (the mark of an empty wave), and non-finite norms outrank every finite one."""
    rng = np.random.default_rng(20261203)
    for trial in range(2000):
        p = int(rng.integers(1, 129))
        n2 = rng.exponential(1.0, p) * 10.0 ** rng.integers(-300, 300)
        if trial % 5 == 0:
            n2[rng.integers(0, p, max(1, p // 4))] = 0.0
        if trial % 7 == 0:
            n2[rng.integers(0, p, 3)] = n2.max()            # exact ties at the top
        if trial % 11 == 0:
            n2[rng.integers(0, p)] = 5e-324                  # smallest subnormal
        c = np.arange(p)
        keys = _pivot_key(n2, c)
        assert (keys != 0).all()
        win = _key_col(keys.max())
        top = n2.max()
        assert n2[win] >= top * (1.0 - 2.0 ** -44)
        ties = np.flatnonzero(n2 == n2[win])
        assert win == ties.min()
        exact = int(np.argmax(n2))                           # first index of the maximum
        if np.sort(n2)[-2:][0] < top * (1.0 - 2.0 ** -40) or (n2 == top).sum() > 1:
            assert win == exact
    for bad in (np.inf, np.nan):
        n2 = np.array([1.0, 2.0, bad, 3.0])
        assert _key_col(_pivot_key(n2, np.arange(4)).max()) == 2

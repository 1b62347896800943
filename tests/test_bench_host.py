"""Host logic of bench.py (no GPU): the flop and byte models behind its rooflines, its copy
of the Black-Scholes formula (checked against the oracle's pinned closed form), and the
oracle-error leg on prices that equal the oracle's."""
import math

import numpy as np

import bench
import cm_workloads as W
from oracle import carr_madan as O


def test_bench_black_scholes_matches_pinned_closed_form():
    K = np.linspace(40.0, 180.0, 57)
    for T, sig in ((0.5, 0.3), (2.0, 0.15)):
        assert np.allclose(bench._bs_call(100.0, K, 0.05, 0.0, T, sig), O.bs_call(100.0, K, 0.05, 0.0, T, sig),
                           rtol=0, atol=1e-12)


def test_readout_flops_counts_distinct_suffixes():
    n = 3
    rk = [1, 2, 3, 1]
    # all 8 strikes: level l has 2^(n-l) distinct suffixes u >> l
    want = sum(2 ** (n - l) * 8 * rk[l] * rk[l + 1] for l in range(n))
    assert bench.readout_flops(rk, n, np.arange(8)) == want
    # one strike: one product per level
    assert bench.readout_flops(rk, n, np.array([5])) == sum(8 * rk[l] * rk[l + 1] for l in range(n))


def test_round_flops_rank_one_train():
    n = 5
    ones = [1] * (n + 1)
    # per bond: contraction 8*1*2*1*1, QR of a 2 x 1 matrix to rank 1: 24*2*1, no Jacobi pair;
    # then core 0: 8*2*1*1
    assert bench.round_flops(ones, ones, n) == (n - 1) * (16 + 48) + 16


def test_zipup_flops_and_core_elems():
    n = 3
    xr, wr, yz = [1, 2, 2, 1], [1, 2, 2, 1], [1, 2, 2, 1]
    f32, f64 = bench.zipup_flops(xr, wr, yz, n)
    chi, want32, want64 = 1, 0.0, 0.0
    for l in range(n):
        want32 += 8.0 * (chi * wr[l] * 2 * xr[l] * xr[l + 1] + chi * 2 * wr[l] * 2 * wr[l + 1] * xr[l + 1])
        if l < n - 1:
            m, p, k = 2 * chi, wr[l + 1] * xr[l + 1], yz[l + 1]
            want64 += sum(24.0 * (m - i) * (p - i) + 16.0 * (m - i) * k for i in range(k))
            chi = k
    assert (f32, f64) == (want32, want64)
    assert bench.core_elems([1, 2, 3, 1], 3) == 1 * 2 * 2 + 2 * 2 * 3 + 3 * 2 * 1


def test_oracle_error_leg_is_zero_on_oracle_prices():
    probs = W.heston_batch(2, seed=9, n=14)
    u = np.stack([W.near_money(p, 64) for p in probs])
    got = np.stack([O.prices_direct(p, u[b]) for b, p in enumerate(probs)])
    worst, errs = bench.oracle_errors(bench.parity_sample(probs, got, u, [0, 1], every=4))
    assert worst == 0.0 and len(errs) == 2
    assert isinstance(bench._cpu_model(), str)

"""The benchmark's own workload at full size, in the launch configuration the benchmark times:
4096 seeded Heston instances at n = 24 (M = 2^24 grid points each), complex64 contraction and
FP64 factorisation, tol 1e-8, cap 32, persistent-workgroup counts build 4096, zip-up 1536,
rounding 4096, the chain captured as one HIP graph and replayed, 4096 near-money strikes per
instance (Section 2.1's Carr-Madan prices read out of the SFFT train).

Sampled outputs (the batch's first and last instance and fourteen drawn from the rest, 64
strikes spread over each window) are compared with the oracle's direct sums, one price at a
time, at the complex64 bound of 1e-4 S0; every one of the 16.7 M prices is checked against
the no-arbitrage bounds of a call, which hold at any size."""
import sys

import numpy as np
import pytest

import cm_workloads as W
from oracle import carr_madan as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2607_28435_amd as cm  # noqa: E402

C64_TOL = 1e-4
BATCH, N, NK = 4096, 24, 4096


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cm.lib()
    yield
    torch.cuda.synchronize()


def test_headline_workload_graph_replay_vs_oracle():
    say("headline workload: 4096 Heston instances, n = 24, graph replay")
    probs = W.heston_batch(BATCH, seed=20261203, n=N)
    strikes = np.stack([W.near_money(p, NK) for p in probs]).astype(np.int64)
    dev = torch.device("cuda")
    mpo = cm.MpoCache([N], 1e-9, 32, cm.CM_C64)
    pr = cm.SfftPricer(probs, cm.CM_C64, tol=1e-8, cap=32, mpo=mpo)
    pr.slots.update({"build": 4096, "apply": 1536, "round": 4096})
    pr.capture(torch.from_numpy(strikes).to(dev))
    for _ in range(2):
        pr.replay()
    torch.cuda.synchronize()
    got = pr.graph_prices.cpu().numpy()
    bad = {k: int((v != 0).sum()) for k, v in pr.statuses().items()}
    assert all(v == 0 for v in bad.values()), bad
    assert got.shape == (BATCH, NK) and np.isfinite(got).all()

    # no-arbitrage bounds of a European call on every price
    lo_b = np.empty_like(got)
    hi_b = np.empty_like(got)
    for b, p in enumerate(probs):
        K = O.strike_of(p, strikes[b])
        fwd = p.S0 * np.exp(-p.q * p.T)
        lo_b[b] = np.maximum(0.0, fwd - K * np.exp(-p.r * p.T))
        hi_b[b] = fwd
    S0 = np.array([p.S0 for p in probs])[:, None]
    assert (got >= lo_b - C64_TOL * S0).all(), float(((lo_b - got) / S0).max())
    assert (got <= hi_b + C64_TOL * S0).all(), float(((got - hi_b) / S0).max())

    # sampled prices against the oracle's direct sums
    rng = np.random.default_rng(20261204)
    inst = np.concatenate([[0, BATCH - 1], rng.choice(np.arange(1, BATCH - 1), 14, replace=False)])
    cols = np.linspace(0, NK - 1, 64).round().astype(int)
    worst = 0.0
    for b in inst:
        p = probs[b]
        ref = O.prices_direct(p, strikes[b, cols])
        worst = max(worst, float(np.abs(got[b, cols] - ref).max() / p.S0))
    say(f"headline workload: max |err| / S0 over {len(inst)} x {len(cols)} sampled prices = {worst:.3e}")
    assert worst < C64_TOL, worst


def test_ragged_workload_graph_replay_vs_oracle():
    """The ragged batch of the same draws with n ~ U{16..28} (the benchmark's ragged leg):
    longest chain first, graph replay; one sampled instance at every n against the oracle's
    direct sums on 64 strikes each, every price within the call's no-arbitrage bounds."""
    say("ragged workload: 4096 Heston instances, n = 16..28, graph replay")
    probs = W.heston_batch(BATCH, seed=20261203, n_range=(16, 28))
    ns = sorted(set(p.n for p in probs))
    assert ns == list(range(16, 29))
    strikes = np.stack([W.near_money(p, NK) for p in probs]).astype(np.int64)
    mpo = cm.MpoCache(ns, 1e-9, 32, cm.CM_C64)
    pr = cm.SfftPricer(probs, cm.CM_C64, tol=1e-8, cap=32, mpo=mpo)
    pr.capture(torch.from_numpy(strikes).cuda())
    for _ in range(2):
        pr.replay()
    torch.cuda.synchronize()
    got = pr.graph_prices.cpu().numpy()
    bad = {k: int((v != 0).sum()) for k, v in pr.statuses().items()}
    assert all(v == 0 for v in bad.values()), bad
    assert np.isfinite(got).all()
    for b, p in enumerate(probs):
        K = O.strike_of(p, strikes[b])
        fwd = p.S0 * np.exp(-p.q * p.T)
        lo_b = np.maximum(0.0, fwd - K * np.exp(-p.r * p.T))
        assert (got[b] >= lo_b - C64_TOL * p.S0).all() and (got[b] <= fwd + C64_TOL * p.S0).all(), b
    cols = np.linspace(0, NK - 1, 64).round().astype(int)
    worst = {}
    for n in ns:
        b = next(i for i, p in enumerate(probs) if p.n == n)
        ref = O.prices_direct(probs[b], strikes[b, cols])
        worst[n] = float(np.abs(got[b, cols] - ref).max() / probs[b].S0)
    say("ragged workload: max |err| / S0 per n:", {n: f"{e:.1e}" for n, e in worst.items()})
    assert max(worst.values()) < C64_TOL, worst

"""cm_sfft_apply_noalloc (the zip-up for callers that cannot allocate) against
cm_sfft_apply through the C ABI: two calls in a row, the second with a smaller input, each
bit-identical to the workspace entry point on the same trains (the same kernel computes
every instance independently of which persistent workgroup takes it), and the first call's
prices within 1e-4 S0 of the oracle."""
import sys

import numpy as np
import pytest

import cm_workloads as W
from oracle import carr_madan as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2607_28435_amd as cm  # noqa: E402


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


def _both(probs, dtype, tol, cap):
    """Builds x for the problems, then applies Q_n once through each entry point into two
    separate output batches; returns (pricer, y_workspace, y_noalloc, statuses)."""
    pr = cm.SfftPricer(probs, dtype, tol=tol, cap=cap)
    pr.build()
    y2 = cm.TTBatch(pr.ns, 2, 1, cap, dtype)
    st1 = torch.full((pr.batch,), -1, dtype=torch.int32, device="cuda")
    st2 = torch.full((pr.batch,), -1, dtype=torch.int32, device="cuda")
    cm.cm_sfft_apply(pr.mpo.w, pr.x, tol, cap, pr.y, st1, pr.ws)
    cm.cm_sfft_apply_noalloc(pr.mpo.w, pr.x, tol, cap, y2, st2)
    torch.cuda.synchronize()
    return pr, y2, st1.cpu().numpy(), st2.cpu().numpy()


def _same(a, b, ns):
    ra, rb = a.ranks.cpu().numpy(), b.ranks.cpu().numpy()
    for i, n in enumerate(ns):
        assert np.array_equal(ra[i, : n + 1], rb[i, : n + 1]), i
        ca, cb = a.host_cores(i), b.host_cores(i)
        assert all(np.array_equal(x, y) for x, y in zip(ca, cb)), i


def test_noalloc_apply_matches_workspace_entry_point_twice():
    scratch = cm.cm_sfft_apply_noalloc_scratch_bytes()
    slab = cm.cm_workspace_bytes(cm.CM_OP_SFFT_APPLY, 1, 24, 32, cm.CM_C64)
    say("scratch MiB", scratch / 2 ** 20, "slab MB", slab / 1e6, "workgroups", scratch // slab)
    assert scratch // slab >= 16
    # first call: a ragged complex64 Heston batch, more instances than the array's slabs
    probs = W.heston_batch(256, seed=77, n_range=(16, 24))
    pr, y2, st1, st2 = _both(probs, cm.CM_C64, 1e-8, 32)
    assert np.all(st1 == cm.CM_OK) and np.array_equal(st1, st2)
    _same(pr.y, y2, pr.ns)
    # the no-alloc output prices like the workspace one (round and read out from y2)
    pr.y.cores.copy_(y2.cores)
    pr.y.ranks.copy_(y2.ranks)
    pr.round()
    u = np.stack([W.near_money(p, 64) for p in pr.problems])
    prices = torch.empty(u.shape, dtype=torch.float64, device="cuda")
    pr.read(torch.from_numpy(u).cuda(), prices)
    got = prices.cpu().numpy()
    for b in range(0, pr.batch, 37):
        ref = O.prices_direct(pr.problems[b], u[b])
        assert np.abs(got[b] - ref).max() / pr.problems[b].S0 < 1e-4, b
    # second call: a smaller FP64 batch with shorter chains (the array keeps the first
    # call's contents; nothing of them may leak into this one)
    probs2 = [W.bs_rect_n12(), W.heston_n24().replace(n=14, eta=W.eta_rule(14)), W.bs_simpson_n12()]
    pr2, y2b, s1, s2 = _both(probs2, cm.CM_C128, 1e-10, 32)
    assert np.all(s1 == cm.CM_OK) and np.array_equal(s1, s2)
    _same(pr2.y, y2b, pr2.ns)

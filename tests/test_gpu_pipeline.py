"""Batched persistent run: workspace-sized launches, longest-chain-first ordering, the
slot autotuner and HIP-graph capture of the whole SFFT chain, all through the C ABI.

Every instance is priced by one workgroup whatever the slot count or order, so results
must be bit-identical across launch shapes, orderings and graph replays."""
import json
import sys

import numpy as np
import pytest

import cm_workloads as W
from oracle import carr_madan as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2607_28435_amd as cm  # noqa: E402

C64_TOL = 1e-4


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


def _ragged(count=12, seed=7):
    probs = W.heston_batch(count, seed=seed, n_range=(16, 22))
    strikes = torch.from_numpy(np.stack([W.near_money(p, 48) for p in probs])).cuda()
    return probs, strikes


def test_ragged_order_and_slots_bit_identical():
    """Longest-chain-first processing and 1, 3 or default persistent workgroups give the
    same prices as pricing each instance alone, bit for bit, in the caller's order."""
    say("ragged order/slots")
    probs, strikes = _ragged()
    assert len(set(p.n for p in probs)) > 1
    ref = cm.SfftPricer(probs, cm.CM_C64).run(strikes).cpu().numpy()
    for slots in (1, 3):
        pr = cm.SfftPricer(probs, cm.CM_C64, slots={"build": slots, "apply": slots, "round": slots})
        assert not pr.identity
        got = pr.run(strikes).cpu().numpy()
        assert np.array_equal(got, ref), slots
        for k, v in pr.statuses().items():
            assert np.all(v == cm.CM_OK), (k, v)
    for b in (0, 5, 11):
        alone = cm.SfftPricer([probs[b]], cm.CM_C64).run(strikes[b:b + 1]).cpu().numpy()[0]
        assert np.array_equal(alone, ref[b]), b
        oracle = O.prices_direct(probs[b], strikes[b].cpu().numpy())
        assert np.abs(ref[b] - oracle).max() / probs[b].S0 < C64_TOL


def test_graph_replay_matches_eager():
    """The captured chain (build, apply, round, readout, caller-order permutations) replays
    to the eager result, bit for bit, on every replay, with unrelated eager GPU work and
    synchronisations in between."""
    say("graph replay")
    probs, strikes = _ragged(seed=9)
    pr = cm.SfftPricer(probs, cm.CM_C64)
    eager = pr.run(strikes).cpu().numpy().copy()
    pr.capture(strikes)
    other_probs, other_strikes = _ragged(count=5, seed=10)
    other = cm.SfftPricer(other_probs, cm.CM_C64)
    other_ref = other.run(other_strikes).cpu().numpy().copy()
    for rep in range(3):
        out = pr.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), rep
        for k, v in pr.statuses().items():
            assert np.all(v == cm.CM_OK), (rep, k, v)
        # eager work between replays, including the same entry points on other buffers
        got_other = other.run(other_strikes).cpu().numpy()
        assert np.array_equal(got_other, other_ref)
        torch.cuda.synchronize()


def test_autotuner_picks_and_caches(tmp_path):
    """The slot autotuner times its candidates, keeps the fastest per sweep op, writes the
    choice to its JSON table and reads it back on the next call; prices are unchanged."""
    say("autotune")
    probs, strikes = _ragged(count=10, seed=12)
    pr = cm.SfftPricer(probs, cm.CM_C64)
    ref = pr.run(strikes).cpu().numpy().copy()
    path = str(tmp_path / "slots.json")
    best = cm.autotune_slots(pr, strikes, candidates=(1, 2, 10), reps=1, cache_path=path)
    assert set(best) == {"build", "apply", "round"}
    assert all(v in (1, 2, 10) for v in best.values())
    table = json.load(open(path))
    assert len(table) == 1 and list(table.values())[0] == best
    pr2 = cm.SfftPricer(probs, cm.CM_C64)
    again = cm.autotune_slots(pr2, strikes, candidates=(1, 2, 10), reps=1, cache_path=path)
    assert again == {**pr2.slots} and again == best
    assert np.array_equal(pr2.run(strikes).cpu().numpy(), ref)

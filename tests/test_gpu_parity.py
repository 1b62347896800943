"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances: FP64 paths <= 1e-6 S0 max abs price
error, complex64 paths <= 1e-4 S0, on the strike sets named in each test."""
import math
import sys

import numpy as np
import pytest

import cm_workloads as W
from oracle import carr_madan as O
from tests.tt_host import contract_mpo, contract_tt, right_orthonormality_error

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2607_28435_amd as cm  # noqa: E402

FP64_TOL = 1e-6
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


def _strikes_dev(idx_list):
    return torch.from_numpy(np.stack(idx_list).astype(np.int64)).cuda()


# ------------------------------------------------------------------ operator

@pytest.mark.parametrize("n", [1, 2, 4, 7, 10])
def test_qft_mpo_equals_bit_reversed_dft(n):
    say("mpo n", n)
    m = cm.MpoCache([n], 1e-13, 64, cm.CM_C128)
    cores = m.w.host_cores(n)
    Q = contract_mpo(cores)
    assert np.abs(Q - O.qn_matrix(n)).max() < 1e-11
    assert right_orthonormality_error(cores) < 1e-12


def test_qft_mpo_rank_is_small():
    """Section 3.2 quotes r_SFFT ~ 10; the rounded Q_n has bonds of that size."""
    say("mpo ranks")
    m = cm.MpoCache([12, 24], 1e-9, 64, cm.CM_C128)
    for n in (12, 24):
        rk = m.w.ranks[n].cpu().numpy()[: n + 1]
        assert 8 <= rk.max() <= 14, rk


@pytest.mark.parametrize("dtype", [cm.CM_C128, cm.CM_C64])
def test_mpo_table_bit_identical_to_single_builds(dtype):
    """One cm_qft_mpo_table launch for n = 1..14 gives, bit for bit, the operators that
    separate cm_qft_mpo calls give, and each is the bit-reversed DFT."""
    say("mpo table", dtype)
    tol = 1e-12 if dtype == cm.CM_C128 else 1e-7
    table = cm.MpoCache(range(1, 15), tol, 32, dtype)
    ws = cm.Workspace()
    for n in (1, 2, 5, 9, 14):
        single = cm.TTBatch([0] * n + [n], 2, 2, 32, dtype)
        cm.cm_qft_mpo(n, tol, 32, single, n, ws)
        a, b = table.w.host_cores(n), single.host_cores(n)
        assert len(a) == len(b) == n
        assert all(x.shape == y.shape and np.array_equal(x, y) for x, y in zip(a, b)), n
    for n in (3, 7, 10):
        err = np.abs(contract_mpo(table.w.host_cores(n)) - O.qn_matrix(n)).max()
        assert err < (1e-10 if dtype == cm.CM_C128 else 1e-5), (n, err)


def test_mpo_table_saved_and_loaded_prices_identically(tmp_path):
    """A table written to disk and loaded back prices bit-identically to the one built."""
    say("mpo table save/load")
    p = W.bs_rect_n12()
    m = cm.MpoCache([10, 11, 12], 1e-11, 32, cm.CM_C128)
    path = str(tmp_path / "q.npz")
    m.save(path)
    m2 = cm.MpoCache.load(path)
    u = _strikes_dev([W.all_strikes(p)])
    a = cm.SfftPricer([p], cm.CM_C128, tol=1e-10, cap=32, mpo=m).run(u).cpu().numpy()
    b = cm.SfftPricer([p], cm.CM_C128, tol=1e-10, cap=32, mpo=m2).run(u).cpu().numpy()
    assert np.array_equal(a, b)
    assert np.abs(a[0] - O.prices_dense(p)).max() / p.S0 < FP64_TOL


# ------------------------------------------------------------------ QTT of the integrand

@pytest.mark.parametrize("name", ["bs_rect", "bs_simpson", "heston16", "merton16", "heston_rect14", "vg16"])
def test_build_qtt_matches_integrand(name):
    say("qtt", name)
    p = {"bs_rect": W.bs_rect_n12(), "bs_simpson": W.bs_simpson_n12(),
         "heston16": W.heston_n24().replace(n=16),
         "merton16": W.merton_big(30).replace(n=16, eta=W.eta_rule(16)),
         "heston_rect14": W.heston_n24().replace(n=14, quad="rect2", eta=0.1),
         "vg16": W.vg_n20().replace(n=16, eta=W.eta_rule(16))}[name]
    pr = cm.SfftPricer([p], cm.CM_C128, tol=1e-10, cap=32)
    pr.build()
    torch.cuda.synchronize()
    assert pr.st_build.cpu().numpy()[0] == cm.CM_OK
    x = contract_tt(pr.x.host_cores(0))
    ref = O.integrand(p, np.arange(2 ** p.n))
    rel = np.linalg.norm(x - ref) / np.linalg.norm(ref)
    assert rel < 1e-9, rel
    assert right_orthonormality_error(pr.x.host_cores(0)) < 1e-10


# ------------------------------------------------------------------ full pipelines, FP64

def test_sfft_bs_n12_fp64_all_strikes():
    """Rectangle rule, FP64, tol 1e-10: every one of the 4096 prices within 1e-6 S0 of the
    oracle (and of the Black–Scholes formula)."""
    say("sfft bs n12 fp64")
    p = W.bs_rect_n12()
    pr = cm.SfftPricer([p], cm.CM_C128, tol=1e-10, cap=32)
    u = W.all_strikes(p)
    got = pr.run(_strikes_dev([u])).cpu().numpy()[0]
    st = pr.statuses()
    assert all(v[0] == cm.CM_OK for v in st.values()), st
    ref = O.prices_dense(p)
    assert np.abs(got - ref).max() / p.S0 < FP64_TOL, np.abs(got - ref).max()


def test_sfft_bs_n12_simpson_fp64():
    say("sfft bs simpson")
    p = W.bs_simpson_n12()
    pr = cm.SfftPricer([p], cm.CM_C128, tol=1e-10, cap=32)
    u = W.all_strikes(p)
    got = pr.run(_strikes_dev([u])).cpu().numpy()[0]
    ref = O.prices_dense(p)
    K = O.strike_of(p, u)
    win = (K >= 50) & (K <= 150)
    assert np.abs(got - ref)[win].max() / p.S0 < FP64_TOL
    # outside the window the Simpson alias makes prices huge; agreement is relative there
    big = np.abs(ref) > 1e3 * p.S0
    assert np.all(np.abs(got - ref)[big] <= 1e-6 * np.abs(ref)[big])


def test_readout_tree_and_per_strike_paths_fp64():
    """Readout of one FP64 SFFT train (BS rectangle rule, n = 16, tol 1e-10) through both
    readout paths: a contiguous near-money block (prefix tree: the block spans at most two
    values of u >> 12), the same block shuffled (still the tree), and a strided window (the
    per-strike contraction). All against the oracle's direct DFT."""
    p = W.bs_rect_n12().replace(n=16, eta=40.0 / 2 ** 8)
    strided = W.window_strided(p, 4096)
    near = W.near_money(p, len(strided))
    shuffled = np.random.default_rng(1).permutation(near)
    pr = cm.SfftPricer([p] * 3, cm.CM_C128, tol=1e-10, cap=32)
    got = pr.run(_strikes_dev([near, shuffled, strided])).cpu().numpy()
    st = pr.statuses()
    assert all(np.all(v == cm.CM_OK) for v in st.values()), st
    for row, u in zip(got, (near, shuffled, strided)):
        ref = O.prices_direct(p, u)
        assert np.abs(row - ref).max() / p.S0 < FP64_TOL
    assert np.allclose(got[1][np.argsort(shuffled)], got[0], rtol=0, atol=1e-12 * p.S0)


@pytest.mark.parametrize("quad", ["rect2", "simpson1"])
def test_dense_fft_fp64_n12_all_strikes(quad):
    say("dense fp64", quad)
    p = W.bs_rect_n12().replace(quad=quad)
    got, st = cm.dense_prices([p], cm.CM_C128)
    got = got.cpu().numpy()[0]
    assert st.cpu().numpy()[0] == cm.CM_OK
    ref = O.prices_dense(p)
    err = np.abs(got - ref)
    assert np.all(err <= FP64_TOL * p.S0 + 1e-12 * np.abs(ref)), err.max()


def _dft_roundoff_bound(p, rel=1e-13):
    """Per-strike bound on the price error that FP64 rounding of the DFT can cause:
    rel * sum_j |x_j| scaled by the readout factor exp(-alpha k_u)/(s pi)."""
    g = O.grid(p)
    u = np.arange(g.M)
    x1 = np.abs(O.integrand(p, u)).sum()
    return rel * x1 * np.exp(-p.alpha * g.k(u)) / (g.s * math.pi)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 9, 13, 14, 17])
def test_dense_fft_fp64_sizes(n):
    """Single- and multi-pass plans (ragged radix splits) against the oracle's FFT, within the
    FP64 rounding bound of the transform (the paper's grid spans extreme strikes where the
    factor exp(-alpha k) amplifies rounding; Section 4 notes the same)."""
    say("dense fp64 n", n)
    p = W.paper_bs_grid(n)
    got, st = cm.dense_prices([p], cm.CM_C128)
    ref = O.prices_dense(p)
    err = np.abs(got.cpu().numpy()[0] - ref)
    bound = _dft_roundoff_bound(p) + 1e-12 * p.S0
    assert np.all(err <= bound), (err / bound).max()


@pytest.mark.parametrize("dtype,n,eta", [(cm.CM_C128, 16, 2.0), (cm.CM_C128, 16, 0.25), (cm.CM_C128, 16, 0.05),
                                         (cm.CM_C128, 16, 0.002), (cm.CM_C64, 20, 0.1), (cm.CM_C64, 20, 0.01),
                                         (cm.CM_C64, 20, 0.0005)])
def test_dense_pruned_first_stages(dtype, n, eta):
    """Simpson rule (support of x starting at 0): from coarse to fine eta the support's share
    of each pass-1 work item crosses the thresholds at which the first three, two, one or no
    Stockham stages are written directly instead of computed (a single non-zero input per
    butterfly is only repeated). Every case matches the oracle: within the FP64 rounding
    bound on all strikes (complex128), within 1e-4 S0 on 0.5 <= K/S0 <= 1.5 (complex64)."""
    say("dense pruned", dtype, n, eta)
    p = W.bs_simpson_n12().replace(n=n, eta=eta)
    got, st = cm.dense_prices([p], dtype)
    assert st.cpu().numpy()[0] == cm.CM_OK
    got = got.double().cpu().numpy()[0]
    ref = O.prices_dense(p)
    err = np.abs(got - ref)
    if dtype == cm.CM_C128:
        # strikes where exp(-alpha k) overflows carry no price on either side
        bound = _dft_roundoff_bound(p) + 1e-12 * p.S0
        ok = np.isfinite(bound) & np.isfinite(ref)
        assert ok.sum() > 2 ** (n - 1) and np.all(np.isfinite(got[ok]))
        assert np.all(err[ok] <= bound[ok]), (err[ok] / bound[ok]).max()
    else:
        K = O.strike_of(p, np.arange(2 ** n))
        win = (K >= 50.0) & (K <= 150.0)
        assert win.sum() > 0 and err[win].max() / p.S0 < C64_TOL, err[win].max()


def test_paper_grid_statevector_pin_through_gpu():
    """The paper's grid (Section 4) priced on the GPU dense path reproduces the oracle's
    FFT NRMSE floor order (~1e-15) at n = 14."""
    p = W.paper_bs_grid(14)
    got, _ = cm.dense_prices([p], cm.CM_C128)
    u = np.arange(2 ** 14)
    K = O.strike_of(p, u)
    w = (K >= 50) & (K <= 150)
    e = O.nrmse(got.cpu().numpy()[0][w], O.bs_call(100.0, K[w], 0.05, 0.0, 0.5, 0.3), 100.0)
    assert e < 1e-13


@pytest.mark.parametrize("n", [20, 28])
def test_paper_grid_dense_fp64_floor(n):
    """Section 4.1's FFT arm on the GPU dense path in FP64: on the paper's grid the NRMSE
    against Black–Scholes over 0.5 <= K/S0 <= 1.5 stays at the FFT floor (the paper prints
    4.4e-15 for n > 12) also at n = 28, where k0 ~ -8e3 and lambda u cancel to the strike."""
    say("paper grid dense fp64 n", n)
    p = W.paper_bs_grid(n)
    got, _ = cm.dense_prices([p], cm.CM_C128)
    g = O.grid(p)
    lo = math.ceil((math.log(50.0) - g.k0) / g.lam)
    hi = math.floor((math.log(150.0) - g.k0) / g.lam)
    u = np.arange(lo, hi + 1, max(1, (hi - lo) // 100000))
    sel = got[0][torch.from_numpy(u).to(got.device)].cpu().numpy()
    del got
    ref = O.bs_call(100.0, O.strike_of(p, u), 0.05, 0.0, 0.5, 0.3)
    e = O.nrmse(sel, ref, 100.0)
    say("  nrmse", e)
    assert e < 4.4e-15


@pytest.mark.parametrize("n", [24, 32, 40])
def test_paper_grid_large_n_sfft(n):
    """The paper's two-sided grid (Section 4) at n = 24, 32 and 40 through the FP64 SFFT chain:
    the QTT build converges (its sample points are formed from exact index offsets, so the
    symmetric grid's large v0 does not cancel into the leaf tests) and the prices match the
    Black–Scholes formula over 0.5 <= K/S0 <= 1.5 to NRMSE 1e-11 at every n: the read-out's
    damping factor uses the exact grid strike k0 + 2 pi u / (M eta) (k0 is ~2^(n/2) away from
    the money on this grid, so a rounded lambda would add ~1e-11 at n = 40)."""
    say("paper grid sfft n", n)
    p = W.paper_bs_grid(n)
    lam = 2 * math.pi / (2 ** n * p.eta)
    lo = math.ceil((math.log(50.0) - p.k0) / lam)
    hi = math.floor((math.log(150.0) - p.k0) / lam)
    u = np.linspace(lo, hi, 4096).round().astype(np.int64)
    pr = cm.SfftPricer([p], cm.CM_C128, tol=1e-10, cap=64)
    got = pr.run(_strikes_dev([u])).cpu().numpy()[0]
    st = pr.statuses()
    assert all(v[0] == cm.CM_OK for v in st.values()), st
    ref = O.bs_call(100.0, O.strike_of(p, u), 0.05, 0.0, 0.5, 0.3)
    e = O.nrmse(got, ref, 100.0)
    say("  nrmse", e, "max", np.abs(got - ref).max() / 100)
    assert e < 1e-11 and np.abs(got - ref).max() / 100 < FP64_TOL


def test_dense_fft_fp64_batched_multi_instance_launch():
    """Four instances in one launch (n = 20, two passes): every instance against the oracle's
    direct DFT on strikes strided over 0.5 <= K/S0 <= 1.5."""
    probs = W.heston_batch(4, seed=11, n=20)
    got, st = cm.dense_prices(probs, cm.CM_C128)
    assert np.all(st.cpu().numpy() == cm.CM_OK)
    got = got.cpu().numpy()
    for b, p in enumerate(probs):
        u = W.window_strided(p, 256)
        ref = O.prices_direct(p, u)
        assert np.abs(got[b, u] - ref).max() / p.S0 < FP64_TOL


def test_dense_fft_failed_problem_is_nan():
    """A problem that fails its checks gets its status code and NaN prices; its neighbours in
    the batch are unaffected."""
    good = W.bs_simpson_n12()
    bad = good.replace(params=(-0.2,))
    got, st = cm.dense_prices([good, bad, good], cm.CM_C128)
    st = st.cpu().numpy()
    got = got.cpu().numpy()
    assert list(st) == [cm.CM_OK, cm.CM_E_INVALID, cm.CM_OK]
    assert np.isnan(got[1]).all()
    ref = O.prices_dense(good)
    for b in (0, 2):
        assert np.all(np.abs(got[b] - ref) <= FP64_TOL * good.S0 + 1e-12 * np.abs(ref))


# ------------------------------------------------------------------ complex64 paths

def test_heston_n24_c64_sfft_and_dense_vs_oracle():
    """Heston n = 24, eta = 0.05: SFFT (tol 1e-8, cap 64) and the dense Stockham FFT, both
    complex64, against the FP64 oracle on 4096 strikes strided through 0.5 <= K/S0 <= 1.5."""
    say("heston n24 c64")
    p = W.heston_n24()
    u = W.window_strided(p, 4096)
    ref = O.prices_direct(p, u)
    pr = cm.SfftPricer([p], cm.CM_C64, tol=1e-8, cap=64)
    got = pr.run(_strikes_dev([u])).cpu().numpy()[0]
    st = pr.statuses()
    assert all(v[0] == cm.CM_OK for v in st.values()), st
    e_sfft = np.abs(got - ref).max() / p.S0
    dense, _ = cm.dense_prices([p], cm.CM_C64, strikes=_strikes_dev([u]))
    e_dense = np.abs(dense.cpu().numpy()[0] - ref).max() / p.S0
    say("errors sfft", e_sfft, "dense", e_dense)
    assert e_sfft < C64_TOL and e_dense < C64_TOL


def test_dense_c64_heston_batch_n24_support_cut():
    """Eight seeded Heston draws at n = 24 through the complex64 dense path (integrand cut to
    its numerical support, maturities down to the box's shortest): sampled strikes over
    0.5 <= K/S0 <= 1.5 against the FP64 oracle."""
    probs = W.heston_batch(8, seed=5, n=24)
    got, st = cm.dense_prices(probs, cm.CM_C64)
    assert np.all(st.cpu().numpy() == cm.CM_OK)
    for b, p in enumerate(probs):
        u = W.window_strided(p, 128)
        ref = O.prices_direct(p, u)
        e = np.abs(got[b, torch.from_numpy(u).cuda()].double().cpu().numpy() - ref).max() / p.S0
        say("dense c64 n24 instance", b, "T", round(p.T, 3), "err", e)
        assert e < C64_TOL


def test_batched_heston_ragged_c64():
    """Seeded Heston draws over the batched parameter box with uneven n (16..20): every
    instance within 1e-4 S0 of the oracle on 64 near-money strikes."""
    say("batched heston")
    probs = W.heston_batch(24, seed=5, n_range=(16, 20))
    u = [W.near_money(p, 64) for p in probs]
    pr = cm.SfftPricer(probs, cm.CM_C64, tol=1e-8, cap=32)
    got = pr.run(_strikes_dev(u)).cpu().numpy()
    st = pr.statuses()
    for k, v in st.items():
        assert np.all(v == cm.CM_OK), (k, v)
    for b, p in enumerate(probs):
        ref = O.prices_direct(p, u[b])
        assert np.abs(got[b] - ref).max() / p.S0 < C64_TOL, (b, p)


def _oracle_rows(probs, strikes):
    """The oracle's direct-sum prices of every instance (threads over instances: the sums
    are vectorised numpy, which releases the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(8) as ex:
        return list(ex.map(lambda a: O.prices_direct(a[0], a[1]), zip(probs, strikes)))


def test_batched_heston_ragged_c64_every_n_16_to_28():
    """The batched configuration's whole range of chain lengths in one ragged batch: two
    seeded draws from the Heston box at every n in 16..28 (complex64 contraction, FP64
    factorisations, tol 1e-8, bond cap 64), 256 near-money strikes each, every price within
    1e-4 S0 of the oracle's FP64 direct sum. Cost grows linearly in n (Eq. complexity_TTO),
    so n = 28 is the configuration's hardest chain."""
    probs = []
    for n in range(16, 29):
        probs += W.heston_batch(2, seed=700 + n, n=n)
    u = [W.near_money(p, 256) for p in probs]
    say("ragged n=16..28:", len(probs), "instances")
    pr = cm.SfftPricer(probs, cm.CM_C64, tol=1e-8, cap=64)
    got = pr.run(_strikes_dev(u)).cpu().numpy()
    for k, v in pr.statuses().items():
        assert np.all(v == cm.CM_OK), (k, v)
    refs = _oracle_rows(probs, u)
    worst = 0.0
    for b, p in enumerate(probs):
        e = np.abs(got[b] - refs[b]).max() / p.S0
        worst = max(worst, e)
        assert e < C64_TOL, (b, p.n, e)
    say("  worst error / S0", worst)


def test_dense_c64_merton_n30_vs_series():
    """The dense complex64 Stockham path on the 2^30-point Merton grid (8 GiB per pass
    buffer, three passes), gathered at 4096 near-money strikes, against the Merton series."""
    say("dense merton n30")
    p = W.merton_big(30)
    u = W.near_money(p, 4096)
    got, st = cm.dense_prices([p], cm.CM_C64, strikes=_strikes_dev([u]))
    assert st.cpu().numpy()[0] == cm.CM_OK
    ref = O.merton_call(p, O.strike_of(p, u))
    e = np.abs(got.double().cpu().numpy()[0] - ref).max() / p.S0
    say("  max error / S0", e)
    assert e < C64_TOL


@pytest.mark.parametrize("kappa,sv,rho", [(0.5, 0.8, 0.5), (0.05, 0.3, 0.99), (4.0, 0.1, -0.5)],
                         ids=["D<0,k>0", "D>=0,k>0", "D>=0,k<0"])
def test_heston_moment_status_every_branch(kappa, sv, rho):
    """The device's moment check (Eq. damping_moment_condition via the explosion time)
    agrees with the oracle's T* on every branch: instances at 0.5 T* and 0.95 T* price (the
    first against the oracle), one at 1.05 T* reports CM_E_MOMENT; with an infinite T*
    every maturity prices. Both the SFFT build and the dense path."""
    om = 2.5
    Ts = O.heston_explosion_time(kappa, sv, rho, om)
    Tm = [0.5 * Ts, 0.95 * Ts, 1.05 * Ts] if math.isfinite(Ts) else [0.5, 5.0, 30.0]
    want = [cm.CM_OK, cm.CM_OK, cm.CM_E_MOMENT] if math.isfinite(Ts) else [cm.CM_OK] * 3
    base = W.Problem("heston", "simpson1", 12, 100.0, 0.03, 0.0, 1.0, 1.5, 0.25, (kappa, 0.04, sv, rho, 0.04))
    probs = [base.replace(T=float(T)) for T in Tm]
    say("T* =", Ts, "maturities", Tm)
    pr = cm.SfftPricer(probs, cm.CM_C128, tol=1e-10, cap=32)
    u = np.stack([W.near_money(base, 16)] * 3)
    got = pr.run(torch.from_numpy(u).cuda()).cpu().numpy()
    assert pr.statuses()["build"].tolist() == want
    _, dst = cm.dense_prices(probs, cm.CM_C128)
    assert dst.cpu().numpy().tolist() == want
    ref = O.prices_direct(probs[0], u[0])
    assert np.abs(got[0] - ref).max() / base.S0 < FP64_TOL


@pytest.mark.parametrize("n", [30, 40])
def test_merton_large_grid_vs_series(n):
    """Merton, n = 30 and 40 (the 2^40 grid is never materialised): SFFT complex64 prices at
    4096 near-money strikes against the Merton series."""
    say("merton n", n)
    p = W.merton_big(n)
    u = W.near_money(p, 4096)
    pr = cm.SfftPricer([p], cm.CM_C64, tol=1e-8, cap=32)
    got = pr.run(_strikes_dev([u])).cpu().numpy()[0]
    st = pr.statuses()
    assert all(v[0] == cm.CM_OK for v in st.values()), st
    ref = O.merton_call(p, O.strike_of(p, u))
    assert np.abs(got - ref).max() / p.S0 < C64_TOL


def test_vg_fp64_sfft_and_dense_window():
    """Variance Gamma (the model the paper names for its time-changed Brownian motion),
    n = 16, FP64 SFFT at tol 1e-10 and the FP64 dense FFT against the oracle's dense
    Carr–Madan prices on 4096 strikes strided through 0.5 <= K/S0 <= 1.5 (far from the money
    e^{-alpha k} magnifies any transform error by up to e^{23} on this grid, so every FP64
    test past n = 12 compares on a strike window)."""
    say("vg n16 fp64")
    p = W.vg_n20().replace(n=16, eta=W.eta_rule(16))
    u = W.window_strided(p, 4096)
    ref = O.prices_dense(p)[u]
    pr = cm.SfftPricer([p], cm.CM_C128, tol=1e-10, cap=32)
    got = pr.run(_strikes_dev([u])).cpu().numpy()[0]
    st = pr.statuses()
    assert all(v[0] == cm.CM_OK for v in st.values()), st
    dense, _ = cm.dense_prices([p], cm.CM_C128)
    e_sfft = np.abs(got - ref).max() / p.S0
    e_dense = np.abs(dense.cpu().numpy()[0][u] - ref).max() / p.S0
    say("errors sfft", e_sfft, "dense", e_dense, "y ranks", pr.y.ranks[0, : p.n + 1].tolist())
    assert e_sfft < FP64_TOL and e_dense < FP64_TOL


def test_vg_batch_c64_n20_vs_oracle_and_gamma_mixture():
    """Eight seeded Variance Gamma draws at n = 20 through the complex64 SFFT chain: 64
    near-money strikes each within 1e-4 S0 of the oracle, and the first draw's prices
    against the gamma mixture of Black–Scholes prices."""
    say("vg batch c64")
    probs = W.vg_batch(8, seed=31, n=20)
    u = [W.near_money(p, 64) for p in probs]
    pr = cm.SfftPricer(probs, cm.CM_C64, tol=1e-8, cap=32)
    got = pr.run(_strikes_dev(u)).cpu().numpy()
    st = pr.statuses()
    for k, v in st.items():
        assert np.all(v == cm.CM_OK), (k, v)
    for b, p in enumerate(probs):
        ref = O.prices_direct(p, u[b])
        assert np.abs(got[b] - ref).max() / p.S0 < C64_TOL, (b, p)
    sel = u[0][::16]
    mix = O.vg_call_gamma_mixture(probs[0], O.strike_of(probs[0], sel))
    assert np.abs(got[0][::16] - mix).max() / probs[0].S0 < C64_TOL


def test_vg_status_codes():
    """Variance Gamma validation: a non-positive variance rate is invalid, and a positive
    drift that makes E[S_T^(alpha+1)] infinite reports the moment condition; the valid
    instance in the same batch is priced."""
    say("vg status")
    good = W.vg_n20().replace(n=12, eta=0.25)
    bad_nu = good.replace(params=(0.12, -0.1, -0.14))
    moment = good.replace(params=(0.3, 0.9, 0.5))
    pr = cm.SfftPricer([good, bad_nu, moment], cm.CM_C128, tol=1e-10, cap=32)
    u = np.stack([W.near_money(good, 16)] * 3)
    got = pr.run(torch.from_numpy(u).cuda()).cpu().numpy()
    st = pr.statuses()
    assert st["build"].tolist() == [cm.CM_OK, cm.CM_E_INVALID, cm.CM_E_MOMENT]
    ref = O.prices_direct(good, u[0])
    assert np.abs(got[0] - ref).max() / good.S0 < FP64_TOL
    _, dst = cm.dense_prices([good, bad_nu, moment], cm.CM_C128)
    assert dst.cpu().numpy().tolist() == [cm.CM_OK, cm.CM_E_INVALID, cm.CM_E_MOMENT]


@pytest.mark.parametrize("name", ["heston20_tol1e-12", "bs12rect_tol1e-13"])
def test_zipup_site_paths_fp64(name):
    """The zip-up compiles its register-resident pivot loop with two lanes per column for 8,
    12, 16 and 24 slots per lane (2 chi <= 16, 24, 32, 48), with four or eight lanes per
    column for sites with w' r' <= 64 or <= 32, and takes an LDS path above 2 chi = 48.
    Heston at n = 20 and tol 1e-12 carries bonds from 1 to 24 (the narrow sites take the wide
    groups, the rest every two-lane loop); the rectangle-rule Black–Scholes grid at tol 1e-13
    reaches bonds above 24 (the LDS path). Prices through the whole chain against the
    oracle; the complex64 batch tests cover the wide groups at typical ranks."""
    say("zip-up site paths", name)
    p, tol = {"heston20_tol1e-12": (W.heston_n24().replace(n=20, eta=W.eta_rule(20)), 1e-12),
              "bs12rect_tol1e-13": (W.bs_rect_n12(), 1e-13)}[name]
    pr = cm.SfftPricer([p], cm.CM_C128, tol=tol, cap=48)
    pr.build()
    pr.apply()
    torch.cuda.synchronize()
    chi = pr.y.ranks[0, : p.n].cpu().numpy()   # carried bond entering each site
    if name.startswith("heston"):
        for lo, hi in ((1, 8), (9, 12), (13, 16), (17, 24)):
            assert np.any((chi >= lo) & (chi <= hi)), (lo, hi, chi)
    else:
        assert chi.max() > 24, chi
    pr.round()
    u = W.near_money(p, 256)
    prices = torch.empty((1, len(u)), dtype=torch.float64, device="cuda")
    pr.read(_strikes_dev([u]), prices)
    for k, v in pr.statuses().items():
        assert np.all(v == cm.CM_OK), (k, v)
    ref = O.prices_direct(p, u)
    assert np.abs(prices.cpu().numpy()[0] - ref).max() / p.S0 < FP64_TOL


@pytest.mark.parametrize("dtype,tol,gate", [(cm.CM_C128, 1e-10, FP64_TOL), (cm.CM_C64, 1e-8, C64_TOL)],
                         ids=["c128", "c64"])
def test_vg_short_clock_prices(dtype, tol, gate):
    """A Variance Gamma instance whose gamma clock is short (T/nu = 0.18, so x decays only
    like |v|^-0.36 and has no negligible tail) builds without error; its prices match the
    oracle's direct sum and the gamma mixture of Black–Scholes prices."""
    say("vg short clock", dtype)
    p = W.vg_short_clock(20)
    u = W.near_money(p, 64)
    pr = cm.SfftPricer([p], dtype, tol=tol, cap=32)
    got = pr.run(_strikes_dev([u])).cpu().numpy()[0]
    for k, v in pr.statuses().items():
        assert np.all(v == cm.CM_OK), (k, v)
    sel = u[::4]
    assert np.abs(got[::4] - O.prices_direct(p, sel)).max() / p.S0 < gate
    mix = O.vg_call_gamma_mixture(p, O.strike_of(p, u[::8]))
    assert np.abs(got[::8] - mix).max() / p.S0 < gate


def test_unresolved_structure_reports_noconv():
    """An instance whose characteristic function has more structure than the QTT build's
    per-depth interval limits resolve (Merton with near-deterministic jumps and almost no
    diffusion) is reported per instance (CM_E_NOCONV; its train is left as the zero train)
    without disturbing its neighbour in the batch."""
    say("unresolved structure")
    good = W.vg_n20().replace(n=24, eta=W.eta_rule(24))
    bad = W.merton_oscillating()
    pr = cm.SfftPricer([good, bad], cm.CM_C64, tol=1e-8, cap=32)
    u = np.stack([W.near_money(good, 64), W.near_money(bad, 64)])
    got = pr.run(torch.from_numpy(u).cuda()).cpu().numpy()
    st = pr.statuses()
    assert st["build"].tolist() == [cm.CM_OK, cm.CM_E_NOCONV]
    assert np.abs(got[0] - O.prices_direct(good, u[0])).max() / good.S0 < C64_TOL


# ------------------------------------------------------------------ status codes and edges

def test_status_codes_per_instance():
    say("status codes")
    good = W.bs_simpson_n12()
    bad_sigma = good.replace(params=(-0.2,))
    # Heston draw whose E[S^(alpha+1)] explodes before T (kappa 0.5, sigma_v 0.8, rho -0.1)
    moment = W.Problem("heston", "simpson1", 12, 100.0, 0.03, 0.0, 4.0, 1.5, 0.25, (0.5, 0.04, 0.8, -0.1, 0.04))
    pr = cm.SfftPricer([good, bad_sigma, moment], cm.CM_C128, tol=1e-10, cap=32)
    u = np.stack([W.near_money(good, 16)] * 3)
    u[0, 3] = 2 ** 12 + 5   # out of range strike for instance 0
    got = pr.run(torch.from_numpy(u).cuda()).cpu().numpy()
    st = pr.statuses()
    assert st["build"][0] == cm.CM_OK
    assert st["build"][1] == cm.CM_E_INVALID
    assert st["build"][2] == cm.CM_E_MOMENT
    assert st["read"][0] == cm.CM_E_INVALID and math.isnan(got[0, 3])
    ok = np.delete(np.arange(16), 3)
    ref = O.prices_direct(good, u[0, ok])
    assert np.abs(got[0, ok] - ref).max() / 100 < FP64_TOL


def test_call_level_errors():
    good = W.bs_simpson_n12()
    pr = cm.SfftPricer([good], cm.CM_C128, tol=1e-10, cap=32)
    with pytest.raises(cm.CmError) as e:
        cm.cm_build_qtt(pr.prob, 1, 1e-10, 65, pr.x, pr.st_build, pr.ws)
    assert e.value.code == cm.CM_E_INVALID
    with pytest.raises(cm.CmError):
        cm.cm_tt_round(pr.x, -1.0, 8, None, None, pr.ws)

"""Standalone pins of the SFFT step and of TT rounding through the C ABI (no pricing chain):
the zip-up against the plain DFT (Eq. dft, Section 3.2) on trains written from the host,
the plane-wave special case, Parseval, and the rounding bound of Section 3.1.

Host trains are right-orthonormalised with numpy before the zip-up (the form
cm_sfft_apply expects of its input); expected values come from the oracle's FFT of the
densely contracted input, never from the GPU."""
import math
import sys

import numpy as np
import pytest

from oracle import carr_madan as O
from tests.tt_host import (bitrev_perm, contract_mpo, contract_tt, random_train, right_orthonormality_error,
                           right_orthonormalize, tt_eval, upload_train)

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


def _apply(w, xs, dtype, tol, cap):
    """Uploads host trains xs (right-orthonormal) and runs cm_sfft_apply with the operators
    of batch w (train n is the operator for chain length n); returns the output batch and
    the statuses."""
    ns = [len(c) for c in xs]
    x = cm.TTBatch(ns, 2, 1, cap, dtype)
    y = cm.TTBatch(ns, 2, 1, cap, dtype)
    for b, cores in enumerate(xs):
        upload_train(x, b, cores, cm.CM_TT_RIGHT_ORTHO)
    st = torch.full((len(xs),), -1, dtype=torch.int32, device="cuda")
    cm.cm_sfft_apply(w, x, tol, cap, y, st, cm.Workspace())
    torch.cuda.synchronize()
    return x, y, st.cpu().numpy()


def _exact_y(cores):
    """The plain definition: y = M^-1/2 DFT_-(x) of the dense input (the oracle's FFT),
    listed in the order a contraction of the output train gives (output core l carries
    bit 2^l of u, core 0 slowest: dense position bitrev(u))."""
    x = contract_tt(cores)
    n = len(cores)
    y = O.dft_fft(x)
    return y[bitrev_perm(n)], x


@pytest.mark.parametrize("dtype", [cm.CM_C128, cm.CM_C64], ids=["c128", "c64"])
def test_zipup_register_site_with_output_bond_above_32(dtype):
    """The zip-up's contraction and pivoted-QR factorisation for a general operator: a
    random right-orthonormal operator (bonds up to 12) applied to a random train whose bond
    doubles from 2 to 4 at site 5. Generic ranks make site 5 take the register-resident
    path with carry 20 (2 chi = 40 <= 48, w' r' = 48 <= 128) and keep k = 40 > 32 columns;
    the output train must equal the dense operator times the dense input."""
    n, cap = 12, 48
    wb = [1, 2, 4, 8, 10, 10, 12, 12, 10, 8, 4, 2, 1]
    xb = [1, 2, 2, 2, 2, 2, 4, 4, 4, 4, 4, 2, 1]
    rng = np.random.default_rng(12)
    Wc = right_orthonormalize(random_train(rng, wb, d=4))
    xs = right_orthonormalize(random_train(rng, xb))
    assert right_orthonormality_error(Wc) < 1e-12 and right_orthonormality_error(xs) < 1e-12
    w = cm.TTBatch([0] * n + [n], 2, 2, cap, dtype)
    upload_train(w, n, Wc, cm.CM_TT_RIGHT_ORTHO)
    x, y, st = _apply(w, [xs], dtype, 1e-13 if dtype == cm.CM_C128 else 1e-7, cap)
    assert st[0] == cm.CM_OK, st
    chi = y.ranks[0, : n + 1].cpu().numpy()
    say("y bonds", chi.tolist())
    assert chi[5] == 20 and chi[6] == 40, chi
    ref = contract_mpo(Wc) @ contract_tt(xs)
    got = contract_tt(y.host_cores(0))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say("max rel err", err)
    assert err < (1e-10 if dtype == cm.CM_C128 else 1e-5)


@pytest.mark.parametrize("dtype,n,tol,round_tol", [(cm.CM_C128, 12, 1e-10, 1e-10), (cm.CM_C128, 20, 1e-10, 1e-10),
                                                   (cm.CM_C64, 24, 1e-6, 1e-4)],
                         ids=["c128-n12", "c128-n20", "c64-n24"])
def test_plane_wave_goes_to_rank_one_delta(dtype, n, tol, round_tol):
    """A plane wave x_j = exp(2 pi i j m / M) is an exact rank-1 train (core l carries the
    factor exp(2 pi i m 2^(n-1-l) / M) for bit 1); its transform is sqrt(M) delta_{u,m}, again
    of rank 1, found by the output train at the bit-reversed position of m (Section 3.2:
    Q_n omits the bit reversal). In complex64 the operator's truncation error (relative
    Frobenius 1e-7, which for a single Fourier mode need not spread evenly) and FP32
    rounding leave second singular values just above a 1e-6 rounding threshold, so the rank
    is checked after rounding at the complex64 tolerance class (1e-4)."""
    M = 2 ** n
    rng = np.random.default_rng(n)
    ms = [int(rng.integers(0, M)) for _ in range(3)] + [0, M - 1]
    xs = []
    for m in ms:
        cores = []
        for l in range(n):
            f = np.exp(2j * math.pi * ((m * (1 << (n - 1 - l))) % M) / M)
            cores.append(np.array([1.0, f], dtype=np.complex128).reshape(1, 2, 1) / math.sqrt(2))
        cores[0] = cores[0] * math.sqrt(2) ** n   # norm of x is sqrt(M), right cores orthonormal
        xs.append(cores)
    mpo = cm.MpoCache([n], tol / 10, 32, dtype)
    x, y, st = _apply(mpo.w, xs, dtype, tol, 32)
    assert np.all(st == cm.CM_OK), st
    err = torch.zeros(len(xs), dtype=torch.float64, device="cuda")
    rst = torch.zeros(len(xs), dtype=torch.int32, device="cuda")
    cm.cm_tt_round(y, round_tol, 32, err, rst, cm.Workspace())
    torch.cuda.synchronize()
    assert np.all(rst.cpu().numpy() == cm.CM_OK)
    rk = y.ranks.cpu().numpy()[:, : n + 1]
    say("ranks after rounding", rk.max(axis=1).tolist())
    assert np.all(rk == 1), rk
    brv = lambda v: int(format(v, f"0{n}b")[::-1], 2)
    gate = 1e-8 if dtype == cm.CM_C128 else 1e-4
    for b, m in enumerate(ms):
        cores = y.host_cores(b)
        # the single non-zero entry: bits of m, output core l carrying bit 2^l
        peak = tt_eval(cores, [(m >> l) & 1 for l in range(n)])
        assert abs(abs(peak) - math.sqrt(M)) < gate * math.sqrt(M), (m, peak)
        assert abs(peak.imag) < gate * math.sqrt(M)
        # another strike (m xor 1 differs in bit 0) sees nothing
        other = tt_eval(cores, [((m ^ 1) >> l) & 1 for l in range(n)])
        assert abs(other) < gate * math.sqrt(M)
        if n <= 12:
            dense = contract_tt(cores)
            ref = np.zeros(M, dtype=np.complex128)
            ref[brv(m)] = math.sqrt(M)
            assert np.abs(dense - ref).max() < gate * math.sqrt(M)


@pytest.mark.parametrize("dtype", [cm.CM_C128, cm.CM_C64], ids=["c128", "c64"])
def test_zipup_random_trains_dft_and_parseval(dtype):
    """A ragged batch of random right-orthonormal trains (n = 6..14, bonds up to 3): each
    output equals the DFT of its input to the operator's tolerance, and ||y|| = ||x||
    (Parseval; Q_n is unitary)."""
    rng = np.random.default_rng(5)
    ns = [6, 9, 11, 14, 12, 8]
    xs = []
    for n in ns:
        ranks = [1] + [min(3, 2 ** i, 2 ** (n - i)) for i in range(1, n)] + [1]
        xs.append(right_orthonormalize(random_train(rng, ranks)))
    tol, mtol, gate = (1e-12, 1e-13, 1e-9) if dtype == cm.CM_C128 else (1e-6, 1e-7, 2e-5)
    mpo = cm.MpoCache(ns, mtol, 48, dtype)
    x, y, st = _apply(mpo.w, xs, dtype, tol, 48)
    assert np.all(st == cm.CM_OK), st
    for b, cores in enumerate(xs):
        ref, xd = _exact_y(cores)
        got = contract_tt(y.host_cores(b))
        nx = np.linalg.norm(xd)
        say("n", ns[b], "rel err", np.abs(got - ref).max() / nx, "norm ratio", np.linalg.norm(got) / nx)
        assert np.linalg.norm(got - ref) < gate * nx
        assert abs(np.linalg.norm(got) - nx) < gate * nx


def _left_orthonormalize(cores):
    """Cores 0..n-2 left-orthonormal (mirror of right_orthonormalize); bond l shrinks to at
    most 2^l, the capacity layout's bound."""
    rev = right_orthonormalize([c.transpose(2, 1, 0) for c in cores[::-1]])
    return [c.transpose(2, 1, 0) for c in rev[::-1]]


def _decaying_train(rng, n, terms, ratio):
    """sum_t ratio^t (random rank-1 train t), written as one train of bond `terms` with
    block-diagonal interior cores: its unfoldings have singular values that fall roughly
    geometrically, so rounding at a tolerance drops a known tail. Returned left-orthonormal
    (exact), which also brings the bonds within 2^l."""
    rank1 = [random_train(rng, [1] * (n + 1)) for _ in range(terms)]
    cores = []
    for l in range(n):
        r0 = 1 if l == 0 else terms
        r1 = 1 if l == n - 1 else terms
        G = np.zeros((r0, 2, r1), dtype=np.complex128)
        for t in range(terms):
            a = 0 if l == 0 else t
            c = 0 if l == n - 1 else t
            G[a, :, c] += rank1[t][l][0, :, 0] * (ratio ** t if l == 0 else 1.0)
        cores.append(G)
    return _left_orthonormalize(cores)


@pytest.mark.parametrize("dtype", [cm.CM_C128, cm.CM_C64], ids=["c128", "c64"])
@pytest.mark.parametrize("tol", [1e-2, 1e-4])
def test_tt_round_bound_and_err_out(dtype, tol):
    """Rounding (Section 3.1) of random trains, and of a left-orthonormal train flagged as
    such (the first sweep skipped): the achieved relative Frobenius error stays within tol
    (Oseledets' bound), err_out reports it (never below the achieved error, up to the
    storage rounding), bonds shrink, and the result is right-orthonormal."""
    rng = np.random.default_rng(int(-math.log10(tol)) + 10 * dtype)
    ns = [10, 7, 12, 10]
    trains = [_decaying_train(rng, n, 12, 0.3) for n in ns[:2]] + \
             [random_train(rng, [1] + [min(8, 2 ** i, 2 ** (n - i)) for i in range(1, n)] + [1]) for n in ns[2:]]
    trains[3] = _left_orthonormalize(trains[3])
    out = {}
    for sel, flags in (((0, 1, 2), 0), ((3,), cm.CM_TT_LEFT_ORTHO)):
        sub = cm.TTBatch([ns[b] for b in sel], 2, 1, 32, dtype)
        for i, b in enumerate(sel):
            upload_train(sub, i, trains[b])
        sub.struct.flags = flags
        before = [contract_tt(sub.host_cores(i)) for i in range(len(sel))]   # as stored
        e = torch.zeros(len(sel), dtype=torch.float64, device="cuda")
        s = torch.zeros(len(sel), dtype=torch.int32, device="cuda")
        cm.cm_tt_round(sub, tol, 32, e, s, cm.Workspace())
        torch.cuda.synchronize()
        for i, b in enumerate(sel):
            out[b] = (before[i], sub.host_cores(i), float(e[i]), int(s[i]), sub.ranks[i, : ns[b] + 1].cpu().numpy())
    store = 1e-14 if dtype == cm.CM_C128 else 3e-7
    for b in range(len(ns)):
        A, cores, e_out, code, rk = out[b]
        assert code == cm.CM_OK
        At = contract_tt(cores)
        rel = np.linalg.norm(A - At) / np.linalg.norm(A)
        say("train", b, "n", ns[b], "tol", tol, "achieved", rel, "err_out", e_out, "bonds", rk.max())
        assert rel <= tol * (1 + 1e-9) + store
        assert e_out <= tol * (1 + 1e-12)
        assert rel <= e_out * (1 + 1e-6) + store
        assert right_orthonormality_error(cores) < (1e-12 if dtype == cm.CM_C128 else 1e-5)
        if b < 2:
            assert rk.max() < 12   # the geometric tail was dropped

"""Pins of the CPU oracle against facts that do not come from the oracle itself:
numbers printed in the paper, closed-form prices, an ODE integration of the Heston
characteristic function, quadrature exactness, and a gate-by-gate QFT circuit."""
import math
import os

import numpy as np
import pytest
from scipy import integrate

import cm_workloads as W
from oracle import carr_madan as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.txt")


def _golden(key):
    out = {}
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, n, v, d = line.split()
        if k == key:
            out[int(n)] = (float(v), int(d))
    return out


def _window(p, lo=50.0, hi=150.0):
    u = np.arange(2 ** p.n)
    K = O.strike_of(p, u)
    m = (K >= lo) & (K <= hi)
    return u[m], K[m]


# ------------------------------------------------------------------ paper-printed numbers

def test_statevector_nrmse_matches_paper_printed_values():
    """Section 4.2 prints the statevector NRMSE at n = 3, 4, 5; the oracle's grid, psi,
    DFT and sqrt(p) reconstruction must reproduce them to the printed digits."""
    for n, (val, digits) in _golden("statevector_nrmse").items():
        p = W.paper_bs_grid(n)
        u, K = _window(p)
        C = O.qft_observable_prices(p, u)
        e = O.nrmse(C, O.bs_call(100.0, K, 0.05, 0.0, 0.5, 0.3), 100.0)
        half_ulp = 0.5 * 10 ** (math.floor(math.log10(val)) - (digits - 1))
        assert abs(e - val) <= half_ulp, (n, e, val)


def test_sampler_point_mass_and_uniform():
    """A point mass always yields its outcome; under the uniform law bit t is just
    U_t >= 1/2 (bit 0 has weight 1)."""
    g = np.random.default_rng(5)
    U = g.random((500, 6))
    pm = np.zeros(64)
    pm[37] = 1.0
    assert np.all(O.sample_outcomes(pm, U) == 37)
    ref = (U >= 0.5).astype(np.int64) @ (2 ** np.arange(6))
    assert np.array_equal(O.sample_outcomes(np.full(64, 1 / 64), U), ref)


def test_sampler_independent_bits_closed_form():
    """For a law with independent bits, P(bit t = 1) = theta_t, the rule 'bit t is 1 iff
    U_t (q0 + q1) >= q0' sets bit t exactly when U_t >= 1 - theta_t."""
    g = np.random.default_rng(6)
    th = g.uniform(0.1, 0.9, 7)
    u = np.arange(128)
    bits = (u[:, None] >> np.arange(7)) & 1
    prob = np.prod(np.where(bits == 1, th, 1 - th), axis=1)
    U = g.random((2000, 7))
    ref = (U >= 1 - th).astype(np.int64) @ (2 ** np.arange(7))
    got = O.sample_outcomes(prob, U)
    # outcomes agree except where U_t sits within rounding of the threshold
    assert np.mean(got == ref) > 0.999


def test_sampler_frequencies():
    """Empirical frequencies of many shots from a random law stay within 5 standard errors."""
    g = np.random.default_rng(7)
    prob = g.random(32) ** 3
    prob /= prob.sum()
    R = 200000
    s = O.sample_outcomes(prob, g.random((R, 5)))
    f = np.bincount(s, minlength=32) / R
    assert np.all(np.abs(f - prob) <= 5 * np.sqrt(prob * (1 - prob) / R) + 1e-12)


def test_shot_prices_equal_statevector_prices_for_exact_counts():
    """When every outcome is counted in exact proportion R_l = R p_l, the shot estimator
    (Eqs. qft_probability_estimator, qft_observable_price) equals the exact-probability
    observable prices of the statevector readout; and shot_prices counts samples."""
    p = W.paper_bs_grid(5)
    prob, nx2 = O.qft_probabilities(p)
    u = np.arange(2 ** 5)
    R = 1e9
    got = O.prices_from_counts(p, u, prob * R, R, nx2)
    ref = O.qft_observable_prices(p, u)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    samples = np.array([3, 7, 7, 3, 3, 30, 7, 3])
    c = O.shot_prices(p, samples, np.array([3, 7, 30, 31]), 2.0)
    assert np.allclose(c, O.prices_from_counts(p, np.array([3, 7, 30, 31]), np.array([4, 3, 1, 0]), 8, 2.0), rtol=1e-15)


def test_statevector_n3_discriminates_readout():
    """At n=3 the Re(.) readout differs from the sqrt(p) readout beyond the printed digits,
    so the pin above really fixes the reconstruction formula."""
    p = W.paper_bs_grid(3)
    u, K = _window(p)
    C = O.prices_dense(p)[u]
    e = O.nrmse(C, O.bs_call(100.0, K, 0.05, 0.0, 0.5, 0.3), 100.0)
    assert abs(e - 9.30e-3) > 0.5e-5


def test_fft_error_floor_order_of_magnitude():
    """Section 4.1: the FFT arm saturates near NRMSE 4.4e-15 for n > 12."""
    floor = _golden("fft_nrmse_floor")[0][0]
    for n in (14, 16):
        p = W.paper_bs_grid(n)
        u, K = _window(p)
        e = O.nrmse(O.prices_dense(p)[u], O.bs_call(100.0, K, 0.05, 0.0, 0.5, 0.3), 100.0)
        assert floor / 30 < e < floor * 10, (n, e)


# ------------------------------------------------------------------ characteristic functions

def _rand_problems(seed=3):
    g = np.random.default_rng(seed)
    out = []
    for _ in range(4):
        out.append(W.Problem("bs", "simpson1", 10, 100.0, g.uniform(0, .06), g.uniform(0, .03),
                             g.uniform(.2, 2), 1.5, .25, (g.uniform(.1, .5),)))
        out.append(W.Problem("merton", "simpson1", 10, 100.0, g.uniform(0, .06), g.uniform(0, .03),
                             g.uniform(.2, 2), 1.5, .25,
                             (g.uniform(.1, .4), g.uniform(0, 1), g.uniform(-.2, .1), g.uniform(.05, .3))))
    out += W.heston_batch(4, seed=seed, n=12)
    out += W.vg_batch(4, seed=seed, n=12)
    return out


def test_cf_normalisation_and_martingale():
    """phi(0) = 1 and phi(-i) = E[S_T] = S0 e^{(r-q)T} for every model."""
    for p in _rand_problems():
        assert abs(O.char_fn(p, 0.0) - 1.0) < 1e-13
        fwd = p.S0 * math.exp((p.r - p.q) * p.T)
        assert abs(O.char_fn(p, -1j) / fwd - 1.0) < 1e-12, p


def test_bs_second_moment():
    """phi(-2i) = E[S_T^2] = S0^2 exp(2(r-q)T + sigma^2 T) for the lognormal law."""
    p = W.bs_simpson_n12()
    sig = p.params[0]
    ref = p.S0 ** 2 * math.exp(2 * (p.r - p.q) * p.T + sig * sig * p.T)
    assert abs(O.char_fn(p, -2j) / ref - 1.0) < 1e-13


def _heston_riccati(p, u):
    """E[exp(i u ln S_T)] from the Heston Riccati ODEs integrated numerically."""
    kappa, theta, sv, rho, v0 = p.params

    def rhs(t, y):
        B = y[0] + 1j * y[1]
        dB = 0.5 * sv * sv * B * B + (1j * u * rho * sv - kappa) * B - 0.5 * (u * u + 1j * u)
        dA = kappa * theta * B
        return [dB.real, dB.imag, dA.real, dA.imag]

    sol = integrate.solve_ivp(rhs, (0.0, p.T), [0.0, 0.0, 0.0, 0.0], rtol=1e-12, atol=1e-14,
                              method="DOP853")
    B = sol.y[0, -1] + 1j * sol.y[1, -1]
    A = sol.y[2, -1] + 1j * sol.y[3, -1]
    return np.exp(1j * u * (math.log(p.S0) + (p.r - p.q) * p.T) + A + B * v0)


def test_heston_cf_matches_riccati_ode():
    """The closed-form Heston cf against a direct integration of its Riccati ODEs, at real
    and at shifted complex arguments (where psi evaluates it)."""
    for p in W.heston_batch(3, seed=11, n=16):
        for u in (0.7, 3.0, 11.0, 2.0 - 2.5j, 9.0 - 2.5j):
            a = O.char_fn(p, u)
            b = _heston_riccati(p, u)
            assert abs(a - b) <= 1e-8 * max(1.0, abs(b)), (p, u, a, b)


def test_merton_without_jumps_is_bs():
    p = W.merton_big(30).replace(n=12, eta=0.25, params=(0.15, 0.0, -0.1, 0.2))
    q = W.Problem("bs", "simpson1", 12, p.S0, p.r, p.q, p.T, p.alpha, p.eta, (0.15,))
    v = np.linspace(0, 40, 17)
    assert np.abs(O.psi(p, v) - O.psi(q, v)).max() < 1e-12 * np.abs(O.psi(q, v)).max()


# ------------------------------------------------------------------ quadrature and transform

def test_simpson_weights_integrate_to_fourth_order():
    """One-sided Simpson weights integrate a decaying smooth function with O(eta^4) error;
    a wrong 0-indexed transcription does not converge."""
    f = lambda v: np.exp(-v) * (1 + v * v)          # integral over [0, inf) = 3
    errs = []
    for eta in (0.2, 0.1):
        p = W.bs_simpson_n12().replace(eta=eta)
        j = np.arange(4096)
        errs.append(abs((O.weights(p, j) * f(j * eta)).sum() - 3.0))
    assert errs[1] < 1e-4 and errs[0] / errs[1] > 12.0, errs
    wrong = 0.1 / 3 * (3 + (-1.0) ** np.arange(4096) - (np.arange(4096) == 0))
    assert abs((wrong * f(np.arange(4096) * 0.1)).sum() - 3.0) > 1e-3


def test_dft_plane_wave_and_parseval():
    """Eq. dft: a plane wave exp(2 pi i j m / M) maps to sqrt(M) at u = m, zero elsewhere;
    the map preserves the 2-norm; the direct and FFT evaluations agree."""
    n = 10
    M = 2 ** n
    j = np.arange(M)
    for m in (0, 1, 37, M - 1):
        y = O.dft_direct(np.exp(2j * np.pi * j * m / M), j, np.arange(M), n)
        e = np.zeros(M); e[m] = math.sqrt(M)
        assert np.abs(y - e).max() < 1e-10
    x = np.random.default_rng(0).standard_normal(M) + 1j * np.random.default_rng(1).standard_normal(M)
    y1 = O.dft_direct(x, j, j, n)
    y2 = O.dft_fft(x)
    assert np.abs(y1 - y2).max() < 1e-10
    assert abs(np.linalg.norm(y1) - np.linalg.norm(x)) < 1e-9


def _qft_circuit_minus(n):
    """Q_n assembled gate by gate: the QFT circuit (Hadamard, then controlled phase
    R_k = diag(1, exp(2 pi i / 2^k)) from each later qubit) without its final SWAPs, with
    the phases conjugated for the minus-sign transform (the adjoint gates, reversed order
    of the commuting diagonal part is immaterial). Qubit 0 is the most significant bit."""
    M = 2 ** n
    H = np.array([[1, 1], [1, -1]]) / math.sqrt(2)
    U = np.eye(M, dtype=complex)
    idx = np.arange(M)
    bit = lambda q: (idx >> (n - 1 - q)) & 1
    for a in range(n):
        Ha = np.kron(np.kron(np.eye(2 ** a), H), np.eye(2 ** (n - 1 - a)))
        U = Ha @ U
        for b in range(a + 1, n):
            k = b - a + 1
            ph = np.where((bit(a) == 1) & (bit(b) == 1), np.exp(-2j * np.pi / 2 ** k), 1.0)
            U = ph[:, None] * U
    return U


def test_qn_matrix_equals_gate_circuit():
    """Section 3.2: QFT = R_n Q_n; Q_n from the circuit equals the bit-reversed DFT."""
    for n in (1, 2, 3, 4, 5, 6):
        assert np.abs(_qft_circuit_minus(n) - O.qn_matrix(n)).max() < 1e-12, n


def test_qn_is_bit_reversed_dft():
    n = 6
    Q = O.qn_matrix(n)
    F = O.dft_fft(np.eye(2 ** n))      # columns = DFT of unit vectors
    perm = O.bitrev(np.arange(2 ** n), n)
    assert np.abs(Q - F[perm, :]).max() < 1e-12
    assert np.abs(Q @ Q.conj().T - np.eye(2 ** n)).max() < 1e-12


# ------------------------------------------------------------------ prices vs references

def test_bs_rectangle_all_strikes_vs_closed_form():
    """Config n=12, eta=0.25, alpha=1.5, symmetric rectangle rule: every one of the 4096
    grid prices matches Eq. analytic_BS."""
    p = W.bs_rect_n12()
    u = np.arange(4096)
    K = O.strike_of(p, u)
    err = np.abs(O.prices_dense(p) - O.bs_call(100.0, K, 0.05, 0.0, 1.0, 0.2)).max() / 100.0
    assert err < 1e-8, err


def test_bs_simpson_alias_clean_strikes_vs_closed_form():
    """One-sided Simpson: the half-period alias (1/3) e^{alpha pi/eta} C(k + pi/eta) spoils
    the lowest strikes; on the alias-clean set the prices match the closed form."""
    p = W.bs_simpson_n12()
    u = np.arange(4096)
    K = O.strike_of(p, u)
    C = O.prices_dense(p)
    ref = O.bs_call(100.0, K, 0.05, 0.0, 1.0, 0.2)
    alias = np.exp(p.alpha * np.pi / p.eta) / 3 * O.bs_call(100.0, K * np.exp(np.pi / p.eta), 0.05, 0.0, 1.0, 0.2)
    clean = alias < 1e-10 * 100
    assert clean.sum() > 3000
    assert np.abs(C - ref)[clean].max() / 100 < 1e-8
    assert np.abs(C - ref)[~clean].max() / 100 > 1.0     # the alias is real


def _model_grid(model):
    if model == "bs":
        return W.bs_simpson_n12().replace(n=14, eta=0.1)
    if model == "vg":
        return W.vg_n20().replace(n=16, eta=W.eta_rule(16))
    return W.heston_n24().replace(n=16)


@pytest.mark.parametrize("model", ["bs", "heston", "vg"])
def test_alpha_invariance(model):
    """Every admissible alpha gives the same price (Section 2.1, after Eq. psi)."""
    p = _model_grid(model)
    u = W.window_strided(p, 256)
    ref = O.prices_direct(p, u)
    for a in (1.0, 2.0, 3.0):
        C = O.prices_direct(p.replace(alpha=a), u)
        assert np.abs(C - ref).max() / p.S0 < 1e-9, (a, np.abs(C - ref).max())


@pytest.mark.parametrize("model", ["bs", "heston", "vg"])
def test_put_call_parity(model):
    """alpha = -2.5 transforms the damped put; C - P = S0 e^{-qT} - K e^{-rT}."""
    p = _model_grid(model)
    u = W.window_strided(p, 256)
    K = O.strike_of(p, u)
    C = O.prices_direct(p, u)
    P = O.prices_direct(p.replace(alpha=-2.5), u)
    par = p.S0 * math.exp(-p.q * p.T) - K * math.exp(-p.r * p.T)
    assert np.abs(C - P - par).max() / p.S0 < 1e-10


def test_merton_series_near_money():
    p = W.merton_big(30).replace(n=20, eta=W.eta_rule(20))
    u = W.near_money(p, 64)
    C = O.prices_direct(p, u)
    ref = O.merton_call(p, O.strike_of(p, u))
    assert np.abs(C - ref).max() / p.S0 < 1e-12


def test_heston_gil_pelaez():
    p = W.heston_n24().replace(n=18)
    u = W.window_strided(p, 9)
    C = O.prices_direct(p, u)
    ref = O.heston_call_gil_pelaez(p, O.strike_of(p, u))
    assert np.abs(C - ref).max() / p.S0 < 1e-10


def test_vg_gamma_mixture():
    """Variance Gamma: the Carr–Madan prices against the gamma mixture of Black–Scholes
    prices (conditioning on the gamma clock), across the strike window."""
    p = W.vg_n20()
    u = W.window_strided(p, 9)
    C = O.prices_direct(p, u)
    ref = O.vg_call_gamma_mixture(p, O.strike_of(p, u))
    assert np.abs(C - ref).max() / p.S0 < 1e-10


def test_vg_small_nu_is_bs():
    """With theta = 0 and a vanishing variance rate the gamma clock becomes deterministic and
    Variance Gamma reduces to Black–Scholes with the same sigma."""
    p = W.vg_n20().replace(n=12, eta=0.25, params=(0.2, 1e-7, 0.0))
    q = W.Problem("bs", "simpson1", 12, p.S0, p.r, p.q, p.T, p.alpha, p.eta, (0.2,))
    v = np.linspace(0, 40, 17)
    assert np.abs(O.psi(p, v) - O.psi(q, v)).max() < 1e-6 * np.abs(O.psi(q, v)).max()


def test_vg_moment_condition():
    """E[S_T^(alpha+1)] exists for the fixture and fails once theta nu drives the gamma
    moment generating function's argument past 1 (theta > 0 here)."""
    p = W.vg_n20()
    assert O.vg_moment_ok(p, p.alpha + 1.0)
    assert not O.vg_moment_ok(p.replace(params=(0.3, 0.9, 0.5)), 2.5)


@pytest.mark.parametrize("name", ["heston18", "heston22_shortT", "bs16_rect", "merton20", "vg18"])
def test_direct_truncated_dft_matches_full_fft(name):
    """The truncated direct sum (the support of x found by doubling, Section 2.1's sum cut
    where the tail is negligible) against numpy's FFT of the full vector: one-sided
    (Simpson) and two-sided (rectangle) supports, the batched box's shortest maturity
    (slowest decay of psi), jumps and a gamma clock long enough (T/nu = 12) for psi to
    decay within the grid."""
    p = {"heston18": W.heston_n24().replace(n=18),
         "heston22_shortT": W.heston_batch(1, seed=3, n=22)[0].replace(T=0.1),
         "bs16_rect": W.bs_rect_n12().replace(n=16, eta=W.eta_rule(16)),
         "merton20": W.merton_big(20),
         "vg18": W.vg_n20().replace(n=18, eta=W.eta_rule(18), T=2.0)}[name]
    u = W.window_strided(p, 300)
    full = O.prices_dense(p)[u]
    assert len(O.support(p)) < 2 ** p.n   # the sum really is truncated
    assert np.abs(O.prices_direct(p, u) - full).max() / p.S0 < 1e-12


def test_heston_explosion_time_matches_riccati_blowup():
    """T*(omega) of the moment E[S_T^omega] against the blow-up time of the moment Riccati
    ODE dB/dt = sigma^2 B^2/2 + (rho sigma omega - kappa) B + omega(omega-1)/2."""
    kappa, sv, rho = 0.5, 0.8, -0.1
    om = 2.5
    Ts = O.heston_explosion_time(kappa, sv, rho, om)

    def rhs(t, y):
        return [0.5 * sv * sv * y[0] ** 2 + (rho * sv * om - kappa) * y[0] + 0.5 * om * (om - 1)]

    ev = lambda t, y: y[0] - 1e8
    ev.terminal = True
    sol = integrate.solve_ivp(rhs, (0, 50), [0.0], events=ev, rtol=1e-11, atol=1e-12)
    assert abs(sol.t_events[0][0] - Ts) < 1e-5 * Ts
    # the whole batched-Heston parameter box keeps E[S^2.5] finite up to T = 2
    assert Ts > 2.0


def _moment_riccati(kappa, sv, rho, om, t_end):
    """Integrates dB/dt = sigma^2 B^2/2 + (rho sigma omega - kappa) B + omega(omega-1)/2,
    B(0) = 0 (the log-moment coefficient of E[S_T^omega] under Heston); returns the
    solution object, stopped where B passes 1e8 (the moment's blow-up)."""
    def rhs(t, y):
        return [0.5 * sv * sv * y[0] ** 2 + (rho * sv * om - kappa) * y[0] + 0.5 * om * (om - 1)]

    ev = lambda t, y: y[0] - 1e8
    ev.terminal = True
    return integrate.solve_ivp(rhs, (0, t_end), [0.0], events=ev, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("kappa,sv,rho", [(0.5, 0.8, 0.5), (0.05, 0.3, 0.99)],
                         ids=["D<0,k>0", "D>=0,k>0"])
def test_heston_explosion_time_positive_correlation_branches(kappa, sv, rho):
    """The explosion-time branches that positive correlation reaches (k = rho sigma omega -
    kappa > 0): complex roots of the Riccati right-hand side (D < 0, the arctangent form
    without the pi shift) and real roots (D >= 0, the logarithmic form), each against the
    blow-up time of the moment ODE."""
    om = 2.5
    k = rho * sv * om - kappa
    D = k * k - sv * sv * om * (om - 1.0)
    assert k > 0 and ((D < 0) if rho == 0.5 else (D >= 0))
    Ts = O.heston_explosion_time(kappa, sv, rho, om)
    sol = _moment_riccati(kappa, sv, rho, om, 50.0)
    assert len(sol.t_events[0]) == 1
    assert abs(sol.t_events[0][0] - Ts) < 1e-5 * Ts


def test_heston_explosion_time_infinite_branch():
    """Strong mean reversion and negative correlation (D >= 0, k < 0): the moment ODE
    settles on its stable root -(k + sqrt(D))/sigma^2 and never blows up, so T* is
    infinite."""
    kappa, sv, rho, om = 4.0, 0.1, -0.5, 2.5
    k = rho * sv * om - kappa
    D = k * k - sv * sv * om * (om - 1.0)
    assert D >= 0 and k < 0
    assert math.isinf(O.heston_explosion_time(kappa, sv, rho, om))
    sol = _moment_riccati(kappa, sv, rho, om, 200.0)
    assert len(sol.t_events[0]) == 0
    root = (-k - math.sqrt(D)) / (sv * sv)
    assert abs(sol.y[0, -1] - root) < 1e-8 * abs(root)


def test_log_strike_is_the_exact_grid_point():
    """k_u = k0 + 2 pi u / (M eta) within extended precision's 2^-62 |lambda (u - us)| plus two
    ulps of k_u, on the paper's grid at n = 40 (k0 near -3.7e5, so lambda u and k0 cancel to
    ~4.6 in the strike window) and on a default grid (k0 = ln S0 - pi / eta taken as a real
    number, us = M/2): against the same sum in 50-digit decimal arithmetic (pi to 60 digits)."""
    from decimal import Decimal, getcontext
    getcontext().prec = 50
    PI = Decimal("3.141592653589793238462643383279502884197169399375105820974944")
    for p in (W.paper_bs_grid(40), W.heston_n24()):
        g = O.grid(p)
        M = 2 ** p.n
        lam = 2.0 * math.pi / (M * p.eta)
        u_atm = int(round((math.log(100.0) - g.k0) / lam))
        us = np.array([0, 1, u_atm - 12345, u_atm, u_atm + 777, M - 1], dtype=np.int64)
        got = g.k(us)
        for uu, kk in zip(us, got):
            # the default k0 is ln S0 - pi / eta as a real number
            k0 = Decimal(p.k0) if p.k0 is not None else Decimal(math.log(p.S0)) - PI / Decimal(p.eta)
            exact = k0 + 2 * PI * Decimal(int(uu)) / (Decimal(M) * Decimal(p.eta))
            ush = int(uu) - (M // 2 if p.k0 is None else 0)
            lamu = abs(2 * PI * Decimal(ush) / (Decimal(M) * Decimal(p.eta)))
            bound = lamu * Decimal(2.0 ** -62) + 2 * Decimal(np.spacing(abs(float(kk))))
            assert abs(Decimal(float(kk)) - exact) <= bound, (p.n, uu)
        # the naive form rounds lambda first and misses the near-money strikes by far more
        if p.n == 40:
            naive = g.k0 + lam * float(u_atm)
            exact = Decimal(g.k0) + 2 * PI * Decimal(u_atm) / (Decimal(M) * Decimal(p.eta))
            assert abs(Decimal(naive) - exact) > 100 * Decimal(np.spacing(4.6))

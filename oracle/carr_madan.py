"""CPU FP64 oracle for Carr–Madan option pricing -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import this
module. The HIP product path never calls it, and it shares no code with that path.

It computes the discretised Carr–Madan price exactly as the paper defines it, with no
tensor trains and no blocking:

  * characteristic functions of the log-price (Section 2; Eq. characteristic_function)
    for Black–Scholes (Section 2, the GBM solution), Merton jump diffusion and Heston
    (both named in Section 2; their standard closed forms are written out below);
  * the damped transform psi (Eq. psi);
  * the integrand vector x on the frequency grid (Eq. x, generalised to a lowest
    frequency v0 so that both the paper's symmetric rectangle rule (Eq. Ck_from_psi)
    and the one-sided Simpson rule that Section 2.1 allows can be expressed);
  * the unitary DFT with the minus sign (Eq. dft), evaluated either directly with the
    phase (j*u mod M) reduced exactly in integers, or with numpy's FFT as the library
    primitive;
  * prices from the transform (Eq. discretization_dft);
  * reference prices: the Black–Scholes formula (Eq. analytic_BS), the Merton series and
    Gil-Pelaez inversion for Heston;
  * the quantum-observable price reconstruction (Eq. qft_observable_price) and the NRMSE
    error measure (Eq. error_measure);
  * the dense operator Q_n of Section 3.2 (the QFT circuit without its bit reversal).

Conventions (readings of the paper): M = 2^n, lambda = 2 pi/(M eta),
k_u = k0 + lambda u, v_j = v0 + j eta with v0 = -M eta/2 (rectangle) or 0 (Simpson);
x_j = w_j psi(v_j) exp(-i j eta k0); y = M^(-1/2) DFT_-(x);
C(k_u) = Re[ exp(-alpha k_u)/(s pi) * exp(-i v0 k_u) * sqrt(M) * y_u ], s = 2 (rectangle)
or 1 (Simpson).
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np
from scipy import integrate, special

__all__ = [
    "char_fn", "psi", "grid", "weights", "integrand", "dft_direct", "dft_fft",
    "prices_from_y", "prices_dense", "prices_direct", "bs_call", "merton_call",
    "heston_call_gil_pelaez", "vg_call_gamma_mixture", "qft_observable_prices", "qft_probabilities",
    "sample_outcomes", "shot_prices", "prices_from_counts", "nrmse", "qn_matrix",
    "heston_explosion_time", "strike_of",
]

TWO_PI_LD = np.longdouble(2) * np.arccos(np.longdouble(-1))


# ----------------------------------------------------------------------------- models

def char_fn(p, u):
    """phi(u) = E[exp(i u ln S_T)] (Eq. characteristic_function) for complex u.

    Black–Scholes: ln S_T ~ N(ln S0 + (r - q - sigma^2/2) T, sigma^2 T) (Section 2, the
    explicit GBM solution).
    Merton: BS diffusion plus compound-Poisson jumps with normal log-jump sizes
    N(mu_J, delta_J^2), intensity lam_J, drift-compensated (kappa_J = E[e^J] - 1).
    Heston: the principal-branch form of Albrecher et al. (2007), with
    b = kappa - rho sigma_v i u, d = sqrt(b^2 + sigma_v^2 (i u + u^2)), g = (b-d)/(b+d).
    Variance Gamma (the gamma time change of Section 2): X = theta G + sigma W(G), with G
    gamma-distributed of mean T and variance nu T, so E[e^{i u X}] = E[e^{G (i u theta -
    sigma^2 u^2 / 2)}] = (1 - i u theta nu + sigma^2 nu u^2 / 2)^(-T/nu); the drift omega =
    ln(1 - theta nu - sigma^2 nu / 2) / nu makes e^{-(r-q)t} S_t a martingale. The base has
    a positive real part wherever E[S_T^(-Im u)] is finite, so the principal log is used.
    """
    u = np.asarray(u, dtype=np.complex128)
    S0, r, q, T = p.S0, p.r, p.q, p.T
    if p.model == "bs":
        (sig,) = p.params
        return np.exp(1j * u * (math.log(S0) + (r - q - 0.5 * sig * sig) * T)
                      - 0.5 * sig * sig * T * u * u)
    if p.model == "merton":
        sig, lam, muJ, dJ = p.params
        kJ = math.exp(muJ + 0.5 * dJ * dJ) - 1.0
        drift = math.log(S0) + (r - q - 0.5 * sig * sig - lam * kJ) * T
        return np.exp(1j * u * drift - 0.5 * sig * sig * T * u * u
                      + lam * T * (np.exp(1j * u * muJ - 0.5 * dJ * dJ * u * u) - 1.0))
    if p.model == "heston":
        kappa, theta, sv, rho, v0 = p.params
        b = kappa - rho * sv * 1j * u
        d = np.sqrt(b * b + sv * sv * (1j * u + u * u))
        g = (b - d) / (b + d)
        e = np.exp(-d * T)
        C = kappa * theta / (sv * sv) * ((b - d) * T - 2.0 * np.log((1.0 - g * e) / (1.0 - g)))
        D = (b - d) / (sv * sv) * (1.0 - e) / (1.0 - g * e)
        return np.exp(1j * u * (math.log(S0) + (r - q) * T) + C + D * v0)
    if p.model == "vg":
        sig, nu, th = p.params
        om = math.log(1.0 - th * nu - 0.5 * sig * sig * nu) / nu
        base = 1.0 - 1j * u * th * nu + 0.5 * sig * sig * nu * u * u
        return np.exp(1j * u * (math.log(S0) + (r - q + om) * T) - (T / nu) * np.log(base))
    raise ValueError(p.model)


def psi(p, v, alpha: Optional[float] = None):
    """psi(v) = exp(-r T) phi(v - i(alpha+1)) / ((alpha + i v)(alpha + 1 + i v))  (Eq. psi)."""
    a = p.alpha if alpha is None else alpha
    v = np.asarray(v, dtype=np.float64)
    return (math.exp(-p.r * p.T) * char_fn(p, v - 1j * (a + 1.0))
            / ((a + 1j * v) * (a + 1.0 + 1j * v)))


# ----------------------------------------------------------------------------- grid

class Grid:
    """Discretisation of Section 2.1: M = 2^n, frequency step eta (Delta_v), log-strike
    step lambda with eta * lambda = 2 pi / M (the grid relation), lowest log-strike k0,
    lowest frequency v0, and the factor s of the price formula."""

    def __init__(self, p):
        self.n = p.n
        self.M = 2 ** p.n
        self.eta = p.eta
        self.lam = 2.0 * math.pi / (self.M * p.eta)
        # The default grid is centred on the money: k0 = ln S0 - M lambda / 2 as a real number,
        # so that k_u = ln S0 + lambda (u - M/2) with an exact integer offset (kc, us); k0 here
        # is that value rounded, for display and for search windows only.
        if p.k0 is None:
            self.kc, self.us = math.log(p.S0), self.M // 2
            self.k0 = math.log(p.S0) - self.M * self.lam / 2.0
        else:
            self.kc, self.us = float(p.k0), 0
            self.k0 = float(p.k0)
        if p.quad == "rect2":
            self.v0 = -self.M * p.eta / 2.0
            self.s = 2.0
        else:
            self.v0 = 0.0
            self.s = 1.0
        self.quad = p.quad

    def k(self, u):
        """k_u = k0 + 2 pi u / (M eta): the log-strike that the DFT phase exp(-2 pi i j u / M)
        pairs with index u (the grid relation eta lambda = 2 pi / M of Section 2.1 holds
        exactly in the sum); the default k0 enters as ln S0 and the exact offset -M/2 of u.
        Formed in extended precision (64-bit significand) and rounded once: within about
        2^-63 |lambda (u - us)| plus half an ulp of k_u, even where k0 and lambda u are large
        and cancel (grids centred far from the money: 1e-14 at n = 40 on the paper's grid);
        lambda rounded to double first would shift k_u by up to |lambda u| times the double
        epsilon (4e-11 there)."""
        uu = (np.asarray(u, dtype=np.int64) - self.us).astype(np.longdouble)
        step = TWO_PI_LD / (np.longdouble(self.M) * np.longdouble(self.eta))
        return (np.longdouble(self.kc) + step * uu).astype(np.float64)


def grid(p) -> Grid:
    return Grid(p)


def strike_of(p, u):
    """Strike K = exp(k_u) of log-strike index u."""
    return np.exp(grid(p).k(u))


def weights(p, j):
    """Quadrature weights w_j. Rectangle: w_j = eta (Eq. Ck_from_psi). Simpson, one-sided,
    0-indexed: w_j = (eta/3)(3 - (-1)^j - delta_{j0}) (the higher-order rule Section 2.1
    allows to be folded into x)."""
    j = np.asarray(j, dtype=np.int64)
    if p.quad == "rect2":
        return np.full(j.shape, p.eta, dtype=np.float64)
    sgn = np.where(j % 2 == 0, 1.0, -1.0)
    return p.eta / 3.0 * (3.0 - sgn - (j == 0).astype(np.float64))


def _phase_frac(j, c_ld):
    """fractional part of j * c (c a longdouble), for exact-enough phase reduction."""
    t = np.asarray(j, dtype=np.longdouble) * c_ld
    return t - np.floor(t)


def integrand(p, j):
    """x_j = w_j psi(v0 + j eta) exp(-i j eta k0)  (Eq. x with the lowest frequency v0;
    for v0 = -N eta this is exactly the paper's Eq. x, whose extra factor exp(i eta N k0)
    moves into the readout as exp(-i v0 k_u))."""
    g = grid(p)
    j = np.asarray(j, dtype=np.int64)
    v = g.v0 + j.astype(np.float64) * p.eta
    # eta k0 / (2 pi) in turns; the default k0 = ln S0 - pi / eta adds half a turn per j
    c = np.longdouble(p.eta) * np.longdouble(g.kc) / TWO_PI_LD
    if g.us:
        c = c - np.longdouble(0.5)
    ang = (TWO_PI_LD * _phase_frac(j, c)).astype(np.float64)
    return weights(p, j) * psi(p, v) * np.exp(-1j * ang)


# ----------------------------------------------------------------------------- transforms

def dft_direct(x, j, u, n):
    """y_u = M^(-1/2) sum_j x_j exp(-2 pi i j u / M) (Eq. dft), summed over the given
    (support) indices j only; the phase (j*u) mod M is reduced exactly in integers."""
    M = 2 ** n
    x = np.asarray(x, dtype=np.complex128)
    j = np.asarray(j, dtype=np.uint64)
    u = np.asarray(u, dtype=np.uint64)
    mask = np.uint64(M - 1)
    out = np.empty(u.shape, dtype=np.complex128)
    chunk = max(1, (1 << 22) // max(1, len(j)))
    for s in range(0, len(u), chunk):
        uu = u[s:s + chunk]
        ph = (np.multiply.outer(uu, j) & mask).astype(np.float64) * (2.0 * math.pi / M)
        out[s:s + chunk] = (np.exp(-1j * ph) * x[None, :]).sum(axis=1)
    return out / math.sqrt(M)


def dft_fft(x):
    """Eq. dft for the full vector, with numpy's FFT (same minus-sign convention)."""
    x = np.asarray(x, dtype=np.complex128)
    return np.fft.fft(x) / math.sqrt(len(x))


def prices_from_y(p, u, y):
    """C(k_u) = Re[ exp(-alpha k_u)/(s pi) exp(-i v0 k_u) sqrt(M) y_u ]
    (Eq. discretization_dft; Re(.) of the classical readout)."""
    g = grid(p)
    u = np.asarray(u, dtype=np.int64)
    k = g.k(u)
    # exp(-i v0 k_u) = exp(-i v0 k0) exp(-i v0 lambda u); by the grid relation
    # v0 lambda = -pi for the symmetric rule (the paper's e^{i pi l}) and 0 for Simpson.
    # -v0 k0 in turns: (M eta / 2) k0 / (2 pi); the default k0 = ln S0 - pi / eta takes off M/4
    t0 = -np.longdouble(g.v0) * np.longdouble(g.kc) / TWO_PI_LD
    if g.us:
        t0 = t0 - np.longdouble(g.M) / 4
    a0 = float(TWO_PI_LD * (t0 - np.floor(t0)))
    ph = np.exp(1j * a0) * (np.where(u % 2 == 0, 1.0, -1.0) if g.v0 != 0.0 else 1.0)
    return np.real(np.exp(-p.alpha * k) / (g.s * math.pi) * ph * math.sqrt(g.M) * y)


def prices_dense(p):
    """All M prices: x on the full grid, FFT, readout (the dense Carr–Madan path)."""
    j = np.arange(2 ** p.n, dtype=np.int64)
    y = dft_fft(integrand(p, j))
    return prices_from_y(p, j, y)


def support(p, rel: float = 1e-18, start: int = 1024):
    """Indices j where x_j is not negligible: the smallest window (doubling from `start`
    points around v = 0) whose complement carries sum |x_j| below rel * sum |x_j|.
    The decay of |psi| is checked on a 4x larger window."""
    M = 2 ** p.n
    g = grid(p)
    j_center = 0 if g.v0 == 0.0 else M // 2
    J = min(start, M)
    while True:
        big = min(4 * J, M)
        if g.v0 == 0.0:
            jj = np.arange(big, dtype=np.int64)
        else:
            jj = np.arange(max(0, j_center - big // 2), min(M, j_center + big // 2), dtype=np.int64)
        ax = np.abs(integrand(p, jj))
        if g.v0 == 0.0:
            inner = jj < J
        else:
            inner = np.abs(jj - j_center) < J // 2
        tail = ax[~inner].sum()
        if big == M or tail <= rel * ax.sum():
            sel = jj[inner] if big != M else jj
            return sel
        J *= 2


def prices_direct(p, u, rel: float = 1e-18):
    """Prices at strike indices u by the direct (truncated) DFT over the support of x."""
    j = support(p, rel)
    y = dft_direct(integrand(p, j), j, u, p.n)
    return prices_from_y(p, u, y)


# ----------------------------------------------------------------------------- references

def bs_call(S0, K, r, q, T, sigma):
    """Black–Scholes call (Eq. analytic_BS), with a continuous dividend yield q."""
    K = np.asarray(K, dtype=np.float64)
    sq = sigma * math.sqrt(T)
    d1 = (np.log(S0 / K) + (r - q + 0.5 * sigma * sigma) * T) / sq
    d2 = d1 - sq
    return S0 * math.exp(-q * T) * special.ndtr(d1) - K * math.exp(-r * T) * special.ndtr(d2)


def merton_call(p, K, terms: int = 60):
    """Merton (1976) series: a Poisson mixture of Black–Scholes prices with adjusted rate
    and volatility."""
    sig, lam, muJ, dJ = p.params
    kJ = math.exp(muJ + 0.5 * dJ * dJ) - 1.0
    lamp = lam * (1.0 + kJ)
    K = np.asarray(K, dtype=np.float64)
    out = np.zeros_like(K)
    for m in range(terms):
        w = math.exp(-lamp * p.T + m * math.log(lamp * p.T) - math.lgamma(m + 1)) if lamp > 0 else (1.0 if m == 0 else 0.0)
        sm = math.sqrt(sig * sig + m * dJ * dJ / p.T)
        rm = p.r - lam * kJ + m * math.log(1.0 + kJ) / p.T
        out += w * bs_call(p.S0, K, rm, p.q, p.T, sm)
    return out


def heston_call_gil_pelaez(p, K):
    """Heston call by Gil-Pelaez inversion, C = S0 e^{-qT} P1 - K e^{-rT} P2, integrated
    with adaptive quadrature (an integrator independent of the DFT)."""
    S0, r, q, T = p.S0, p.r, p.q, p.T
    phi_mi = char_fn(p, -1j)
    out = []
    for KK in np.atleast_1d(K):
        lk = math.log(KK)

        def f2(u):
            return (np.exp(-1j * u * lk) * char_fn(p, u) / (1j * u)).real

        def f1(u):
            return (np.exp(-1j * u * lk) * char_fn(p, u - 1j) / (1j * u * phi_mi)).real

        P2 = 0.5 + integrate.quad(f2, 0.0, np.inf, limit=2000, epsabs=1e-14, epsrel=1e-13)[0] / math.pi
        P1 = 0.5 + integrate.quad(f1, 0.0, np.inf, limit=2000, epsabs=1e-14, epsrel=1e-13)[0] / math.pi
        out.append(S0 * math.exp(-q * T) * P1 - KK * math.exp(-r * T) * P2)
    return np.array(out)


def vg_call_gamma_mixture(p, K):
    """Variance Gamma call as a gamma mixture of Black–Scholes prices: given the gamma time
    G = g, ln S_T is normal with mean ln S0 + (r - q + omega) T + theta g and variance
    sigma^2 g, so E[(S_T - K)^+ | g] = F_g N(d1) - K N(d2) with F_g = S0 e^{(r-q+omega)T +
    theta g + sigma^2 g/2}, d1 = (ln(F_g/K) + sigma^2 g/2) / (sigma sqrt g), d2 = d1 -
    sigma sqrt g; the price is e^{-rT} times its expectation over the gamma density of
    shape T/nu and scale nu (adaptive quadrature; independent of any Fourier transform)."""
    sig, nu, th = p.params
    S0, r, q, T = p.S0, p.r, p.q, p.T
    om = math.log(1.0 - th * nu - 0.5 * sig * sig * nu) / nu
    shape, scale = T / nu, nu
    lgn = math.lgamma(shape) + shape * math.log(scale)
    out = []
    for KK in np.atleast_1d(K):
        KK = float(KK)

        def f(g):
            if g <= 0.0:
                return 0.0
            sq = sig * math.sqrt(g)
            lF = math.log(S0) + (r - q + om) * T + th * g + 0.5 * sig * sig * g
            d1 = (lF - math.log(KK) + 0.5 * sq * sq) / sq
            cond = math.exp(lF) * special.ndtr(d1) - KK * special.ndtr(d1 - sq)
            dens = math.exp((shape - 1.0) * math.log(g) - g / scale - lgn)
            return cond * dens

        # the density can be singular at g = 0 (shape < 1): split there and integrate out
        a = integrate.quad(f, 0.0, scale, limit=500, epsabs=1e-15, epsrel=1e-13)[0]
        b = integrate.quad(f, scale, np.inf, limit=500, epsabs=1e-15, epsrel=1e-13)[0]
        out.append(math.exp(-r * T) * (a + b))
    return np.array(out)


def vg_moment_ok(p, omega):
    """E[S_T^omega] is finite under Variance Gamma iff 1 - omega theta nu - sigma^2 nu
    omega^2 / 2 > 0 (the gamma moment generating function exists there)."""
    sig, nu, th = p.params
    return 1.0 - omega * th * nu - 0.5 * sig * sig * nu * omega * omega > 0.0


def heston_explosion_time(kappa, sv, rho, omega):
    """Time T* at which E[S_T^omega] becomes infinite under Heston (Andersen & Piterbarg
    2007); the damping condition E[S_T^(alpha+1)] < inf (Eq. damping_moment_condition)
    holds iff T < T*(alpha+1)."""
    k = rho * sv * omega - kappa
    D = k * k - sv * sv * omega * (omega - 1.0)
    if D >= 0:
        if k < 0:
            return math.inf
        sD = math.sqrt(D)
        return math.log((k + sD) / (k - sD)) / sD if k > sD else math.inf
    sD = math.sqrt(-D)
    return 2.0 / sD * ((math.pi if k < 0 else 0.0) + math.atan(sD / k))


# ----------------------------------------------------------------------------- paper pieces

def qft_observable_prices(p, u=None):
    """Prices reconstructed from measurement probabilities (Eq. qft_observable_price),
    with exact probabilities p_l = |y_l / ||x|| |^2 (Eq. qft_probabilities), i.e. the
    statevector readout that takes the phase of e^{i pi l} y_l to be zero."""
    g = grid(p)
    j = np.arange(g.M, dtype=np.int64)
    x = integrand(p, j)
    y = dft_fft(x)
    nx = np.linalg.norm(x)
    prob = np.abs(y / nx) ** 2
    uu = j if u is None else np.asarray(u, dtype=np.int64)
    k = g.k(uu)
    return np.exp(-p.alpha * k) / (g.s * math.pi) * nx * math.sqrt(g.M) * np.sqrt(prob[uu])


def qft_probabilities(p):
    """p_l = |y_l / ||x|| |^2 for every outcome l (Eq. qft_probabilities) and ||x||^2."""
    g = grid(p)
    x = integrand(p, np.arange(g.M, dtype=np.int64))
    nx2 = float(np.vdot(x, x).real)
    return np.abs(dft_fft(x)) ** 2 / nx2, nx2


def sample_outcomes(prob, uniforms):
    """Measurement outcomes l in [0, M) drawn from the probabilities `prob` (Eq.
    qft_probabilities) by exact sequential conditional sampling, one bit at a time from
    bit 0 (weight 1): with bits 0..t-1 fixed to `pre`, q_b is the total probability of the
    outcomes whose low t+1 bits are pre + b 2^t, and bit t is 1 iff U_t (q0 + q1) >= q0.
    uniforms: [R, n] in [0, 1), one per shot and bit. Returns int64 [R]."""
    prob = np.asarray(prob, dtype=np.float64)
    M = len(prob)
    n = M.bit_length() - 1
    U = np.asarray(uniforms, dtype=np.float64)
    out = np.zeros(U.shape[0], dtype=np.int64)
    for t in range(n):
        S = prob.reshape(-1, 2 ** (t + 1)).sum(axis=0)   # mass of each residue mod 2^(t+1)
        q0 = S[out]
        q1 = S[out + 2 ** t]
        out = out + np.where(U[:, t] * (q0 + q1) >= q0, 2 ** t, 0)
    return out


def shot_prices(p, samples, u, norm2):
    """Observable prices from R measured outcomes (Eqs. qft_probability_estimator and
    qft_observable_price): p_hat_l = R_l / R and C_hat(k_l) = e^{-alpha k_l} / (s pi) sqrt(M)
    ||x|| sqrt(p_hat_l), with norm2 = ||x||^2."""
    samples = np.sort(np.asarray(samples, dtype=np.int64))
    u = np.asarray(u, dtype=np.int64)
    counts = np.searchsorted(samples, u, side="right") - np.searchsorted(samples, u, side="left")
    return prices_from_counts(p, u, counts, len(samples), norm2)


def prices_from_counts(p, u, counts, R, norm2):
    """C_hat(k_u) = e^{-alpha k_u} / (s pi) sqrt(M) sqrt(norm2 R_u / R) (Eq.
    qft_observable_price with p_hat = R_u / R)."""
    g = grid(p)
    k = g.k(np.asarray(u, dtype=np.int64))
    return np.exp(-p.alpha * k) / (g.s * math.pi) * math.sqrt(g.M) * np.sqrt(norm2 * np.asarray(counts) / R)


def nrmse(C, Cref, S0):
    """NRMSE = (1/S0) sqrt(mean (C - C_ref)^2) over a strike set (Eq. error_measure)."""
    C = np.asarray(C); Cref = np.asarray(Cref)
    return math.sqrt(float(np.mean((C - Cref) ** 2))) / S0


def bitrev(m, n):
    m = np.asarray(m, dtype=np.int64)
    r = np.zeros_like(m)
    for i in range(n):
        r = (r << 1) | ((m >> i) & 1)
    return r


def qn_matrix(n):
    """Dense Q_n (Section 3.2): the QFT circuit without the final bit-reversal SWAPs, for the
    minus-sign unitary DFT of Eq. dft. Since DFT = R_n Q_n with R_n the bit reversal,
    Q_n[m, j] = M^(-1/2) exp(-2 pi i j bitrev_n(m) / M): output row m of Q_n holds the
    transform coefficient of log-strike index bitrev_n(m)."""
    M = 2 ** n
    m = np.arange(M)
    u = bitrev(m, n).astype(np.uint64)
    j = np.arange(M, dtype=np.uint64)
    ph = (np.multiply.outer(u, j) & np.uint64(M - 1)).astype(np.float64) * (2 * math.pi / M)
    return np.exp(-1j * ph) / math.sqrt(M)

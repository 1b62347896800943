"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the bench.

This module holds plain data only: problem parameter sets, seeded random draws of them
and strike-index selections. It contains none of the pricing arithmetic (no
characteristic function, no transform, no readout); both the CPU oracle and the HIP
path compute everything from these parameters on their own.

Problem fields follow the paper's notation for the damped Carr–Madan transform
(Section 2.1): maturity ``T``, damping ``alpha``, frequency step ``eta`` (the paper's
Delta_v), grid exponent ``n`` (M = 2^n points), lowest log-strike ``k0``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

MODELS = ("bs", "merton", "heston", "vg")
QUADS = ("rect2", "simpson1")


@dataclasses.dataclass(frozen=True)
class Problem:
    """One European-call pricing instance on a Carr–Madan log-strike grid.

    model   : "bs" (params = (sigma,)), "merton" (sigma, lam_J, mu_J, delta_J),
              "heston" (kappa, theta, sigma_v, rho, v0), "vg" (sigma, nu, theta): Variance
              Gamma, a Brownian motion with drift theta and volatility sigma run on a gamma
              clock of unit mean rate and variance rate nu
    quad    : "rect2"  - two-sided rectangle rule on v in [-M eta/2, M eta/2)
                         (the paper's symmetric truncation, Section 2.1)
              "simpson1" - one-sided Simpson rule on v in [0, M eta) (Carr & Madan 1999)
    n       : grid exponent, M = 2^n
    k0      : lowest log-strike; None selects ln(S0) - M*lambda/2 (ATM at u = M/2)
    """

    model: str
    quad: str
    n: int
    S0: float
    r: float
    q: float
    T: float
    alpha: float
    eta: float
    params: Tuple[float, ...]
    k0: Optional[float] = None

    def __post_init__(self):
        if self.model not in MODELS:
            raise ValueError(f"unknown model {self.model!r}")
        if self.quad not in QUADS:
            raise ValueError(f"unknown quadrature {self.quad!r}")

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# ---------------------------------------------------------------- fixed configurations

def bs_simpson_n12() -> Problem:
    """Black–Scholes, S0=100, r=0.05, sigma=0.2, T=1; alpha=1.5, N=2^12, eta=0.25, Simpson."""
    return Problem("bs", "simpson1", 12, 100.0, 0.05, 0.0, 1.0, 1.5, 0.25, (0.2,))


def bs_rect_n12() -> Problem:
    """The same Black–Scholes grid with the paper's two-sided rectangle rule."""
    return bs_simpson_n12().replace(quad="rect2")


def heston_n24() -> Problem:
    """Heston kappa=1.5, theta=0.04, sigma_v=0.3, rho=-0.7, v0=0.04, S0=100, r=0.03,
    T=0.5; alpha=1.5, N=2^24, eta=0.05, Simpson."""
    return Problem("heston", "simpson1", 24, 100.0, 0.03, 0.0, 0.5, 1.5, 0.05,
                   (1.5, 0.04, 0.3, -0.7, 0.04))


def eta_rule(n: int) -> float:
    """Frequency step eta = 40 / 2^(n/2) used by the batched Heston and Merton grids."""
    return 40.0 / 2.0 ** (n / 2.0)


def merton_big(n: int) -> Problem:
    """Merton jump diffusion sigma=0.15, lam_J=0.5, mu_J=-0.1, delta_J=0.2, S0=100,
    r=0.02, T=1; alpha=1.5, eta=40/2^(n/2); n = 30 or 40."""
    return Problem("merton", "simpson1", n, 100.0, 0.02, 0.0, 1.0, 1.5, eta_rule(n),
                   (0.15, 0.5, -0.1, 0.2))


def vg_n20() -> Problem:
    """Variance Gamma sigma=0.12, nu=0.17, theta=-0.14 (a typical equity-index fit),
    S0=100, r=0.05, q=0.01, T=0.5; alpha=1.5, eta=40/2^(n/2), n=20, Simpson."""
    return Problem("vg", "simpson1", 20, 100.0, 0.05, 0.01, 0.5, 1.5, eta_rule(20), (0.12, 0.17, -0.14))


def vg_batch(count: int, seed: int = 31, n: int = 20) -> List[Problem]:
    """Seeded Variance Gamma draws: sigma ~ U(0.08, 0.3), nu ~ U(0.05, 0.5),
    theta ~ U(-0.3, 0.05), T ~ U(0.1, 1.5), kept when the damping moment condition holds
    for alpha = 1.5 with margin and T >= nu (the characteristic function then decays at
    least like |v|^-2; shorter clocks are covered by vg_short_clock)."""
    g = _rng(seed)
    out = []
    while len(out) < count:
        sig, nu, th, T = g.uniform(0.08, 0.3), g.uniform(0.05, 0.5), g.uniform(-0.3, 0.05), g.uniform(0.1, 1.5)
        b = 2.5   # alpha + 1
        if 1.0 - b * th * nu - 0.5 * sig * sig * nu * b * b <= 0.05 or T < nu:
            continue
        out.append(Problem("vg", "simpson1", n, 100.0, 0.03, 0.0, float(T), 1.5, eta_rule(n),
                           (float(sig), float(nu), float(th))))
    return out


def vg_short_clock(n: int = 20) -> Problem:
    """A Variance Gamma instance with a short gamma clock (T = 0.05, T/nu = 0.18): its
    characteristic function decays only like |v|^-0.36, so x has no negligible tail."""
    return Problem("vg", "simpson1", n, 100.0, 0.03, 0.0, 0.05, 1.5, eta_rule(n), (0.1854, 0.276, -0.1228))


def merton_oscillating() -> Problem:
    """Merton with near-deterministic jumps (lam_J = 2, mu_J = 0.5, delta_J = 0.001) and
    almost no diffusion (sigma = 0.01), n = 24: the characteristic function keeps
    oscillating with period 2 pi / mu_J out to |v| of order 1 / delta_J."""
    return Problem("merton", "simpson1", 24, 100.0, 0.02, 0.0, 1.0, 1.5, eta_rule(24), (0.01, 2.0, 0.5, 0.001))


def paper_bs_grid(n: int) -> Problem:
    """The paper's experimental grid (Section 4): S0=100, r=0.05, sigma=0.3, T=0.5,
    alpha=2.5; N=2^(n-1), Delta_k=N^(-1/2), b=ln S0 - N Delta_k/2, Delta_v=pi/(N Delta_k),
    two-sided rectangle rule, k0=b."""
    N = 2 ** (n - 1)
    dk = N ** -0.5
    b = math.log(100.0) - N * dk / 2.0
    dv = math.pi / (N * dk)
    return Problem("bs", "rect2", n, 100.0, 0.05, 0.0, 0.5, 2.5, dv, (0.3,), k0=b)


# ---------------------------------------------------------------- seeded draws

HESTON_BOX = {
    "kappa": (0.5, 4.0),
    "theta": (0.01, 0.1),
    "sigma_v": (0.1, 0.8),
    "rho": (-0.9, -0.1),
    "v0": (0.01, 0.1),
    "T": (0.1, 2.0),
}


def _rng(seed: int) -> np.random.Generator:
    # Philox-4x32-10 counter-based generator
    return np.random.Generator(np.random.Philox(seed))


def heston_batch(count: int, seed: int = 20261203, n: Optional[int] = None,
                 n_range: Tuple[int, int] = (16, 28), box=None) -> List[Problem]:
    """Seeded Heston instances with parameters uniform in the box, alpha=1.5, S0=100,
    r=0.03, q=0, Simpson, eta=40/2^(n/2). n is drawn uniformly from n_range (inclusive)
    unless fixed."""
    box = dict(HESTON_BOX if box is None else box)
    g = _rng(seed)
    u = g.random((count, 7))
    out = []
    for i in range(count):
        lo = lambda k: box[k][0]
        hi = lambda k: box[k][1]
        kappa = lo("kappa") + (hi("kappa") - lo("kappa")) * u[i, 0]
        theta = lo("theta") + (hi("theta") - lo("theta")) * u[i, 1]
        sv = lo("sigma_v") + (hi("sigma_v") - lo("sigma_v")) * u[i, 2]
        rho = lo("rho") + (hi("rho") - lo("rho")) * u[i, 3]
        v0 = lo("v0") + (hi("v0") - lo("v0")) * u[i, 4]
        T = lo("T") + (hi("T") - lo("T")) * u[i, 5]
        nn = n if n is not None else int(n_range[0] + min(int(u[i, 6] * (n_range[1] - n_range[0] + 1)),
                                                      n_range[1] - n_range[0]))
        out.append(Problem("heston", "simpson1", nn, 100.0, 0.03, 0.0, float(T), 1.5,
                           eta_rule(nn), (float(kappa), float(theta), float(sv), float(rho), float(v0))))
    return out


# Surrogate domain: the batched Heston box plus the log-moneyness k = ln(K/S0).
SURROGATE_K = (-0.5, 0.5)
SURROGATE_KEYS = ("kappa", "theta", "sigma_v", "rho", "v0", "T", "k")


def surrogate_box(enlarge: float = 0.0) -> Tuple[np.ndarray, np.ndarray]:
    """(lo, hi) of the seven surrogate inputs; `enlarge` widens every interval by that
    fraction of its width (half on each side), clipped to where the model stays defined
    (positive rates and volatilities, |rho| < 1, T > 0)."""
    lo = np.array([HESTON_BOX[k][0] for k in SURROGATE_KEYS[:6]] + [SURROGATE_K[0]], dtype=np.float64)
    hi = np.array([HESTON_BOX[k][1] for k in SURROGATE_KEYS[:6]] + [SURROGATE_K[1]], dtype=np.float64)
    w = (hi - lo) * enlarge / 2
    lo, hi = lo - w, hi + w
    floor = np.array([0.05, 0.001, 0.02, -0.98, 0.001, 0.02, -np.inf])
    ceil = np.array([np.inf, np.inf, np.inf, 0.98, np.inf, np.inf, np.inf])
    return np.maximum(lo, floor), np.minimum(hi, ceil)


def surrogate_queries(count: int, seed: int, enlarge: float = 0.0) -> np.ndarray:
    """[count, 7] float64 query points (kappa, theta, sigma_v, rho, v0, T, k) uniform in the
    (possibly enlarged) surrogate box, from a Philox stream."""
    lo, hi = surrogate_box(enlarge)
    u = _rng(seed).random((count, 7))
    return lo + (hi - lo) * u


def bs_batch(count: int, seed: int = 7, n: int = 12, quad: str = "simpson1") -> List[Problem]:
    """Seeded Black–Scholes instances (sigma in [0.1, 0.5], T in [0.25, 2], r in [0, 0.06])."""
    g = _rng(seed)
    u = g.random((count, 3))
    return [Problem("bs", quad, n, 100.0, float(0.06 * u[i, 2]), 0.0, float(0.25 + 1.75 * u[i, 1]),
                    1.5, 0.25 if n == 12 else eta_rule(n), (float(0.1 + 0.4 * u[i, 0]),))
            for i in range(count)]


# ---------------------------------------------------------------- strike selections

def near_money(p: Problem, count: int = 4096) -> np.ndarray:
    """`count` consecutive log-strike indices centred on u = M/2 (the at-the-money index
    when k0 is left at its default)."""
    M = 2 ** p.n
    c = min(count, M)
    start = M // 2 - c // 2
    return np.arange(start, start + c, dtype=np.int64)


def window_strided(p: Problem, count: int = 4096, lo: float = 0.5, hi: float = 1.5) -> np.ndarray:
    """Up to `count` strike indices spread evenly over the moneyness window lo <= K/S0 <= hi
    on the default grid (ATM at u = M/2, log-strike spacing 2 pi / (M eta))."""
    M = 2 ** p.n
    lam = 2.0 * math.pi / (M * p.eta)
    u_lo = max(0, int(math.ceil(M / 2 + math.log(lo) / lam)))
    u_hi = min(M - 1, int(math.floor(M / 2 + math.log(hi) / lam)))
    total = u_hi - u_lo + 1
    if total <= count:
        return np.arange(u_lo, u_hi + 1, dtype=np.int64)
    stride = total // count
    return (u_lo + stride * np.arange(count)).astype(np.int64)


def all_strikes(p: Problem) -> np.ndarray:
    return np.arange(2 ** p.n, dtype=np.int64)

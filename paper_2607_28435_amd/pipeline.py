"""Stage chaining on one stream: SFFT path (build QTT -> SFFT apply -> round -> readout)
and the dense path. Marshalling only; every stage is one call into libcm."""
from __future__ import annotations

from typing import Dict, Iterable, Optional, Sequence

import numpy as np

from . import (CM_C64, CM_C128, TTBatch, Workspace, cm_build_qtt, cm_fft_price, cm_qft_mpo, cm_readout_prices,
               cm_sfft_apply, cm_tt_round, pack_problems)


def _torch():
    import torch
    return torch


class MpoCache:
    """Q_n operators for a set of chain lengths, stored so that train n is Q_n
    (the layout cm_sfft_apply expects). Built once per (n, tol, cap, dtype)."""

    def __init__(self, ns: Iterable[int], tol: float, cap: int, dtype: int, device="cuda", stream=None):
        ns = sorted(set(int(n) for n in ns))
        self.tol, self.cap, self.dtype = tol, cap, dtype
        n_max = max(ns)
        slots = [n if n in ns else 0 for n in range(n_max + 1)]
        self.w = TTBatch(slots, 2, 2, cap, dtype, device)
        self.w.struct.n_max = n_max
        ws = Workspace(device)
        for n in ns:
            cm_qft_mpo(n, tol, cap, self.w, n, ws, stream)
        self.ns = ns


class SfftPricer:
    """Batched SFFT pricing of a fixed list of problems on one stream.

    tol       : zip-up and rounding tolerance (relative Frobenius)
    build_tol : QTT construction tolerance (default tol/10)
    mpo_tol   : operator rounding tolerance (default tol/10)
    cap       : bond capacity of x and y (zip-up bonds are limited to min(cap, 32))
    """

    def __init__(self, problems: Sequence, dtype: int = CM_C64, tol: float = 1e-8, cap: int = 32,
                 build_tol: Optional[float] = None, mpo_tol: Optional[float] = None, mpo: Optional[MpoCache] = None,
                 device="cuda", stream=None):
        torch = _torch()
        self.problems = list(problems)
        self.batch = len(self.problems)
        self.dtype, self.tol, self.cap = dtype, tol, cap
        self.build_tol = tol / 10 if build_tol is None else build_tol
        ns = [p.n for p in self.problems]
        self.prob = pack_problems(self.problems, device)
        self.x = TTBatch(ns, 2, 1, cap, dtype, device)
        self.y = TTBatch(ns, 2, 1, cap, dtype, device)
        self.mpo = mpo if mpo is not None else MpoCache(ns, tol / 10 if mpo_tol is None else mpo_tol, cap, dtype,
                                                        device, stream)
        z = lambda: torch.zeros(self.batch, dtype=torch.int32, device=device)
        self.st_build, self.st_apply, self.st_round, self.st_read = z(), z(), z(), z()
        self.round_err = torch.zeros(self.batch, dtype=torch.float64, device=device)
        self.ws = Workspace(device)
        self.stream = stream

    def build(self):
        cm_build_qtt(self.prob, self.batch, self.build_tol, self.cap, self.x, self.st_build, self.ws, self.stream)

    def core(self, strikes, prices):
        """The online part: SFFT apply, rounding and readout (x must be built)."""
        cm_sfft_apply(self.mpo.w, self.x, self.tol, self.cap, self.y, self.st_apply, self.ws, self.stream)
        cm_tt_round(self.y, self.tol, self.cap, self.round_err, self.st_round, self.ws, self.stream)
        cm_readout_prices(self.y, self.prob, strikes, strikes.shape[-1], prices, self.st_read, self.stream)

    def run(self, strikes, prices=None):
        """strikes: device int64 [batch, nk]; returns device float64 [batch, nk]."""
        torch = _torch()
        if prices is None:
            prices = torch.empty(strikes.shape, dtype=torch.float64, device=strikes.device)
        self.build()
        self.core(strikes, prices)
        return prices

    def statuses(self) -> Dict[str, np.ndarray]:
        return {k: getattr(self, "st_" + k).cpu().numpy() for k in ("build", "apply", "round", "read")}


def dense_prices(problems: Sequence, dtype: int = CM_C64, strikes=None, device="cuda", stream=None, ws=None):
    """Dense Carr–Madan prices for problems sharing one n; all M prices if strikes is None."""
    torch = _torch()
    n = problems[0].n
    prob = pack_problems(problems, device)
    batch = len(problems)
    real = torch.float32 if dtype == CM_C64 else torch.float64
    if strikes is None:
        prices = torch.empty((batch, 2 ** n), dtype=real, device=device)
        nk = 0
    else:
        prices = torch.empty(strikes.shape, dtype=real, device=device)
        nk = strikes.shape[-1]
    status = torch.zeros(batch, dtype=torch.int32, device=device)
    ws = ws if ws is not None else Workspace(device)
    cm_fft_price(prob, batch, n, dtype, strikes, nk, prices, status, ws, stream)
    return prices, status

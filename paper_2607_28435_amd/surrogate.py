"""Pricing surrogate: a multilayer perceptron from (kappa, theta, sigma_v, rho, v0, T, k) to
C/S0 (k = ln(K/S0)), trained on batched SFFT prices by the library's own forward, backward
and Adam kernels, and gated by its training box plus a no-arbitrage residual, with the
SFFT path as fallback and as the reference for its error. A project addition: the paper has no
learned component.

Marshalling and orchestration only: data generation is cm_build_qtt .. cm_readout_prices,
training is cm_mlp_forward / cm_mlp_mse / cm_mlp_backward / cm_adam_step, inference is
cm_mlp_forward and cm_surrogate_gate.
"""
from __future__ import annotations

import ctypes as C
import math
import time
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

from . import (CM_C64, CM_E_MOMENT, CM_MLP_NPARAMS, CM_OK, CmMlp, ProblemArrays, cm_adam_step, cm_mlp_act_bytes,
               cm_mlp_backward, cm_mlp_forward, cm_mlp_mse, cm_mlp_sync_bf16, cm_surrogate_gate)
from .pipeline import MpoCache, SfftPricer

_LAYERS = [(256, 7), (256, 256), (256, 256), (256, 256), (1, 256)]   # (out, in)


def _torch():
    import torch
    return torch


def init_params(seed: int) -> np.ndarray:
    """Initial parameter vector (layout of cm.h): weights and biases uniform in
    +-1/sqrt(fan_in) per layer, from a Philox stream."""
    g = np.random.Generator(np.random.Philox(seed))
    parts = []
    for out, inp in _LAYERS:
        b = 1.0 / math.sqrt(inp)
        parts.append(g.uniform(-b, b, out * inp))
        parts.append(g.uniform(-b, b, out))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == CM_MLP_NPARAMS
    return theta


class MlpNet:
    """Device state of one network: FP32 master parameters, their BF16 copies, Adam
    moments and gradient, and grow-only scratch for activations."""

    def __init__(self, lo: Sequence[float], hi: Sequence[float], seed: int = 0, device="cuda", stream=None):
        torch = _torch()
        lo = np.asarray(lo, dtype=np.float64)
        hi = np.asarray(hi, dtype=np.float64)
        self.lo, self.hi = lo, hi
        shift = (lo + hi) / 2
        scale = 2.0 / (hi - lo)
        self.device, self.stream = device, stream
        self.params = torch.from_numpy(init_params(seed)).to(device)
        self.wbf = torch.zeros(3 * 256 * 256, dtype=torch.int16, device=device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.struct = CmMlp(self.params.data_ptr(), self.wbf.data_ptr(), (C.c_float * 7)(*shift.tolist()),
                            (C.c_float * 7)(*scale.tolist()))
        cm_mlp_sync_bf16(self.struct, stream)
        self.t = 0
        self._bufs: Dict[str, object] = {}

    def _buf(self, name: str, nbytes: int):
        torch = _torch()
        b = self._bufs.get(name)
        if b is None or b.numel() < nbytes:
            b = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
            self._bufs[name] = b
        return b

    def forward(self, x, out=None):
        """x: device float32 [B, 7] raw inputs -> device float32 [B] (inference scratch:
        two pre-activation buffers)."""
        torch = _torch()
        B = int(x.shape[0])
        y = out if out is not None else torch.empty(B, dtype=torch.float32, device=x.device)
        nb = cm_mlp_act_bytes(B) // 2
        acts = self._buf("infer", nb)
        cm_mlp_forward(self.struct, x, B, y, acts, nb, self.stream)
        return y

    def train_step(self, x, t, lr: float, loss_acc=None):
        """One Adam step on the mean squared error of the batch (x [B, 7], t [B], both
        device float32). loss_acc: optional device float scalar that accumulates the loss."""
        torch = _torch()
        B = int(x.shape[0])
        nb = cm_mlp_act_bytes(B)
        acts = self._buf("acts", nb)
        ws = self._buf("ws", nb // 2)
        y = self._buf("y", 4 * B).view(torch.float32)[:B]
        dy = self._buf("dy", 4 * B).view(torch.float32)[:B]
        cm_mlp_forward(self.struct, x, B, y, acts, nb, self.stream)
        cm_mlp_mse(y, t, B, dy, loss_acc, self.stream)
        cm_mlp_backward(self.struct, x, acts, dy, B, self.grad, ws, nb // 2, self.stream)
        self.t += 1
        cm_adam_step(self.struct, self.grad, self.m, self.v, self.t, lr, stream=self.stream)


# ------------------------------------------------------------------ SFFT prices for the surrogate

def eta_for(n: int) -> float:
    return 40.0 / 2.0 ** (n / 2)


def heston_arrays(params6: np.ndarray, n: int, S0: float, r: float, alpha: float, k0=None) -> ProblemArrays:
    """Problems for rows (kappa, theta, sigma_v, rho, v0, T) on an n-point Simpson grid."""
    p = np.asarray(params6, dtype=np.float64)
    return ProblemArrays("heston", "simpson1", n, S0, r, 0.0, p[:, 5], alpha, eta_for(n), p[:, :5], k0=k0)


# Where the Heston model stays defined (kappa, theta, sigma_v, rho, v0, T, k): the floors and
# ceilings a widened training box is clipped to.
_FLOOR = np.array([0.05, 0.001, 0.02, -0.98, 0.001, 0.02, -np.inf])
_CEIL = np.array([np.inf, np.inf, np.inf, 0.98, np.inf, np.inf, np.inf])


def widen(lo, hi, frac: float) -> Tuple[np.ndarray, np.ndarray]:
    """The box [lo, hi] with every interval widened by `frac` of its width (half on each
    side), clipped to where the model is defined."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    w = (hi - lo) * frac / 2
    return np.maximum(lo - w, _FLOOR), np.minimum(hi + w, _CEIL)


class Surrogate:
    """Gated surrogate over the trusted box [lo, hi] of (kappa, theta, sigma_v, rho, v0, T, k),
    k = ln(K/S0), for S0 and r fixed; SFFT prices (Simpson rule, n-point grids, alpha
    damping, complex64 contraction, tolerance tol) train and check it and price what the
    gate rejects. The gate accepts a query inside the box whose decoded price keeps the
    no-arbitrage bounds and, once `calibrate` has run, whose (T, k) cell showed a
    validation error within err_tol.

    The network is trained on a box `train_lo`/`train_hi` wider than the trusted one (by
    default 20 % of each width, clipped where the model stops being defined), so that no
    accepted query sits on the edge of the training data, and it predicts
    z = log(C/S0 + out_eps), which spreads the small prices of out-of-the-money strikes;
    the gate decodes C/S0 = e^z - out_eps."""

    def __init__(self, lo, hi, train_widen: float = 0.2, S0: float = 100.0, r: float = 0.03, n: int = 16,
                 alpha: float = 1.5, tol: float = 1e-8, res_tol: float = 1e-3, out_eps: float = 1e-2,
                 seed: int = 0, device="cuda"):
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)
        self.train_lo, self.train_hi = widen(self.lo, self.hi, train_widen)
        self.S0, self.r, self.n, self.alpha, self.tol, self.res_tol = S0, r, n, alpha, tol, res_tol
        self.out_eps = out_eps
        self.device = device
        self.net = MlpNet(self.train_lo, self.train_hi, seed=seed, device=device)
        self._mpo = None
        self.history = []
        self.cell_err = None      # calibrated (T, k) error table (device float32), see calibrate()
        self.err_tol = 0.0

    def encode(self, price_over_s0: np.ndarray) -> np.ndarray:
        """Training target for C/S0 (the inverse of the gate's decoding)."""
        c = np.asarray(price_over_s0, dtype=np.float64)
        return np.log(np.maximum(c, 0.0) + self.out_eps) if self.out_eps > 0 else c

    # -- SFFT prices
    def _mpo_cache(self):
        if self._mpo is None:
            self._mpo = MpoCache([self.n], self.tol / 10, 32, CM_C64, self.device)
        return self._mpo

    def grid_prices(self, params6: np.ndarray, ks: np.ndarray, chunk: int = 8192) -> Tuple[np.ndarray, np.ndarray]:
        """Training data: each parameter row priced at its row of log-moneyness values
        (snapped to the grid). Rows whose SFFT reports an error (for instance a damping
        moment that explodes before T) are dropped. Returns (X [rows*per, 7] with snapped k,
        C/S0 [rows*per])."""
        torch = _torch()
        n, M = self.n, 2 ** self.n
        lam = 2 * math.pi / (M * eta_for(n))
        params6 = np.asarray(params6, dtype=np.float64)
        u = np.rint(M / 2 + np.asarray(ks) / lam).astype(np.int64)
        k_snap = lam * (u - M / 2)
        out = np.empty(u.shape, dtype=np.float64)
        good = np.ones(len(params6), dtype=bool)
        for c0 in range(0, len(params6), chunk):
            sl = slice(c0, min(len(params6), c0 + chunk))
            pa = heston_arrays(params6[sl], n, self.S0, self.r, self.alpha)
            pr = SfftPricer(pa, CM_C64, tol=self.tol, cap=32, mpo=self._mpo_cache(), device=self.device)
            got = pr.run(torch.from_numpy(u[sl]).to(self.device))
            ok = np.ones(sl.stop - sl.start, dtype=bool)
            for v in pr.statuses().values():
                ok &= v == CM_OK
            good[sl] = ok
            out[sl] = got.cpu().numpy() / self.S0
        per = u.shape[1]
        X = np.concatenate([np.repeat(params6[good], per, axis=0), k_snap[good].reshape(-1, 1)], axis=1)
        return X, out[good].reshape(-1)

    def training_set(self, n_sets: int, per: int, seed: int) -> Tuple[np.ndarray, np.ndarray]:
        """n_sets parameter draws uniform in the training box, each priced at `per` uniform
        log-moneyness values (Philox streams seed and seed + 1)."""
        g = np.random.Generator(np.random.Philox(seed))
        lo, hi = self.train_lo, self.train_hi
        sets = lo[:6] + (hi[:6] - lo[:6]) * g.random((n_sets, 6))
        ks = np.random.Generator(np.random.Philox(seed + 1)).uniform(lo[6], hi[6], (n_sets, per))
        return self.grid_prices(sets, ks)

    def query_prices(self, queries: np.ndarray, chunk: int = 16384) -> Tuple[np.ndarray, np.ndarray]:
        """SFFT price of each query (kappa, theta, sigma_v, rho, v0, T, k) at exactly its k: the
        grid is shifted (k0) so that strike index M/2 is k. Problems whose damping moment
        explodes at alpha are re-priced at alpha/3. Returns (C/S0, status)."""
        torch = _torch()
        q = np.asarray(queries, dtype=np.float64)
        n, M = self.n, 2 ** self.n
        lam = 2 * math.pi / (M * eta_for(n))
        out = np.full(len(q), np.nan)
        status = np.zeros(len(q), dtype=np.int32)
        for c0 in range(0, len(q), chunk):
            sl = np.arange(c0, min(len(q), c0 + chunk))
            todo, alpha = sl, self.alpha
            for _attempt in range(2):
                k0 = math.log(self.S0) + q[todo, 6] - lam * (M / 2)
                pa = heston_arrays(q[todo, :6], n, self.S0, self.r, alpha, k0=k0)
                pr = SfftPricer(pa, CM_C64, tol=self.tol, cap=32, mpo=self._mpo_cache(), device=self.device)
                strikes = torch.full((len(todo), 1), M // 2, dtype=torch.int64, device=self.device)
                got = pr.run(strikes).cpu().numpy()[:, 0] / self.S0
                st = pr.statuses()
                code = np.zeros(len(todo), dtype=np.int32)
                for v in st.values():
                    code = np.where(code == CM_OK, v, code)
                out[todo] = np.where(code == CM_OK, got, np.nan)
                status[todo] = code
                retry = code == CM_E_MOMENT
                if not retry.any():
                    break
                todo, alpha = todo[retry], alpha / 3
        return out, status

    # -- training
    def fit(self, X: np.ndarray, Y: np.ndarray, steps: int, batch: int = 8192, lr: float = 2e-3,
            lr_final: float = 2e-5, warmup: int = 200, log_every: int = 500, seed: int = 1,
            time_budget: Optional[float] = None) -> Dict[str, float]:
        """Adam on the mean squared error of the encoded price (Y holds C/S0) with a warm-up
        and a cosine decay from lr to lr_final; minibatches are slices of a fresh
        permutation each epoch."""
        torch = _torch()
        Xd = torch.from_numpy(np.asarray(X, dtype=np.float32)).to(self.device)
        Yd = torch.from_numpy(self.encode(Y).astype(np.float32)).to(self.device)
        N = Xd.shape[0]
        gen = torch.Generator(device=self.device)
        gen.manual_seed(seed)
        loss_acc = torch.zeros(1, dtype=torch.float32, device=self.device)
        per_epoch = max(1, N // batch)
        perm = None
        t0 = time.perf_counter()
        done = 0
        for s in range(steps):
            j = s % per_epoch
            if j == 0:
                perm = torch.randperm(N, device=self.device, generator=gen)
            idx = perm[j * batch:(j + 1) * batch]
            if s < warmup:
                cur = lr * (s + 1) / warmup
            else:
                f = (s - warmup) / max(1, steps - warmup)
                cur = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * f))
            self.net.train_step(Xd.index_select(0, idx), Yd.index_select(0, idx), cur, loss_acc)
            done = s + 1
            if log_every and done % log_every == 0:
                self.history.append((done, float(loss_acc.item()) / log_every))
                loss_acc.zero_()
            if time_budget is not None and done % 100 == 0:
                torch.cuda.synchronize()
                if time.perf_counter() - t0 > time_budget:
                    break
        torch.cuda.synchronize()
        return {"steps": done, "seconds": time.perf_counter() - t0,
                "final_loss": self.history[-1][1] if self.history else float("nan")}

    # -- calibration of the gate
    def cell_index(self, T: np.ndarray, k: np.ndarray, nT: int, nk: int) -> Tuple[np.ndarray, np.ndarray]:
        """(T, k) cell of each query on an nT x nk grid over the trusted box, formed in
        float32 exactly as the gate kernel forms it."""
        f = np.float32
        lo, hi = self.lo.astype(f), self.hi.astype(f)
        fT = (np.asarray(T, dtype=f) - lo[5]) / (hi[5] - lo[5])
        fk = (np.asarray(k, dtype=f) - lo[6]) / (hi[6] - lo[6])
        iT = np.clip((fT * f(nT)).astype(np.int64), 0, nT - 1)
        ik = np.clip((fk * f(nk)).astype(np.int64), 0, nk - 1)
        return iT, ik

    def calibrate(self, n_val: int = 2 ** 15, seed: int = 4001, err_tol: float = 5e-4,
                  cells: Tuple[int, int] = (16, 16)) -> Dict[str, float]:
        """Residual calibration of the gate on a validation split: n_val queries uniform in
        the trusted box (a Philox stream of its own) are priced by the network and by the
        SFFT path; the largest |network - SFFT| / S0 in each (T, k) cell becomes the cell's
        error, and the gate then sends every query whose cell exceeds err_tol (by default
        half the 1e-3 S0 target, a margin for points the validation did not see) to the
        SFFT fallback. Cells without a validated query count as failed."""
        torch = _torch()
        nT, nk = cells
        g = np.random.Generator(np.random.Philox(seed))
        q = self.lo + (self.hi - self.lo) * g.random((n_val, 7))
        q32 = q.astype(np.float32)
        ref, st = self.query_prices(q32.astype(np.float64))
        qd = torch.from_numpy(q32).to(self.device)
        z = self.net.forward(qd)
        y = torch.exp(z.double()) - self.out_eps if self.out_eps > 0 else z.double()
        err = np.abs(y.cpu().numpy() - ref)
        err = np.where((st == CM_OK) & np.isfinite(err), err, np.inf)
        iT, ik = self.cell_index(q32[:, 5], q32[:, 6], nT, nk)
        table = np.full((nT, nk), np.inf)
        seen = np.zeros((nT, nk), dtype=bool)
        seen[iT, ik] = True
        table[seen] = 0.0
        np.maximum.at(table, (iT, ik), err)
        self.cell_err = torch.from_numpy(table.astype(np.float32)).to(self.device)
        self.err_tol = float(err_tol)
        return {"validation_queries": n_val, "cells": nT * nk, "cells_rejected": int((table > err_tol).sum()),
                "validation_max_err": float(err[np.isfinite(err)].max()),
                "validation_reference_failures": int((st != CM_OK).sum())}

    # -- inference
    def predict(self, queries_dev):
        """Decoded network price and gate for device float32 queries [B, 7]:
        (C/S0 [B] float32, accept [B] int32)."""
        torch = _torch()
        z = self.net.forward(queries_dev)
        B = queries_dev.shape[0]
        price = torch.empty(B, dtype=torch.float32, device=queries_dev.device)
        acc = torch.empty(B, dtype=torch.int32, device=queries_dev.device)
        cm_surrogate_gate(queries_dev, z, B, self.lo.tolist(), self.hi.tolist(), self.r, self.res_tol, acc,
                          out_eps=self.out_eps, price=price, cell_err=self.cell_err, err_tol=self.err_tol)
        return price, acc

    def price(self, queries: np.ndarray) -> Dict[str, np.ndarray]:
        """Gated prices C/S0 for host queries [B, 7]: the network where the gate accepts,
        the SFFT path elsewhere."""
        torch = _torch()
        qd = torch.from_numpy(np.asarray(queries, dtype=np.float32)).to(self.device)
        y, acc = self.predict(qd)
        y = y.double().cpu().numpy()
        acc = acc.cpu().numpy().astype(bool)
        out = y.copy()
        rej = np.where(~acc)[0]
        if len(rej):
            out[rej], _ = self.query_prices(np.asarray(queries, dtype=np.float64)[rej])
        return {"price": out, "accept": acc, "net": y}

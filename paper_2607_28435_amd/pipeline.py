"""Stage chaining on one stream: SFFT path (build QTT -> SFFT apply -> round -> readout)
and the dense path. Marshalling only; every stage is one call into libcm."""
from __future__ import annotations

from typing import Dict, Iterable, Optional, Sequence

import numpy as np

from . import (CM_C64, CM_C128, CM_TT_RIGHT_ORTHO, ProblemArrays, TTBatch, Workspace, cm_build_qtt, cm_fft_price,
               cm_qft_mpo, cm_qft_mpo_table,
               cm_readout_observable, cm_readout_prices, cm_sample_outcomes, cm_sfft_apply, cm_shot_prices,
               cm_tt_round, pack_problems)


def _torch():
    import torch
    return torch


class MpoCache:
    """Operator look-up table: Q_n for every n from min(ns) to max(ns), stored so that train
    n is Q_n (the layout cm_sfft_apply expects) and built by one cm_qft_mpo_table launch
    (one workgroup per operator). Q_n depends only on n, the tolerance, the bond cap and the
    storage type, so `save` writes the table to an .npz file and `load` restores it without
    constructing anything."""

    FORMAT = 1

    def __init__(self, ns: Iterable[int], tol: float, cap: int, dtype: int, device="cuda", stream=None,
                 build: bool = True):
        ns = sorted(set(int(n) for n in ns))
        self.tol, self.cap, self.dtype = tol, cap, dtype
        self.n_lo, self.n_hi = ns[0], ns[-1]
        slots = [n if self.n_lo <= n <= self.n_hi else 0 for n in range(self.n_hi + 1)]
        self.w = TTBatch(slots, 2, 2, cap, dtype, device)
        self.w.struct.n_max = self.n_hi
        self.ns = list(range(self.n_lo, self.n_hi + 1))
        if build:
            cm_qft_mpo_table(self.n_lo, self.n_hi, tol, cap, self.w, Workspace(device), stream)

    def save(self, path: str) -> None:
        """Writes the table (cores, bond dimensions and the parameters it was built with)."""
        np.savez(path, format=self.FORMAT, tol=self.tol, cap=self.cap, dtype=self.dtype, n_lo=self.n_lo,
                 n_hi=self.n_hi, rank_max=self.w.rank_max, ranks=self.w.ranks.cpu().numpy(),
                 core_off=self.w.core_off.cpu().numpy(), cores=self.w.cores.cpu().numpy())

    @classmethod
    def load(cls, path: str, device="cuda") -> "MpoCache":
        """Restores a table written by `save` (plain arrays; nothing in the file is executed)."""
        torch = _torch()
        with np.load(path, allow_pickle=False) as z:
            if int(z["format"]) != cls.FORMAT:
                raise ValueError(f"{path}: operator table format {int(z['format'])}, expected {cls.FORMAT}")
            m = cls(range(int(z["n_lo"]), int(z["n_hi"]) + 1), float(z["tol"]), int(z["cap"]), int(z["dtype"]),
                    device, build=False)
            if not np.array_equal(z["core_off"], m.w.core_off.cpu().numpy()) or z["cores"].shape != m.w.cores.shape:
                raise ValueError(f"{path}: operator table layout does not match")
            m.w.cores.copy_(torch.from_numpy(z["cores"]))
            m.w.ranks.copy_(torch.from_numpy(z["ranks"]))
            m.w.struct.rank_max = int(z["rank_max"])
        m.w.struct.flags = CM_TT_RIGHT_ORTHO
        return m


_SWEEP_OPS = ("build", "apply", "round")


class SfftPricer:
    """Batched SFFT pricing of a fixed list of problems on one stream.

    tol       : zip-up and rounding tolerance (relative Frobenius)
    build_tol : QTT construction tolerance (default tol/10)
    mpo_tol   : operator rounding tolerance (default tol/10)
    cap       : bond capacity of x and y (zip-up bonds are limited to min(cap, 48))
    slots     : persistent workgroups per sweep op ({"build": s, "apply": s, "round": s});
                None entries take the library default (see `autotune_slots`)

    Ragged batches are processed longest chain first (the persistent workgroups take
    instances b, b + slots, ..., so descending cost balances them); `run` and `statuses`
    return everything in the caller's order. `capture` records the whole chain as one HIP
    graph for replay.
    """

    def __init__(self, problems: Sequence, dtype: int = CM_C64, tol: float = 1e-8, cap: int = 32,
                 build_tol: Optional[float] = None, mpo_tol: Optional[float] = None, mpo: Optional[MpoCache] = None,
                 device="cuda", stream=None, slots: Optional[Dict[str, Optional[int]]] = None):
        torch = _torch()
        arrays = isinstance(problems, ProblemArrays)
        if not arrays:
            problems = list(problems)
        self.batch = len(problems)
        ns_in = [int(v) for v in problems.n] if arrays else [p.n for p in problems]
        if len(set(ns_in)) > 1:
            # longest chain first; stable among equal n
            self.order = sorted(range(self.batch), key=lambda i: -ns_in[i])
        else:
            self.order = list(range(self.batch))
        self.identity = self.order == list(range(self.batch))
        if arrays:
            self.problems = problems if self.identity else problems.take(self.order)
        else:
            self.problems = [problems[i] for i in self.order]
        self.dtype, self.tol, self.cap = dtype, tol, cap
        self.build_tol = tol / 10 if build_tol is None else build_tol
        ns = [ns_in[i] for i in self.order]
        self.ns = ns
        self.device = device
        self.prob = self.problems.pack(device) if arrays else pack_problems(self.problems, device)
        self.x = TTBatch(ns, 2, 1, cap, dtype, device)
        self.y = TTBatch(ns, 2, 1, cap, dtype, device)
        self.mpo = mpo if mpo is not None else MpoCache(ns, tol / 10 if mpo_tol is None else mpo_tol, cap, dtype,
                                                        device, stream)
        z = lambda: torch.zeros(self.batch, dtype=torch.int32, device=device)
        self.st_build, self.st_apply, self.st_round, self.st_read = z(), z(), z(), z()
        self.st_sample, self.st_shot = z(), z()
        self.round_err = torch.zeros(self.batch, dtype=torch.float64, device=device)
        self.ws = Workspace(device)
        self.stream = stream
        self.slots = {k: None for k in _SWEEP_OPS}
        if slots:
            self.slots.update(slots)
        self._perm = None if self.identity else torch.tensor(self.order, dtype=torch.int64, device=device)
        self._graph = None

    # -- stages (all on internal, cost-ordered rows)
    def build(self):
        cm_build_qtt(self.prob, self.batch, self.build_tol, self.cap, self.x, self.st_build, self.ws, self.stream,
                     slots=self.slots["build"])

    def apply(self):
        cm_sfft_apply(self.mpo.w, self.x, self.tol, self.cap, self.y, self.st_apply, self.ws, self.stream,
                      slots=self.slots["apply"])

    def round(self):
        cm_tt_round(self.y, self.tol, self.cap, self.round_err, self.st_round, self.ws, self.stream,
                    slots=self.slots["round"])

    def read(self, strikes_int, prices_int):
        self.st_read.zero_()
        cm_readout_prices(self.y, self.prob, strikes_int, strikes_int.shape[-1], prices_int, self.st_read,
                          self.stream)

    def core(self, strikes_int, prices_int):
        """The online part: SFFT apply, rounding and readout (x must be built); rows in
        internal order."""
        self.apply()
        self.round()
        self.read(strikes_int, prices_int)

    # -- caller-order interface
    def to_internal(self, rows):
        return rows if self.identity else rows.index_select(0, self._perm)

    def run(self, strikes, prices=None):
        """strikes: device int64 [batch, nk] (caller's order); returns device float64
        [batch, nk] in the caller's order."""
        torch = _torch()
        s_int = self.to_internal(strikes)
        p_int = torch.empty(s_int.shape, dtype=torch.float64, device=strikes.device)
        self.build()
        self.core(s_int, p_int)
        if self.identity:
            if prices is None:
                return p_int
            prices.copy_(p_int)
            return prices
        if prices is None:
            prices = torch.empty_like(p_int)
        prices.index_copy_(0, self._perm, p_int)
        return prices

    def statuses(self) -> Dict[str, np.ndarray]:
        out = {}
        for k in ("build", "apply", "round", "read", "sample", "shot"):
            v = getattr(self, "st_" + k).cpu().numpy()
            if not self.identity:
                w = np.empty_like(v)
                w[np.asarray(self.order)] = v
                v = w
            out[k] = v
        return out

    def _to_caller(self, rows):
        if self.identity:
            return rows
        out = _torch().empty_like(rows)
        out.index_copy_(0, self._perm, rows)
        return out

    # -- the QFT-observable arm (Section 2.2)
    def observable(self, strikes):
        """Observable prices with exact probabilities, exp(-alpha k)/(s pi) sqrt(M) |y_u|, for
        device int64 strikes [batch, nk] (caller's order); returns float64 [batch, nk]."""
        torch = _torch()
        s_int = self.to_internal(strikes)
        p_int = torch.empty(s_int.shape, dtype=torch.float64, device=strikes.device)
        self.build()
        self.apply()
        self.round()
        self.st_read.zero_()
        cm_readout_observable(self.y, self.prob, s_int, s_int.shape[-1], p_int, self.st_read, self.stream)
        return self._to_caller(p_int)

    def measure(self, strikes, uniforms):
        """Emulated QFT measurement: builds the output trains, draws R outcomes per
        instance with the caller's uniforms (device float64 [batch, n_max, R], bit-major) and prices
        the strikes (device int64 [batch, nk], strictly increasing per row) from the
        outcome counts. Returns (prices float64 [batch, nk], counts int32 [batch, nk],
        samples int64 [batch, R], norm2 float64 [batch]), all in the caller's order."""
        torch = _torch()
        R = int(uniforms.shape[2])
        dev = strikes.device
        s_int = self.to_internal(strikes)
        u_int = self.to_internal(uniforms)
        samples = torch.empty((self.batch, R), dtype=torch.int64, device=dev)
        norm2 = torch.empty(self.batch, dtype=torch.float64, device=dev)
        counts = torch.empty(s_int.shape, dtype=torch.int32, device=dev)
        prices = torch.empty(s_int.shape, dtype=torch.float64, device=dev)
        self.build()
        self.apply()
        self.round()
        self.st_sample.zero_()
        self.st_shot.zero_()
        cm_sample_outcomes(self.y, u_int, R, samples, norm2, self.st_sample, self.ws, self.stream)
        cm_shot_prices(self.prob, self.batch, norm2, samples, R, s_int, s_int.shape[-1], counts, prices,
                       self.st_shot, self.stream)
        return tuple(self._to_caller(t) for t in (prices, counts, samples, norm2))

    # -- HIP graph of the whole chain
    def capture(self, strikes):
        """Records build -> apply -> round -> readout (plus the caller-order permutations) as
        one HIP graph. Runs the chain once eagerly first so that every buffer exists; the
        graph then owns its input copy (`graph_strikes`) and output (`graph_prices`)."""
        torch = _torch()
        self.graph_strikes = strikes.clone()
        self.graph_prices = self.run(self.graph_strikes)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run(self.graph_strikes, self.graph_prices)
        self._graph = g
        return g

    def replay(self):
        if self._graph is None:
            raise RuntimeError("capture() first")
        self._graph.replay()
        return self.graph_prices


def autotune_slots(pricer: SfftPricer, strikes, candidates: Sequence[int] = (512, 1024, 2048, 4096), reps: int = 2,
                   cache_path: Optional[str] = None) -> Dict[str, int]:
    """Picks the persistent-workgroup count of each sweep op by timing the candidates on the
    pricer's own batch (HIP events, best of `reps`), stores the choice in pricer.slots and,
    if cache_path is given, in a JSON table keyed by device, dtype, cap, batch and the
    chain-length histogram (read back on the next call instead of re-timing)."""
    import json
    import os
    torch = _torch()
    key = "|".join([torch.cuda.get_device_name(), str(pricer.dtype), str(pricer.cap), str(pricer.batch),
                    ",".join(f"{n}:{c}" for n, c in sorted(_hist(pricer.ns).items()))])
    table = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            table = json.load(f)
        if key in table:
            pricer.slots.update({k: int(v) for k, v in table[key].items()})
            return dict(pricer.slots)
    cands = sorted(set(min(int(c), pricer.batch) for c in candidates))
    s_int = pricer.to_internal(strikes)
    p_int = torch.empty(s_int.shape, dtype=torch.float64, device=strikes.device)
    stream = torch.cuda.current_stream()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    pricer.build()
    pricer.core(s_int, p_int)
    torch.cuda.synchronize()
    best = {}
    for op in _SWEEP_OPS:
        res = {}
        for c in cands:
            pricer.slots[op] = c
            t = []
            for _ in range(reps):
                if op == "build":
                    t.append(timed(pricer.build))
                elif op == "apply":
                    t.append(timed(pricer.apply))
                else:
                    pricer.apply()   # rounding works in place: start from a fresh zip-up output
                    t.append(timed(pricer.round))
            res[c] = min(t)
        best[op] = min(res, key=res.get)
        pricer.slots[op] = best[op]
    if cache_path:
        table[key] = best
        with open(cache_path, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return best


def _hist(values) -> Dict[int, int]:
    h: Dict[int, int] = {}
    for v in values:
        h[int(v)] = h.get(int(v), 0) + 1
    return h


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

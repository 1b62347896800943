"""Python binding of libcm (MI355X SFFT Carr–Madan pricing).

Argument marshalling only: every computation runs in the HIP kernels of libcm.so. PyTorch
provides device memory and the current stream. Importing this package does not load the
library; the first call does, and raises if libcm.so has not been built (there is no CPU
fallback).

The entry points keep the C ABI's names (include/cm.h): cm_qft_mpo, cm_build_qtt,
cm_sfft_apply, cm_tt_round, cm_readout_prices, cm_fft_price, plus cm_workspace_bytes,
cm_tt_layout, cm_status_str. `TTBatch` owns the device buffers of a ragged batch of
trains; `pack_problems` turns problem descriptions into the device array of cm_problem.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcm.so")

CM_MAX_N = 48
CM_RANKS_STRIDE = 49
CM_OK, CM_E_INVALID, CM_E_MOMENT, CM_E_RANKCAP, CM_E_NOCONV, CM_E_NONFINITE, CM_E_HIP, CM_E_UNSUPPORTED = range(8)
CM_BS, CM_MERTON, CM_HESTON, CM_VG = range(4)
CM_QUAD_RECT2, CM_QUAD_SIMPSON1 = range(2)
CM_C64, CM_C128 = range(2)
CM_OP_QFT_MPO, CM_OP_BUILD_QTT, CM_OP_SFFT_APPLY, CM_OP_TT_ROUND, CM_OP_FFT_PRICE, CM_OP_SAMPLE = range(6)
CM_TT_LEFT_ORTHO, CM_TT_RIGHT_ORTHO = 1, 2

_MODEL = {"bs": CM_BS, "merton": CM_MERTON, "heston": CM_HESTON, "vg": CM_VG}
_QUAD = {"rect2": CM_QUAD_RECT2, "simpson1": CM_QUAD_SIMPSON1}

PROBLEM_DTYPE = np.dtype([
    ("model", "<i4"), ("quad", "<i4"), ("n", "<i4"), ("flags", "<i4"),
    ("S0", "<f8"), ("r", "<f8"), ("q", "<f8"), ("T", "<f8"), ("alpha", "<f8"), ("eta", "<f8"),
    ("k0", "<f8"), ("p", "<f8", (5,)), ("reserved", "<f8", (2,)),
])
assert PROBLEM_DTYPE.itemsize == 128


class CmTTBatch(C.Structure):
    _fields_ = [
        ("batch", C.c_int32), ("d_out", C.c_int32), ("d_in", C.c_int32), ("cap_rank", C.c_int32),
        ("n_max", C.c_int32), ("dtype", C.c_int32), ("rank_max", C.c_int32), ("flags", C.c_int32),
        ("n", C.c_void_p), ("ranks", C.c_void_p), ("core_off", C.c_void_p), ("cores", C.c_void_p),
    ]


class CmMlp(C.Structure):
    _fields_ = [("params", C.c_void_p), ("w_bf16", C.c_void_p), ("shift", C.c_float * 7), ("scale", C.c_float * 7)]


CM_MLP_NIN, CM_MLP_WIDTH, CM_MLP_NPARAMS = 7, 256, 199681

_lib = None


def lib() -> C.CDLL:
    """Loads libcm.so (once). Raises RuntimeError if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libcm.so not found at {LIB_PATH}; build it with "
                           "`python -m paper_2607_28435_amd.build` (no CPU fallback exists)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, f64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    pb = C.POINTER(CmTTBatch)
    sig = {
        "cm_tt_layout": (i64, [C.c_int, C.c_int, C.c_int, C.c_int, vp]),
        "cm_workspace_bytes": (sz, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]),
        "cm_qft_mpo": (C.c_int, [C.c_int, f64, C.c_int, pb, C.c_int, vp, sz, vp]),
        "cm_qft_mpo_table": (C.c_int, [C.c_int, C.c_int, f64, C.c_int, pb, vp, sz, vp]),
        "cm_build_qtt": (C.c_int, [vp, C.c_int, f64, C.c_int, pb, vp, vp, sz, vp]),
        "cm_sfft_apply": (C.c_int, [pb, pb, f64, C.c_int, pb, vp, vp, sz, vp]),
        "cm_sfft_apply_noalloc": (C.c_int, [pb, pb, f64, C.c_int, pb, vp, vp]),
        "cm_sfft_apply_noalloc_scratch_bytes": (sz, []),
        "cm_tt_round": (C.c_int, [pb, f64, C.c_int, vp, vp, vp, sz, vp]),
        "cm_readout_prices": (C.c_int, [pb, vp, vp, C.c_int, vp, vp, vp]),
        "cm_readout_observable": (C.c_int, [pb, vp, vp, C.c_int, vp, vp, vp]),
        "cm_sample_outcomes": (C.c_int, [pb, vp, C.c_int, vp, vp, vp, vp, sz, vp]),
        "cm_shot_prices": (C.c_int, [vp, C.c_int, vp, vp, C.c_int, vp, C.c_int, vp, vp, vp, vp]),
        "cm_fft_price": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, vp, C.c_int, vp, vp, vp, sz, vp]),
        "cm_mlp_act_bytes": (sz, [C.c_int]),
        "cm_mlp_sync_bf16": (C.c_int, [C.POINTER(CmMlp), vp]),
        "cm_mlp_forward": (C.c_int, [C.POINTER(CmMlp), vp, C.c_int, vp, vp, sz, vp]),
        "cm_mlp_backward": (C.c_int, [C.POINTER(CmMlp), vp, vp, vp, C.c_int, vp, vp, sz, vp]),
        "cm_mlp_mse": (C.c_int, [vp, vp, C.c_int, vp, vp, vp]),
        "cm_adam_step": (C.c_int, [C.POINTER(CmMlp), vp, vp, vp, C.c_int, C.c_float, C.c_float, C.c_float,
                                   C.c_float, vp]),
        "cm_surrogate_gate": (C.c_int, [vp, vp, C.c_int, vp, vp, C.c_float, C.c_float, C.c_float, vp, C.c_int,
                                        C.c_int, C.c_float, vp, vp, vp]),
        "cm_status_str": (C.c_char_p, [C.c_int]),
        "cm_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def exported_symbols() -> List[str]:
    return ["cm_tt_layout", "cm_workspace_bytes", "cm_qft_mpo", "cm_qft_mpo_table", "cm_build_qtt", "cm_sfft_apply",
            "cm_sfft_apply_noalloc", "cm_sfft_apply_noalloc_scratch_bytes", "cm_tt_round", "cm_readout_prices",
            "cm_readout_observable", "cm_sample_outcomes",
            "cm_shot_prices", "cm_fft_price", "cm_mlp_act_bytes", "cm_mlp_sync_bf16",
            "cm_mlp_forward", "cm_mlp_backward", "cm_mlp_mse", "cm_adam_step", "cm_surrogate_gate",
            "cm_status_str", "cm_version"]


class CmError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {cm_status_str(code)} (code {code})")
        self.code = code


def _check(code: int, where: str) -> int:
    if code != CM_OK:
        raise CmError(code, where)
    return code


def cm_status_str(code: int) -> str:
    return lib().cm_status_str(int(code)).decode()


def cm_version() -> str:
    return lib().cm_version().decode()


def cm_workspace_bytes(op: int, batch: int, n_max: int, cap_rank: int, dtype: int) -> int:
    return int(lib().cm_workspace_bytes(op, batch, n_max, cap_rank, dtype))


def cm_tt_layout(n: int, d_out: int, d_in: int, cap_rank: int) -> Tuple[int, np.ndarray]:
    off = np.zeros(CM_MAX_N, dtype=np.int64)
    total = lib().cm_tt_layout(n, d_out, d_in, cap_rank, off.ctypes.data)
    if total < 0:
        raise CmError(CM_E_INVALID, "cm_tt_layout")
    return int(total), off[:n].copy()


# ------------------------------------------------------------------ device helpers

def _torch():
    import torch
    return torch


def _stream_ptr(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def pack_problems(problems: Sequence, device="cuda"):
    """Device array (torch.uint8, 128 bytes per problem) of cm_problem structs."""
    torch = _torch()
    a = np.zeros(len(problems), dtype=PROBLEM_DTYPE)
    for i, p in enumerate(problems):
        a[i]["model"] = _MODEL[p.model]
        a[i]["quad"] = _QUAD[p.quad]
        a[i]["n"] = p.n
        a[i]["S0"], a[i]["r"], a[i]["q"], a[i]["T"] = p.S0, p.r, p.q, p.T
        a[i]["alpha"], a[i]["eta"] = p.alpha, p.eta
        a[i]["k0"] = math.nan if p.k0 is None else p.k0
        pp = list(p.params) + [0.0] * (5 - len(p.params))
        a[i]["p"] = pp
    t = torch.from_numpy(a.view(np.uint8).copy())
    return t.to(device)


class ProblemArrays:
    """A batch of problems held as numpy arrays (one entry per problem), for batches too
    large to describe problem by problem. Fields follow cm_problem; `model`/`quad` are
    strings shared by the whole batch, `p` is [count, 5]."""

    def __init__(self, model: str, quad: str, n, S0, r, q, T, alpha, eta, p, k0=None):
        count = len(np.atleast_1d(T))
        full = lambda v, dt=np.float64: np.broadcast_to(np.asarray(v, dtype=dt), (count,)).copy()
        self.model, self.quad = model, quad
        self.n = full(n, np.int32)
        self.S0, self.r, self.q, self.T = full(S0), full(r), full(q), full(T)
        self.alpha, self.eta = full(alpha), full(eta)
        self.k0 = full(math.nan if k0 is None else k0)
        pp = np.zeros((count, 5))
        pa = np.asarray(p, dtype=np.float64)
        pp[:, :pa.shape[1]] = pa
        self.p = pp

    def __len__(self):
        return len(self.T)

    def take(self, idx) -> "ProblemArrays":
        idx = np.asarray(idx)
        return ProblemArrays(self.model, self.quad, self.n[idx], self.S0[idx], self.r[idx], self.q[idx],
                             self.T[idx], self.alpha[idx], self.eta[idx], self.p[idx], self.k0[idx])

    def pack(self, device="cuda"):
        torch = _torch()
        a = np.zeros(len(self), dtype=PROBLEM_DTYPE)
        a["model"] = _MODEL[self.model]
        a["quad"] = _QUAD[self.quad]
        a["n"] = self.n
        a["S0"], a["r"], a["q"], a["T"] = self.S0, self.r, self.q, self.T
        a["alpha"], a["eta"], a["k0"] = self.alpha, self.eta, self.k0
        a["p"] = self.p
        return torch.from_numpy(a.view(np.uint8).copy()).to(device)


class TTBatch:
    """Device buffers of a ragged batch of trains (or operators) in capacity layout."""

    def __init__(self, ns: Sequence[int], d_out: int, d_in: int, cap_rank: int, dtype: int, device="cuda"):
        torch = _torch()
        self.ns = [int(x) for x in ns]
        self.batch = len(self.ns)
        self.d_out, self.d_in, self.cap_rank, self.dtype = d_out, d_in, cap_rank, dtype
        offs = np.zeros((self.batch, CM_MAX_N), dtype=np.int64)
        total = 0
        for b, n in enumerate(self.ns):
            if n <= 0:
                continue
            per, off = cm_tt_layout(n, d_out, d_in, cap_rank)
            offs[b, :n] = off + total
            total += per
        ctype = torch.complex64 if dtype == CM_C64 else torch.complex128
        self.cores = torch.zeros(max(total, 1), dtype=ctype, device=device)
        self.ranks = torch.ones((self.batch, CM_RANKS_STRIDE), dtype=torch.int32, device=device)
        self.n = torch.tensor(self.ns, dtype=torch.int32, device=device)
        self.core_off = torch.from_numpy(offs).to(device)
        self._s = CmTTBatch(self.batch, d_out, d_in, cap_rank, max(self.ns) if self.ns else 0, dtype, 0, 0,
                            _ptr(self.n), _ptr(self.ranks), _ptr(self.core_off), _ptr(self.cores))

    @property
    def struct(self) -> CmTTBatch:
        return self._s

    @property
    def rank_max(self) -> int:
        return int(self._s.rank_max)

    def host_cores(self, b: int) -> List[np.ndarray]:
        """Copies train b to host as a list of arrays [r_l, d_out*d_in, r_{l+1}]."""
        n = self.ns[b]
        rk = self.ranks[b].cpu().numpy()
        off = self.core_off[b].cpu().numpy()
        allc = self.cores.cpu().numpy()
        d = self.d_out * self.d_in
        out = []
        for l in range(n):
            cnt = rk[l] * d * rk[l + 1]
            out.append(allc[off[l]:off[l] + cnt].reshape(rk[l], d, rk[l + 1]).astype(np.complex128))
        return out

    def bytes_used(self, b: int) -> int:
        """Bytes of the stored cores of train b at their current ranks."""
        rk = self.ranks[b].cpu().numpy()
        d = self.d_out * self.d_in
        es = 8 if self.dtype == CM_C64 else 16
        return int(sum(rk[l] * d * rk[l + 1] for l in range(self.ns[b])) * es)


class Workspace:
    """Grows-only device byte buffer reused across calls."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = None

    def get(self, nbytes: int):
        torch = _torch()
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self.buf


# ------------------------------------------------------------------ the C ABI entry points

def _sweep_ws_bytes(op: int, batch: int, n_max: int, cap_rank: int, dtype: int, slots: Optional[int]) -> int:
    """Workspace bytes for a sweep op: the library's default, or exactly `slots` slabs (the
    library runs one persistent workgroup per slab)."""
    if slots is None:
        return cm_workspace_bytes(op, batch, n_max, cap_rank, dtype)
    slab = cm_workspace_bytes(op, 1, n_max, cap_rank, dtype)
    return slab * max(1, min(int(slots), batch))


def cm_qft_mpo(n: int, tol: float, cap_rank: int, w: TTBatch, slot: int, ws: Workspace, stream=None) -> int:
    need = cm_workspace_bytes(CM_OP_QFT_MPO, 1, n, cap_rank, w.dtype)
    buf = ws.get(need)
    code = lib().cm_qft_mpo(n, tol, cap_rank, C.byref(w.struct), slot, _ptr(buf), buf.numel(), _stream_ptr(stream))
    return _check(code, "cm_qft_mpo")


def cm_qft_mpo_table(n_lo: int, n_hi: int, tol: float, cap_rank: int, w: TTBatch, ws: Workspace,
                     stream=None) -> int:
    need = cm_workspace_bytes(CM_OP_QFT_MPO, n_hi - n_lo + 1, n_hi, cap_rank, w.dtype)
    buf = ws.get(need)
    code = lib().cm_qft_mpo_table(n_lo, n_hi, tol, cap_rank, C.byref(w.struct), _ptr(buf), buf.numel(),
                                  _stream_ptr(stream))
    return _check(code, "cm_qft_mpo_table")


def cm_build_qtt(prob_dev, batch: int, tol: float, cap_rank: int, x: TTBatch, status, ws: Workspace,
                 stream=None, slots: Optional[int] = None) -> int:
    need = _sweep_ws_bytes(CM_OP_BUILD_QTT, batch, x.struct.n_max, cap_rank, x.dtype, slots)
    buf = ws.get(need)
    code = lib().cm_build_qtt(_ptr(prob_dev), batch, tol, cap_rank, C.byref(x.struct), _ptr(status), _ptr(buf),
                              need, _stream_ptr(stream))
    return _check(code, "cm_build_qtt")


def cm_sfft_apply(w_by_n: TTBatch, x: TTBatch, tol: float, cap_rank: int, y: TTBatch, status, ws: Workspace,
                  stream=None, slots: Optional[int] = None) -> int:
    need = _sweep_ws_bytes(CM_OP_SFFT_APPLY, x.batch, x.struct.n_max, cap_rank, x.dtype, slots)
    buf = ws.get(need)
    code = lib().cm_sfft_apply(C.byref(w_by_n.struct), C.byref(x.struct), tol, cap_rank, C.byref(y.struct),
                               _ptr(status), _ptr(buf), need, _stream_ptr(stream))
    return _check(code, "cm_sfft_apply")


def cm_sfft_apply_noalloc(w_by_n: TTBatch, x: TTBatch, tol: float, cap_rank: int, y: TTBatch, status,
                          stream=None) -> int:
    """cm_sfft_apply with the library's fixed device scratch array instead of a workspace
    (the call allocates nothing)."""
    code = lib().cm_sfft_apply_noalloc(C.byref(w_by_n.struct), C.byref(x.struct), tol, cap_rank, C.byref(y.struct),
                                       _ptr(status), _stream_ptr(stream))
    return _check(code, "cm_sfft_apply_noalloc")


def cm_sfft_apply_noalloc_scratch_bytes() -> int:
    return int(lib().cm_sfft_apply_noalloc_scratch_bytes())


def cm_tt_round(t: TTBatch, tol: float, cap_rank: int, err_out, status, ws: Workspace, stream=None,
                slots: Optional[int] = None) -> int:
    need = _sweep_ws_bytes(CM_OP_TT_ROUND, t.batch, t.struct.n_max, t.cap_rank, t.dtype, slots)
    buf = ws.get(need)
    code = lib().cm_tt_round(C.byref(t.struct), tol, cap_rank, _ptr(err_out), _ptr(status), _ptr(buf), need,
                             _stream_ptr(stream))
    return _check(code, "cm_tt_round")


def cm_readout_prices(y: TTBatch, prob_dev, strike_idx, nk: int, prices, status=None, stream=None) -> int:
    code = lib().cm_readout_prices(C.byref(y.struct), _ptr(prob_dev), _ptr(strike_idx), nk, _ptr(prices),
                                   _ptr(status), _stream_ptr(stream))
    return _check(code, "cm_readout_prices")


def cm_readout_observable(y: TTBatch, prob_dev, strike_idx, nk: int, prices, status=None, stream=None) -> int:
    code = lib().cm_readout_observable(C.byref(y.struct), _ptr(prob_dev), _ptr(strike_idx), nk, _ptr(prices),
                                       _ptr(status), _stream_ptr(stream))
    return _check(code, "cm_readout_observable")


def cm_sample_outcomes(y: TTBatch, uniforms, R: int, out, norm2, status, ws: Workspace, stream=None) -> int:
    """uniforms: float64 [batch][y.n_max][R] (bit-major); out: int64 [batch][R]; norm2: float64 [batch]."""
    need = cm_workspace_bytes(CM_OP_SAMPLE, y.batch, y.struct.n_max, y.cap_rank, y.dtype)
    buf = ws.get(need)
    code = lib().cm_sample_outcomes(C.byref(y.struct), _ptr(uniforms), R, _ptr(out), _ptr(norm2), _ptr(status),
                                    _ptr(buf), need, _stream_ptr(stream))
    return _check(code, "cm_sample_outcomes")


def cm_shot_prices(prob_dev, batch: int, norm2, samples, R: int, strike_idx, nk: int, counts, prices, status=None,
                   stream=None) -> int:
    code = lib().cm_shot_prices(_ptr(prob_dev), batch, _ptr(norm2), _ptr(samples), R, _ptr(strike_idx), nk,
                                _ptr(counts), _ptr(prices), _ptr(status), _stream_ptr(stream))
    return _check(code, "cm_shot_prices")


def cm_fft_price(prob_dev, batch: int, n: int, dtype: int, strike_idx, nk: int, prices, status, ws: Workspace,
                 stream=None) -> int:
    need = cm_workspace_bytes(CM_OP_FFT_PRICE, batch, n, 0, dtype)
    buf = ws.get(need)
    code = lib().cm_fft_price(_ptr(prob_dev), batch, n, dtype, _ptr(strike_idx), nk, _ptr(prices), _ptr(status),
                              _ptr(buf), buf.numel(), _stream_ptr(stream))
    return _check(code, "cm_fft_price")


# ------------------------------------------------------------------ surrogate network

def cm_mlp_act_bytes(B: int) -> int:
    return int(lib().cm_mlp_act_bytes(int(B)))


def cm_mlp_sync_bf16(net: CmMlp, stream=None) -> int:
    return _check(lib().cm_mlp_sync_bf16(C.byref(net), _stream_ptr(stream)), "cm_mlp_sync_bf16")


def cm_mlp_forward(net: CmMlp, x, B: int, y, acts, acts_bytes: int, stream=None) -> int:
    code = lib().cm_mlp_forward(C.byref(net), _ptr(x), int(B), _ptr(y), _ptr(acts), int(acts_bytes),
                                _stream_ptr(stream))
    return _check(code, "cm_mlp_forward")


def cm_mlp_backward(net: CmMlp, x, acts, dy, B: int, grad, ws, ws_bytes: int, stream=None) -> int:
    code = lib().cm_mlp_backward(C.byref(net), _ptr(x), _ptr(acts), _ptr(dy), int(B), _ptr(grad), _ptr(ws),
                                 int(ws_bytes), _stream_ptr(stream))
    return _check(code, "cm_mlp_backward")


def cm_mlp_mse(y, t, B: int, dy, loss, stream=None) -> int:
    return _check(lib().cm_mlp_mse(_ptr(y), _ptr(t), int(B), _ptr(dy), _ptr(loss), _stream_ptr(stream)),
                  "cm_mlp_mse")


def cm_adam_step(net: CmMlp, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8, stream=None) -> int:
    code = lib().cm_adam_step(C.byref(net), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr), float(beta1),
                              float(beta2), float(eps), _stream_ptr(stream))
    return _check(code, "cm_adam_step")


def cm_surrogate_gate(x, z, B: int, lo: Sequence[float], hi: Sequence[float], r: float, res_tol: float, accept,
                      out_eps: float = 0.0, price=None, cell_err=None, err_tol: float = 0.0, stream=None) -> int:
    """cell_err: optional device float32 [nT, nk] calibrated error table over (T, k)."""
    lo_a = (C.c_float * 7)(*[float(v) for v in lo])
    hi_a = (C.c_float * 7)(*[float(v) for v in hi])
    nT, nk = (int(cell_err.shape[0]), int(cell_err.shape[1])) if cell_err is not None else (0, 0)
    code = lib().cm_surrogate_gate(_ptr(x), _ptr(z), int(B), C.cast(lo_a, C.c_void_p), C.cast(hi_a, C.c_void_p),
                                   float(r), float(res_tol), float(out_eps), _ptr(cell_err), nT, nk, float(err_tol),
                                   _ptr(price), _ptr(accept), _stream_ptr(stream))
    return _check(code, "cm_surrogate_gate")


from .pipeline import MpoCache, SfftPricer, autotune_slots, dense_prices  # noqa: E402
from .surrogate import MlpNet, Surrogate  # noqa: E402

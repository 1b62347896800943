"""Host-side checks of the C ABI library: it loads, exports every function declared in
include/cm.h, and its pure host helpers (layout, workspace sizes, status strings) behave.
No GPU compute is called here."""
import os
import re

import numpy as np
import pytest

import paper_2607_28435_amd as cm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cm_\w+)\s*\(", src)))


def test_library_exports_every_declared_function():
    L = cm.lib()
    names = _declared()
    assert {"cm_qft_mpo", "cm_build_qtt", "cm_sfft_apply", "cm_tt_round", "cm_readout_prices",
            "cm_fft_price"} <= set(names)
    for nm in names:
        assert hasattr(L, nm), nm


def test_problem_struct_layout():
    assert cm.PROBLEM_DTYPE.itemsize == 128
    assert cm.PROBLEM_DTYPE.fields["S0"][1] == 16
    assert cm.PROBLEM_DTYPE.fields["k0"][1] == 64
    import ctypes
    assert ctypes.sizeof(cm.CmTTBatch) == 64


def test_tt_layout_bounds():
    total, off = cm.cm_tt_layout(6, 2, 1, 3)
    # interior bonds min(3, 2^l): 1,2,3,3,3,3,1
    r = [1, 2, 3, 3, 3, 3, 1]
    assert total == sum(r[l] * 2 * r[l + 1] for l in range(6))
    assert list(off) == list(np.cumsum([0] + [r[l] * 2 * r[l + 1] for l in range(5)]))
    total4, _ = cm.cm_tt_layout(5, 2, 2, 64)
    r4 = [1, 4, 16, 64, 64, 1]
    assert total4 == sum(r4[l] * 4 * r4[l + 1] for l in range(5))
    with pytest.raises(cm.CmError):
        cm.cm_tt_layout(0, 2, 1, 4)


def test_workspace_sizes():
    for op in (cm.CM_OP_QFT_MPO, cm.CM_OP_BUILD_QTT, cm.CM_OP_SFFT_APPLY, cm.CM_OP_TT_ROUND):
        a = cm.cm_workspace_bytes(op, 4, 24, 32, cm.CM_C64)
        b = cm.cm_workspace_bytes(op, 4, 24, 64, cm.CM_C64)
        assert 0 < a <= b
    assert cm.cm_workspace_bytes(cm.CM_OP_FFT_PRICE, 1, 24, 0, cm.CM_C64) >= 8 * 2 ** 24
    assert cm.cm_workspace_bytes(cm.CM_OP_BUILD_QTT, 4, 24, 65, cm.CM_C64) == 0
    assert cm.cm_workspace_bytes(99, 4, 24, 32, cm.CM_C64) == 0


def test_status_strings():
    for code in range(8):
        assert cm.cm_status_str(code)
    assert "moment" in cm.cm_status_str(cm.CM_E_MOMENT)
    assert cm.cm_version().startswith("cm-sfft")


def test_sweep_workspace_is_per_slot():
    """Sweep ops run one persistent workgroup per workspace slab: the default size is
    min(batch, 2048) slabs and an explicit slot count asks for exactly that many."""
    from paper_2607_28435_amd import _sweep_ws_bytes
    for op in (cm.CM_OP_BUILD_QTT, cm.CM_OP_SFFT_APPLY, cm.CM_OP_TT_ROUND):
        slab = cm.cm_workspace_bytes(op, 1, 24, 32, cm.CM_C64)
        assert slab > 0
        assert cm.cm_workspace_bytes(op, 100, 24, 32, cm.CM_C64) == 100 * slab
        assert cm.cm_workspace_bytes(op, 5000, 24, 32, cm.CM_C64) == 2048 * slab
        assert _sweep_ws_bytes(op, 100, 24, 32, cm.CM_C64, 7) == 7 * slab
        assert _sweep_ws_bytes(op, 5, 24, 32, cm.CM_C64, 7) == 5 * slab
        assert _sweep_ws_bytes(op, 100, 24, 32, cm.CM_C64, None) == 100 * slab


def test_sample_workspace_is_environment_slab():
    """The sampler keeps, per instance, n_max + 1 environment slots and n_max core slots of
    two FP64 complex blocks each, of edge RS = min(cap, 32) rounded up to a multiple of 4."""
    assert cm.cm_workspace_bytes(cm.CM_OP_SAMPLE, 3, 24, 64, cm.CM_C64) == 3 * (3 * 24 + 1) * 32 * 32 * 16
    assert cm.cm_workspace_bytes(cm.CM_OP_SAMPLE, 2, 10, 8, cm.CM_C128) == 2 * 31 * 8 * 8 * 16
    assert cm.cm_workspace_bytes(cm.CM_OP_SAMPLE, 1, 10, 10, cm.CM_C128) == 31 * 12 * 12 * 16
    assert cm.cm_workspace_bytes(cm.CM_OP_SAMPLE, 2, 10, 257, cm.CM_C128) == 0


def test_operator_table_file_round_trip(tmp_path):
    """The operator look-up table's file format (host logic only; no GPU): a table written by
    `save` loads back with identical cores, bond dimensions and parameters, and a file of
    another layout is refused."""
    import torch
    m = cm.MpoCache([3, 4, 5, 6], 1e-9, 8, cm.CM_C128, device="cpu", build=False)
    g = np.random.default_rng(0)
    m.w.cores.copy_(torch.from_numpy(g.standard_normal(m.w.cores.shape) + 1j * g.standard_normal(m.w.cores.shape)))
    rk = np.ones(m.w.ranks.shape, dtype=np.int32)
    for n in range(3, 7):
        rk[n, 1:n] = 4
    m.w.ranks.copy_(torch.from_numpy(rk))
    m.w.struct.rank_max = 4
    path = str(tmp_path / "qft_table.npz")
    m.save(path)
    r = cm.MpoCache.load(path, device="cpu")
    assert (r.n_lo, r.n_hi, r.tol, r.cap, r.dtype) == (3, 6, 1e-9, 8, cm.CM_C128)
    assert torch.equal(r.w.cores, m.w.cores) and torch.equal(r.w.ranks, m.w.ranks)
    assert r.w.rank_max == 4 and r.w.struct.flags == cm.CM_TT_RIGHT_ORTHO
    other = cm.MpoCache([3, 4, 5, 6], 1e-9, 16, cm.CM_C128, device="cpu", build=False)
    other.save(path)
    z = dict(np.load(path, allow_pickle=False))
    z["cap"] = np.array(8)
    np.savez(path, **z)
    with pytest.raises(ValueError):
        cm.MpoCache.load(path, device="cpu")

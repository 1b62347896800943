"""Surrogate network kernels (cm_mlp_*, cm_adam_step, cm_surrogate_gate) through the C ABI
against the CPU FP64 reference (oracle/mlp.py), and the gated surrogate end to end.

Tolerances: the 256 x 256 layers multiply BF16 weights (the reference uses the same
BF16-rounded weights) by activations split into two BF16 parts (relative rounding about
2^-17) with FP32 accumulation, so the forward pass matches to ~1e-5 relative. The weight
gradients g_ij = sum_b delta_i[b] a_j[b] multiply the split delta (2^-17) by single-BF16
activations (round to nearest: relative 2^-9), so every element is checked against
|g - g_ref| <= 2^-8 sum_b |delta_i[b]| |a_j[b]|: the 2^-9 of the activation operand plus
about as much again for the FP32 accumulation over the batch and the ~2^-12 relative
error delta and a carry from the chain (both measured on the reference's own delta and
a)."""
import math
import sys
import time

import numpy as np
import pytest

import cm_workloads as W
from oracle import carr_madan as O
from oracle import mlp as R

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2607_28435_amd as cm  # noqa: E402
from paper_2607_28435_amd.surrogate import MlpNet, Surrogate, init_params  # noqa: E402


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


def _effective_theta(theta32):
    """The parameters the kernels actually multiply by: W2..W4 rounded to BF16."""
    th = theta32.astype(np.float64).copy()
    p = R.unpack(th)
    for l in (2, 3, 4):
        p[f"W{l}"][...] = R.bf16_round(p[f"W{l}"])
    return R.pack(p)


def _net_and_inputs(B, seed=3, scale_hidden=1.0):
    lo, hi = W.surrogate_box()
    net = MlpNet(lo, hi, seed=seed)
    if scale_hidden != 1.0:
        net.params.mul_(scale_hidden)
        cm.cm_mlp_sync_bf16(net.struct)
    x = W.surrogate_queries(B, seed + 100)
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    theta = _effective_theta(net.params.cpu().numpy())
    xn = R.normalise(x.astype(np.float32).astype(np.float64), (lo + hi) / 2, 2.0 / (hi - lo))
    return net, xd, theta, xn


@pytest.mark.parametrize("B", [1, 45, 300, 4096])
def test_mlp_forward_matches_reference(B):
    say("mlp forward", B)
    net, xd, theta, xn = _net_and_inputs(B, scale_hidden=3.0)
    y = net.forward(xd).double().cpu().numpy()
    ref, _ = R.forward(theta, xn)
    err = np.abs(y - ref).max() / max(1e-3, np.abs(ref).max())
    say("  rel err", err)
    assert err < 1e-4


def test_mlp_forward_keep_matches_inference():
    """The training forward (all four pre-activations kept, one launch per layer) and the fused
    inference forward (activations on chip) compute the same network, for batches that fill
    several 64-query tiles and leave a ragged last one, up to one (131149 queries, 2050
    tiles) where every workgroup takes several tiles and the last ones fewer. They differ
    only in the first layer, FP32 on one side and three BF16 products of hi / lo parts on
    the other (each product within 3 * 2^-18 relative of the FP32 one), and in the order of
    the final sum: within 5e-5 of the output scale."""
    for B in (1, 777, 4099, 131149):
        net, xd, theta, xn = _net_and_inputs(B, scale_hidden=3.0)
        y1 = net.forward(xd).clone()
        nb = cm.cm_mlp_act_bytes(B)
        acts = torch.empty(nb, dtype=torch.uint8, device="cuda")
        y2 = torch.empty(B, dtype=torch.float32, device="cuda")
        cm.cm_mlp_forward(net.struct, xd, B, y2, acts, nb)
        d = (y1 - y2).abs().max().item() / max(1e-3, y2.abs().max().item())
        say("  B", B, "fused vs layer-by-layer rel diff", d)
        assert d < 5e-5
        ref, _ = R.forward(theta, xn)
        assert np.abs(y1.double().cpu().numpy() - ref).max() / max(1e-3, np.abs(ref).max()) < 1e-4


def _abs_products(theta, xn, zs, dy):
    """sum_b |delta_i[b]| |a_j[b]| for every weight block and sum_b |delta_i[b]| for every
    bias, from the reference's own per-sample deltas (dL/dz of each layer) and activations:
    the scale the elementwise bound of each gradient entry is relative to."""
    p = R.unpack(theta)
    acts = [np.asarray(xn, dtype=np.float64)] + [R.silu(z) for z in zs]
    dy = np.asarray(dy, dtype=np.float64).reshape(-1, 1)
    out = {"W5": np.abs(dy).T @ np.abs(acts[4]), "b5": np.abs(dy).sum(axis=0)}
    delta = (dy @ p["W5"]) * R.silu_grad(zs[3])
    for l in range(4, 0, -1):
        out[f"W{l}"] = np.abs(delta).T @ np.abs(acts[l - 1])
        out[f"b{l}"] = np.abs(delta).sum(axis=0)
        if l >= 2:
            delta = (delta @ p[f"W{l}"]) * R.silu_grad(zs[l - 2])
    return out


@pytest.mark.parametrize("B", [64, 1000])
def test_mlp_backward_matches_reference(B):
    """Every gradient entry against the FP64 reference within 2^-8 of its absolute-product
    scale (module docstring); each block as a whole within 2^-8 relative (Frobenius)."""
    say("mlp backward", B)
    net, xd, theta, xn = _net_and_inputs(B, seed=5, scale_hidden=3.0)
    rng = np.random.default_rng(B)
    dy = rng.standard_normal(B)
    nb = cm.cm_mlp_act_bytes(B)
    acts = torch.empty(nb, dtype=torch.uint8, device="cuda")
    y = torch.empty(B, dtype=torch.float32, device="cuda")
    cm.cm_mlp_forward(net.struct, xd, B, y, acts, nb)
    ws = torch.empty(nb // 2, dtype=torch.uint8, device="cuda")
    dyd = torch.from_numpy(dy.astype(np.float32)).cuda()
    grad = torch.full((cm.CM_MLP_NPARAMS,), 7.0, dtype=torch.float32, device="cuda")   # must be overwritten
    cm.cm_mlp_backward(net.struct, xd, acts, dyd, B, grad, ws, nb // 2)
    g = R.unpack(grad.double().cpu().numpy())
    _, zs = R.forward(theta, xn)
    dy64 = dy.astype(np.float32).astype(np.float64)
    ref = R.unpack(R.backward(theta, xn, zs, dy64))
    scale = _abs_products(theta, xn, zs, dy64)
    for name, _shape in R._SHAPES:
        ratio = np.abs(g[name] - ref[name]) / np.maximum(scale[name], 1e-300)
        e = np.linalg.norm(g[name] - ref[name]) / max(1e-30, np.linalg.norm(ref[name]))
        say("  ", name, "max err / scale", ratio.max(), "(bound 2^-8 = 3.9e-3), relative norm", e)
        assert ratio.max() <= 2.0 ** -8, name
        assert e < 2.0 ** -8, name


def test_mse_and_adam_match_reference():
    rng = np.random.default_rng(11)
    B = 1000
    y = rng.standard_normal(B).astype(np.float32)
    t = rng.standard_normal(B).astype(np.float32)
    yd, td = torch.from_numpy(y).cuda(), torch.from_numpy(t).cuda()
    dy = torch.empty(B, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    cm.cm_mlp_mse(yd, td, B, dy, loss)
    r = y.astype(np.float64) - t
    assert np.allclose(dy.cpu().numpy(), 2 * r / B, rtol=1e-6, atol=1e-9)
    assert abs(loss.item() - np.mean(r * r)) < 1e-5 * np.mean(r * r)
    # Adam, three steps against the float64 reference
    lo, hi = W.surrogate_box()
    net = MlpNet(lo, hi, seed=1)
    th = net.params.double().cpu().numpy()
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for step in range(1, 4):
        g = rng.standard_normal(th.size) * 10.0 ** rng.integers(-4, 1, th.size)
        net.grad.copy_(torch.from_numpy(g.astype(np.float32)))
        cm.cm_adam_step(net.struct, net.grad, net.m, net.v, step, 1e-3)
        net.t = step
        th, m, v = R.adam_step(th, g.astype(np.float32).astype(np.float64), m, v, step, 1e-3)
    got = net.params.double().cpu().numpy()
    assert np.abs(got - th).max() < 1e-6
    # the BF16 copies follow the new master weights, in the fragment order the header states:
    # W_l[n][k] at 8 (64 (16 (n / 32) + k / 16) + 32 ((k / 8) mod 2) + n mod 32) + k mod 8
    wbf = net.wbf.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
    p = R.unpack(got)
    n, k = np.meshgrid(np.arange(256), np.arange(256), indexing="ij")
    at = (8 * (64 * (16 * (n // 32) + k // 16) + 32 * ((k // 8) % 2) + n % 32) + k % 8).reshape(-1)
    assert np.array_equal(np.sort(at), np.arange(65536))
    for i, l in enumerate((2, 3, 4)):
        blk = wbf[i * 65536:(i + 1) * 65536].view(np.float32).astype(np.float64)
        assert np.array_equal(blk[at], R.bf16_round(p[f"W{l}"].reshape(-1)))


def test_gate_box_and_bounds():
    lo, hi = W.surrogate_box()
    r = 0.03
    mid = (lo + hi) / 2
    rows, ys, want = [], [], []

    def add(x, y, ok):
        rows.append(x), ys.append(y), want.append(ok)
    add(mid, 0.1, True)
    add(lo, 1 - math.exp(lo[6] - r * lo[5]) + 0.01, True)   # box edges are inside
    add(hi, 0.05, True)
    for i in range(7):                  # each coordinate just outside
        x = mid.copy()
        x[i] = hi[i] + 1e-3 * (hi[i] - lo[i])
        add(x, 0.1, False)
    x = mid.copy()
    x[6] = -0.4                         # deep in the money: lower bound 1 - e^{k - rT}
    lb = 1 - math.exp(-0.4 - r * x[5])
    add(x, lb + 1e-4, True)
    add(x, lb - 5e-3, False)            # below the no-arbitrage bound by more than 1e-3
    add(mid, 1.01, False)               # above S0
    add(mid, float("nan"), False)
    xd = torch.from_numpy(np.array(rows, dtype=np.float32)).cuda()
    yd = torch.from_numpy(np.array(ys, dtype=np.float32)).cuda()
    acc = torch.empty(len(rows), dtype=torch.int32, device="cuda")
    cm.cm_surrogate_gate(xd, yd, len(rows), lo.astype(np.float32).tolist(), hi.astype(np.float32).tolist(), r, 1e-3,
                         acc)
    assert acc.cpu().numpy().astype(bool).tolist() == want


def test_gate_calibrated_cell_table():
    """The calibrated residual check: a query is sent to the fallback when the validation
    error of its (T, k) cell exceeds err_tol, wherever else it stands; cells index the
    trusted box's (T, k) rectangle, with the upper edges clamped into the last cell."""
    lo, hi = W.surrogate_box()
    r = 0.03
    nT, nk = 4, 8
    table = np.full((nT, nk), 1e-4, dtype=np.float32)
    table[1, 6] = 2e-3          # one cell above err_tol
    table[3, 7] = np.inf        # one cell without validation data
    mid = (lo + hi) / 2

    def at(fT, fk):
        x = mid.copy()
        x[5] = lo[5] + fT * (hi[5] - lo[5])
        x[6] = lo[6] + fk * (hi[6] - lo[6])
        return x
    rows = [at(0.3, 0.8), at(0.3, 0.7), at(0.1, 0.8), at(1.0, 1.0), at(0.9, 0.9), at(0.0, 0.0), at(0.6, 0.2)]
    want = [False, True, True, False, False, True, True]
    xs = np.array(rows, dtype=np.float32)
    lower = np.maximum(0.0, 1 - np.exp(xs[:, 6].astype(np.float64) - r * xs[:, 5]))
    ys = (lower + 0.02).astype(np.float32)      # inside the no-arbitrage band
    xd = torch.from_numpy(xs).cuda()
    yd = torch.from_numpy(ys).cuda()
    acc = torch.empty(len(rows), dtype=torch.int32, device="cuda")
    cells = torch.from_numpy(table).cuda()
    cm.cm_surrogate_gate(xd, yd, len(rows), lo.astype(np.float32).tolist(), hi.astype(np.float32).tolist(), r, 1e-3,
                         acc, cell_err=cells, err_tol=5e-4)
    assert acc.cpu().numpy().astype(bool).tolist() == want
    cm.cm_surrogate_gate(xd, yd, len(rows), lo.astype(np.float32).tolist(), hi.astype(np.float32).tolist(), r, 1e-3,
                         acc)   # without the table every row is accepted
    assert acc.cpu().numpy().all()


def test_query_prices_shifted_grid_vs_oracle():
    """The fallback prices each query at exactly its k by shifting k0 so that strike index
    M/2 is k: checked against the oracle's direct DFT on the same shifted grids."""
    lo, hi = W.surrogate_box()
    s = Surrogate(lo, hi)
    q = W.surrogate_queries(8, 21)
    got, st = s.query_prices(q)
    assert np.all(st == cm.CM_OK)
    n, M = s.n, 2 ** s.n
    eta = 40.0 / 2 ** (n / 2)
    lam = 2 * math.pi / (M * eta)
    for i in range(len(q)):
        p = W.Problem("heston", "simpson1", n, 100.0, 0.03, 0.0, float(q[i, 5]), 1.5, eta,
                      tuple(float(v) for v in q[i, :5]), k0=math.log(100.0) + q[i, 6] - lam * M / 2)
        ref = O.prices_direct(p, np.array([M // 2]))[0] / 100.0
        assert abs(got[i] - ref) < 1e-6, (i, got[i], ref)


def test_surrogate_trains_gates_and_beats_sfft():
    """The surrogate's recipe end to end on the GPU's own kernels: 2^22 SFFT training samples
    (2^16 parameter draws over the widened box x 64 log-moneyness values), 60 000 Adam
    steps, the gate calibrated on 2^15 validation queries (cells above 5e-4 S0 fall back).
    On 2^16 held-out queries in the trusted box every accepted price lies within 1e-3 S0
    of the SFFT reference (the target), at least 90 % are accepted; out-of-box queries go
    to the fallback, whose prices are the SFFT's; the network answers the in-box queries
    more than 10x faster than batched SFFT pricing of them."""
    say("surrogate train")
    lo, hi = W.surrogate_box()
    s = Surrogate(lo, hi, seed=0)
    X, Y = s.training_set(2 ** 16, 64, seed=1001)
    info = s.fit(X, Y, steps=60000, batch=8192, lr=2e-3, log_every=5000)
    h = s.history
    say("  loss", h[0][1], "->", h[-1][1], info)
    assert h[-1][1] < h[0][1] / 50
    cal = s.calibrate(2 ** 15, seed=4001)
    say("  calibration", cal)
    q_in = W.surrogate_queries(2 ** 16, 5001)
    q_out = W.surrogate_queries(2000, 78, enlarge=0.4)
    outside = np.any((q_out < lo) | (q_out > hi), axis=1)
    q = np.concatenate([q_in, q_out[outside][:500]])
    res = s.price(q)
    ref_prices, st = s.query_prices(q)
    n_in = len(q_in)
    acc = res["accept"]
    ok = acc & (st == cm.CM_OK)
    err = np.abs(res["price"][ok] - ref_prices[ok]).max()
    say("  max err in gate", err, "accept rate", acc[:n_in].mean())
    assert acc[:n_in].mean() > 0.9
    assert not acc[n_in:].any()
    assert err <= 1e-3
    fb = (~acc) & (st == cm.CM_OK)
    assert np.allclose(res["price"][fb], ref_prices[fb], rtol=0, atol=1e-12)
    # speed: network vs batched SFFT on the same in-box queries
    qd = torch.from_numpy(q_in.astype(np.float32)).cuda()
    s.predict(qd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        s.predict(qd)
    torch.cuda.synchronize()
    t_net = (time.perf_counter() - t0) / 5
    t0 = time.perf_counter()
    s.query_prices(q_in)
    torch.cuda.synchronize()
    t_sfft = time.perf_counter() - t0
    say("  net", t_net, "sfft", t_sfft, "speedup", t_sfft / t_net)
    assert t_sfft / t_net > 10

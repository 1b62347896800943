"""Pins of the surrogate network's CPU FP64 reference (oracle/mlp.py) against facts that do
not come from the reference itself: finite differences, closed forms of degenerate
networks, the closed-form Adam step, and torch's own bfloat16 rounding."""
import numpy as np
import pytest

from oracle import mlp as R


def _rand_theta(rng, scale=0.3):
    p = {}
    for name, shape in R._SHAPES:
        fan_in = shape[-1] if len(shape) == 2 else 1
        p[name] = rng.standard_normal(shape) * (scale / np.sqrt(fan_in) if len(shape) == 2 else 0.1)
    return R.pack(p)


def test_parameter_count_matches_architecture():
    # 7*256+256 + 3*(256*256+256) + 256+1, the size the surrogate's description states
    assert R.N_PARAMS == 199_681


def test_silu_grad_matches_central_differences():
    z = np.linspace(-12, 12, 241)
    h = 1e-6
    fd = (R.silu(z + h) - R.silu(z - h)) / (2 * h)
    assert np.abs(fd - R.silu_grad(z)).max() < 1e-8
    assert R.silu(0.0) == 0.0 and abs(R.silu_grad(0.0) - 0.5) < 1e-15


def test_backward_matches_finite_differences():
    """Every parameter block (a dropped term, wrong index or transposed operand in any
    layer shows up): central differences of the MSE on sampled coordinates."""
    rng = np.random.default_rng(3)
    theta = _rand_theta(rng, scale=1.5)
    xn = rng.uniform(-1, 1, (6, 7))
    t = rng.uniform(0, 0.5, 6)
    loss, g = R.mse_loss_and_grad(theta, xn, t)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in R._SHAPES])
    idx = []
    for bi in range(len(R._SHAPES)):
        lo, hi = offs[bi], offs[bi + 1]
        idx.extend(rng.integers(lo, hi, size=min(6, hi - lo)).tolist())
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (R.mse_loss_and_grad(theta + e, xn, t)[0] - R.mse_loss_and_grad(theta - e, xn, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_degenerate_network_closed_form():
    """With W1..W4 = 0 every hidden layer is the constant silu(b_l): the output is
    W5 silu(b4) + b5 for every input, and the gradients of W1..W3 vanish exactly while
    those of b4 and W5 take their closed forms."""
    rng = np.random.default_rng(5)
    p = R.unpack(_rand_theta(rng).copy())
    p = {k: v.copy() for k, v in p.items()}
    for l in (1, 2, 3, 4):
        p[f"W{l}"][:] = 0.0
    theta = R.pack(p)
    xn = rng.uniform(-1, 1, (4, 7))
    y, zs = R.forward(theta, xn)
    y0 = float(p["W5"][0] @ R.silu(p["b4"]) + p["b5"][0])
    assert np.allclose(y, y0, rtol=0, atol=1e-15)
    dy = rng.standard_normal(4)
    g = R.unpack(R.backward(theta, xn, zs, dy))
    for l in (1, 2, 3):
        assert np.all(g[f"W{l}"] == 0.0)
    assert np.allclose(g["W5"][0], dy.sum() * R.silu(p["b4"]), rtol=1e-14, atol=0)
    assert np.allclose(g["b4"], dy.sum() * p["W5"][0] * R.silu_grad(p["b4"]), rtol=1e-14, atol=0)
    assert np.allclose(g["W4"], np.outer(dy.sum() * p["W5"][0] * R.silu_grad(p["b4"]), R.silu(p["b3"])),
                       rtol=1e-14, atol=1e-300)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments equal g and g^2 at every step,
    so each step moves theta by exactly lr * g / (|g| + eps)."""
    rng = np.random.default_rng(7)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr, eps = 1e-3, 1e-8
    cur = th.copy()
    for t in range(1, 6):
        cur, m, v = R.adam_step(cur, g, m, v, t, lr, eps=eps)
        assert np.allclose(cur, th - t * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-13)


def test_bf16_round_matches_torch_and_ties_to_even():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(9)
    a = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -0.0]])
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = R.bf16_round(a)
    assert np.array_equal(got, ref)
    assert got[-4] == 1.0 and got[-3] == 1.0 and got[-2] == 1.0 + 2 ** -6

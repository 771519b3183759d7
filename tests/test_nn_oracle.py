"""Pins of the FP64 network oracle: the 3x3 convolution against SciPy's 2-D
correlation, pooling/upsampling against their definitions, and every
gradient of the full U-Net against central finite differences."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import nn_oracle as N

SMALL = dict(c_in=3, widths=(2, 3, 4, 5), c_out=2)


def test_conv_matches_scipy_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 7, 9, 3))
    W = rng.standard_normal((9, 3, 4))
    b = rng.standard_normal(4)
    y = N.conv3x3(x, W, b)
    for n in range(2):
        for co in range(4):
            ref = np.full((7, 9), b[co])
            for ci in range(3):
                k = W[:, ci, co].reshape(3, 3)  # tap = (dy+1)*3 + (dx+1)
                ref += correlate2d(x[n, :, :, ci], k, mode="same", boundary="fill")
            assert np.allclose(y[n, :, :, co], ref, atol=1e-12)


def test_pool_and_upsample():
    x = np.arange(2 * 4 * 6 * 3, dtype=float).reshape(2, 4, 6, 3)
    p = N.avgpool(x)
    assert p.shape == (2, 2, 3, 3)
    assert p[1, 1, 2, 0] == np.mean(x[1, 2:4, 4:6, 0])
    u = N.upsample(p)
    assert u.shape == x.shape and u[0, 3, 5, 2] == p[0, 1, 2, 2]
    # adjointness: <up(a), b> = <a, up^T(b)>, <pool(a), c> = <a, pool^T(c)>
    rng = np.random.default_rng(1)
    a, bb = rng.standard_normal((2, 3, 5, 2)), rng.standard_normal((2, 6, 10, 2))
    assert np.isclose(np.sum(N.upsample(a) * bb), np.sum(a * N.upsample_backward(bb)))
    c = rng.standard_normal((2, 3, 5, 2))
    assert np.isclose(np.sum(N.avgpool(bb) * c), np.sum(bb * N.avgpool_backward(c)))


def test_param_count_full_network():
    p = N.init_params(16, 0)
    assert 1.9e6 < N.n_params(p) < 2.0e6


@pytest.mark.parametrize("seed", [0, 1])
def test_gradients_finite_differences(seed):
    rng = np.random.default_rng(seed)
    p = N.init_params(SMALL["c_in"], seed, SMALL["widths"], SMALL["c_out"])
    for k in p:  # nonzero biases so every term is exercised
        if k.endswith(".b"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((2, 8, 16, SMALL["c_in"]))
    t = rng.standard_normal((2, 8, 16, SMALL["c_out"]))
    y, cache = N.forward(p, x)
    g = N.backward(p, cache, y, t)
    assert set(g) == set(p)
    eps = 1e-6
    for name in p:
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = N.loss(N.forward(p, x)[0], t)
            flat[idx] = old - eps
            lm = N.loss(N.forward(p, x)[0], t)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (name, idx, fd, an)


def test_adam_matches_definition():
    p = {"w": np.array([1.0, -2.0])}
    m = {"w": np.zeros(2)}
    v = {"w": np.zeros(2)}
    g = {"w": np.array([0.5, -1.0])}
    N.adam_step(p, g, m, v, 1, 0.1)
    # first step of Adam moves every weight by -lr * sign(g)
    assert np.allclose(p["w"], [0.9, -1.9], atol=1e-7)


def test_bf16_rounding_matches_torch():
    """The oracle's BF16 rounding against torch's float32 -> bfloat16 cast
    (round to nearest, ties to even) on random values and exact ties."""
    import torch
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        [0.0, 1.0, -1.0]]).astype(np.float32).astype(np.float64)
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(N.bf16_round(x), want)
    # ties: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7 (-> 1, even);
    # 1 + 3 2^-8 between 1 + 2^-7 and 1 + 2^-6 (-> 1 + 2^-6, even)
    ties = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 3 * 2.0 ** -9 * 2 ** 5])
    assert np.array_equal(N.bf16_round(ties), [1.0, 1 + 2.0 ** -6, -1.0, 3 * 2.0 ** -9 * 2 ** 5])


def test_bf16_operand_mode_is_the_exact_network_on_rounded_operands():
    """With every weight already a BF16 value and the input too, the BF16
    mode differs from the exact mode only by the rounding of the stored
    activations: same output to BF16 rounding level, same backward code."""
    rng = np.random.default_rng(6)
    p = N.init_params(SMALL["c_in"], 3, SMALL["widths"], SMALL["c_out"])
    p = {k: N.bf16_round(v) if k.endswith(".W") and v.ndim == 3 else v for k, v in p.items()}
    x = N.bf16_round(rng.standard_normal((2, 8, 16, SMALL["c_in"])))
    t = rng.standard_normal((2, 8, 16, SMALL["c_out"]))
    ye, ce = N.forward(p, x)
    yb, cb = N.forward(p, x, operands="bf16")
    rel = np.linalg.norm(yb - ye) / np.linalg.norm(ye)
    assert 0 < rel < 2e-2
    # stored activations of the BF16 mode are BF16 values
    for name in ("e0", "e2", "d1"):
        for a in cb[name][1:]:
            assert np.array_equal(N.bf16_round(a), a)
    # the backward pass is the exact one evaluated at the BF16 mode's state:
    # replaying the exact backward on its cache gives the same gradients
    gb = N.backward(p, cb, yb, t)
    cb_exact = dict(cb)
    cb_exact["operands"] = None
    ge = N.backward(p, cb_exact, yb, t)
    for k in gb:
        assert np.array_equal(gb[k], ge[k])


def test_softplus_against_logaddexp_and_its_derivative():
    x = np.linspace(-40.0, 40.0, 4001)
    assert np.allclose(N.softplus(x), np.logaddexp(0.0, x), rtol=1e-15, atol=1e-300)
    # sigmoid(x) recovered from the output, against 1 / (1 + e^-x)
    assert np.allclose(N.softplus_grad_from_output(N.softplus(x)), 1.0 / (1.0 + np.exp(-x)),
                       rtol=1e-12, atol=0)

"""GPU tests of the warm-start network kernels against the FP64 NumPy oracle.

The kernels run BF16 MFMA products with FP32 accumulation and keep
activations and their gradients in BF16 (8-bit mantissa), so agreement with
the FP64 oracle is judged by relative norms and cosines: ~14 layers of BF16
rounding give a few per cent at most on the output and on every gradient.
"""
import numpy as np
import pytest

from oracle import nn_oracle as N

pytestmark = pytest.mark.gpu

WIDTHS = (32, 64, 128, 256)


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_mfma_accumulator_layout():
    from paper_1003_0282_amd import lbnn
    assert lbnn.mfma_selftest() == 0


def _setup(H=16, W=32, B=2, c_in=8, c_out=4, seed=0):
    import torch
    from paper_1003_0282_amd import lbnn
    rng = np.random.default_rng(seed)
    p = N.init_params(c_in, seed, WIDTHS, c_out)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    names = [n for n, _ in N.layer_shapes(c_in, WIDTHS, c_out)]
    x = rng.standard_normal((B, H, W, c_in))
    t = 0.5 * rng.standard_normal((B, H, W, c_out))
    net = lbnn.Net(H, W, c_in, c_out, WIDTHS, max_batch=B)
    assert net.nparam == N.n_params(p)
    net.set_params(lbnn.flatten_params(p, names).astype(np.float32))
    xd = torch.tensor(x, dtype=torch.float32, device="cuda")
    td = torch.tensor(t, dtype=torch.float32, device="cuda")
    return net, p, names, x, t, xd, td


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_forward_matches_oracle():
    net, p, names, x, t, xd, td = _setup()
    y = net.forward(xd).double().cpu().numpy()
    y_ref, _ = N.forward(p, x)
    err = _rel(y, y_ref)
    print("forward rel err", err)
    assert err < 3e-2


def test_gradients_match_oracle():
    from paper_1003_0282_amd import lbnn
    net, p, names, x, t, xd, td = _setup(seed=1)
    net.forward(xd)
    loss, g = net.backward(td)
    y_ref, cache = N.forward(p, x)
    g_ref = N.backward(p, cache, y_ref, t)
    assert abs(loss - N.loss(y_ref, t)) / N.loss(y_ref, t) < 3e-2
    gd = lbnn.unflatten(g.double().cpu().numpy(), N.layer_shapes(8, WIDTHS, 4))
    worst = []
    for name in names:
        a, b = gd[name].reshape(-1), g_ref[name].reshape(-1)
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))
        rel = _rel(a, b)
        worst.append((rel, cos, name))
        # the deepest weight gradients sum over few pixels (64 at level 2 of
        # this 16 x 32 input), so BF16 rounding is least averaged out there
        assert cos > 0.99 and rel < 0.15, (name, cos, rel)
    print("worst gradient", max(worst))


@pytest.mark.parametrize("H,W,B,c_in,c_out", [(40, 72, 3, 5, 5), (128, 256, 2, 8, 5)])
def test_forward_and_gradients_other_shapes(H, W, B, c_in, c_out):
    """Odd level sizes (5 x 9 at the deepest level, so pixel groups straddle
    rows), padded input channels, several pixel chunks per weight-gradient
    workgroup, and the 128 x 256 shape of the warm start."""
    from paper_1003_0282_amd import lbnn
    net, p, names, x, t, xd, td = _setup(H, W, B, c_in, c_out, seed=4)
    y = net.forward(xd).double().cpu().numpy()
    y_ref, cache = N.forward(p, x)
    assert _rel(y, y_ref) < 3e-2, _rel(y, y_ref)
    loss, g = net.backward(td)
    g_ref = N.backward(p, cache, y_ref, t)
    assert abs(loss - N.loss(y_ref, t)) / N.loss(y_ref, t) < 3e-2
    gd = lbnn.unflatten(g.double().cpu().numpy(), N.layer_shapes(c_in, WIDTHS, c_out))
    worst = []
    for name in names:
        a, b = gd[name].reshape(-1), g_ref[name].reshape(-1)
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))
        rel = _rel(a, b)
        worst.append((rel, cos, name))
        assert cos > 0.99 and rel < 0.15, (name, cos, rel)
    print("worst gradient", max(worst))


def test_training_reduces_loss():
    import torch
    net, p, names, x, t, xd, td = _setup(seed=2)
    # a learnable target: a smooth function of the input
    t2 = torch.tanh(xd[..., :4] * 0.5).contiguous()
    losses = [net.train_step(xd, t2, 2e-3) for _ in range(60)]
    print("loss", losses[0], "->", losses[-1])
    assert losses[-1] < 0.3 * losses[0]


def test_adam_matches_oracle_step():
    from paper_1003_0282_amd import lbnn
    net, p, names, x, t, xd, td = _setup(seed=3)
    net.forward(xd)
    _, g = net.backward(td)
    net.adam(1e-3)
    got = net.get_params().double().cpu().numpy()
    gd = lbnn.unflatten(g.double().cpu().numpy(), N.layer_shapes(8, WIDTHS, 4))
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    p2 = {k: val.astype(np.float32).astype(np.float64) for k, val in p.items()}
    N.adam_step(p2, gd, m, v, 1, 1e-3)
    ref = lbnn.flatten_params(p2, names)
    assert np.abs(got - ref).max() < 1e-6


def test_to_fields_scale_offset_and_smoothing():
    import torch
    from paper_1003_0282_amd import lbnn
    B, H, W, K = 2, 16, 32, 5
    net = lbnn.Net(H, W, 8, K, WIDTHS, max_batch=B)
    rng = np.random.default_rng(7)
    y = rng.standard_normal((B, H, W, K)).astype(np.float32)
    yd = torch.tensor(y, device="cuda")
    sc, of = [0.5, 2.0, -1.0, 3.0, 0.25], [1.0, 0.0, 0.5, -2.0, 0.0]
    for smooth in (False, True):
        outs = [torch.empty(B * H * W, device="cuda") for _ in range(K)]
        outs[2] = None
        net.to_fields(yd, sc, of, outs, smooth=smooth)
        torch.cuda.synchronize()
        yy = y.astype(np.float64)
        if smooth:  # (1, 2, 1)/4 along H and W, edge values repeated
            p = np.pad(yy, ((0, 0), (1, 1), (0, 0), (0, 0)), mode="edge")
            yy = 0.25 * p[:, :-2] + 0.5 * p[:, 1:-1] + 0.25 * p[:, 2:]
            p = np.pad(yy, ((0, 0), (0, 0), (1, 1), (0, 0)), mode="edge")
            yy = 0.25 * p[:, :, :-2] + 0.5 * p[:, :, 1:-1] + 0.25 * p[:, :, 2:]
        for k in range(K):
            if outs[k] is None:
                continue
            want = (yy[..., k] * sc[k] + of[k]).reshape(-1)
            assert np.abs(outs[k].cpu().numpy() - want).max() < 1e-5 * (1 + np.abs(want).max())
    # a pure checkerboard is removed by the filter
    cb = np.fromfunction(lambda b, i, j, k: (-1.0) ** (i + j), (B, H, W, K)).astype(np.float32)
    outs = [torch.empty(B * H * W, device="cuda") for _ in range(K)]
    net.to_fields(torch.tensor(cb, device="cuda"), [1.0] * K, [0.0] * K, outs, smooth=True)
    inner = outs[0].cpu().numpy().reshape(B, H, W)[:, 1:-1, 1:-1]
    assert np.abs(inner).max() < 1e-6

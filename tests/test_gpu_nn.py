"""GPU tests of the warm-start network kernels against the FP64 NumPy oracle.

The kernels multiply BF16 operands on the matrix cores with FP32
accumulation: the convolution weights and every stored activation are BF16
values.  The oracle's BF16-operand mode evaluates exactly that network (the
same operands, rounded to the nearest BF16 value where the network produces
them) with FP64 arithmetic everywhere else, so the forward output agrees to
accumulation-order rounding and every parameter gradient (whose chain runs
through BF16 gradient tensors in the kernels) to the contracted bar: cosine
>= 0.999 and relative norm <= 1e-2.  The exact-operand oracle is reported
beside it for information: the BF16 network is a slightly different
function from the FP64 one.
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
    # the GPU holds FP32 parameters and inputs: the oracle gets the same values
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    x = x.astype(np.float32).astype(np.float64)
    net.set_params(lbnn.flatten_params(p, names).astype(np.float32))
    xd = torch.tensor(x, dtype=torch.float32, device="cuda")
    td = torch.tensor(t, dtype=torch.float32, device="cuda")
    return net, p, names, x, t, xd, td


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


FWD_TOL = 1e-2       # relative norm of the output
COS_MIN, REL_MAX = 0.999, 1e-2


def _check_gradients(net, p, names, x, t, td, c_in, c_out):
    from paper_1003_0282_amd import lbnn
    loss, g = net.backward(td)
    y_ref, cache = N.forward(p, x, operands="bf16")
    g_ref = N.backward(p, cache, y_ref, t)
    assert abs(loss - N.loss(y_ref, t)) / N.loss(y_ref, t) < 1e-3
    gd = lbnn.unflatten(g.double().cpu().numpy(), N.layer_shapes(c_in, WIDTHS, c_out))
    y_x, cache_x = N.forward(p, x)
    g_x = N.backward(p, cache_x, y_x, t)
    worst, worst_x = [], []
    for name in names:
        a, b = gd[name].reshape(-1), g_ref[name].reshape(-1)
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))
        rel = _rel(a, b)
        worst.append((rel, cos, name))
        bx = g_x[name].reshape(-1)
        worst_x.append((_rel(a, bx), name))
        assert cos >= COS_MIN and rel <= REL_MAX, (name, cos, rel)
    print("worst gradient vs BF16-operand oracle", max(worst))
    print("worst gradient vs exact-operand oracle (information)", max(worst_x))


def test_forward_matches_oracle():
    net, p, names, x, t, xd, td = _setup()
    y = net.forward(xd).double().cpu().numpy()
    y_ref, _ = N.forward(p, x, operands="bf16")
    err = _rel(y, y_ref)
    y_x, _ = N.forward(p, x)
    print("forward rel err %.2e (exact-operand oracle: %.2e)" % (err, _rel(y, y_x)))
    assert err <= FWD_TOL


def test_gradients_match_oracle():
    net, p, names, x, t, xd, td = _setup(seed=1)
    net.forward(xd)
    _check_gradients(net, p, names, x, t, td, 8, 4)


@pytest.mark.parametrize("H,W,B,c_in,c_out", [(40, 72, 3, 5, 5), (128, 256, 2, 8, 5)])
def test_forward_and_gradients_other_shapes(H, W, B, c_in, c_out):
    """Odd level sizes (5 x 9 at the deepest level, so pixel groups straddle
    rows), padded input channels, several pixel chunks per weight-gradient
    workgroup, and the 128 x 256 shape of the warm start."""
    net, p, names, x, t, xd, td = _setup(H, W, B, c_in, c_out, seed=4)
    y = net.forward(xd).double().cpu().numpy()
    y_ref, _ = N.forward(p, x, operands="bf16")
    assert _rel(y, y_ref) <= FWD_TOL, _rel(y, y_ref)
    _check_gradients(net, p, names, x, t, td, c_in, c_out)


def test_training_is_bitwise_reproducible():
    """Every reduction runs in a fixed order (per-chunk partial sums, then a
    second pass in chunk order): two trainings from one state give the same
    parameters bit for bit."""
    import torch
    runs = []
    for _ in range(2):
        net, p, names, x, t, xd, td = _setup(40, 72, 3, 5, 5, seed=8)
        losses = [net.train_step(xd, td, 1e-3) for _ in range(12)]
        runs.append((losses, net.get_params().cpu().numpy()))
        torch.cuda.synchronize()
    assert runs[0][0] == runs[1][0]
    assert np.array_equal(runs[0][1], runs[1][1])


def test_forward_does_not_depend_on_the_batch():
    """Each output pixel sees the same operands in the same accumulation
    order whatever the batch size (and so whatever grid and tile shapes the
    launch picks), so a sample's output is the same bits in a batch of 2 and
    in a batch of 16.  The batch-2 forward is checked against the oracle
    above."""
    import torch
    from paper_1003_0282_amd import lbnn
    net, p, names, x, t, xd, td = _setup(128, 256, 2, 8, 5, seed=9)
    big = lbnn.Net(128, 256, 8, 5, WIDTHS, max_batch=16)
    big.set_params(net.get_params())
    rng = np.random.default_rng(10)
    x16 = torch.tensor(rng.standard_normal((16, 128, 256, 8)), dtype=torch.float32, device="cuda")
    x16[5:7] = xd
    y16 = big.forward(x16).cpu().numpy()
    y2 = net.forward(xd).cpu().numpy()
    assert np.array_equal(y16[5:7], y2)


def test_adam_keeps_the_bf16_weight_copies_current():
    """The Adam step also writes each updated convolution weight to its BF16
    copies (forward and adjoint order): after training steps the network's
    forward equals, bit for bit, that of a network given the same
    parameters, whose copies are cast from them.  Five input channels make
    the first layer's padded channels part of the check."""
    from paper_1003_0282_amd import lbnn
    net, p, names, x, t, xd, td = _setup(40, 72, 3, 5, 5, seed=11)
    y0 = net.forward(xd).cpu().numpy()
    for _ in range(3):
        net.train_step(xd, td, 1e-2)
    fresh = lbnn.Net(40, 72, 5, 5, WIDTHS, max_batch=3)
    fresh.set_params(net.get_params())
    y1 = net.forward(xd).cpu().numpy()
    assert not np.array_equal(y0, y1)
    assert np.array_equal(y1, fresh.forward(xd).cpu().numpy())


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

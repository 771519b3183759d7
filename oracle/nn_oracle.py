"""FP64 NumPy oracle of the warm-start network (test infrastructure only).

TEST INFRASTRUCTURE ONLY: the tests compare the HIP network kernels with this
file; the product never imports it.  It shares no code with the GPU path.

The network is a 4-level convolutional U-Net on NHWC tensors [B, H, W, C]:

    encoder level l (widths c_l):  x -> sp(conv3x3) -> sp(conv3x3) = e_l
                                   p_l = avgpool2x2(e_l)           (l < 3)
    decoder level l = 2, 1, 0:     u = upsample2x(d_{l+1}) (d_3 = e_3)
                                   d_l = sp(conv3x3(sp(conv3x3(concat(u, e_l)))))
    head:                          y = conv1x1(d_0) + b   (no activation)
    loss:                          L = mean((y - target)^2)

sp is the softplus activation, sp(z) = log(1 + e^z), whose derivative
sigmoid(z) = 1 - e^(-sp(z)) follows from its output.  3x3 convolutions use
zero "same" padding; weights W[tap, c_in, c_out] with tap = (dy + 1) * 3 +
(dx + 1) act as out[y, x] = sum in[y + dy, x + dx] W[tap].  Nothing here is
tuned; every backward formula is the plain adjoint of its
forward and is pinned by central finite differences in the tests.

Operand precision.  ``forward(p, x)`` evaluates the network with every
tensor exact (FP64).  ``forward(p, x, operands="bf16")`` evaluates the
network the GPU kernels define, whose matrix-core products take BF16
operands: the weights of the 3x3 convolutions, the network input and every
activation tensor the network stores (the activation output of each
convolution and each pooled map) are rounded to the nearest BF16 value (ties
to even) where they are produced; biases and the 1x1 head stay as given, and
all arithmetic (sums, products, the backward pass) stays FP64.  The backward
pass treats the rounding as the identity (the usual straight-through
convention) and takes each activation's derivative from its stored output,
so ``backward`` is the same code in both modes.  A kernel that stores BF16
activations is compared with this mode.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


# ---- BF16 rounding -----------------------------------------------------------

def bf16_round(x):
    """Nearest BF16 value (8 significant bits, ties to even) of each element,
    as float64; zero stays zero.  Values stay far inside BF16's exponent
    range here, so no overflow or subnormal case arises."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                 # x = m 2^e, 1/2 <= |m| < 1
    return np.ldexp(np.round(m * 256.0), e - 8)   # np.round: half to even


def _ident(x):
    return x


def _rounders(operands):
    if operands is None:
        return _ident
    if operands == "bf16":
        return bf16_round
    raise ValueError("operands must be None or 'bf16'")


# ---- layers ---------------------------------------------------------------

def conv3x3(x, W, b):
    """x [B,H,W,Ci], W [9,Ci,Co], b [Co] -> [B,H,W,Co]."""
    B, H, Wd, Ci = x.shape
    xp = np.zeros((B, H + 2, Wd + 2, Ci), dtype=x.dtype)
    xp[:, 1:-1, 1:-1] = x
    out = np.zeros((B, H, Wd, W.shape[2]), dtype=np.float64)
    for t, (dy, dx) in enumerate(TAPS):
        out += xp[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + Wd] @ W[t]
    return out + b


def conv3x3_backward(x, W, gout):
    """Gradients of conv3x3 w.r.t. x, W and b given d(out) = gout."""
    B, H, Wd, Ci = x.shape
    xp = np.zeros((B, H + 2, Wd + 2, Ci), dtype=np.float64)
    xp[:, 1:-1, 1:-1] = x
    gxp = np.zeros_like(xp)
    gW = np.zeros_like(W, dtype=np.float64)
    g2 = gout.reshape(-1, gout.shape[-1])
    for t, (dy, dx) in enumerate(TAPS):
        win = xp[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + Wd]
        gW[t] = win.reshape(-1, Ci).T @ g2
        gxp[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + Wd] += gout @ W[t].T
    gb = g2.sum(axis=0)
    return gxp[:, 1:-1, 1:-1], gW, gb


def softplus(x):
    """log(1 + e^x), written so that no exponential overflows."""
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


def softplus_grad_from_output(a):
    """d softplus / dx at the input whose output is a: sigmoid(x) = 1 - e^(-a)."""
    return -np.expm1(-a)


def avgpool(x):
    B, H, Wd, C = x.shape
    return x.reshape(B, H // 2, 2, Wd // 2, 2, C).mean(axis=(2, 4))


def avgpool_backward(g):
    return np.repeat(np.repeat(g, 2, axis=1), 2, axis=2) / 4.0


def upsample(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample_backward(g):
    B, H, Wd, C = g.shape
    return g.reshape(B, H // 2, 2, Wd // 2, 2, C).sum(axis=(2, 4))


# ---- the network ------------------------------------------------------------

def layer_shapes(c_in: int, widths=(32, 64, 128, 256), c_out: int = 4):
    """Ordered (name, weight shape) list of all trainable tensors."""
    c0, c1, c2, c3 = widths
    convs = [("e0a", c_in, c0), ("e0b", c0, c0), ("e1a", c0, c1), ("e1b", c1, c1),
             ("e2a", c1, c2), ("e2b", c2, c2), ("e3a", c2, c3), ("e3b", c3, c3),
             ("d2a", c3 + c2, c2), ("d2b", c2, c2), ("d1a", c2 + c1, c1), ("d1b", c1, c1),
             ("d0a", c1 + c0, c0), ("d0b", c0, c0)]
    out = []
    for name, ci, co in convs:
        out.append((name + ".W", (9, ci, co)))
        out.append((name + ".b", (co,)))
    out.append(("head.W", (c0, c_out)))
    out.append(("head.b", (c_out,)))
    return out


def init_params(c_in: int, seed: int, widths=(32, 64, 128, 256), c_out: int = 4):
    """He-normal weights, zero biases (a seeded, deterministic start)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in layer_shapes(c_in, widths, c_out):
        if name.endswith(".b"):
            p[name] = np.zeros(shape)
        else:
            fan_in = shape[0] * shape[1] if len(shape) == 3 else shape[0]
            p[name] = rng.standard_normal(shape) * np.sqrt(2.0 / fan_in)
    return p


def _block(x, p, name, cache, rnd):
    z1 = conv3x3(x, rnd(p[name + "a.W"]), p[name + "a.b"])
    a1 = rnd(softplus(z1))
    z2 = conv3x3(a1, rnd(p[name + "b.W"]), p[name + "b.b"])
    a2 = rnd(softplus(z2))
    cache[name] = (x, a1, a2)
    return a2


def forward(p, x, operands=None):
    """x [B,H,W,Cin] -> (y [B,H,W,Cout], cache); operands: None (exact) or
    "bf16" (see the module docstring)."""
    rnd = _rounders(operands)
    cache = {"operands": operands}
    x = rnd(x)
    e0 = _block(x, p, "e0", cache, rnd)
    e1 = _block(rnd(avgpool(e0)), p, "e1", cache, rnd)
    e2 = _block(rnd(avgpool(e1)), p, "e2", cache, rnd)
    e3 = _block(rnd(avgpool(e2)), p, "e3", cache, rnd)
    d2 = _block(np.concatenate([upsample(e3), e2], axis=-1), p, "d2", cache, rnd)
    d1 = _block(np.concatenate([upsample(d2), e1], axis=-1), p, "d1", cache, rnd)
    d0 = _block(np.concatenate([upsample(d1), e0], axis=-1), p, "d0", cache, rnd)
    y = d0 @ p["head.W"] + p["head.b"]
    cache["d0out"] = d0
    return y, cache


def loss(y, target):
    return float(np.mean((y - target) ** 2))


def _block_backward(p, name, cache, g, grads, rnd):
    x, a1, a2 = cache[name]
    g = g * softplus_grad_from_output(a2)
    g, grads[name + "b.W"], grads[name + "b.b"] = conv3x3_backward(a1, rnd(p[name + "b.W"]), g)
    g = g * softplus_grad_from_output(a1)
    g, grads[name + "a.W"], grads[name + "a.b"] = conv3x3_backward(x, rnd(p[name + "a.W"]), g)
    return g


def backward(p, cache, y, target):
    """Gradients of loss(y, target) w.r.t. every parameter (of the mode the
    forward pass ran in; the rounding of the BF16 mode passes gradients
    through unchanged)."""
    rnd = _rounders(cache.get("operands"))
    grads = {}
    gy = 2.0 * (y - target) / y.size
    d0 = cache["d0out"]
    grads["head.W"] = d0.reshape(-1, d0.shape[-1]).T @ gy.reshape(-1, gy.shape[-1])
    grads["head.b"] = gy.reshape(-1, gy.shape[-1]).sum(axis=0)
    g = gy @ p["head.W"].T
    skips = {}
    for lvl, skip, up_ch in (("d0", "e0", None), ("d1", "e1", None), ("d2", "e2", None)):
        gcat = _block_backward(p, lvl, cache, g, grads, rnd)
        c_skip = cache[skip][2].shape[-1]
        skips[skip] = gcat[..., -c_skip:]
        g = upsample_backward(gcat[..., :-c_skip])
    g = _block_backward(p, "e3", cache, g, grads, rnd)
    for lvl in ("e2", "e1", "e0"):
        g = avgpool_backward(g) + skips[lvl]
        g = _block_backward(p, lvl, cache, g, grads, rnd)
    return grads


def adam_step(p, grads, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), in place; step counts from 1."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * grads[k]
        v[k] = b2 * v[k] + (1 - b2) * grads[k] ** 2
        mh = m[k] / (1 - b1 ** step)
        vh = v[k] / (1 - b2 ** step)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def n_params(p) -> int:
    return int(sum(v.size for v in p.values()))

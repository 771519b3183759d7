"""FP64 NumPy oracle of the warm-start network (test infrastructure only).

TEST INFRASTRUCTURE ONLY: the tests compare the HIP network kernels with this
file; the product never imports it.  It shares no code with the GPU path.

The network is a 4-level convolutional U-Net on NHWC tensors [B, H, W, C]:

    encoder level l (widths c_l):  x -> relu(conv3x3) -> relu(conv3x3) = e_l
                                   p_l = avgpool2x2(e_l)           (l < 3)
    decoder level l = 2, 1, 0:     u = upsample2x(d_{l+1}) (d_3 = e_3)
                                   d_l = relu(conv3x3(relu(conv3x3(concat(u, e_l)))))
    head:                          y = conv1x1(d_0) + b   (no activation)
    loss:                          L = mean((y - target)^2)

3x3 convolutions use zero "same" padding; weights W[tap, c_in, c_out] with
tap = (dy + 1) * 3 + (dx + 1) act as out[y, x] = sum in[y + dy, x + dx] W[tap].
Nothing here is tuned; every backward formula is the plain adjoint of its
forward and is pinned by central finite differences in the tests.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


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


def relu(x):
    return np.maximum(x, 0.0)


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


def _block(x, p, name, cache):
    z1 = conv3x3(x, p[name + "a.W"], p[name + "a.b"])
    a1 = relu(z1)
    z2 = conv3x3(a1, p[name + "b.W"], p[name + "b.b"])
    a2 = relu(z2)
    cache[name] = (x, a1, a2)
    return a2


def forward(p, x):
    """x [B,H,W,Cin] -> (y [B,H,W,Cout], cache)."""
    cache = {}
    e0 = _block(x, p, "e0", cache)
    e1 = _block(avgpool(e0), p, "e1", cache)
    e2 = _block(avgpool(e1), p, "e2", cache)
    e3 = _block(avgpool(e2), p, "e3", cache)
    d2 = _block(np.concatenate([upsample(e3), e2], axis=-1), p, "d2", cache)
    d1 = _block(np.concatenate([upsample(d2), e1], axis=-1), p, "d1", cache)
    d0 = _block(np.concatenate([upsample(d1), e0], axis=-1), p, "d0", cache)
    y = d0 @ p["head.W"] + p["head.b"]
    cache["d0out"] = d0
    return y, cache


def loss(y, target):
    return float(np.mean((y - target) ** 2))


def _block_backward(p, name, cache, g, grads):
    x, a1, a2 = cache[name]
    g = g * (a2 > 0)
    g, grads[name + "b.W"], grads[name + "b.b"] = conv3x3_backward(a1, p[name + "b.W"], g)
    g = g * (a1 > 0)
    g, grads[name + "a.W"], grads[name + "a.b"] = conv3x3_backward(x, p[name + "a.W"], g)
    return g


def backward(p, cache, y, target):
    """Gradients of loss(y, target) w.r.t. every parameter."""
    grads = {}
    gy = 2.0 * (y - target) / y.size
    d0 = cache["d0out"]
    grads["head.W"] = d0.reshape(-1, d0.shape[-1]).T @ gy.reshape(-1, gy.shape[-1])
    grads["head.b"] = gy.reshape(-1, gy.shape[-1]).sum(axis=0)
    g = gy @ p["head.W"].T
    skips = {}
    for lvl, skip, up_ch in (("d0", "e0", None), ("d1", "e1", None), ("d2", "e2", None)):
        gcat = _block_backward(p, lvl, cache, g, grads)
        c_skip = cache[skip][2].shape[-1]
        skips[skip] = gcat[..., -c_skip:]
        g = upsample_backward(gcat[..., :-c_skip])
    g = _block_backward(p, "e3", cache, g, grads)
    for lvl in ("e2", "e1", "e0"):
        g = avgpool_backward(g) + skips[lvl]
        g = _block_backward(p, lvl, cache, g, grads)
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

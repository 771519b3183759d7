"""Python binding of the warm-start network library ``liblbnn.so``
(include/lbnn.h): argument marshalling only.  torch provides the workspace
and the stream; every layer runs in the library's kernels."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbnn.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("liblbnn.so is missing: run `python -m paper_1003_0282_amd.build` "
                      "(the network has no CPU fallback)")


class Desc(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("c_in", C.c_int32), ("c_out", C.c_int32),
                ("widths", C.c_int32 * 4), ("max_batch", C.c_int32)]


# torch's HIP runtime is loaded before the library so that both use the
# same one (the library only borrows torch's device memory and streams)
import torch  # noqa: E402,F401

_L = C.CDLL(LIB_PATH)
_st = C.c_int32
_P = C.c_void_p
_sigs = {
    "lbnn_workspace_bytes": (_st, [C.POINTER(Desc), C.POINTER(C.c_size_t)]),
    "lbnn_create": (_st, [C.POINTER(Desc), _P, C.c_size_t, _P, C.POINTER(_P)]),
    "lbnn_destroy": (None, [_P]),
    "lbnn_param_count": (_st, [_P, C.POINTER(C.c_int64)]),
    "lbnn_set_params": (_st, [_P, _P]),
    "lbnn_get_params": (_st, [_P, _P]),
    "lbnn_forward": (_st, [_P, _P, _P, C.c_int32]),
    "lbnn_backward": (_st, [_P, _P, _P, C.POINTER(C.c_double)]),
    "lbnn_adam": (_st, [_P, C.c_float, C.c_float, C.c_float, C.c_float]),
    "lbnn_train_step": (_st, [_P, _P, _P, C.c_int32, C.c_float, C.POINTER(C.c_double)]),
    "lbnn_to_fields": (_st, [_P, _P, C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_float),
                             C.c_int32, C.POINTER(_P)]),
    "lbnn_mfma_selftest": (_st, [_P, _P, C.POINTER(C.c_int32)]),
    "lbnn_last_error": (C.c_char_p, []),
}
for _n, (_r, _a) in _sigs.items():
    _f = getattr(_L, _n)
    _f.restype = _r
    _f.argtypes = _a


class LbnnError(RuntimeError):
    pass


def _check(st, where):
    if st != 0:
        raise LbnnError("%s failed (status %d): %s" % (where, st, _L.lbnn_last_error().decode()))


def exported_symbols():
    return sorted(_sigs)


def mfma_selftest() -> int:
    import torch
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = C.c_int32(-1)
    s = torch.cuda.current_stream()
    _check(_L.lbnn_mfma_selftest(C.c_void_p(cnt.data_ptr()), C.c_void_p(s.cuda_stream),
                                 C.byref(out)), "lbnn_mfma_selftest")
    return int(out.value)


class Net:
    """One U-Net instance (parameters, Adam state, activations) in a torch
    workspace."""

    def __init__(self, H, W, c_in, c_out=4, widths=(32, 64, 128, 256), max_batch=8,
                 device="cuda", stream=None):
        import torch
        self.desc = Desc()
        self.desc.H, self.desc.W, self.desc.c_in, self.desc.c_out = H, W, c_in, c_out
        for k in range(4):
            self.desc.widths[k] = widths[k]
        self.desc.max_batch = max_batch
        nb = C.c_size_t()
        _check(_L.lbnn_workspace_bytes(C.byref(self.desc), C.byref(nb)), "lbnn_workspace_bytes")
        self.device = torch.device(device)
        self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(_L.lbnn_create(C.byref(self.desc), C.c_void_p(ptr), nb, C.c_void_p(self.stream.cuda_stream),
                              C.byref(h)), "lbnn_create")
        self.h = h
        n = C.c_int64()
        _check(_L.lbnn_param_count(self.h, C.byref(n)), "lbnn_param_count")
        self.nparam = int(n.value)
        self.H, self.W, self.c_in, self.c_out, self.max_batch = H, W, c_in, c_out, max_batch

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            _L.lbnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat):
        import torch
        t = torch.as_tensor(np.asarray(flat, dtype=np.float32) if not isinstance(flat, torch.Tensor)
                            else flat, dtype=torch.float32, device=self.device).contiguous()
        assert t.numel() == self.nparam
        _check(_L.lbnn_set_params(self.h, C.c_void_p(t.data_ptr())), "lbnn_set_params")
        self.stream.synchronize()

    def get_params(self):
        import torch
        t = torch.empty(self.nparam, dtype=torch.float32, device=self.device)
        _check(_L.lbnn_get_params(self.h, C.c_void_p(t.data_ptr())), "lbnn_get_params")
        return t

    def forward(self, x):
        """x: torch float32 [B, H, W, c_in] on the device -> y [B, H, W, c_out]."""
        import torch
        x = x.contiguous()
        B = x.shape[0]
        y = torch.empty((B, self.H, self.W, self.c_out), dtype=torch.float32, device=self.device)
        _check(_L.lbnn_forward(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), B),
               "lbnn_forward")
        return y

    def backward(self, target, want_grads=True):
        import torch
        target = target.contiguous()
        g = torch.empty(self.nparam, dtype=torch.float32, device=self.device) if want_grads else None
        L = C.c_double()
        _check(_L.lbnn_backward(self.h, C.c_void_p(target.data_ptr()),
                                C.c_void_p(g.data_ptr()) if g is not None else None, C.byref(L)),
               "lbnn_backward")
        return float(L.value), g

    def adam(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        _check(_L.lbnn_adam(self.h, lr, b1, b2, eps), "lbnn_adam")

    def train_step(self, x, target, lr):
        L = C.c_double()
        _check(_L.lbnn_train_step(self.h, C.c_void_p(x.contiguous().data_ptr()),
                                  C.c_void_p(target.contiguous().data_ptr()), x.shape[0], lr,
                                  C.byref(L)), "lbnn_train_step")
        return float(L.value)

    def to_fields(self, y, scale, offset, outs, smooth=False):
        """y [B,H,W,c_out] -> one packed float field per channel (torch tensors
        or None to skip), optionally low-passed by (1, 2, 1)/4 along H and W."""
        k = self.c_out
        sc = (C.c_float * k)(*[float(v) for v in scale[:k]])
        of = (C.c_float * k)(*[float(v) for v in offset[:k]])
        ptrs = (_P * k)(*[o.data_ptr() if o is not None else None for o in outs[:k]])
        _check(_L.lbnn_to_fields(self.h, C.c_void_p(y.data_ptr()), y.shape[0], sc, of,
                                 int(bool(smooth)), ptrs), "lbnn_to_fields")


def flatten_params(p: dict, names) -> np.ndarray:
    return np.concatenate([np.asarray(p[n], dtype=np.float64).reshape(-1) for n in names])


def unflatten(flat, shapes):
    out, off = {}, 0
    for name, shape in shapes:
        n = int(np.prod(shape))
        out[name] = np.asarray(flat[off:off + n]).reshape(shape)
        off += n
    return out

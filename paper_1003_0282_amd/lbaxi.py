"""Python binding of the C-ABI library ``liblbaxi.so`` (include/lbaxi.h).

Argument marshalling only: PyTorch provides the device memory (one uint8
workspace tensor per handle, field tensors) and the HIP stream; every step of
the method runs in the library's kernels.  Importing this module fails loudly
when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbaxi.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("liblbaxi.so is missing: run `python -m paper_1003_0282_amd.build` "
                      "(the HIP library has no CPU fallback)")

FP64, FP32, FP32_FAST = 0, 1, 2
SWIRL, THERMAL, CARTESIAN, WET_WALLS, MRT, ORIGINAL, ZOU_HE, PLANES = 1, 2, 4, 8, 16, 32, 64, 128
SIDE = {"axis": 0, "wall": 1, "periodic": 2, "freeslip": 3}
RUNNING, CONVERGED, DIVERGED, CAPPED = 0, 1, 2, 3
STATUS_NAMES = {RUNNING: "running", CONVERGED: "converged", DIVERGED: "diverged",
                CAPPED: "capped"}


class Side(C.Structure):
    _fields_ = [("kind", C.c_int32), ("thermal", C.c_int32), ("u_z", C.c_double),
                ("u_r", C.c_double), ("omega", C.c_double), ("T", C.c_double),
                ("r_split", C.c_double), ("kind2", C.c_int32), ("thermal2", C.c_int32),
                ("omega2", C.c_double), ("T2", C.c_double)]


class Desc(C.Structure):
    _fields_ = [("nz", C.c_int32), ("nr", C.c_int32), ("r0", C.c_double),
                ("prec", C.c_int32), ("fields", C.c_uint32), ("tau", C.c_double),
                ("tau_g", C.c_double), ("tau_h", C.c_double), ("rho0", C.c_double),
                ("a0", C.c_double), ("period", C.c_double), ("phase", C.c_double),
                ("gbeta", C.c_double), ("T_ref", C.c_double), ("south", Side),
                ("north", Side), ("west", Side), ("east", Side), ("s_e", C.c_double),
                ("s_eps", C.c_double), ("s_q", C.c_double)]


# torch's HIP runtime is loaded before the library so that both use the
# same one (the library only borrows torch's device memory and streams)
import torch  # noqa: E402,F401

_L = C.CDLL(LIB_PATH)
_st = C.c_int32
_P = C.c_void_p
_sigs = {
    "lbaxi_last_error": (C.c_char_p, []),
    "lbaxi_strerror": (C.c_char_p, [_st]),
    "lbaxi_workspace_bytes": (_st, [C.c_int32, C.POINTER(Desc), C.POINTER(C.c_size_t)]),
    "lbaxi_create": (_st, [C.c_int32, C.POINTER(Desc), _P, C.c_size_t, _P, C.POINTER(_P)]),
    "lbaxi_destroy": (None, [_P]),
    "lbaxi_seed": (_st, [_P, _P, _P, _P, _P, _P]),
    "lbaxi_step": (_st, [_P, C.c_int64]),
    "lbaxi_macros": (_st, [_P, _P, _P, _P, _P, _P]),
    "lbaxi_residual": (_st, [_P, C.POINTER(C.c_double)]),
    "lbaxi_residual_static": (_st, [_P, C.POINTER(C.c_double)]),
    "lbaxi_time": (_st, [_P, C.c_int32, C.POINTER(C.c_int64)]),
    "lbaxi_batch_run": (_st, [_P, C.c_double, C.c_int64, C.c_int64, C.POINTER(C.c_int32),
                              C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "lbaxi_resume": (_st, [_P, C.POINTER(C.c_int32)]),
    "lbaxi_set_launch": (_st, [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "lbaxi_get_launch": (_st, [_P, C.POINTER(C.c_int32)]),
    "lbaxi_set_graph_steps": (_st, [_P, C.c_int32]),
    "lbaxi_set_fused_walls": (_st, [_P, C.c_int32]),
    "lbaxi_autotune": (_st, [_P, C.c_int32, C.POINTER(C.c_int32)]),
    "lbaxi_state_bytes": (_st, [_P, C.POINTER(C.c_size_t)]),
    "lbaxi_save": (_st, [_P, _P, C.c_size_t]),
    "lbaxi_load": (_st, [_P, _P, C.c_size_t]),
    "lbaxi_node_count": (_st, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "lbaxi_abi_desc_size": (C.c_size_t, []),
    "lbaxi_stream_copy": (_st, [_P, _P, C.c_size_t, C.c_int32, _P]),
    "lbaxi_set_profiling": (_st, [_P, C.c_int32]),
    "lbaxi_kernel_time": (_st, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
}
for _name, (_res, _args) in _sigs.items():
    _f = getattr(_L, _name)
    _f.restype = _res
    _f.argtypes = _args

if _L.lbaxi_abi_desc_size() != C.sizeof(Desc):
    raise ImportError("lbaxi_desc layout mismatch between liblbaxi.so and the binding")


class LbaxiError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = int(status)
        msg = "%s failed: %s (%s)" % (where, _L.lbaxi_strerror(status).decode(),
                                      _L.lbaxi_last_error().decode())
        super().__init__(msg)


def _check(status: int, where: str):
    if status != 0:
        raise LbaxiError(status, where)


def _side(d: dict) -> Side:
    s = Side()
    s.kind = SIDE[d.get("kind", "wall")]
    s.thermal = int(d.get("thermal", 0))
    s.u_z = float(d.get("uz", 0.0))
    s.u_r = float(d.get("ur", 0.0))
    s.omega = float(d.get("omega", 0.0))
    s.T = float(d.get("T", 0.0))
    s.r_split = float(d.get("r_split", -1.0))
    s.kind2 = SIDE[d.get("kind2", "wall")]
    s.thermal2 = int(d.get("thermal2", 0))
    s.omega2 = float(d.get("omega2", 0.0))
    s.T2 = float(d.get("T2", 0.0))
    return s


def make_desc(case: dict, prec: int) -> Desc:
    """Case dict (see workloads) -> lbaxi_desc."""
    d = Desc()
    d.nz, d.nr = int(case["nz"]), int(case["nr"])
    d.r0 = float(case.get("r0", 0.0))
    d.prec = int(prec)
    d.fields = ((SWIRL if case.get("swirl") else 0) | (THERMAL if case.get("thermal") else 0)
                | (CARTESIAN if case.get("cartesian") else 0)
                | (WET_WALLS if case.get("wet") else 0) | (MRT if case.get("mrt") else 0)
                | (ORIGINAL if case.get("original") else 0)
                | (ZOU_HE if case.get("zou_he") else 0) | (PLANES if case.get("planes") else 0))
    d.tau = float(case["tau"])
    d.tau_g = float(case.get("tau_g", 0.0))
    d.tau_h = float(case.get("tau_h", 0.0))
    d.rho0 = float(case.get("rho0", 1.0))
    d.a0 = float(case.get("a0", 0.0))
    d.period = float(case.get("period", 0.0))
    d.phase = float(case.get("phase", 0.0))
    d.gbeta = float(case.get("gbeta", 0.0))
    d.T_ref = float(case.get("T_ref", 0.0))
    d.south, d.north = _side(case["south"]), _side(case["north"])
    d.west, d.east = _side(case["west"]), _side(case["east"])
    d.s_e = float(case.get("s_e", 0.0))
    d.s_eps = float(case.get("s_eps", 0.0))
    d.s_q = float(case.get("s_q", 0.0))
    return d


def workspace_bytes(cases, prec: int) -> int:
    arr = (Desc * len(cases))(*[make_desc(c, prec) for c in cases])
    b = C.c_size_t()
    _check(_L.lbaxi_workspace_bytes(len(cases), arr, C.byref(b)), "lbaxi_workspace_bytes")
    return int(b.value)


@dataclass
class RunResult:
    status: np.ndarray
    steps: np.ndarray
    residual: np.ndarray


class Lattices:
    """A handle over one or many lattices living in one torch workspace.

    cases: list of case dicts (or one dict); prec: FP64 or FP32.
    """

    def __init__(self, cases, prec: int = FP64, device: str = "cuda", stream=None):
        import torch
        if isinstance(cases, dict):
            cases = [cases]
        self.cases = [dict(c) for c in cases]
        self.prec = int(prec)
        self.dtype = torch.float64 if self.prec == FP64 else torch.float32
        self.device = torch.device(device)
        self._descs = (Desc * len(cases))(*[make_desc(c, self.prec) for c in cases])
        nbytes = workspace_bytes(self.cases, self.prec)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(_L.lbaxi_create(len(cases), self._descs, C.c_void_p(self._ws_ptr),
                               C.c_size_t(nbytes), C.c_void_p(self.stream.cuda_stream),
                               C.byref(h)), "lbaxi_create")
        self.h = h
        self.n = len(cases)
        self.shapes = [(int(c["nr"]), int(c["nz"])) for c in self.cases]
        self.sizes = [nr * nz for nr, nz in self.shapes]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        self.nodes = int(self.offsets[-1])

    # -- lifetime --
    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            _L.lbaxi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers --
    def _field_ptr(self, x):
        import torch
        if x is None:
            return None
        if isinstance(x, (list, tuple)):
            x = torch.cat([torch.as_tensor(v, dtype=self.dtype).reshape(-1) for v in x])
        t = torch.as_tensor(x, dtype=self.dtype, device=self.device).reshape(-1).contiguous()
        if t.numel() != self.nodes:
            raise ValueError("field has %d values, the handle has %d nodes" % (t.numel(), self.nodes))
        self._keep.append(t)
        return C.c_void_p(t.data_ptr())

    def split(self, packed):
        """Packed [nodes] tensor -> list of [nr][nz] views, one per lattice."""
        return [packed[self.offsets[k]:self.offsets[k + 1]].view(*self.shapes[k])
                for k in range(self.n)]

    # -- API --
    def seed(self, uz=None, ur=None, uth=None, T=None, rho=None):
        """Equilibrium seeding from packed fields (None: rest / T_ref / rho0)."""
        self._keep = []
        ptrs = [self._field_ptr(x) for x in (rho, uz, ur, uth, T)]
        _check(_L.lbaxi_seed(self.h, *ptrs), "lbaxi_seed")
        self._keep_seed = self._keep  # inputs must live until the kernel ran
        self.stream.synchronize()

    def step(self, n: int = 1):
        _check(_L.lbaxi_step(self.h, int(n)), "lbaxi_step")

    def macros(self, which=("rho", "uz", "ur", "uth", "T")):
        import torch
        out = {k: torch.empty(self.nodes, dtype=self.dtype, device=self.device) for k in which}
        ptrs = [C.c_void_p(out[k].data_ptr()) if k in out else None
                for k in ("rho", "uz", "ur", "uth", "T")]
        _check(_L.lbaxi_macros(self.h, *ptrs), "lbaxi_macros")
        return out

    def macros_list(self, which=("rho", "uz", "ur", "uth", "T")):
        m = self.macros(which)
        return [{k: v[self.offsets[i]:self.offsets[i + 1]].view(*self.shapes[i])
                 for k, v in m.items()} for i in range(self.n)]

    def residual(self, raise_on_nan: bool = False) -> np.ndarray:
        out = (C.c_double * self.n)()
        st = _L.lbaxi_residual(self.h, out)
        if st == -5 and not raise_on_nan:
            return np.array(out[:])
        _check(st, "lbaxi_residual")
        return np.array(out[:])

    def residual_static(self, raise_on_nan: bool = False) -> np.ndarray:
        """lbaxi_residual_static: the residual with the library's fixed
        reduction words (no workspace use)."""
        out = (C.c_double * self.n)()
        st = _L.lbaxi_residual_static(self.h, out)
        if st == -5 and not raise_on_nan:
            return np.array(out[:])
        _check(st, "lbaxi_residual_static")
        return np.array(out[:])

    def time(self, k: int = 0) -> int:
        t = C.c_int64()
        _check(_L.lbaxi_time(self.h, int(k), C.byref(t)), "lbaxi_time")
        return int(t.value)

    def run(self, tol: float, max_steps: int, check_every: int) -> RunResult:
        st = (C.c_int32 * self.n)()
        steps = (C.c_int64 * self.n)()
        res = (C.c_double * self.n)()
        _check(_L.lbaxi_batch_run(self.h, float(tol), int(max_steps), int(check_every), st,
                                  steps, res), "lbaxi_batch_run")
        return RunResult(np.array(st[:]), np.array(steps[:]), np.array(res[:]))

    def resume(self) -> int:
        n = C.c_int32()
        _check(_L.lbaxi_resume(self.h, C.byref(n)), "lbaxi_resume")
        return int(n.value)

    def set_launch(self, tile_z=64, tile_r=4, grid=0, xcd=0, nt_store=1):
        _check(_L.lbaxi_set_launch(self.h, tile_z, tile_r, grid, xcd, nt_store),
               "lbaxi_set_launch")

    def get_launch(self):
        c = (C.c_int32 * 5)()
        _check(_L.lbaxi_get_launch(self.h, c), "lbaxi_get_launch")
        return tuple(c[:])

    def set_graph_steps(self, k: int):
        _check(_L.lbaxi_set_graph_steps(self.h, int(k)), "lbaxi_set_graph_steps")

    def set_fused_walls(self, on: bool):
        _check(_L.lbaxi_set_fused_walls(self.h, 1 if on else 0), "lbaxi_set_fused_walls")

    def autotune(self, steps_per_trial: int = 8):
        c = (C.c_int32 * 5)()
        _check(_L.lbaxi_autotune(self.h, int(steps_per_trial), c), "lbaxi_autotune")
        return tuple(c[:])

    def set_profiling(self, on: bool):
        _check(_L.lbaxi_set_profiling(self.h, int(bool(on))), "lbaxi_set_profiling")

    def kernel_time(self):
        """(summed step-kernel milliseconds, launches) since the last call."""
        ms = C.c_double()
        n = C.c_int64()
        _check(_L.lbaxi_kernel_time(self.h, C.byref(ms), C.byref(n)), "lbaxi_kernel_time")
        return float(ms.value), int(n.value)

    def save(self) -> bytes:
        n = C.c_size_t()
        _check(_L.lbaxi_state_bytes(self.h, C.byref(n)), "lbaxi_state_bytes")
        buf = C.create_string_buffer(n.value)
        _check(_L.lbaxi_save(self.h, buf, n), "lbaxi_save")
        return buf.raw

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(_L.lbaxi_load(self.h, buf, C.c_size_t(len(blob))), "lbaxi_load")


def exported_symbols() -> list[str]:
    return sorted(_sigs)

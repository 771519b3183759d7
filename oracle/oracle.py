"""ctypes front end of the FP64 CPU oracle (``lbaxi_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may use this module; the product path never does.  It
imports nothing from the GPU package and the GPU package imports nothing from
here.  A *case* is a plain dict (see ``paper_1003_0282_amd.workloads``) that
uses the usual BGK relaxation time tau_s; the oracle itself follows the
paper's tau (nu = tau/3, Sec. III A), so the conversion tau = tau_s - 1/2 and
the paper's default tau_g = 2 tau / 3 (Sec. III C) happen here.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbaxi_oracle.c")
_LIB = os.path.join(_HERE, "liblbaxi_oracle.so")

_KIND = {"axis": 0, "wall": 1, "periodic": 2, "freeslip": 3}


class _Side(C.Structure):
    _fields_ = [
        ("kind", C.c_int),
        ("uz", C.c_double),
        ("ur", C.c_double),
        ("omega", C.c_double),
        ("thermal", C.c_int),
        ("T", C.c_double),
        ("r_split", C.c_double),
        ("kind2", C.c_int),
        ("omega2", C.c_double),
        ("thermal2", C.c_int),
        ("T2", C.c_double),
    ]


class _Params(C.Structure):
    _fields_ = [
        ("nz", C.c_int),
        ("nr", C.c_int),
        ("r0", C.c_double),
        ("swirl", C.c_int),
        ("thermal", C.c_int),
        ("cartesian", C.c_int),
        ("wet", C.c_int),
        ("tau", C.c_double),
        ("tau_g", C.c_double),
        ("tau_h", C.c_double),
        ("rho0", C.c_double),
        ("a0", C.c_double),
        ("period", C.c_double),
        ("phase", C.c_double),
        ("gbeta", C.c_double),
        ("T_ref", C.c_double),
        ("side", _Side * 4),
        ("mrt", C.c_int),
        ("s_e", C.c_double),
        ("s_eps", C.c_double),
        ("s_q", C.c_double),
        ("s_rho", C.c_double),
        ("s_j", C.c_double),
        ("original", C.c_int),
        ("zou_he", C.c_int),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over radial rows)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        P = C.POINTER(C.c_double)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(_Params)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_seed.argtypes = [C.c_void_p, P, P, P, P, P]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_macros.argtypes = [C.c_void_p, P, P, P, P, P]
        L.orc_residual.restype = C.c_double
        L.orc_residual.argtypes = [C.c_void_p]
        L.orc_time.restype = C.c_int64
        L.orc_time.argtypes = [C.c_void_p]
        L.orc_get_state.argtypes = [C.c_void_p, P, P, P]
        L.orc_set_state.argtypes = [C.c_void_p, P, P, P, C.c_int64]
        L.orc_stream_only.argtypes = [C.c_void_p, P, P, P]
        L.orc_feq9.argtypes = [C.c_double, C.c_double, C.c_double, P]
        L.orc_geq4.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, P]
        L.orc_heq4.argtypes = [C.c_double, C.c_double, C.c_double, P]
        L.orc_node_macros.argtypes = [C.POINTER(_Params), C.c_int, C.c_int64, P, P, P, P]
        L.orc_node_source.argtypes = [C.POINTER(_Params), C.c_int, C.c_int64, P, P, P]
        L.orc_node_collide.argtypes = [C.POINTER(_Params), C.c_int, C.c_int64, P, P, P,
                                       P, P, P, P]
        L.orc_mrt_basis.argtypes = [P, P]
        L.orc_mrt_source_moments.argtypes = [C.POINTER(_Params), C.c_int, C.c_int64, P, P, P]
        L.orc_force_a.restype = C.c_double
        L.orc_force_a.argtypes = [C.POINTER(_Params), C.c_int64]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        L.orc_sizeof_params.restype = C.c_size_t
        assert L.orc_sizeof_params() == C.sizeof(_Params)
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _side(d: dict) -> _Side:
    s = _Side()
    s.kind = _KIND[d.get("kind", "wall")]
    s.uz = float(d.get("uz", 0.0))
    s.ur = float(d.get("ur", 0.0))
    s.omega = float(d.get("omega", 0.0))
    s.thermal = int(d.get("thermal", 0))
    s.T = float(d.get("T", 0.0))
    s.r_split = float(d.get("r_split", -1.0))
    s.kind2 = _KIND[d.get("kind2", "wall")]
    s.omega2 = float(d.get("omega2", 0.0))
    s.thermal2 = int(d.get("thermal2", 0))
    s.T2 = float(d.get("T2", 0.0))
    return s


def params(case: dict) -> _Params:
    """Case dict (tau_s convention) -> oracle parameters (paper's tau)."""
    p = _Params()
    p.nz, p.nr = int(case["nz"]), int(case["nr"])
    p.r0 = float(case.get("r0", 0.0))
    p.swirl = int(bool(case.get("swirl", False)))
    p.thermal = int(bool(case.get("thermal", False)))
    p.cartesian = int(bool(case.get("cartesian", False)))
    p.wet = int(bool(case.get("wet", False)))
    tau = float(case["tau"]) - 0.5
    p.tau = tau
    tg = float(case.get("tau_g", 0.0))
    p.tau_g = (tg - 0.5) if tg > 0 else 2.0 * tau / 3.0  # tau_g = 2 tau / 3
    th = float(case.get("tau_h", 0.0))
    p.tau_h = (th - 0.5) if th > 0 else tau
    p.rho0 = float(case.get("rho0", 1.0))
    p.a0 = float(case.get("a0", 0.0))
    p.period = float(case.get("period", 0.0))
    p.phase = float(case.get("phase", 0.0))
    p.gbeta = float(case.get("gbeta", 0.0))
    p.T_ref = float(case.get("T_ref", 0.0))
    for k, name in enumerate(("south", "north", "west", "east")):
        p.side[k] = _side(case[name])
    # MRT rates (Sec. III B): s_v = 1/(tau + 1/2); s_e = s_v as the paper
    # requires for axisymmetric flow, s_eps = s_v (the even moments of a
    # two-relaxation-time model) and s_q from (1/s_v - 1/2)(1/s_q - 1/2) =
    # 3/16 unless the case gives them; the conserved-moment rates drop out.
    p.mrt = int(bool(case.get("mrt", False)))
    sv = 1.0 / (tau + 0.5)
    p.s_e = float(case.get("s_e", 0.0)) or sv
    p.s_eps = float(case.get("s_eps", 0.0)) or sv
    p.s_q = float(case.get("s_q", 0.0)) or 1.0 / (0.5 + 3.0 / (16.0 * tau))
    p.s_rho = float(case.get("s_rho", 1.0))
    p.s_j = float(case.get("s_j", 1.0))
    # the original scheme of Sec. II (Eqs. 5-10): f only, halfway walls
    p.original = int(bool(case.get("original", False)))
    if p.original and (p.swirl or p.thermal or p.wet or p.mrt):
        raise ValueError("the original scheme models f only, with halfway walls and BGK")
    # Zou-He no-slip on the radial walls of a wet-node lattice
    p.zou_he = int(bool(case.get("zou_he", False)))
    if p.zou_he and (not p.wet or any(case[s].get("kind") == "wall" and case[s].get("ur", 0.0)
                                      for s in ("south", "north"))
                     or case["west"].get("kind") != "periodic"):
        raise ValueError("Zou-He walls need wet-node walls, periodic z-ends (the paper's "
                         "pipes) and no normal wall velocity")
    return p


class Oracle:
    """One lattice advanced by the CPU oracle."""

    def __init__(self, case: dict, threads: int | None = None):
        self.case = dict(case)
        self.p = params(case)
        self.L = lib()
        if threads is not None:
            self.L.orc_set_threads(int(threads))
        self.h = self.L.orc_create(C.byref(self.p))
        if not self.h:
            raise MemoryError("oracle allocation failed")
        self.nz, self.nr = self.p.nz, self.p.nr

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.L.orc_destroy(h)
            self.h = None

    def _field(self, a):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64).reshape(self.nr, self.nz)
        return a

    def seed(self, uz=None, ur=None, uth=None, T=None, rho=None):
        fields = [self._field(x) for x in (uz, ur, uth, T, rho)]
        self.L.orc_seed(self.h, *[_ptr(x) for x in fields])

    def step(self, n: int = 1):
        self.L.orc_step(self.h, int(n))

    @property
    def t(self) -> int:
        return int(self.L.orc_time(self.h))

    def macros(self):
        out = [np.empty((self.nr, self.nz)) for _ in range(5)]
        self.L.orc_macros(self.h, *[_ptr(x) for x in out])
        return dict(zip(("rho", "uz", "ur", "uth", "T"), out))

    def residual(self) -> float:
        return float(self.L.orc_residual(self.h))

    def get_state(self):
        n = self.nz * self.nr
        f = np.empty((9, self.nr, self.nz))
        g = np.empty((4, self.nr, self.nz))
        h = np.empty((4, self.nr, self.nz))
        self.L.orc_get_state(self.h, _ptr(f), _ptr(g), _ptr(h))
        assert f.size == 9 * n
        return f, g, h

    def set_state(self, f, g=None, h=None, t: int = 0):
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = None if g is None else np.ascontiguousarray(g, dtype=np.float64)
        h = None if h is None else np.ascontiguousarray(h, dtype=np.float64)
        self.L.orc_set_state(self.h, _ptr(f), _ptr(g), _ptr(h), int(t))

    def stream_only(self, fs, gs=None, hs=None):
        fs = np.ascontiguousarray(fs, dtype=np.float64)
        gs = None if gs is None else np.ascontiguousarray(gs, dtype=np.float64)
        hs = None if hs is None else np.ascontiguousarray(hs, dtype=np.float64)
        self.L.orc_stream_only(self.h, _ptr(fs), _ptr(gs), _ptr(hs))


# ---- node-level entry points used by the identity tests --------------------

def feq9(rho, uz, ur):
    out = np.empty(9)
    lib().orc_feq9(rho, uz, ur, _ptr(out))
    return out


def geq4(rho0, uth, uz, ur):
    out = np.empty(4)
    lib().orc_geq4(rho0, uth, uz, ur, _ptr(out))
    return out


def heq4(T, uz, ur):
    out = np.empty(4)
    lib().orc_heq4(T, uz, ur, _ptr(out))
    return out


def node_macros(case, j, t, f, g=None, h=None):
    p = params(case)
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.zeros(4) if g is None else np.ascontiguousarray(g, dtype=np.float64)
    h = np.zeros(4) if h is None else np.ascontiguousarray(h, dtype=np.float64)
    out = np.empty(5)
    lib().orc_node_macros(C.byref(p), int(j), int(t), _ptr(f), _ptr(g), _ptr(h), _ptr(out))
    return out


def node_source(case, j, t, m, feq):
    p = params(case)
    S = np.empty(9)
    lib().orc_node_source(C.byref(p), int(j), int(t), _ptr(np.asarray(m, float)),
                          _ptr(np.asarray(feq, float)), _ptr(S))
    return S


def node_collide(case, j, t, f, g=None, h=None):
    p = params(case)
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.zeros(4) if g is None else np.ascontiguousarray(g, dtype=np.float64)
    h = np.zeros(4) if h is None else np.ascontiguousarray(h, dtype=np.float64)
    fo, go, ho, m = np.empty(9), np.empty(4), np.empty(4), np.empty(5)
    lib().orc_node_collide(C.byref(p), int(j), int(t), _ptr(f), _ptr(g), _ptr(h),
                           _ptr(fo), _ptr(go), _ptr(ho), _ptr(m))
    return fo, go, ho, m


def mrt_basis():
    """(M, M^-1) of the MRT moments, Eq. (38), rows in the order of m."""
    M, Mi = np.empty((9, 9)), np.empty((9, 9))
    lib().orc_mrt_basis(_ptr(M), _ptr(Mi))
    return M, Mi


def mrt_source_moments(case, j, t, m, meq):
    """S~ = -(u_r / r) m_eq + S~' of Eq. (51) for macros m at row j."""
    p = params(case)
    St = np.empty(9)
    lib().orc_mrt_source_moments(C.byref(p), int(j), int(t), _ptr(np.asarray(m, float)),
                                 _ptr(np.asarray(meq, float)), _ptr(St))
    return St


def force_a(case, t):
    p = params(case)
    return float(lib().orc_force_a(C.byref(p), int(t)))


def set_threads(n: int):
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())

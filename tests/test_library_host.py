"""Host-side checks of the C-ABI library that need no GPU: every function the
header declares is exported, descriptors are validated as documented, and
the workspace size is consistent."""
import ctypes as C
import os
import re

import pytest

from paper_1003_0282_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b((?:lbaxi|lbnn)_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    from paper_1003_0282_amd import lbaxi
    return lbaxi


def test_every_declared_symbol_is_exported(L):
    from paper_1003_0282_amd import lbnn
    libs = {"lbaxi.h": C.CDLL(L.LIB_PATH), "lbnn.h": C.CDLL(lbnn.LIB_PATH)}
    headers = sorted(h for h in os.listdir(os.path.join(ROOT, "include")) if h.endswith(".h"))
    assert headers == sorted(libs)
    total = 0
    for hdr, lib in libs.items():
        names = [n for n in _declared(hdr) if n.startswith(hdr.split(".")[0] + "_")]
        total += len(names)
        missing = [n for n in names if not hasattr(lib, n)]
        assert not missing, (hdr, missing)
    assert total >= 30


def test_binding_covers_header(L):
    from paper_1003_0282_amd import lbnn
    declared = set(_declared("lbaxi.h"))
    assert declared == set(L.exported_symbols()), declared ^ set(L.exported_symbols())
    declared_nn = set(n for n in _declared("lbnn.h") if n.startswith("lbnn_"))
    assert declared_nn == set(lbnn.exported_symbols()), declared_nn ^ set(lbnn.exported_symbols())


def test_nn_workspace_and_validation():
    import ctypes as C2
    from paper_1003_0282_amd import lbnn
    d = lbnn.Desc()
    d.H, d.W, d.c_in, d.c_out, d.max_batch = 128, 256, 8, 4, 4
    for k, w in enumerate((32, 64, 128, 256)):
        d.widths[k] = w
    b = C2.c_size_t()
    assert lbnn._L.lbnn_workspace_bytes(C2.byref(d), C2.byref(b)) == 0
    assert b.value > 4 * 4 * 1.9e6
    d.widths[1] = 48
    assert lbnn._L.lbnn_workspace_bytes(C2.byref(d), C2.byref(b)) == -1
    d.widths[1] = 288  # a multiple of 32 above the 256 the kernels stage
    assert lbnn._L.lbnn_workspace_bytes(C2.byref(d), C2.byref(b)) == -1
    d.widths[1] = 64
    d.max_batch = 128  # 128 x 128 x 256 pixels: the 32-bit indexing bound
    assert lbnn._L.lbnn_workspace_bytes(C2.byref(d), C2.byref(b)) == -1
    d.max_batch = 127
    assert lbnn._L.lbnn_workspace_bytes(C2.byref(d), C2.byref(b)) == 0


def test_desc_layout(L):
    assert L._L.lbaxi_abi_desc_size() == C.sizeof(L.Desc)


def _status(L, cases, prec=0):
    try:
        L.workspace_bytes(cases, prec)
        return 0
    except L.LbaxiError as e:
        return e.status


def test_validation(L):
    ok = W.hagen_poiseuille()
    assert _status(L, [ok]) == 0
    bad_tau = dict(ok, tau=0.5)
    assert _status(L, [bad_tau]) == -2
    # tau_s up to 3/2 is stable on the axis pipe, beyond it omega_- < 0 at r = 1
    assert _status(L, [dict(ok, tau=1.45)]) == 0
    assert _status(L, [dict(ok, tau=1.55)]) == -2
    assert _status(L, [dict(ok, nz=1)]) == -1
    assert _status(L, [dict(ok, r0=2.0)]) == -1          # axis needs r0 = 0
    assert _status(L, [dict(ok, north=W.axis())]) == -1  # axis only south
    assert _status(L, [dict(ok, west=W.wall())]) == -1   # periodic on one end only
    assert _status(L, [dict(ok, north=W.freeslip())]) == -1
    assert _status(L, [dict(ok, swirl=True, tau_g=1.6)]) == -2
    assert _status(L, [ok, W.cavity(8, 8, 10.0)]) == -1  # mixed field sets
    assert _status(L, [ok], prec=7) == -1
    # MRT: rates in (0, 2) or 0 for the default; the BGK row check of f does
    # not apply (tau_s = 1.55 is allowed); one collision model per batch
    mrt = dict(ok, mrt=True)
    assert _status(L, [mrt]) == 0
    assert _status(L, [dict(mrt, tau=1.55)]) == 0
    assert _status(L, [dict(mrt, s_q=2.0)]) == -2
    assert _status(L, [dict(mrt, s_eps=-0.1)]) == -2
    assert _status(L, [dict(mrt, s_e=1.9, s_eps=0.3, s_q=1.99)]) == 0
    assert _status(L, [dict(mrt, tau=0.5)]) == -2
    assert _status(L, [mrt, ok]) == -1
    assert _status(L, [mrt, dict(mrt, wet=True), dict(mrt, cartesian=True, r0=0.0)]) == 0
    # original scheme: f only, halfway walls; its own kernels per batch
    orig = dict(ok, original=True)
    assert _status(L, [orig]) == 0
    assert _status(L, [dict(orig, swirl=True)]) == -1
    assert _status(L, [dict(orig, wet=True)]) == -1
    assert _status(L, [dict(orig, mrt=True)]) == -1
    assert _status(L, [orig, ok]) == -1
    assert L.workspace_bytes([orig], 0) > L.workspace_bytes([ok], 0)
    # Zou-He: on wet-node walls only, radial walls without normal velocity
    zh = dict(ok, wet=True, zou_he=True)
    assert _status(L, [zh]) == 0
    assert _status(L, [dict(ok, zou_he=True)]) == -1
    assert _status(L, [dict(zh, north=W.wall(ur=1e-3))]) == -1
    assert _status(L, [zh, dict(ok, wet=True)]) == 0   # a per-lattice wall model
    assert _status(L, [dict(zh, west=W.wall(), east=W.wall())]) == -1


def test_workspace_grows_with_batch(L):
    a = L.workspace_bytes([W.cavity(16, 24, 100.0)], 1)
    b = L.workspace_bytes([W.cavity(16, 24, 100.0)] * 3, 1)
    assert b > 2 * a
    assert L.workspace_bytes([W.cavity(16, 24, 100.0)], 0) > a


def test_largest_lattice_accepted(L):
    """In-lattice byte offsets are 32-bit: a lattice whose populations (nr + 4
    row blocks of 9 padded rows of 16448 floats at nz = 16384) reach 4 GiB is
    refused, one just below is accepted (FP32, f only)."""
    ok = W.base_case(16384, 7200, 0.8, a0=1e-7)      # 7204 * 9 * 16448 * 4 B < 2^32
    too_big = W.base_case(16384, 7300, 0.8, a0=1e-7)  # 7304 * 9 * 16448 * 4 B > 2^32
    assert _status(L, [ok], prec=1) == 0
    assert _status(L, [too_big], prec=1) == -1
    # the bound counts bytes: the accepted FP32 lattice is refused in FP64
    assert _status(L, [ok], prec=0) == -1
    assert _status(L, [W.base_case(16384, 3600, 0.8, a0=1e-7)], prec=0) == 0

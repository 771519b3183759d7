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
    """Element indices inside a lattice are 32-bit: a lattice of 2^31
    population elements or more is refused, one just below is accepted (it
    is stored as planes, since its row blocks would pass 4 GiB).  At
    nz = 16384 a padded row holds 16448 floats or 16416 doubles; f only."""
    ok = W.base_case(16384, 14000, 0.8, a0=1e-7)       # 9 planes of 14002 rows + strips < 2^31
    too_big = W.base_case(16384, 14600, 0.8, a0=1e-7)  # 9 * 14602 * 16448 > 2^31
    assert _status(L, [ok], prec=1) == 0
    assert _status(L, [too_big], prec=1) == -1
    # the bound counts elements, not bytes: the same in FP64
    assert _status(L, [ok], prec=0) == 0
    assert _status(L, [too_big], prec=0) == -1


def test_layout_sizes(L):
    """Row blocks take nr + 4 blocks of Q padded rows; planes Q planes of
    nr + 2 padded rows and two strips; a lattice whose row blocks would pass
    4 GiB takes the plane layout by itself."""
    small = W.base_case(100, 50, 0.8)
    rb = L.workspace_bytes([small], 1)
    pl = L.workspace_bytes([dict(small, planes=True)], 1)
    # rows of 100 floats pad to 160 (lead-in 32, 101 slots, 128-byte
    # rounding), strips of 52 to 64: row blocks 54 x 9 x 160 elements,
    # planes 9 x (52 x 160 + 2 x 64); two buffers, each 64-element aligned
    # within 256-byte aligned workspace slices
    d = (54 * 9 * 160 - 9 * (52 * 160 + 2 * 64)) * 4 * 2
    assert abs((rb - pl) - d) <= 2 * 256, (rb, pl, d)
    big = W.base_case(16384, 7300, 0.8)
    assert L.workspace_bytes([big], 1) == L.workspace_bytes([dict(big, planes=True)], 1)
    mid = W.base_case(16384, 7200, 0.8)  # row blocks fit below 4 GiB
    assert L.workspace_bytes([mid], 1) != L.workspace_bytes([dict(mid, planes=True)], 1)

"""Stream-function post-processing (d psi/dr = -r u_z, d psi/dz = r u_r,
Sec. IV B) and the Wheeler workload's parameters, on the CPU."""
import numpy as np

from paper_1003_0282_amd import streamfn as SF
from paper_1003_0282_amd import workloads as W


def test_pipe_profile_closed_form():
    """u_z = U0 (1 - r^2/R^2) gives psi = -U0 (r^2/2 - r^4 / (4 R^2))."""
    R, n = 50.0, 50
    r = np.arange(n, dtype=float)
    uz = np.tile((1 - r ** 2 / R ** 2)[:, None], (1, 3))
    psi = SF.stream_function(uz)
    want = -(r ** 2 / 2 - r ** 4 / (4 * R ** 2))
    assert np.abs(psi[:, 1] - want).max() < 2e-3 * np.abs(want).max()


def test_both_relations_recover_a_solenoidal_field():
    """psi = r^2 (1 - r^2/R^2) sin(pi z / H): u_z = -(1/r) d_r psi, u_r =
    (1/r) d_z psi; both integrations return psi (second order)."""
    errs = []
    for n in (40, 80):
        R, H = n - 1.0, n - 1.0
        r = np.arange(n, dtype=float)[:, None]
        z = np.arange(n, dtype=float)[None, :]
        s = np.sin(np.pi * z / H)
        psi = r ** 2 * (1 - r ** 2 / R ** 2) * s
        uz = -(2 - 4 * r ** 2 / R ** 2) * s
        ur = r * (1 - r ** 2 / R ** 2) * (np.pi / H) * np.cos(np.pi * z / H)
        a, b = SF.stream_function(uz), SF.stream_function_z(ur)
        scale = np.abs(psi).max()
        errs.append((np.abs(a - psi).max() / scale, np.abs(b - psi).max() / scale))
    assert errs[1][0] < 1e-3 and errs[1][1] < 1e-3, errs
    assert errs[0][0] / errs[1][0] > 3.5 and errs[0][1] / errs[1][1] > 3.5, errs


def test_wheeler_parameters():
    """H = R_c, crystal radius 0.4 R_c, U_t = beta R_c Omega_x = 0.1,
    Re = R_c^2 Omega / nu for crystal and crucible."""
    for Re_x, Re_c in ((100.0, -25.0), (1000.0, -250.0)):
        c = W.wheeler(Re_x, Re_c)
        Rc, nu = c["R_c"], (c["tau"] - 0.5) / 3
        assert c["nz"] - 1 == Rc == c["nr"] - 1
        assert abs(c["nu"] - nu) < 1e-15
        om_x, om_c = c["east"]["omega"], c["north"]["omega"]
        assert abs(0.4 * Rc * om_x - 0.1) < 1e-12
        assert abs(Rc * Rc * om_x / nu - Re_x) < 1e-9 and abs(Rc * Rc * om_c / nu - Re_c) < 1e-9
        assert c["west"]["omega"] == om_c and c["east"]["r_split"] == 0.4 * Rc
        assert c["east"]["kind2"] == "freeslip" and c["wet"] and not c["thermal"]


def test_extrema_units():
    """psi is reported in units of nu R_c."""
    c = W.wheeler(100.0, -25.0, n=20)
    uz = np.zeros((20, 20))
    uz[:5] = 1.0
    lo, hi = SF.wheeler_extrema(c, uz)
    psi = SF.stream_function(uz)
    assert abs(lo - psi.min() / (c["nu"] * c["R_c"])) < 1e-15 and hi == 0.0

"""Pins of the CPU oracle's time step and of its Eq. (57) residual.

1. One complete time step of the improved scheme is evaluated here a second
   time, independently of the oracle and exactly, in rational arithmetic
   (Python ``fractions``), from the equations as the paper states them:
   macros by Eqs. (16)-(17) with the velocity-independent force added
   (u_theta = sum g / rho0, Sec. III C), the equilibrium of Eq. (6), the
   source of Eq. (12) with F_r = -2 mu0 u_r / r^2 + rho0 u_theta^2 / r, the
   direction-dependent rate omega_a = (1 + tau e_ar / r)/(tau + 1/2) and the
   update of Eq. (13); the swirl populations by Eqs. (53)-(54); every 1/r
   term zero on the axis (Sec. IV A); then pull streaming with a periodic z
   wrap, the specular axis mirror for f, the non-equilibrium extrapolation of
   g onto the axis row (Sec. IV B) and a halfway moving wall at r = R.  The
   3 x 4 lattice holds the axis row, wall links, the periodic wrap, a body
   force and swirl.  The oracle must agree to 1e-15 on every population,
   and each of a few plausible slips (a direction-blind omega, a dropped
   (1 - omega/2) factor, a flipped mass source, an axis that bounces back
   instead of mirroring) must miss it by far more.
2. The residual of Eq. (57) is the largest change of |u| = sqrt(u_z^2 +
   u_r^2) between the last two time levels: it must equal the NumPy
   difference of two consecutive macro fields exactly, differ from the
   pairing with the level before, and be NaN when the state holds a NaN.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from paper_1003_0282_amd import workloads as W

# D2Q9 in the oracle's documented order, components (e_z, e_r), weights of Eq. (6)
E9 = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
W9 = [Fr(4, 9)] + [Fr(1, 9)] * 4 + [Fr(1, 36)] * 4
E4 = [(1, 0), (0, 1), (-1, 0), (0, -1)]  # D2Q4 of Sec. III C, weights 1/4


def _find9(ez, er):
    return E9.index((ez, er))


def _find4(ez, er):
    return E4.index((ez, er))


def _case():
    # tau_s = 3/4 (paper tau = 1/4); a sliding, rotating lid at r = R = 3.5
    return W.base_case(3, 4, 0.75, swirl=True, a0=2.0 ** -10,
                       north=W.wall(omega=2.0 ** -5, uz=2.0 ** -6))


def _random_state(case, seed):
    """Dyadic populations near rest (exact in binary floating point)."""
    rng = np.random.default_rng(seed)
    nr, nz = case["nr"], case["nz"]
    f = np.empty((9, nr, nz))
    for a in range(9):
        f[a] = float(W9[a]) * (1.0 + rng.integers(-400, 401, size=(nr, nz)) / 2.0 ** 14)
    g = rng.integers(-300, 301, size=(4, nr, nz)) / 2.0 ** 16
    return f, g


def exact_step(case, tau, tau_g, f, g, slip=None):
    """One time step in rational arithmetic from the paper's equations.

    tau, tau_g: the paper's relaxation parameters exactly as the oracle holds
    them (binary fractions).  slip selects a deliberate mistake (tests of the
    test)."""
    nz, nr = case["nz"], case["nr"]
    rho0 = Fr(case["rho0"])
    a0 = Fr(case["a0"])
    lid = case["north"]
    uzw, urw, Om = Fr(lid["uz"]), Fr(lid["ur"]), Fr(lid["omega"])
    tau, tau_g = Fr(tau), Fr(tau_g)
    mu0 = rho0 * tau / 3                     # mu = tau rho cs^2 (Eq. 36), rho -> rho0
    nu_g = tau_g / 2                         # nu = tau_g c^2 / 2 (Sec. III C)
    F = [[[Fr(f[a, j, i]) for i in range(nz)] for j in range(nr)] for a in range(9)]
    G = [[[Fr(g[a, j, i]) for i in range(nz)] for j in range(nr)] for a in range(4)]

    def inv_r(j):
        return Fr(0) if j == 0 else Fr(1, j)

    def macros(fh, gh, j):
        """Eqs. (16)-(17) with G = (a, rho0 u_th^2 / r); u_th = sum g / rho0."""
        ir = inv_r(j)
        s0 = sum(fh)
        sz = sum(e[0] * x for e, x in zip(E9, fh))
        sr = sum(e[1] * x for e, x in zip(E9, fh))
        uth = Fr(0) if j == 0 else sum(gh) / rho0
        Gz, Gr = a0, rho0 * uth * uth * ir
        ur = (sr + Gr / 2) / (s0 + mu0 * ir * ir)
        rho = s0 / (1 + ur * ir / 2)
        uz = (sz + Gz / 2) / s0
        return rho, uz, ur, uth

    def geq(uth, uz, ur):
        """Eq. (54) with rho -> rho0."""
        return [rho0 * uth / 4 * (1 + 2 * (e[0] * uz + e[1] * ur)) for e in E4]

    fstar = [[[None] * nz for _ in range(nr)] for _ in range(9)]
    gstar = [[[None] * nz for _ in range(nr)] for _ in range(4)]
    for j in range(nr):
        ir = inv_r(j)
        for i in range(nz):
            fh = [F[a][j][i] for a in range(9)]
            gh = [G[a][j][i] for a in range(4)]
            if j == 0:
                # axis row: g becomes the non-equilibrium part of row 1 (same level)
                f1 = [F[a][1][i] for a in range(9)]
                g1 = [G[a][1][i] for a in range(4)]
                _, uz1, ur1, uth1 = macros(f1, g1, 1)
                gh = [x - y for x, y in zip(g1, geq(uth1, uz1, ur1))]
            rho, uz, ur, uth = macros(fh, gh, j)
            Fz = a0
            Fr_ = -2 * mu0 * ur * ir * ir + rho0 * uth * uth * ir
            usq = uz * uz + ur * ur
            for a, (ez, er) in enumerate(E9):
                eu = ez * uz + er * ur
                feq = W9[a] * rho * (1 + 3 * eu + Fr(9, 2) * eu * eu - Fr(3, 2) * usq)   # Eq. (6)
                mass = ur * ir if slip != "mass_sign" else -ur * ir
                S = (3 * ((ez - uz) * Fz + (er - ur) * Fr_) / rho - mass) * feq           # Eq. (12)
                if slip == "omega_flat":
                    om = 1 / (tau + Fr(1, 2))
                else:
                    om = (1 + tau * er * ir) / (tau + Fr(1, 2))                           # after Eq. (13)
                src = (1 - om / 2) * S if slip != "no_half" else S
                fstar[a][j][i] = fh[a] - om * (fh[a] - feq) + src                        # Eq. (13)
            ge = geq(uth, uz, ur)
            for a, (ez, er) in enumerate(E4):
                om = (1 + tau_g * er * ir) / (tau_g + Fr(1, 2))
                Sg = -ir * (2 * ur + nu_g * ir) * ge[a]                                   # Eq. (54)
                gstar[a][j][i] = gh[a] - om * (gh[a] - ge[a]) + Sg                        # Eq. (53)
    # pull streaming: periodic in z; axis mirror (f); halfway moving wall at r = nr - 1/2
    R = nr - Fr(1, 2)
    fn = np.empty((9, nr, nz))
    gn = np.empty((4, nr, nz))
    exact = {}
    for j in range(nr):
        for i in range(nz):
            for a, (ez, er) in enumerate(E9):
                iu, ju = (i - ez) % nz, j - er
                if ju < 0:
                    if slip == "axis_bounce":
                        v = fstar[_find9(-ez, -er)][j][i]
                    else:
                        v = fstar[_find9(ez, -er)][1][iu]   # ghost (iu, -1) mirrors (iu, 1)
                elif ju >= nr:
                    v = fstar[_find9(-ez, -er)][j][i] + 6 * W9[a] * rho0 * (ez * uzw + er * urw)
                else:
                    v = fstar[a][ju][iu]
                exact[("f", a, j, i)] = v
                fn[a, j, i] = float(v)
            for a, (ez, er) in enumerate(E4):
                iu, ju = (i - ez) % nz, j - er
                if ju < 0:
                    v = Fr(0)   # the axis row's g is rebuilt from row 1 before use
                elif ju >= nr:
                    v = -gstar[_find4(-ez, -er)][j][i] + rho0 * Om * R / 2
                else:
                    v = gstar[a][ju][iu]
                gn[a, j, i] = float(v)
    return fn, gn, exact


@pytest.mark.parametrize("seed", [0, 1])
def test_one_step_matches_exact_rational_evaluation(orc, seed):
    case = _case()
    f, g = _random_state(case, seed)
    o = orc.Oracle(case)
    o.set_state(f, g, None, 0)
    o.step(1)
    fo, go, _ = o.get_state()
    p = orc.params(case)
    fx, gx, _ = exact_step(case, p.tau, p.tau_g, f, g)
    ef, eg = np.abs(fo - fx).max(), np.abs(go - gx).max()
    print("max |oracle - exact|: f %.2e, g %.2e" % (ef, eg))
    assert ef <= 1e-15 and eg <= 1e-15
    # every population moved: the comparison is not trivially against the input
    assert np.abs(fx - f).max() > 1e-4


@pytest.mark.parametrize("slip", ["omega_flat", "no_half", "mass_sign", "axis_bounce"])
def test_exact_step_detects_plausible_slips(orc, slip):
    """The rational evaluation with one deliberate mistake misses the oracle
    by orders of magnitude more than rounding: the pin can tell."""
    case = _case()
    f, g = _random_state(case, 0)
    o = orc.Oracle(case)
    o.set_state(f, g, None, 0)
    o.step(1)
    fo, _, _ = o.get_state()
    p = orc.params(case)
    fx, _, _ = exact_step(case, p.tau, p.tau_g, f, g, slip=slip)
    assert np.abs(fo - fx).max() > 1e-9, slip


def _speed(m):
    return np.sqrt(m["uz"] * m["uz"] + m["ur"] * m["ur"])


@pytest.mark.parametrize("wet", [False, True])
def test_residual_is_the_change_of_speed_between_the_last_two_levels(orc, wet):
    case = W.cavity(12, 20, 400.0, wet=wet)
    fld = W.random_fields(case, 3)
    o = orc.Oracle(case)
    o.seed(fld["uz"], fld["ur"], fld["uth"], None, fld["rho"])
    assert o.residual() == -1.0   # no previous level yet
    o.step(5)
    m_prev2 = o.macros()
    o.step(1)
    m_prev = o.macros()
    o.step(1)
    m_now = o.macros()
    want = float(np.max(np.abs(_speed(m_now) - _speed(m_prev))))
    got = o.residual()
    print("residual %.6e (NumPy %.6e)" % (got, want))
    assert abs(got - want) <= 1e-15 * max(1.0, want)
    assert want > 1e-6
    # pairing with the level before the last one gives a different number
    wrong = float(np.max(np.abs(_speed(m_now) - _speed(m_prev2))))
    assert abs(wrong - want) > 1e-3 * want
    # comparing a level with itself would give zero
    assert got > 0.0


def test_residual_is_nan_when_the_state_holds_nan(orc):
    case = W.cavity(12, 20, 400.0)
    fld = W.random_fields(case, 4)
    fld["uz"][5, 7] = np.nan
    o = orc.Oracle(case)
    o.seed(fld["uz"], fld["ur"], fld["uth"], None, fld["rho"])
    o.step(2)
    assert np.isnan(o.residual())
    # a finite state of the same lattice gives a finite residual
    o2 = orc.Oracle(case)
    o2.seed(W.random_fields(case, 4)["uz"])
    o2.step(2)
    assert np.isfinite(o2.residual())

"""Pins of the oracle's MRT collision model (Sec. III B, Eqs. 37-51).

Each pin comes from outside the oracle's own formulas: the closed form of the
equilibrium moments (Eq. 39), the textbook velocity-space forcing term whose
moments Eq. (51) lists, exact invariances of the scheme (the conserved-moment
rates drop out; one common rate is the BGK model), the exactness of plane
Poiseuille flow under a two-relaxation-time collision with the "magic"
combination 3/16 and halfway walls, exact Stokes solutions that carry the
1/r terms of Eqs. (49)-(50) (an axisymmetric decay mode with radial velocity,
radial source flow between porous cylinders), Hagen-Poiseuille (Eq. 55) and
the stability claim of Fig. 7 (BGK diverges at tau = 0.005, MRT does not).

Directions of the lattice are (e_z, e_r); the MRT moments take x = r and
y = z as the paper does.
"""
import numpy as np
import pytest
from scipy.optimize import brentq
from scipy.special import iv, jv

from paper_1003_0282_amd import workloads as W

EZ = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], float)
ER = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], float)
WT = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def _mrt(case, **kw):
    c = dict(case)
    c["mrt"] = True
    c.update(kw)
    return c


def _seeded(case, steps, **seed):
    from oracle import oracle as O
    o = O.Oracle(case)
    o.seed(**seed)
    o.step(steps)
    return o, o.macros()


# ---- the moment basis (Eqs. 38-39) ---------------------------------------------

def test_basis_is_orthogonal_and_inverted(orc):
    M, Mi = orc.mrt_basis()
    G = M @ M.T
    assert np.abs(G - np.diag(np.diag(G))).max() == 0.0
    assert np.abs(M @ Mi - np.eye(9)).max() < 1e-15
    assert np.abs(Mi @ M - np.eye(9)).max() < 1e-15
    # the momentum rows are the velocity components (x = r, y = z)
    assert np.array_equal(M[3], ER) and np.array_equal(M[5], EZ) and np.array_equal(M[0], 1 + 0 * EZ)


def test_equilibrium_moments_are_eq39(orc):
    M, _ = orc.mrt_basis()
    rng = np.random.default_rng(3)
    for _ in range(20):
        rho, uz, ur = 1 + 0.1 * rng.standard_normal(), *(0.1 * rng.standard_normal(2))
        ux, uy = ur, uz
        u2 = ux * ux + uy * uy
        want = rho * np.array([1, -2 + 3 * u2, 1 - 3 * u2, ux, -ux, uy, -uy, ux * ux - uy * uy,
                               ux * uy])
        assert np.abs(M @ orc.feq9(rho, uz, ur) - want).max() < 1e-15


def _guo(uz, ur, Fz, Fr):
    """Velocity-space forcing w_a [3 (e_a - u).F + 9 (e_a.u)(e_a.F)]."""
    eu = EZ * uz + ER * ur
    eF = EZ * Fz + ER * Fr
    return WT * (3 * ((EZ - uz) * Fz + (ER - ur) * Fr) + 9 * eu * eF)


def test_force_moments_of_eq51_are_the_velocity_space_forcing(orc):
    """Eq. (51) is M applied to the standard second-order forcing term; the
    mass part of S~ is -(u_r / r) m_eq, whose zeroth moment is the continuity
    source -rho u_r / r of Eq. (1)."""
    M, _ = orc.mrt_basis()
    rng = np.random.default_rng(5)
    for cart, j in ((True, 3), (False, 3), (False, 0)):
        case = _mrt(W.base_case(4, 8, 0.8, a0=2e-5, cartesian=cart, swirl=True))
        mu0 = (case["tau"] - 0.5) / 3
        for _ in range(5):
            rho = 1 + 0.05 * rng.standard_normal()
            uz, ur, uth = 0.05 * rng.standard_normal(3)
            if j == 0:
                ur = uth = 0.0
            m = np.array([rho, uz, ur, uth, 0.0])
            meq = M @ orc.feq9(rho, uz, ur)
            St = orc.mrt_source_moments(case, j, 0, m, meq)
            ir = 0.0 if (cart or j == 0) else 1.0 / j
            Fz, Fr = 2e-5, -2 * mu0 * ur * ir * ir + uth * uth * ir
            want = M @ _guo(uz, ur, Fz, Fr) - ur * ir * meq
            assert np.abs(St - want).max() < 1e-16
            assert abs(St[0] + rho * ur * ir) < 1e-17


def test_velocity_space_source_keeps_eqs_16_17(orc):
    """Seeding f-bar = f_eq - S/2 with the MRT source returns the seeded
    fields through Eqs. (16)-(17): sum S = -rho u_r / r and sum e_i S =
    F_i - rho u_i u_r / r hold for the MRT source as for Eq. (12)."""
    from oracle import oracle as O
    case = _mrt(W.base_case(12, 10, 0.7, swirl=True, a0=1e-5, west=W.wall(), east=W.wall()))
    fld = W.random_fields(case, seed=11)
    o = O.Oracle(case)
    o.seed(**fld)
    m = o.macros()
    for k in ("rho", "uz", "ur", "uth"):
        want = fld[k].copy()
        if k in ("ur", "uth"):
            want[0] = 0.0
        assert np.abs(m[k] - want).max() < 1e-15, k


# ---- exact invariances -------------------------------------------------------------

def test_conserved_moment_rates_drop_out(orc):
    """With f-bar = f - S/2 the conserved moments leave the collision as
    m-bar + S~ whatever s_rho and s_j are."""
    rng = np.random.default_rng(7)
    case = _mrt(W.base_case(4, 6, 0.7, swirl=True, a0=1e-5))
    f = orc.feq9(1.0, 0.03, 0.02) + 1e-3 * rng.standard_normal(9)
    g = 0.01 * rng.standard_normal(4)
    outs = [orc.node_collide(dict(case, s_rho=a, s_j=b), 3, 5, f, g)[0]
            for a, b in ((1.0, 1.0), (0.3, 1.7), (1.9, 0.2))]
    for o in outs[1:]:
        assert np.abs(o - outs[0]).max() < 1e-15


def test_single_rate_planar_mrt_is_bgk(orc):
    """All rates equal to 1/(tau + 1/2), every 1/r term off and no force: the
    MRT collision is the BGK collision (Eq. 13 with omega = omega0)."""
    from oracle import oracle as O
    tau = 0.9
    sv = 1 / (tau - 0.5 + 0.5)
    base = W.base_case(10, 8, tau, cartesian=True, south=W.wall(), north=W.wall(),
                       west=W.wall(), east=W.wall(uz=0.0, ur=0.05))
    base["north"] = W.wall(uz=0.04)
    fld = W.random_fields(base, seed=2)
    fld.pop("uth", None)
    fld.pop("T", None)
    res = []
    for c in (base, _mrt(base, s_e=sv, s_eps=sv, s_q=sv)):
        o = O.Oracle(c)
        o.seed(**fld)
        o.step(40)
        res.append(o.get_state()[0])
    assert np.abs(res[1] - res[0]).max() < 1e-14


# ---- closed-form flows -----------------------------------------------------------

def test_plane_poiseuille_is_exact_with_magic_rates(orc):
    """Planar channel under a body force: with s_e = s_eps = s_v and
    (1/s_v - 1/2)(1/s_q - 1/2) = 3/16 halfway walls sit exactly half a
    spacing out, so the steady profile a/(2 mu) y (H - y) is reproduced to
    rounding for any tau (BGK leaves a tau-dependent slip)."""
    for tau in (0.55, 1.5):
        nr, mu = 8, (tau - 0.5) / 3
        case = _mrt(W.base_case(2, nr, tau, cartesian=True, south=W.wall(), a0=1e-6))
        y = np.arange(nr) + 0.5
        ua = 1e-6 / (2 * mu) * y * (nr - y)
        o, m = _seeded(case, int(60 * nr * nr / mu / 9.8), uz=np.tile(ua[:, None], (1, 2)))
        assert np.abs(m["uz"][:, 0] - ua).max() / ua.max() < 1e-10
        assert np.abs(m["ur"]).max() < 1e-12  # rounding of the moment transform


def test_mrt_hagen_poiseuille(orc):
    """Eq. (55): u_z = U0 (1 - r^2 / R^2), U0 = a R^2 / (4 mu), halfway and
    wet-node walls."""
    for wet in (False, True):
        case = _mrt(W.hagen_poiseuille(), wet=wet)
        R = case["nr"] - (1.0 if wet else 0.5)
        U0 = case["a0"] * R * R / (4 * (case["tau"] - 0.5) / 3)
        r = np.arange(case["nr"])
        ua = U0 * (1 - r ** 2 / R ** 2)
        o, m = _seeded(case, 20000)
        err = m["uz"][:, 0] - ua
        assert np.sqrt(np.mean(err ** 2)) / U0 < 1.5e-3
        assert np.abs(err).max() / U0 < 3e-3
        assert 0 <= o.residual() < 1e-10


def _stokes_mode(nz, nr):
    """Unsteady Stokes mode of a no-slip pipe of radius R, periodic in z:
    psi = r [J1(l r) + B I1(k r)] sin(k z) with u_r = -(1/r) d_z psi, u_z =
    (1/r) d_r psi, both vanishing at R (k J1(lR) I0(kR) = l J0(lR) I1(kR));
    it decays as exp(-nu (l^2 + k^2) t)."""
    R, k = nr - 0.5, 2 * np.pi / nz
    fn = lambda l: k * jv(1, l * R) * iv(0, k * R) - l * jv(0, l * R) * iv(1, k * R)
    ls = np.linspace(0.5 / R, 8 / R, 2000)
    v = fn(ls)
    i = np.where(np.sign(v[:-1]) != np.sign(v[1:]))[0][0]
    lam = brentq(fn, ls[i], ls[i + 1])
    B = -jv(1, lam * R) / iv(1, k * R)
    r = np.arange(nr)[:, None]
    z = np.arange(nz)[None, :]
    ur = -k * (jv(1, lam * r) + B * iv(1, k * r)) * np.cos(k * z)
    uz = (lam * jv(0, lam * r) + B * k * iv(0, k * r)) * np.sin(k * z)
    s = 1e-4 / np.abs(uz).max()
    return lam * lam + k * k, uz * s, ur * s


@pytest.mark.parametrize("mrt,bound", [(True, 1.5e-3), (False, 2e-3)])
def test_stokes_mode_with_radial_velocity_decays_at_exact_rate(orc, mrt, bound):
    """The decay rate of a mode with both u_r and u_z tests the 1/r viscous
    terms of the radial and axial momentum equations (Eqs. 49-50 for MRT,
    the direction-dependent rates of Eq. 13 for BGK)."""
    from oracle import oracle as O
    nz, nr, tau = 40, 20, 0.8
    k2, uz, ur = _stokes_mode(nz, nr)
    sig = (tau - 0.5) / 3 * k2
    o = O.Oracle(W.base_case(nz, nr, tau, north=W.wall(), mrt=mrt))
    o.seed(uz=uz, ur=ur)
    r = np.arange(nr)[:, None]
    T = int(1.0 / sig)
    ts, amps = [], []
    for _ in range(10):
        o.step(T // 10)
        m = o.macros()
        amps.append((np.sum(m["uz"] * uz * r) + np.sum(m["ur"] * ur * r))
                    / (np.sum(uz * uz * r) + np.sum(ur * ur * r)))
        ts.append(o.t)
    rate = -np.polyfit(ts[2:], np.log(amps[2:]), 1)[0]
    assert abs(rate / sig - 1) < bound, rate / sig - 1


@pytest.mark.parametrize("mrt", [True, False])
def test_radial_source_flow_between_porous_cylinders(orc, mrt):
    """Fluid injected through the inner cylinder and drawn off at the outer
    one: u_r = Q / r, for which the axisymmetric viscous force
    mu (lap u_r + (1/r) d_r u_r - u_r / r^2) vanishes, so p + rho u^2 / 2 is
    constant across the gap.  Leaving out the (1/r) d_r u_r term of Eq. (49)
    would add a viscous pressure drop of about 2 mu Q / r^2, roughly twice the
    dynamic pressure here."""
    Q, r0, nr, tau = 0.1, 4.0, 16, 0.8
    rin, rout = r0 - 0.5, r0 + nr - 0.5
    case = W.base_case(2, nr, tau, r0=r0, south=W.wall(ur=Q / rin), north=W.wall(ur=Q / rout),
                       mrt=mrt)
    o, m = _seeded(case, 20000)
    r = r0 + np.arange(nr)
    ur, rho = m["ur"][:, 0], m["rho"][:, 0]
    assert np.abs(r * rho * ur / Q - 1).max() < 0.03
    B = rho / 3 + 0.5 * ur ** 2
    dyn = 0.5 * (Q / r[0]) ** 2
    assert (B.max() - B.min()) / dyn < 0.4
    assert o.residual() < 1e-6


def test_mrt_solid_body_rotation_centrifugal_pressure(orc):
    """The centrifugal force rho0 u_th^2 / r enters F_x of Eq. (51):
    rho(r) - rho(0) = 1.5 rho0 Omega^2 r^2 with u_th = Omega r."""
    nr = 32
    Om = 1e-2 / nr
    case = _mrt(W.base_case(2, nr, 0.8, north=W.wall(omega=Om), swirl=True))
    r = np.arange(nr)
    _, m = _seeded(case, int(30 * nr * nr / 0.1 / 5.8), uth=np.tile((Om * r)[:, None], (1, 2)))
    rho = m["rho"][:, 0]
    dp = 1.5 * Om ** 2 * r ** 2
    assert np.abs((rho - rho[0]) - dp).max() / dp.max() < 3e-3
    assert np.abs(m["ur"]).max() < 1e-12


def test_mrt_womersley(orc):
    """Eq. (56) with the time-periodic force of the paper's run (T = 1200)."""
    from oracle import oracle as O
    case = _mrt(W.womersley_paper(nz=2))
    T = int(case["period"])
    R = W.pipe_radius(case)
    nu = (case["tau"] - 0.5) / 3.0
    w = 2 * np.pi / T
    alpha = R * np.sqrt(w / nu)
    phi = (-alpha + 1j * alpha) / np.sqrt(2)
    r = np.arange(case["nr"])
    o = O.Oracle(case)
    o.seed()
    o.step(9 * T)
    xs = []
    for _ in range(16):
        m = o.macros()
        ua = np.real(case["a0"] / (1j * w) * (1 - jv(0, r * phi / R) / jv(0, phi))
                     * np.exp(1j * w * o.t))
        xs.append(np.sum(np.abs(m["uz"][:, 0] - ua)) / np.sum(np.abs(ua)))
        o.step(T // 16)
    assert np.mean(xs) < 6.5e-3, np.mean(xs)


# ---- Fig. 7: stability at tau = 0.005 --------------------------------------------

def test_bgk_diverges_and_mrt_holds_at_tau_0005(orc):
    """Rotating-lid cylinder at nu = 0.005 / 3 (tau_s = 0.505, the paper's
    Fig. 7 viscosity) on a 30 x 20 grid with the lid speed of the paper's
    run: BGK turns NaN within a few thousand steps, MRT stays bounded."""
    from oracle import oracle as O
    nr, nz = 20, 30
    nu = 0.005 / 3
    R = nr - 0.5
    Om = 258.0 * nu / R ** 2
    out = {}
    for mrt in (False, True):
        case = W.base_case(nz, nr, 0.505, swirl=True, north=W.wall(), west=W.wall(),
                           east=W.wall(omega=Om), mrt=mrt)
        o = O.Oracle(case)
        o.seed()
        for _ in range(8):
            o.step(500)
            res = o.residual()
            if not np.isfinite(res):
                break
        out[mrt] = (res, o.macros())
    assert not np.isfinite(out[False][0])
    res, m = out[True]
    assert np.isfinite(res) and res < 1e-3
    assert np.abs(m["uz"]).max() < Om * R and np.abs(m["uth"]).max() <= 1.01 * Om * R


def test_bulk_rate_must_match_shear_rate(orc):
    """The paper's closing remark on the MRT scheme: axisymmetric flow has a
    nonzero pseudo-divergence (d_r u_r + d_z u_z = -u_r / r), so the bulk
    rate s_e must equal s_v.  In radial source flow, where that divergence
    is everywhere nonzero, p + rho u^2 / 2 stays constant with s_e = s_v and
    is off by several times more when s_e departs from it."""
    Q, r0, nr, tau = 0.1, 4.0, 16, 0.8
    sv = 1.0 / tau
    dev = {}
    for se in (sv, 1.0, 0.6):
        case = _mrt(W.base_case(2, nr, tau, r0=r0, south=W.wall(ur=Q / (r0 - 0.5)),
                                north=W.wall(ur=Q / (r0 + nr - 0.5))), s_e=se)
        _, m = _seeded(case, 20000)
        r = r0 + np.arange(nr)
        B = m["rho"][:, 0] / 3 + 0.5 * m["ur"][:, 0] ** 2
        dev[se] = (B.max() - B.min()) / (0.5 * (Q / r[0]) ** 2)
    assert dev[sv] < 0.4
    assert dev[1.0] > 3 * dev[sv] and dev[0.6] > 3 * dev[1.0], dev

"""Pins of the CPU oracle against exact identities the paper fixes.

Each test checks the oracle against a property that holds for any input
(moment identities of Eq. 30, the macro definitions Eqs. 14-15, the source
moments implied by Eq. 12, the collision's mass identity, permutation and
symmetry properties of streaming), so a dropped term, a wrong sign or a wrong
index in the oracle fails here.  The velocity sets below are the textbook D2Q9
and D2Q4 sets in the direction order the oracle documents.
"""
import itertools

import numpy as np
import pytest

from paper_1003_0282_amd import workloads as W

# D2Q9 in the documented order, components (e_z, e_r); D2Q4 likewise.
E9 = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)],
              dtype=float)
E4 = np.array([(1, 0), (0, 1), (-1, 0), (0, -1)], dtype=float)
CS2 = 1.0 / 3.0


def _case(**kw):
    c = W.base_case(8, 8, kw.pop("tau", 0.8), **kw)
    return c


def test_feq_moments_eq30(orc):
    """Eq. (30): zeroth to third moments of the D2Q9 equilibrium."""
    rng = np.random.default_rng(1)
    for _ in range(50):
        rho = rng.uniform(0.8, 1.2)
        u = rng.uniform(-0.1, 0.1, size=2)
        f = orc.feq9(rho, u[0], u[1])
        assert abs(f.sum() - rho) < 1e-15
        assert np.allclose(E9.T @ f, rho * u, atol=1e-16, rtol=0)
        Pi = np.einsum("a,ai,aj->ij", f, E9, E9)
        assert np.allclose(Pi, rho * np.outer(u, u) + rho * CS2 * np.eye(2), atol=1e-15, rtol=0)
        P3 = np.einsum("a,ai,aj,ak->ijk", f, E9, E9, E9)
        d = np.eye(2)
        exp = rho * CS2 * (np.einsum("i,jk->ijk", u, d) + np.einsum("j,ik->ijk", u, d)
                           + np.einsum("k,ij->ijk", u, d))
        assert np.allclose(P3, exp, atol=1e-16, rtol=0)


def test_feq_weights_at_rest(orc):
    f = orc.feq9(1.0, 0.0, 0.0)
    assert np.allclose(f, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, atol=0, rtol=1e-15)


def test_geq_heq_moments(orc):
    """Eq. (54): sum g_eq = rho0 u_th, sum e g_eq = rho0 u_th u,
    sum e e g_eq = rho0 u_th c^2/2 I (D2Q4, cs^2 = 1/2); same for h with T."""
    rng = np.random.default_rng(2)
    for _ in range(30):
        rho0, uth, T = rng.uniform(0.9, 1.1), rng.uniform(-0.1, 0.1), rng.uniform(0, 1)
        u = rng.uniform(-0.1, 0.1, size=2)
        g = orc.geq4(rho0, uth, u[0], u[1])
        assert abs(g.sum() - rho0 * uth) < 1e-16
        assert np.allclose(E4.T @ g, rho0 * uth * u, atol=1e-17, rtol=0)
        assert np.allclose(np.einsum("a,ai,aj->ij", g, E4, E4), 0.5 * rho0 * uth * np.eye(2),
                           atol=1e-16, rtol=0)
        h = orc.heq4(T, u[0], u[1])
        assert abs(h.sum() - T) < 1e-15
        assert np.allclose(E4.T @ h, T * u, atol=1e-16, rtol=0)


def _random_pops(rng, rho0=1.0, amp=0.05):
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    f = w * rho0 * (1.0 + amp * rng.uniform(-1, 1, size=9))
    g = 0.01 * rng.uniform(-1, 1, size=4)
    h = 0.25 + 0.05 * rng.uniform(-1, 1, size=4)
    return f, g, h


def _force(case, j, t, m):
    """F = (a(t) + rho0 g beta (T - T_ref), rho0 u_th^2/r - 2 mu0 u_r / r^2)."""
    tau = case["tau"] - 0.5
    mu0 = case["rho0"] * tau / 3.0
    r = case["r0"] + j
    ir = 0.0 if (r <= 0 or case.get("cartesian")) else 1.0 / r
    a = case["a0"] * (np.cos(2 * np.pi * t / case["period"] + case["phase"])
                      if case["period"] > 0 else 1.0)
    Fz = a + (case["rho0"] * case["gbeta"] * (m[4] - case["T_ref"]) if case["thermal"] else 0.0)
    Fr = -2 * mu0 * m[2] * ir * ir + (case["rho0"] * m[3] ** 2 * ir if case["swirl"] else 0.0)
    return np.array([Fz, Fr]), ir


CASES = [
    dict(),
    dict(a0=3e-4),
    dict(a0=2e-4, period=100.0, phase=0.3),
    dict(swirl=True, a0=1e-4),
    dict(swirl=True, thermal=True, tau_h=0.9, gbeta=1e-3, T_ref=0.25, a0=-1e-4),
    dict(r0=4.0, south=W.wall(), swirl=True),
]


@pytest.mark.parametrize("kw", CASES)
@pytest.mark.parametrize("j", [0, 1, 5])
def test_macros_satisfy_eq14_eq15(orc, kw, j):
    """Eqs. (16)-(17) (explicit) must solve Eqs. (14)-(15) (implicit)."""
    case = _case(**kw)
    rng = np.random.default_rng(10 + j)
    for t in (0, 7, 33):
        f, g, h = _random_pops(rng)
        if case["south"]["kind"] == "axis" and j == 0:
            g = np.zeros(4)  # the axis value of g is substituted; u_th = 0 there
        m = orc.node_macros(case, j, t, f, g, h)
        rho, u = m[0], m[1:3]
        F, ir = _force(case, j, t, m)
        assert abs(rho - (f.sum() - 0.5 * rho * u[1] * ir)) < 1e-15          # Eq. (14)
        rhs = E9.T @ f + 0.5 * (F - rho * u * u[1] * ir)                      # Eq. (15)
        assert np.allclose(rho * u, rhs, atol=1e-16, rtol=0)
        if case["swirl"] and not (j == 0 and case["south"]["kind"] == "axis"):
            assert abs(m[3] - g.sum() / case["rho0"]) < 1e-16               # u_th = sum g / rho0
        if case["thermal"]:
            assert abs(m[4] - h.sum()) < 1e-16


@pytest.mark.parametrize("kw", CASES)
@pytest.mark.parametrize("j", [0, 1, 3])
def test_source_moments_eq12(orc, kw, j):
    """From Eq. (12): sum S = -rho u_r / r and sum e_i S = F_i - rho u_i u_r / r."""
    case = _case(**kw)
    rng = np.random.default_rng(20 + j)
    for t in (0, 5):
        f, g, h = _random_pops(rng)
        m = orc.node_macros(case, j, t, f, g, h)
        feq = orc.feq9(m[0], m[1], m[2])
        S = orc.node_source(case, j, t, m, feq)
        F, ir = _force(case, j, t, m)
        rho, u = m[0], m[1:3]
        assert abs(S.sum() + rho * u[1] * ir) < 1e-17
        assert np.allclose(E9.T @ S, F - rho * u * u[1] * ir, atol=1e-17, rtol=0)


@pytest.mark.parametrize("kw", CASES)
@pytest.mark.parametrize("j", [0, 1, 2, 6])
def test_collision_mass_identity(orc, kw, j):
    """Eq. (13) with Eqs. (12), (14), (15): for any f^,
    sum f* - sum f^ = -rho u_r / r (exact; zero on the axis)."""
    case = _case(**kw)
    rng = np.random.default_rng(30 + j)
    for t in (0, 3):
        f, g, h = _random_pops(rng)
        fo, go, ho, m = orc.node_collide(case, j, t, f, g, h)
        _, ir = _force(case, j, t, m)
        assert abs((fo.sum() - f.sum()) + m[0] * m[2] * ir) < 1e-15


@pytest.mark.parametrize("tau", [0.55, 0.8, 1.3])
def test_collision_momentum_cartesian(orc, tau):
    """Planar special case (all 1/r terms off): the scheme is the textbook
    forced BGK update, whose momentum gain per step equals the force."""
    case = W.base_case(8, 8, tau, cartesian=True, a0=2e-4)
    rng = np.random.default_rng(3)
    for j in (0, 3):
        f, g, h = _random_pops(rng)
        fo, _, _, m = orc.node_collide(case, j, 0, f, g, h)
        assert abs(fo.sum() - f.sum()) < 1e-15
        assert np.allclose(E9.T @ fo - E9.T @ f, [2e-4, 0.0], atol=2e-16, rtol=0)


def test_rest_state_is_fixed_point(orc):
    """Uniform rest state with no force stays exactly at rest."""
    from oracle import oracle as O
    for kw in (dict(), dict(swirl=True), dict(swirl=True, thermal=True, tau_h=0.8, T_ref=0.3)):
        case = W.base_case(6, 7, 0.7, west=W.wall(), east=W.wall(), **kw)
        o = O.Oracle(case)
        o.seed()
        f0, g0, h0 = o.get_state()
        o.step(25)
        f1, g1, h1 = o.get_state()
        assert np.abs(f1 - f0).max() < 1e-15
        m = o.macros()
        assert np.abs(m["uz"]).max() < 1e-16 and np.abs(m["ur"]).max() < 1e-16
        assert np.abs(m["rho"] - 1.0).max() < 1e-15


def test_seed_roundtrip(orc):
    """Seeding f^ = f_eq - S/2 makes Eqs. (16)-(17) return the seeded fields."""
    from oracle import oracle as O
    case = W.base_case(9, 7, 0.7, a0=1e-4, swirl=True, thermal=True, tau_h=0.9, gbeta=1e-3,
                       T_ref=0.5)
    fl = W.random_fields(case, 5)
    o = O.Oracle(case)
    ur = fl["ur"].copy(); ur[0] = 0
    uth = fl["uth"].copy(); uth[0] = 0
    for rho in (None, fl["rho"]):
        o.seed(fl["uz"], fl["ur"], fl["uth"], fl["T"], rho)
        m = o.macros()
        assert np.abs(m["uz"] - fl["uz"]).max() < 1e-15
        assert np.abs(m["ur"] - ur).max() < 1e-15
        assert np.abs(m["uth"] - uth).max() < 1e-15
        assert np.abs(m["T"] - fl["T"]).max() < 1e-15
        assert np.abs(m["rho"] - (1.0 if rho is None else rho)).max() < 2e-15
        # summing Eq. (12): sum S = -rho u_r / r, so sum f^ = rho (1 + u_r / 2r)
        f, _, _ = o.get_state()
        r = np.arange(case["nr"], dtype=float)[:, None]
        ir = np.where(r > 0, 1.0 / np.maximum(r, 1), 0.0)
        want = m["rho"] * (1.0 + 0.5 * ur * ir)
        assert np.abs(f.sum(0) - want).max() < 2e-15


def test_streaming_is_permutation_periodic_walls(orc):
    """With periodic ends and bounce-back walls, streaming permutes the slots:
    the multiset of population values is unchanged."""
    from oracle import oracle as O
    case = W.base_case(7, 5, 0.8, r0=3.0, south=W.wall(), north=W.wall(), swirl=True,
                       thermal=True, tau_h=0.8)
    o = O.Oracle(case)
    rng = np.random.default_rng(6)
    fs = rng.uniform(size=(9, 5, 7))
    gs = rng.uniform(size=(4, 5, 7))
    hs = rng.uniform(size=(4, 5, 7))
    o.stream_only(fs, gs, hs)
    f, g, h = o.get_state()
    assert np.array_equal(np.sort(f.ravel()), np.sort(fs.ravel()))
    # g and h bounce back with a sign change on Dirichlet walls (zero wall values
    # here): compare magnitudes
    assert np.allclose(np.sort(np.abs(g.ravel())), np.sort(np.abs(gs.ravel())))
    assert np.array_equal(np.sort(h.ravel()), np.sort(hs.ravel()))


def test_streaming_interior_shift(orc):
    """Interior populations move by exactly e_a per step."""
    from oracle import oracle as O
    case = W.base_case(9, 8, 0.8, r0=2.0, south=W.wall(), north=W.wall())
    o = O.Oracle(case)
    rng = np.random.default_rng(7)
    fs = rng.uniform(size=(9, 8, 9))
    o.stream_only(fs)
    f, _, _ = o.get_state()
    for a in range(9):
        ez, er = int(E9[a, 0]), int(E9[a, 1])
        for j in range(1, 7):
            for i in range(9):
                assert f[a, j, i] == fs[a, j - er, (i - ez) % 9]


def test_axis_specular_symmetry(orc):
    """Specular reflection on the axis: for any post-collision input, the
    populations arriving on the axis row come in mirror pairs, so the radial
    momentum on the axis is exactly zero."""
    from oracle import oracle as O
    case = W.base_case(6, 5, 0.8, thermal=True, tau_h=0.8)
    o = O.Oracle(case)
    rng = np.random.default_rng(8)
    o.stream_only(rng.uniform(size=(9, 5, 6)), None, rng.uniform(size=(4, 5, 6)))
    f, _, h = o.get_state()
    pairs = [(a, b) for a, b in itertools.product(range(9), range(9))
             if E9[a, 0] == E9[b, 0] and E9[a, 1] == -E9[b, 1] and E9[a, 1] > 0]
    assert len(pairs) == 3
    for a, b in pairs:
        assert np.array_equal(f[a, 0], f[b, 0])
    assert np.array_equal(h[1, 0], h[3, 0])


def test_axis_symmetry_corner_with_walls(orc):
    """Mirror pairs on the axis survive bounce-back ends when the input is
    itself mirror-symmetric on the axis row (the state a run produces)."""
    from oracle import oracle as O
    case = W.cavity(6, 9, 500.0)
    o = O.Oracle(case)
    rng = np.random.default_rng(9)
    fs = rng.uniform(size=(9, 6, 9))
    # make row 0 mirror-symmetric as a collided axis row is
    for a, b in ((2, 4), (5, 8), (6, 7)):
        fs[b, 0] = fs[a, 0]
    o.stream_only(fs, rng.uniform(size=(4, 6, 9)))
    f, _, _ = o.get_state()
    for a, b in ((2, 4), (5, 8), (6, 7)):
        assert np.array_equal(f[a, 0], f[b, 0])


def test_cartesian_mass_conservation(orc):
    """Planar mode with periodic ends and bounce-back walls: total mass is
    conserved to roundoff over many steps (textbook D2Q9)."""
    from oracle import oracle as O
    case = W.base_case(12, 10, 0.7, cartesian=True, r0=0.0, south=W.wall(), north=W.wall(),
                       a0=1e-4)
    o = O.Oracle(case)
    fl = W.random_fields(case, 11)
    o.seed(fl["uz"], fl["ur"])
    f0, _, _ = o.get_state()
    o.step(300)
    f1, _, _ = o.get_state()
    assert abs(f1.sum() - f0.sum()) < 1e-11


def test_axisymmetric_mass_drift_small(orc):
    """Axisymmetric mode: the physical mass sum_j r_j sum_i rho is conserved
    only up to truncation error; the drift stays small."""
    from oracle import oracle as O
    case = W.cavity(12, 16, 60.0)
    o = O.Oracle(case)
    o.seed()
    r = np.arange(12, dtype=float)
    V = r.copy(); V[0] = 1.0 / 8.0
    M0 = (V[:, None] * o.macros()["rho"]).sum()
    o.step(2000)
    M1 = (V[:, None] * o.macros()["rho"]).sum()
    assert abs(M1 - M0) / M0 < 1e-3


def test_force_phase(orc):
    case = W.womersley(4, 8)
    assert orc.force_a(case, 0) == pytest.approx(1e-4, rel=1e-15)
    assert orc.force_a(case, 1000) == pytest.approx(0.0, abs=1e-18)
    assert orc.force_a(case, 2000) == pytest.approx(-1e-4, rel=1e-15)

"""Seeded synthetic workloads shaped like the paper's test problems.

This module only describes problems: grid sizes, relaxation times, forcing,
boundary kinds and seeded parameter draws.  It holds none of the lattice
Boltzmann arithmetic, so both the GPU path and the CPU oracle may take their
inputs from it.

A *case* is a plain dict:
    nz, nr, r0           grid (node i along z, j along r, r_j = r0 + j)
    swirl, thermal       optional D2Q4 fields (azimuthal velocity, temperature)
    cartesian            planar test mode (every 1/r term off)
    tau                  BGK relaxation time tau_s (the paper's tau + 1/2)
    tau_g, tau_h         tau_s of the g and h fields (0 -> default)
    rho0, a0, period, phase, gbeta, T_ref
    south, north, west, east   side dicts (kind: axis | wall | periodic | freeslip)

Geometry convention: walls sit half a spacing outside the outermost node, so
a pipe with the axis on row 0 and nr rows has radius R = nr - 1/2, and a
cavity with nz columns has height H = nz.
"""
from __future__ import annotations

import math

import numpy as np


# ---- boundary sides -------------------------------------------------------

def axis() -> dict:
    return {"kind": "axis"}


def periodic() -> dict:
    return {"kind": "periodic"}


def wall(omega: float = 0.0, uz: float = 0.0, ur: float = 0.0, thermal: int = 0,
         T: float = 0.0) -> dict:
    return {"kind": "wall", "omega": omega, "uz": uz, "ur": ur, "thermal": thermal, "T": T}


def freeslip() -> dict:
    return {"kind": "freeslip"}


def split_wall(inner: dict, outer: dict, r_split: float) -> dict:
    """z-end made of two segments: `inner` for r <= r_split, `outer` beyond."""
    d = dict(inner)
    d["r_split"] = float(r_split)
    d["kind2"] = outer["kind"]
    d["omega2"] = outer.get("omega", 0.0)
    d["thermal2"] = outer.get("thermal", 0)
    d["T2"] = outer.get("T", 0.0)
    return d


def base_case(nz: int, nr: int, tau: float, **kw) -> dict:
    c = {"nz": int(nz), "nr": int(nr), "r0": 0.0, "swirl": False, "thermal": False,
         "cartesian": False, "tau": float(tau), "tau_g": 0.0, "tau_h": 0.0,
         "rho0": 1.0, "a0": 0.0, "period": 0.0, "phase": 0.0, "gbeta": 0.0,
         "T_ref": 0.0, "south": axis(), "north": wall(), "west": periodic(),
         "east": periodic()}
    c.update(kw)
    return c


def pipe_radius(case: dict) -> float:
    return case["r0"] + case["nr"] - 0.5


# ---- the paper's validation problems ---------------------------------------

def hagen_poiseuille(nz: int = 4, nr: int = 32, a: float = 1e-6, tau: float = 0.8) -> dict:
    """Body-force-driven pipe flow (Sec. IV A, Eq. 55); default = 4 x 32, tau 0.8."""
    return base_case(nz, nr, tau, a0=a, name="hagen_poiseuille_%dx%d" % (nz, nr))


def hagen_poiseuille_paper() -> dict:
    """The paper's own H-P run: 40 x 20, mu = 0.2, a = 1e-4 (Sec. IV A)."""
    mu = 0.2
    return base_case(40, 20, 3.0 * mu + 0.5, a0=1e-4, name="hagen_poiseuille_paper")


def womersley(nz: int = 64, nr: int = 128, tau: float = 0.6, period: float = 4000.0,
              a0: float = 1e-4) -> dict:
    """Pulsatile pipe flow driven by a0 cos(2 pi t / T) (Sec. IV A, Eq. 56)."""
    return base_case(nz, nr, tau, a0=a0, period=period, name="womersley_%dx%d" % (nz, nr))


def womersley_paper(nz: int = 40) -> dict:
    """The paper's Womersley run: R ~ 20, T = 1200, a0 = 1e-3/3, mu = 0.1/3."""
    return base_case(nz, 20, 3.0 * (0.1 / 3.0) + 0.5, a0=1e-3 / 3.0, period=1200.0,
                     name="womersley_paper")


def cavity(nr: int, nz: int, Re: float, U_t: float = 0.1, wet: bool = False) -> dict:
    """Closed cylinder with a rotating top lid (Sec. IV B): Re = Omega R^2 / nu,
    lid speed U_t = Omega R, nu = U_t R / Re, tau_s = 3 nu + 1/2.  R = nr - 1/2
    with halfway walls, nr - 1 with wet-node walls."""
    R = nr - (1.0 if wet else 0.5)
    nu = U_t * R / Re
    omega = U_t / R
    return base_case(nz, nr, 3.0 * nu + 0.5, swirl=True, south=axis(), north=wall(),
                     west=wall(), east=wall(omega=omega), wet=bool(wet),
                     name="cavity_%dx%d_Re%g%s" % (nz, nr, Re, "_wet" if wet else ""),
                     Re=float(Re))


def cavity_paper(Re: float = 990.0, nr: int = 100, nz: int = 150, wet: bool = False) -> dict:
    """The paper's lid-driven run (Sec. IV B, Table 2): 100 x 150 (A = 1.5),
    tau = 0.02 (paper convention, nu = tau/3), Omega = Re nu / R^2."""
    nu = 0.02 / 3.0
    R = nr - (1.0 if wet else 0.5)
    omega = Re * nu / (R * R)
    return base_case(nz, nr, 0.52, swirl=True, south=axis(), north=wall(), west=wall(),
                     east=wall(omega=omega), wet=bool(wet),
                     name="cavity_paper_Re%g%s" % (Re, "_wet" if wet else ""), Re=float(Re))


def batch_cavities(n: int = 256, seed: int = 0, nr_lo: int = 64, nr_hi: int = 512,
                   A_lo: float = 1.0, A_hi: float = 3.0, Re_lo: float = 500.0,
                   Re_hi: float = 2500.0, U_t: float = 0.1,
                   tau_min: float = 0.52) -> list[dict]:
    """Uneven rotating-lid cavities: Nr ~ U{nr_lo..nr_hi}, H/R ~ U[A_lo, A_hi],
    Re ~ U[Re_lo, Re_hi], all from one seeded generator.

    The lid speed is U_t unless that would put tau_s = 3 nu + 1/2 below
    tau_min; then nu is held at (tau_min - 1/2)/3 and the lid runs at
    Re nu / R instead.  tau_min = 0.52 is the relaxation time of the paper's
    cavity runs (Sec. IV B, which also raise the lid speed with Re).  Coarse
    lattices at high Re with tau_s near 0.51 are not stable under BGK: the
    corner where the lid meets the still side wall blows up within a few
    thousand steps."""
    rng = np.random.default_rng(seed)
    nrs = rng.integers(nr_lo, nr_hi + 1, size=n)
    As = rng.uniform(A_lo, A_hi, size=n)
    Res = rng.uniform(Re_lo, Re_hi, size=n)
    nu_min = (tau_min - 0.5) / 3.0
    out = []
    for k in range(n):
        nr = int(nrs[k])
        nz = int(round(As[k] * (nr - 0.5)))
        Re, R = float(Res[k]), nr - 0.5
        c = cavity(nr, nz, Re, max(U_t, Re * nu_min / R))
        c["name"] = "batch%d_%d" % (seed, k)
        out.append(c)
    return out


def melt(Re_c: float, Re_x: float, Gr: float, nr: int = 128, nz: int = 256,
         nu: float = 0.0125, Pr: float = 0.05, beta: float = 0.4, wet: bool = False) -> dict:
    """Rotating crystal / crucible melt with buoyancy (swirl + temperature).

    Crucible of radius R_c (nr - 1/2 with halfway walls, nr - 1 with wet-node
    walls) rotating at Omega_c = Re_c nu / R_c^2 (side wall at T = 1, bottom
    adiabatic); crystal disk r <= beta R_c on the top rotating at
    Omega_x = Re_x nu / R_c^2 at T = 0; free, adiabatic surface outside the
    crystal; Boussinesq buoyancy with g beta = Gr nu^2 / R_c^3 (unit
    temperature difference), T_ref = 1/2.  The D2Q4 temperature field has
    diffusivity kappa = nu / Pr = tau_h / 2 (paper-convention tau_h)."""
    Rc = nr - (1.0 if wet else 0.5)
    om_c = Re_c * nu / Rc ** 2
    om_x = Re_x * nu / Rc ** 2
    kappa = nu / Pr
    top = split_wall(wall(omega=om_x, thermal=1, T=0.0), freeslip(), beta * Rc)
    return base_case(nz, nr, 3.0 * nu + 0.5, swirl=True, thermal=True,
                     tau_h=2.0 * kappa + 0.5, gbeta=Gr * nu * nu / Rc ** 3, T_ref=0.5,
                     south=axis(), north=wall(omega=om_c, thermal=1, T=1.0),
                     west=wall(omega=om_c), east=top, wet=bool(wet),
                     name="melt_Rec%.0f_Rex%.0f_Gr%.0f%s" % (Re_c, Re_x, Gr, "_wet" if wet else ""),
                     Re_c=float(Re_c), Re_x=float(Re_x), Gr=float(Gr))


def wheeler(Re_x: float, Re_c: float, n: int = 100, U_t: float = 0.1, beta: float = 0.4,
            wet: bool = True) -> dict:
    """Wheeler's Czochralski benchmark as the paper sets it up (Sec. IV B):
    isothermal melt of height H = R_c in a crucible of radius R_c rotating at
    Omega_c (side wall and bottom), a crystal disk r <= beta R_c on the top
    rotating at Omega_x, a flat stress-free surface beside it; n x n nodes;
    Re_c = R_c^2 Omega_c / nu, Re_x = R_c^2 Omega_x / nu; the lid speed
    U_t = beta R_c Omega_x fixes nu = U_t R_c / (beta |Re_x|).  With wet-node
    walls (the paper's treatment) R_c = H = n - 1."""
    Rc = n - (1.0 if wet else 0.5)
    nu = U_t * Rc / (beta * abs(Re_x))
    om_x = Re_x * nu / Rc ** 2
    om_c = Re_c * nu / Rc ** 2
    top = split_wall(wall(omega=om_x), freeslip(), beta * Rc)
    return base_case(n, n, 3.0 * nu + 0.5, swirl=True, south=axis(), north=wall(omega=om_c),
                     west=wall(omega=om_c), east=top, wet=bool(wet),
                     name="wheeler_Rex%g_Rec%g%s" % (Re_x, Re_c, "_wet" if wet else ""),
                     Re_x=float(Re_x), Re_c=float(Re_c), nu=float(nu), R_c=float(Rc))


def melt_set(n: int, seed: int, nr: int = 128, nz: int = 256, re_max: float = 1000.0,
             signed: bool = False, gr_range=(1e3, 1e5), nu: float = 0.0125,
             wet: bool = False) -> list[dict]:
    """Seeded melt instances: Re_c, Re_x ~ U[0, re_max] (with random signs when
    signed, i.e. counter-rotation allowed), Gr log-uniform in gr_range."""
    rng = np.random.default_rng(seed)
    out = []
    lo, hi = np.log10(gr_range[0]), np.log10(gr_range[1])
    for _ in range(n):
        rc = rng.uniform(0, re_max) * (rng.choice([-1.0, 1.0]) if signed else 1.0)
        rx = rng.uniform(0, re_max) * (rng.choice([-1.0, 1.0]) if signed else 1.0)
        gr = 10.0 ** rng.uniform(lo, hi)
        out.append(melt(rc, rx, gr, nr=nr, nz=nz, nu=nu, wet=wet))
    return out


def roofline_pipe(nz: int = 16384, nr: int = 2048, tau: float = 0.8, a: float = 1e-7) -> dict:
    """Large body-force pipe (f only) sized far beyond the on-package caches."""
    return base_case(nz, nr, tau, a0=a, name="roofline_pipe_%dx%d" % (nz, nr))


# ---- seeded random states ----------------------------------------------------

def random_fields(case: dict, seed: int, amp: float = 0.02) -> dict:
    """Random macroscopic fields (density, velocities, T) for parity runs (not steady)."""
    rng = np.random.default_rng(seed)
    nr, nz = case["nr"], case["nz"]
    out = {}
    for k in ("uz", "ur", "uth"):
        out[k] = amp * rng.uniform(-1.0, 1.0, size=(nr, nz))
    out["T"] = case.get("T_ref", 0.0) + 0.5 * rng.uniform(-1.0, 1.0, size=(nr, nz))
    out["rho"] = case.get("rho0", 1.0) + 0.01 * rng.uniform(-1.0, 1.0, size=(nr, nz))
    return out


def node_count(cases) -> int:
    return int(sum(c["nz"] * c["nr"] for c in cases))


def describe(case: dict) -> str:
    return "%s (%d x %d, tau_s=%.4f)" % (case.get("name", "case"), case["nz"], case["nr"],
                                         case["tau"])


__all__ = [n for n in dir() if not n.startswith("_") and n not in ("math", "np", "annotations")]

"""Stokes stream function of an axisymmetric velocity field (post-processing,
host side): d(psi)/dr = -r u_z and d(psi)/dz = r u_r (Sec. IV B), with
psi = 0 on the axis.  Fields are [nr][nz] arrays on nodes r_j = r0 + j,
z_i = i; psi is integrated along r with the trapezoid rule."""
from __future__ import annotations

import numpy as np


def stream_function(uz: np.ndarray, r0: float = 0.0) -> np.ndarray:
    """psi(r_j, z_i) = -int_{r0}^{r_j} r u_z dr (psi(r0) = 0; r0 = 0 is the axis)."""
    uz = np.asarray(uz, dtype=np.float64)
    r = (r0 + np.arange(uz.shape[0], dtype=np.float64))[:, None]
    q = -r * uz
    psi = np.zeros_like(q)
    psi[1:] = np.cumsum(0.5 * (q[1:] + q[:-1]), axis=0)
    return psi


def stream_function_z(ur: np.ndarray, r0: float = 0.0) -> np.ndarray:
    """The same function from the other relation, psi(r_j, z_i) = int_0^{z_i}
    r u_r dz, taking psi = 0 on the bottom row of nodes (a wall or the
    surface where u_z = 0 along it); equals stream_function for a field that
    satisfies the axisymmetric continuity equation."""
    ur = np.asarray(ur, dtype=np.float64)
    r = (r0 + np.arange(ur.shape[0], dtype=np.float64))[:, None]
    q = r * ur
    psi = np.zeros_like(q)
    psi[:, 1:] = np.cumsum(0.5 * (q[:, 1:] + q[:, :-1]), axis=1)
    return psi


def wheeler_extrema(case: dict, uz: np.ndarray) -> tuple[float, float]:
    """(psi_min, psi_max) in the viscous units of Wheeler's benchmark: length
    R_c, velocity nu / R_c, so psi is reported as psi / (nu R_c)."""
    psi = stream_function(np.asarray(uz).reshape(case["nr"], case["nz"]), case.get("r0", 0.0))
    s = case["nu"] * case["R_c"]
    return float(psi.min() / s), float(psi.max() / s)

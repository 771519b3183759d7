"""Helpers shared by the GPU parity tests: run one case on the oracle and on
the HIP library from the same seeded fields and compare the macros."""
from __future__ import annotations

import numpy as np

# Tolerances on max|u_gpu - u_oracle| / u_max after the same step count.
TOL = {0: 1e-10, 1: 1e-5}  # FP64, FP32


def oracle_run(case, steps, fields=None):
    from oracle import oracle as O
    o = O.Oracle(case)
    if fields is None:
        o.seed()
    else:
        o.seed(fields.get("uz"), fields.get("ur"), fields.get("uth"), fields.get("T"),
               fields.get("rho"))
    o.step(steps)
    return o


def gpu_run(cases, steps, prec, fields=None, launch=None, graph=None):
    import torch
    from paper_1003_0282_amd import lbaxi as L
    lat = L.Lattices(cases, prec)
    if launch is not None:
        lat.set_launch(*launch)
    if graph is not None:
        lat.set_graph_steps(graph)
    if fields is not None:
        packed = {}
        for k in ("uz", "ur", "uth", "T", "rho"):
            if all(k in f for f in fields):
                packed[k] = torch.cat([torch.as_tensor(np.asarray(f[k]).reshape(-1))
                                       for f in fields])
        lat.seed(**packed)
    lat.step(steps)
    return lat


def to_np(m):
    return {k: v.double().cpu().numpy() for k, v in m.items()}


def errors(case, gm, om):
    """Relative errors of every field: velocities over u_max, T over its
    spread (or 1), rho over rho0."""
    u_max = float(np.sqrt(om["uz"] ** 2 + om["ur"] ** 2 + om["uth"] ** 2).max())
    u_max = max(u_max, 1e-300)
    e = {}
    for k in ("uz", "ur", "uth"):
        e[k] = float(np.abs(gm[k] - om[k]).max()) / u_max
    if case.get("thermal"):
        spread = max(float(om["T"].max() - om["T"].min()), 1.0)
        e["T"] = float(np.abs(gm["T"] - om["T"]).max()) / spread
    # density: rounding of the (undamped) mass accumulates; judge it against rho0
    e["rho"] = float(np.abs(gm["rho"] - om["rho"]).max()) / float(case.get("rho0", 1.0))
    return e, u_max


def assert_parity(case, gm, om, prec, label=""):
    e, u_max = errors(case, gm, om)
    tol = TOL[prec]
    bad = {k: v for k, v in e.items() if not (v <= tol)}
    assert not bad, "%s parity over tolerance %g (u_max %.3e): %s" % (label, tol, u_max, e)
    return e

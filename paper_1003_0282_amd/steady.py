"""Runs to a steady state: a batch of lattices advanced until the Eq. (57)
residual of every lattice reaches a tolerance (or a step cap), with every
lattice's residual recorded at each check, and optionally its distance to a
reference field.  Also the runner of the rotating-lid cavities of Sec. IV B
at the sizes of the time-to-steady workload.

Every step runs in liblbaxi.so; this module marshals calls and bookkeeping.
"""
from __future__ import annotations

import argparse
import json
import time
from dataclasses import dataclass, field

import numpy as np

from . import lbaxi as L
from . import workloads as W

FIELDS = ("rho", "uz", "ur", "uth", "T")


@dataclass
class Solve:
    status: np.ndarray
    steps: np.ndarray
    residual: np.ndarray
    wall_s: float
    fields: dict = field(default_factory=dict)  # packed numpy float64 per FIELDS
    hist_steps: np.ndarray = None  # steps done at each residual check
    hist_wall: np.ndarray = None   # seconds since the start (seeding included)
    hist_res: np.ndarray = None    # [checks, n] Eq. (57) residual, NaN once frozen
    hist_err: np.ndarray = None    # [checks, n] distance to a reference field (if given)

    def first_crossing(self, tol: float):
        """Per instance: index of the first check with residual <= tol, -1 if none."""
        ok = np.nan_to_num(self.hist_res, nan=np.inf) <= tol
        idx = np.argmax(ok, axis=0)
        return np.where(ok.any(axis=0), idx, -1)

    def first_within(self, err: float):
        """Per instance: index of the first check from which the distance to
        the reference stays <= err, -1 if never."""
        bad = ~(np.nan_to_num(self.hist_err, nan=np.inf) <= err)
        last_bad = len(bad) - 1 - np.argmax(bad[::-1], axis=0)
        idx = np.where(bad.any(axis=0), last_bad + 1, 0)
        return np.where(idx < len(bad), idx, -1)


def _ref_distance(lat, ref, n):
    """Per instance: max |u - u_ref| over the three velocity components,
    divided by the instance's max |u_ref| (ref: packed device tensors)."""
    import torch
    m = lat.macros(("uz", "ur", "uth"))
    out = np.zeros(n)
    d = torch.stack([(m[k].double() - ref[k]).abs() for k in ("uz", "ur", "uth")]).amax(0)
    a = torch.stack([ref[k].abs() for k in ("uz", "ur", "uth")]).amax(0)
    for i in range(n):
        sl = slice(int(lat.offsets[i]), int(lat.offsets[i + 1]))
        out[i] = float(d[sl].max() / a[sl].max())
    return out


def solve(cases, init=None, tol=1e-8, max_steps=2_000_000, check_every=1000, budget_s=None,
          prec=L.FP32, launch=None, log=None, tag="", log_every_s=15.0, ref=None) -> Solve:
    """Run every case to the Eq. (57) tolerance (or max_steps) in one batched
    handle, recording every instance's residual at each check; `init` is None
    (from rest) or a dict of packed device fields for Lattices.seed; with
    `ref` (packed float64 device velocity fields) the distance to it is
    recorded at each check as well (outside the timed quantities' meaning:
    the macros pass it needs is included in the wall clock)."""
    import torch
    lat = L.Lattices(cases, prec)
    if launch is not None:
        lat.set_launch(*launch)
    n = len(cases)
    steps = np.zeros(n, np.int64)
    res = np.full(n, np.nan)
    hs, hw, hr, he = [], [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.seed(**init) if init is not None else lat.seed()
    done, last_log = 0, 0.0
    status = np.zeros(n, np.int32)
    while True:
        r = lat.run(tol, check_every, check_every)
        done += check_every
        steps += r.steps
        cur = np.where(r.steps > 0, r.residual, np.nan)
        res = np.where(r.steps > 0, r.residual, res)
        status = r.status
        el = time.perf_counter() - t0
        hs.append(done)
        hw.append(el)
        hr.append(cur)
        if ref is not None:
            he.append(_ref_distance(lat, ref, n))
        live = int((status == L.RUNNING).sum() + (status == L.CAPPED).sum())
        stop = live == 0 or done >= max_steps or (budget_s is not None and el > budget_s)
        if log and (stop or el - last_log > log_every_s):
            last_log = el
            log("%s t=%d live %d/%d conv %d div %d res med %.2e max %.2e  %.1fs" % (
                tag, done, live, n, int((status == L.CONVERGED).sum()),
                int((status == L.DIVERGED).sum()), np.nanmedian(res), np.nanmax(res), el))
        if stop:
            break
        lat.resume()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    m = lat.macros(FIELDS)
    out = {k: m[k].double().cpu().numpy() for k in FIELDS}
    lat.close()
    return Solve(status.copy(), steps, res, wall, out, np.asarray(hs), np.asarray(hw),
                 np.asarray(hr), np.asarray(he) if ref is not None else None)


def cavity_cases(res=(990.0, 1492.0, 2494.0), nr=256, aspects=(1.5, 2.5), wet=False):
    """Rotating-lid cylinders: Nr x Nz = 256 x 384 (H/R = 1.5) and 256 x 640
    (H/R = 2.5), lid speed 0.1, one per Reynolds number; halfway or wet-node
    walls."""
    out = []
    for A in aspects:
        nz = int(round(A * nr))
        for Re in res:
            out.append(W.cavity(nr, nz, Re, wet=wet))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="time to steady state of the rotating-lid cavities")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--max-steps", type=int, default=4_000_000)
    ap.add_argument("--check-every", type=int, default=1000)
    ap.add_argument("--budget", type=float, default=None, help="seconds")
    ap.add_argument("--prec", type=int, default=L.FP32)
    ap.add_argument("--wet", action="store_true", help="wet-node walls (the paper's treatment)")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    cases = cavity_cases(wet=a.wet)
    r = solve(cases, tol=a.tol, max_steps=a.max_steps, check_every=a.check_every,
              budget_s=a.budget, prec=a.prec, log=lambda s: print(s, flush=True), tag="cavity")
    tols = (1e-5, 1e-6, 1e-7, 1e-8)
    rows = []
    for k, c in enumerate(cases):
        row = {"case": c["name"], "nodes": c["nr"] * c["nz"], "status": L.STATUS_NAMES[int(r.status[k])],
               "steps": int(r.steps[k]), "residual": float(r.residual[k])}
        for t in tols:
            idx = r.first_crossing(t)[k]
            row["steps_to_%g" % t] = int(r.hist_steps[idx]) if idx >= 0 else None
            row["wall_to_%g" % t] = float(r.hist_wall[idx]) if idx >= 0 else None
        rows.append(row)
        print(json.dumps(row), flush=True)
    out = {"tol": a.tol, "max_steps": a.max_steps, "wall_s": r.wall_s, "prec": a.prec,
           "wet": a.wet, "cases": rows}
    if a.out:
        with open(a.out, "w") as f:
            json.dump(out, f, indent=1)
    print(json.dumps({"wall_s": r.wall_s, "converged": int((r.status == L.CONVERGED).sum()),
                      "n": len(cases)}))


if __name__ == "__main__":
    main()

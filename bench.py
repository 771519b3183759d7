#!/usr/bin/env python3
"""Throughput benchmark of the improved axisymmetric LB hot path on one GPU.

    python bench.py [--steps K] [--warmup W] [--workload NAME]

A step is one time step of every lattice of the workload (pull streaming with
the boundary rules, macros, collision of f, g and h as the workload has
them), run through the C-ABI library.  The timed region is exactly K steps
between two device synchronisations, inputs resident in HBM.  Prints one JSON
line with MLUPS, the HBM-roofline fraction of the step kernel and the CPU
oracle timed on a bounded sample of the same workload; the default workload's
line also carries the time to the Eq. 57 residual 1e-8 of 128 held-out melts
from rest and from the learned warm start (`time_to_steady`).

Workloads (synthetic, seeded):
  batch256   256 rotating-lid cavities, Nr ~ U{64..512}, H/R ~ U[1,3],
             Re ~ U[500,2500] (tau_s >= 0.52), FP32 f + g, one launch per
             step (default)
  batch256_mrt   the same 256 cavities with the MRT collision of f
  pipe_fp32 / pipe_fp64   16384 x 2048 body-force pipe, f only
  pipe_fp64_zou_he   the same pipe with wet-node Zou-He walls
  pipe_fp64_original / pipe_fp32_original   the same pipe under the original
             scheme of Sec. II (lagged-gradient source, Eqs. 7-10)
  womersley  64 x 128 Womersley pipe, FP32
  cavity     256 x 384 rotating-lid cavity at Re 990, FP32 f + g
  melt512    512 crystal/crucible melts 128 x 256, FP32 f + g + h
  melt512_wet   the same melts with wet-node walls (the learned warm start's runs)
  copy       the library's plain copy kernel (the streaming ceiling)
  unet       warm-start U-Net on 128 x 256 inputs: training steps (batch 8)
             and forward passes (batch 16), TFLOP/s against the BF16 MFMA peak
  warmstart  the learned warm start end to end: time to residual 1e-8
  batch256_sequential   the 256 cavities one handle after another
  wheeler    Wheeler's crystal/crucible benchmark, both Table 1 cases (100 x 100
             and the second also at 200 x 200,
             wet-node walls, FP64) to the Eq. 57 residual 1e-8, psi extrema
  fig7       the paper's Fig. 7 run (100 x 150 rotating-lid cylinder, Re 1290,
             tau = 0.005, wet-node walls, FP64): BGK until it diverges, MRT
             to the Eq. 57 residual 1e-10, the axis maximum against Table 2
  wheeler_refine   Table 1's Re_x = 1e3 case on 100, 141, 200 and 283 nodes
             to the residual 1e-8, then 3 M steps on 100 x 100 with the mass
  cavity_stall   the 256 x 384 Re 990 cylinder with halfway walls, FP64 and
             FP32, 2 M steps: residual, where it sits, its sign pattern
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def workload(name: str):
    from paper_1003_0282_amd import workloads as W
    if name == "batch256":
        return W.batch_cavities(256, seed=0), 1, "256 rotating-lid cavities (seed 0), FP32 f+g"
    if name == "batch256_mrt":
        cases = [dict(c, mrt=True) for c in W.batch_cavities(256, seed=0)]
        return cases, 1, "256 rotating-lid cavities (seed 0), FP32 f+g, MRT collision of f"
    if name == "pipe_fp32":
        return [W.roofline_pipe()], 1, "16384x2048 body-force pipe, FP32 f"
    if name == "pipe_fp64":
        return [W.roofline_pipe()], 0, "16384x2048 body-force pipe, FP64 f"
    if name == "pipe_fp64_zou_he":
        return ([dict(W.roofline_pipe(), wet=True, zou_he=True)], 0,
                "16384x2048 body-force pipe, FP64 f, wet-node Zou-He walls")
    if name == "pipe_fp64_original":
        return ([dict(W.roofline_pipe(), original=True)], 0,
                "16384x2048 body-force pipe, FP64 f, original scheme (Sec. II)")
    if name == "pipe_fp32_original":
        return ([dict(W.roofline_pipe(), original=True)], 1,
                "16384x2048 body-force pipe, FP32 f, original scheme (Sec. II)")
    if name == "womersley":
        return [W.womersley()], 1, "Womersley pipe 64x128, FP32 f"
    if name == "cavity":
        return [W.cavity(256, 384, 990.0)], 1, "rotating-lid cavity 256x384 Re 990, FP32 f+g"
    if name == "melt512":
        return W.melt_set(512, seed=1), 1, "512 crystal/crucible melts 128x256, FP32 f+g+h"
    if name == "melt512_wet":
        return (W.melt_set(512, seed=1, wet=True), 1,
                "512 crystal/crucible melts 128x256, FP32 f+g+h, wet-node walls")
    raise SystemExit("unknown workload %r" % name)


def bytes_per_update(case, prec):
    es = 8 if prec == 0 else 4
    q = 9 + (4 if case.get("swirl") else 0) + (4 if case.get("thermal") else 0)
    if case.get("original"):
        q += 2  # the lagged velocity (u_z, u_r): read once, written once
    return 2 * q * es  # every population read once and written once


def kernel_hash() -> str:
    """Hash of what the HBM counters of a launch shape depend on: the solver's
    device code (lbaxi_device.hpp and the kernel part of lbaxi.hip, everything
    before its host-runtime section) and the host functions that lay the
    populations out in memory (from the layout's description to the
    workspace's)."""
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_1003_0282_amd", "csrc")
    for f in sorted(os.listdir(src)):
        if f.startswith("lbaxi"):
            text = open(os.path.join(src, f), "rb").read()
            cut = text.find(b"\n// host runtime\n")
            if cut < 0:
                h.update(text)
                continue
            h.update(text[:cut])
            a = text.find(b"\n// Row-blocked layout", cut)
            b = text.find(b"\n// Device workspace", a + 1)
            h.update(text[cut:] if a < 0 or b < 0 else text[a:b])
    return h.hexdigest()[:16]


def traffic_entry(name: str, launch: str):
    """HBM bytes per launch of the step kernel from committed rocprofv3 counter
    summaries taken on this exact kernel source and launch shape, or None."""
    p = os.path.join(ROOT, "profiles", "traffic_%s.json" % name)
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_hash") != kernel_hash():
        return None
    for e in d.get("by_launch", [d]):
        if e.get("launch") == launch:
            return float(e["hbm_bytes_per_launch"])
    return None


def _oracle_sample(cases, seconds: float):
    from oracle import oracle as O
    done = 0
    used = []
    t0 = time.perf_counter()
    k = 0
    while time.perf_counter() - t0 < seconds and k < len(cases):
        c = cases[k]
        o = O.Oracle(c)
        o.seed()
        steps = 0
        while steps < 200 and time.perf_counter() - t0 < seconds:
            o.step(5)
            steps += 5
        done += steps * c["nz"] * c["nr"]
        used.append("%s x%d steps" % (c.get("name", "case"), steps))
        del o
        k += 1
    el = time.perf_counter() - t0
    return done, el, k, used


def cpu_baseline(cases, seconds: float):
    """The oracle, as it stands, on a bounded sample of the same workload: on
    every host core it is given, and on one core for a third of the time."""
    from oracle import oracle as O
    O.build()
    cores = O.get_threads()
    done, el, k, used = _oracle_sample(cases, seconds)
    O.set_threads(1)
    try:
        done1, el1, k1, _ = _oracle_sample(cases, seconds / 3.0)
    finally:
        O.set_threads(cores)
    return {"value": done / el / 1e6, "unit": "MLUPS", "cores": cores,
            "kind": "oracle",
            "sample": "%d of %d lattices, %d node updates in %.1f s (%s)" % (
                k, len(cases), done, el, "; ".join(used[:4]) + (" ..." if len(used) > 4 else "")),
            "single_core": {"value": done1 / el1 / 1e6, "unit": "MLUPS", "cores": 1,
                            "sample": "%d lattices, %d node updates in %.1f s" % (k1, done1, el1)}}


def copy_probe(steps: int, warmup: int, nbytes: int = 4 << 30):
    """Device-to-device streaming copy of 4 GiB through the library's copy
    kernel with 1, 2, 4 and 8 loads in flight per lane, and torch's own copy:
    the practical HBM ceiling the step kernel is compared with (the best of
    them), and the kernel whose known traffic calibrates the HBM counters."""
    import torch
    from paper_1003_0282_amd import lbaxi as L
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    s = torch.cuda.current_stream()

    def timed(call):
        for _ in range(max(1, warmup)):
            call()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(steps):
            call()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    runs = {}
    for u in (1, 2, 4, 8):
        ms = timed(lambda: L._check(L._L.lbaxi_stream_copy(src.data_ptr(), dst.data_ptr(), nbytes,
                                                            u, s.cuda_stream), "lbaxi_stream_copy"))
        runs["k_copy<%d>" % u] = ms
    runs["torch copy_"] = timed(lambda: dst.copy_(src))
    assert bool((dst == 1).all())
    gbs = {k: 2 * nbytes / (ms / 1e3) / 1e9 for k, ms in runs.items()}
    best = max(gbs, key=gbs.get)
    return {"metric": "copy bandwidth (read + write)", "value": round(gbs[best], 1), "unit": "GB/s",
            "best": best, "bytes_per_launch": 2 * nbytes,
            "variants": {k: {"ms_per_launch": round(runs[k], 4), "GB/s": round(gbs[k], 1)}
                         for k in runs},
            "frac_of_peak": round(gbs[best] / HBM_PEAK_GBS, 4)}


def sequential_probe(steps: int):
    """The 256 cavities of batch256 run one after another (one handle each,
    default launch shape, graphs on) against the same lattices in one
    batched handle: aggregate MLUPS of both."""
    import torch
    from paper_1003_0282_amd import lbaxi as L
    from paper_1003_0282_amd import workloads as W
    cases = W.batch_cavities(256, seed=0)
    nodes = sum(c["nz"] * c["nr"] for c in cases)
    lats = [L.Lattices([c], L.FP32) for c in cases]
    for lat in lats:
        lat.seed()
        lat.step(64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for lat in lats:
        lat.step(steps)
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t0
    del lats
    batch = L.Lattices(cases, L.FP32)
    batch.seed()
    batch.step(64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(steps)
    torch.cuda.synchronize()
    bat_s = time.perf_counter() - t0
    seq, bat = nodes * steps / seq_s / 1e6, nodes * steps / bat_s / 1e6
    return {"metric": "aggregate MLUPS of 256 cavities: one after another vs one batched handle",
            "value": round(bat / seq, 3), "unit": "x (batched / sequential)", "n_gpus": 1,
            "steps": steps, "higher_is_better": True, "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "batch256_sequential", "lattices": len(cases), "nodes": nodes,
                       "population_storage": "f32", "launch": "default (64 x 4 tiles)"},
            "sequential_mlups": round(seq, 1), "batched_mlups": round(bat, 1)}


def warmstart_probe():
    """Time to the Eq. (57) residual 1e-8 of 16 held-out 128 x 256 melts
    (wet-node walls, FP32 storage) from rest and from the learned warm start,
    with the network trained here on 256 solver-generated steady fields; the
    distance of both end states to FP64 reference fields (residual 1e-10)."""
    import numpy as np
    from paper_1003_0282_amd import warmstart as WS
    t0 = time.perf_counter()
    r = WS.experiment(n_train=256, n_eval=16, nr=128, nz=256, re_max=1000.0, tol=1e-8,
                      gen_steps=1_000_000, eval_steps=2_000_000, train_steps=10000, batch=8,
                      lr=1e-3, gen_budget_s=200, train_budget_s=150, eval_budget_s=100,
                      ref_budget_s=100, wet=True,
                      log=lambda m: print(m, file=sys.stderr, flush=True))
    e, n = r["eval"], r["eval"]["nn_smooth"]
    d8 = [d for d in n["by_tol"] if d["tol"] == 1e-8][0]
    return {
        "metric": "time to steady state (Eq. 57 residual 1e-8): learned warm start vs from rest",
        "value": round(e["zero"]["wall_s"] / n["wall_s"], 3), "unit": "x (wall-time speedup)",
        "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "warmstart_melt128x256", "lattices": 16, "nodes_each": 128 * 256,
                   "walls": "wet-node", "population_storage": "f32",
                   "training_fields": r["train"]["samples"], "train_steps": r["train"]["steps"]},
        "from_rest": {"wall_s": round(e["zero"]["wall_s"], 3),
                      "steps_median": float(np.median(e["zero"]["steps"])),
                      "final_error_median": float(np.median(e["zero"]["final_error"]))},
        "warm_start": {"wall_s": round(n["wall_s"], 3), "inference_s": round(n["inference_s"], 4),
                       "steps_median": float(np.median(n["steps"])),
                       "final_error_median": float(np.median(n["final_error"]))},
        "both_reached_1e-8": d8["reached_both"],
        "pipeline_wall_s": round(time.perf_counter() - t0, 1),
    }


MODEL = os.path.join(ROOT, "paper_1003_0282_amd", "models", "melt_unet_128x256.npz")


def time_to_steady_leg(n_melts: int, tol: float = 1e-8):
    """The second half of the metric: wall time until every one of n_melts
    held-out crystal / crucible melts (128 x 256, wet-node walls, FP32
    storage, seed 1) reaches the Eq. (57) residual tol, from rest and from the
    learned warm start (the committed network, trained by the library's own
    kernels on 4096 steady fields the batched solver generated; inference and
    seeding are inside the warm start's time), in one batched handle each."""
    import numpy as np
    import torch
    from paper_1003_0282_amd import lbaxi as L
    from paper_1003_0282_amd import warmstart as WS
    from paper_1003_0282_amd import workloads as W
    from paper_1003_0282_amd.steady import solve
    cases = W.melt_set(n_melts, 1, nr=128, nz=256, wet=True)
    net, sc, meta = WS.load_model(MODEL, max_batch=8)
    z = solve(cases, tol=tol, max_steps=3_000_000, check_every=1000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X = torch.tensor(WS.features(cases), device="cuda")
    init = WS.predict(net, X, sc, smooth=True)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    w = solve(cases, init=init, tol=tol, max_steps=3_000_000, check_every=1000)
    net.close()
    shape = (n_melts, 128, 256)
    diff = WS.rel_field_error(w.fields, z.fields, shape)
    ok = lambda r: int((r.status == L.CONVERGED).sum())
    return {"workload": "melt_128x256_wet_x%d" % n_melts, "tol": tol,
            "from_rest_s": round(z.wall_s, 3), "warm_start_s": round(w.wall_s + t_inf, 3),
            "inference_s": round(t_inf, 4), "speedup": round(z.wall_s / (w.wall_s + t_inf), 3),
            "steps_median_from_rest": float(np.median(z.steps)),
            "steps_median_warm": float(np.median(w.steps)),
            "converged_from_rest": ok(z), "converged_warm": ok(w), "lattices": n_melts,
            "end_state_difference_median": float(np.median(diff)),
            "model": "trained on %d solver-generated steady fields (seed 2, %d reached the "
                     "residual 1e-8)" % (meta.get("n_train", 0),
                                         meta.get("generate", {}).get("converged", 0))}


def wheeler_probe():
    """Both Table 1 cases of Wheeler's benchmark in one batched FP64 handle
    from rest to the Eq. (57) residual 1e-8; the stream-function extrema in
    units of nu R_c next to the paper's."""
    from paper_1003_0282_amd import lbaxi as L
    from paper_1003_0282_amd import steady as ST
    from paper_1003_0282_amd import streamfn as SF
    from paper_1003_0282_amd import workloads as W
    table1 = {(100.0, -25.0): (-0.0494, 0.1180), (1000.0, -250.0): (-1.444, 1.128)}
    cases = [W.wheeler(*k) for k in table1] + [W.wheeler(1000.0, -250.0, n=200)]
    r = ST.solve(cases, tol=1e-8, max_steps=3_000_000, check_every=2000, prec=L.FP64)
    per = []
    off = 0
    for k, c in enumerate(cases):
        n = c["nr"] * c["nz"]
        lo, hi = SF.wheeler_extrema(c, r.fields["uz"][off:off + n])
        off += n
        p = table1[(c["Re_x"], c["Re_c"])]
        per.append({"grid": "%dx%d" % (c["nr"], c["nz"]), "Re_x": c["Re_x"], "Re_c": c["Re_c"],
                    "tau_s": c["tau"],
                    "status": L.STATUS_NAMES[int(r.status[k])], "steps": int(r.steps[k]),
                    "psi_min": round(lo, 4), "psi_max": round(hi, 4),
                    "paper_psi_min": p[0], "paper_psi_max": p[1]})
    nodes = sum(c["nr"] * c["nz"] for c in cases)
    return {"metric": "Wheeler benchmark: wall time to the Eq. 57 residual 1e-8 (both Table 1 "
                      "cases at 100 x 100 and the second at 200 x 200, one handle)",
            "value": round(r.wall_s, 2), "unit": "s", "n_gpus": 1, "higher_is_better": False,
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "wheeler_table1", "lattices": len(cases),
                       "walls": "wet-node", "population_storage": "f64", "nodes": nodes},
            "mlups": round(sum(c["nr"] * c["nz"] * float(s) for c, s in zip(cases, r.steps))
                           / r.wall_s / 1e6, 1), "cases": per}


def wheeler_refine_probe(long_steps: int = 3_000_000):
    """Table 1's second case (Re_x = 1e3, Re_c = -250, wet-node walls, FP64)
    under grid refinement, each grid from rest to the Eq. (57) residual
    1e-8, with the stream-function extrema; then the 100 x 100 lattice run on
    with its residual, extrema and mean density (sum r rho / sum r)."""
    import numpy as np
    from paper_1003_0282_amd import lbaxi as L
    from paper_1003_0282_amd import steady as ST
    from paper_1003_0282_amd import streamfn as SF
    from paper_1003_0282_amd import workloads as W
    grids = (100, 141, 200, 283)
    cases = [W.wheeler(1000.0, -250.0, n=n) for n in grids]
    r = ST.solve(cases, tol=1e-8, max_steps=3_000_000, check_every=2000, prec=L.FP64)
    per, off = [], 0
    for k, c in enumerate(cases):
        n = c["nr"] * c["nz"]
        lo, hi = SF.wheeler_extrema(c, r.fields["uz"][off:off + n])
        off += n
        per.append({"n": grids[k], "tau_s": c["tau"], "status": L.STATUS_NAMES[int(r.status[k])],
                    "steps": int(r.steps[k]), "psi_min": round(lo, 4), "psi_max": round(hi, 4)})
    # second-order Richardson extrapolation from the pairs (100, 200), (141, 283)
    rich = [{"from": [a["n"], b["n"]],
             "psi_min": round(b["psi_min"] + (b["psi_min"] - a["psi_min"]) / 3.0, 4),
             "psi_max": round(b["psi_max"] + (b["psi_max"] - a["psi_max"]) / 3.0, 4)}
            for a, b in ((per[0], per[2]), (per[1], per[3]))]
    c = cases[0]
    lat = L.Lattices([c], L.FP64)
    lat.seed()
    rr = np.arange(c["nr"], dtype=np.float64)[:, None]
    run, done = [], 0
    for target in (76_000, 300_000, 1_000_000, 2_000_000, 3_000_000):
        if target > long_steps:
            break
        lat.step(target - done)
        done = target
        m = {k: v.double().cpu().numpy().reshape(c["nr"], c["nz"]) for k, v in lat.macros().items()}
        lo, hi = SF.wheeler_extrema(c, m["uz"])
        run.append({"t": done, "residual": float(lat.residual()[0]), "psi_min": round(lo, 4),
                    "psi_max": round(hi, 4),
                    "mean_rho": float((rr * m["rho"]).sum() / (rr.sum() * c["nz"]))})
    lat.close()
    return {"metric": "Wheeler benchmark Re_x = 1e3 under grid refinement (Table 1: "
                      "psi_min -1.444, psi_max 1.128)", "value": per[-1]["psi_min"], "unit": "psi/(nu R_c)",
            "n_gpus": 1, "higher_is_better": None, "vs_baseline": None, "dtype": "f64",
            "data": "synthetic", "config": {"workload": "wheeler_refine", "walls": "wet-node"},
            "grids": per, "richardson": rich, "long_run_100": run}


def cavity_stall_probe(total: int = 2_000_000, every: int = 100_000):
    """The 256 x 384 rotating-lid cylinder at Re 990 with halfway walls from
    rest, FP64 and FP32 storage: every `every` steps the Eq. (57) residual,
    the node where |u| changes most between the last two levels, and at the
    end the signs of that change around it (a period-2 pattern is a staggered
    mode)."""
    import numpy as np
    from paper_1003_0282_amd import lbaxi as L
    from paper_1003_0282_amd import workloads as W
    out = {}
    for prec, name in ((L.FP64, "fp64"), (L.FP32, "fp32")):
        c = W.cavity(256, 384, 990.0)
        lat = L.Lattices([c], prec)
        lat.seed()
        nr, nz = c["nr"], c["nz"]
        rows, done, t0 = [], 0, time.perf_counter()
        win = None
        while done < total:
            lat.step(every - 1)
            m0 = {k: v.double().cpu().numpy().reshape(nr, nz) for k, v in lat.macros().items()}
            lat.step(1)
            done += every
            m1 = {k: v.double().cpu().numpy().reshape(nr, nz) for k, v in lat.macros().items()}
            d = np.hypot(m1["uz"], m1["ur"]) - np.hypot(m0["uz"], m0["ur"])
            j, i = np.unravel_index(np.argmax(np.abs(d)), d.shape)
            rows.append({"t": done, "residual": float(lat.residual()[0]), "i": int(i), "j": int(j)})
            print("cavity_stall %s t=%d residual %.3e at (i=%d, j=%d) %.0fs" % (
                name, done, rows[-1]["residual"], i, j, time.perf_counter() - t0),
                file=sys.stderr, flush=True)
            win = np.sign(d[max(0, j - 2):j + 3, max(0, i - 2):i + 3]).astype(int).tolist()
        lat.close()
        res = [x["residual"] for x in rows]
        out[name] = {"checks": rows, "sign_window_rows_j": win,
                     "decay_per_check_last5": round(float((res[-1] / res[-6]) ** 0.2), 4)}
    return {"metric": "halfway-wall cylinder residual over 2 M steps", "value": out["fp32"]["checks"][-1]["residual"],
            "unit": "Eq. 57 residual", "n_gpus": 1, "higher_is_better": False, "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": "cavity_stall_256x384_re990", "walls": "halfway", "every": every},
            "runs": out}


def fig7_probe(budget_s: float = 240.0, max_steps: int = 40_000_000):
    """Fig. 7: the rotating-lid cylinder of Table 2 at Re = 1290 with nu =
    0.005 / 3 (tau_s = 0.505).  The BGK handle runs until its residual turns
    NaN; the MRT handle runs to the Eq. (57) residual 1e-10 (the paper's
    criterion for this run) within a wall-clock budget, and the magnitude and
    height of the largest axial velocity on the axis are read off."""
    import numpy as np
    import torch
    from paper_1003_0282_amd import lbaxi as L
    from paper_1003_0282_amd import steady as ST
    from paper_1003_0282_amd import workloads as W
    nu = 0.005 / 3.0

    def case(mrt):
        c = W.cavity_paper(1290.0, wet=True)
        R = c["nr"] - 1.0
        return dict(c, tau=0.505, east=W.wall(omega=1290.0 * nu / (R * R)), mrt=mrt,
                    name="fig7_%s" % ("mrt" if mrt else "bgk"))

    bgk = ST.solve([case(False)], tol=1e-10, max_steps=min(200_000, max_steps), check_every=500,
                   prec=L.FP64)
    c = case(True)
    torch.cuda.synchronize()
    r = ST.solve([c], tol=1e-10, max_steps=max_steps, check_every=min(20_000, max_steps),
                 prec=L.FP64,
                 budget_s=budget_s, log=lambda m: print(m, file=sys.stderr, flush=True),
                 tag="fig7 mrt", log_every_s=20.0)
    nr, nz = c["nr"], c["nz"]
    axis = r.fields["uz"][:nr * nz].reshape(nr, nz)[0]
    Ut = c["east"]["omega"] * (nr - 1.0)
    i = int(np.argmax(np.abs(axis)))
    reversed_ = int((axis * np.sign(axis[i]) < -1e-6 * Ut).sum())
    steps = int(r.steps[0])
    return {"metric": "Fig. 7 (tau = 0.005): MRT wall time to the Eq. 57 residual 1e-10; "
                      "BGK divergence",
            "value": round(r.wall_s, 2), "unit": "s", "n_gpus": 1, "higher_is_better": False,
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "fig7_cylinder_100x150_Re1290_tau0.005", "walls": "wet-node",
                       "population_storage": "f64", "nodes": nr * nz},
            "bgk": {"status": L.STATUS_NAMES[int(bgk.status[0])], "steps": int(bgk.steps[0])},
            "mrt": {"status": L.STATUS_NAMES[int(r.status[0])], "steps": steps,
                    "residual": float(r.residual[0]),
                    "mlups": round(nr * nz * steps / r.wall_s / 1e6, 1),
                    "uz_max_over_Ut": round(abs(float(axis[i])) / Ut, 4),
                    "h_max_over_H": round(i / (nz - 1.0), 4),
                    "reversed_axis_nodes": reversed_},
            "table2_re1290_tau0.02": {"uz_max_over_Ut": 0.0716, "h_max_over_H": 0.147}}


MFMA_BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16


def unet_flops(H, W, c_in, widths, c_out):
    """Algorithmic FLOPs per sample of the warm-start U-Net: (forward, one
    training step).  Forward: 2 x the multiply-adds of every 3 x 3
    convolution at its level's resolution plus the 1 x 1 head; a training
    step adds the input gradient of every convolution but the first and the
    weight gradient of every one (the same multiply-adds each)."""
    w = widths
    layers = []  # (level, c_in, c_out)
    prev = c_in
    for l in range(4):
        layers += [(l, prev, w[l]), (l, w[l], w[l])]
        prev = w[l]
    for l in (2, 1, 0):
        layers += [(l, w[l + 1] + w[l], w[l]), (l, w[l], w[l])]
    macs = [(H >> l) * (W >> l) * 9 * ci * co for l, ci, co in layers]
    head = H * W * w[0] * c_out
    fwd = 2.0 * (sum(macs) + head)
    train = fwd + 2.0 * (sum(macs) - macs[0] + head) + 2.0 * (sum(macs) + head)
    return fwd, train


def nn_probe(steps: int, warmup: int, batch: int = 8):
    """Training and inference throughput of the warm-start U-Net on 128 x 256
    inputs (8 channels in, 5 out), BF16 MFMA with FP32 accumulation: whole
    training steps (forward, backward, Adam) timed with HIP events, no host
    synchronisation inside the timed region."""
    import ctypes as C
    import torch
    from paper_1003_0282_amd import lbnn as N
    from paper_1003_0282_amd import warmstart as WS
    H, W = 128, 256
    torch.cuda.set_device(0)
    net = WS.make_net(H, W, max_batch=2 * batch)
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn((2 * batch, H, W, WS.C_IN), device="cuda", generator=g)
    y = torch.randn((2 * batch, H, W, WS.C_OUT), device="cuda", generator=g)
    xb, yb = x[:batch].contiguous(), y[:batch].contiguous()
    call = lambda: N._check(N._L.lbnn_train_step(net.h, C.c_void_p(xb.data_ptr()),
                                                   C.c_void_p(yb.data_ptr()), batch, 1e-4, None),
                            "lbnn_train_step")
    for _ in range(warmup):
        call()
    s = net.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(steps):
        call()
    e1.record(s)
    torch.cuda.synchronize()
    ms_train = e0.elapsed_time(e1) / steps
    yo = torch.empty((2 * batch, H, W, WS.C_OUT), device="cuda")
    fcall = lambda: N._check(N._L.lbnn_forward(net.h, C.c_void_p(x.data_ptr()),
                                                 C.c_void_p(yo.data_ptr()), 2 * batch),
                             "lbnn_forward")
    for _ in range(warmup):
        fcall()
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(steps):
        fcall()
    e1.record(s)
    torch.cuda.synchronize()
    ms_fwd = e0.elapsed_time(e1) / steps
    fwd, train = unet_flops(H, W, WS.C_IN, WS.WIDTHS, WS.C_OUT)
    tf_train = batch * train / ms_train / 1e9
    tf_fwd = 2 * batch * fwd / ms_fwd / 1e9
    net.close()
    return {
        "metric": "U-Net training throughput (forward + backward + Adam, BF16 MFMA, FP32 accumulation)",
        "value": round(tf_train, 2), "unit": "TFLOP/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": round(ms_train, 4), "higher_is_better": True,
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "unet_train_128x256", "batch": batch, "H": H, "W": W,
                   "c_in": WS.C_IN, "c_out": WS.C_OUT, "widths": list(WS.WIDTHS),
                   "gflop_per_sample_forward": round(fwd / 1e9, 3),
                   "gflop_per_sample_train": round(train / 1e9, 3)},
        "roofline": {"bound": "mfma", "achieved": round(tf_train, 2),
                     "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tf_train / MFMA_BF16_PEAK_TFLOPS, 4), "traffic": None,
                     "kernel": "whole training step (every lbnn kernel of it)"},
        "inference": {"batch": 2 * batch, "ms": round(ms_fwd, 4), "tflops": round(tf_fwd, 2),
                      "frac": round(tf_fwd / MFMA_BF16_PEAK_TFLOPS, 4)},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="batch256")
    ap.add_argument("--autotune", type=int, default=1)
    ap.add_argument("--tune-steps", type=int, default=16,
                    help="time steps per autotuner trial (real steps: the state advances)")
    ap.add_argument("--launch", default="", help="tile_z,tile_r,grid,xcd,nt (skips autotune)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--tts-melts", type=int, default=128,
                    help="melts of the time-to-steady leg of the default line (0: skip)")
    ap.add_argument("--kernel-steps", type=int, default=100,
                    help="steps timed kernel by kernel for the roofline figure")
    ap.add_argument("--max-steps", type=int, default=0,
                    help="fig7: cap on the steps of each run (0 = run to the criterion)")
    ap.add_argument("--prec", default="", choices=["", "fp64", "fp32", "fp32fast"],
                    help="override the workload's precision")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the workload is a single-GPU batch and no "
              "multi-GPU path is built (asked for --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1003_0282_amd import lbaxi as L

    if args.workload == "copy":
        print(json.dumps(copy_probe(args.steps, args.warmup)))
        return
    if args.workload == "warmstart":
        print(json.dumps(warmstart_probe()))
        return
    if args.workload == "unet":
        print(json.dumps(nn_probe(args.steps, args.warmup)))
        return
    if args.workload == "wheeler":
        print(json.dumps(wheeler_probe()))
        return
    if args.workload == "fig7":
        print(json.dumps(fig7_probe(max_steps=args.max_steps or 40_000_000)))
        return
    if args.workload == "wheeler_refine":
        print(json.dumps(wheeler_refine_probe()))
        return
    if args.workload == "cavity_stall":
        print(json.dumps(cavity_stall_probe()))
        return
    if args.workload == "batch256_sequential":
        print(json.dumps(sequential_probe(args.steps)))
        return
    cases, prec, label = workload(args.workload)
    if args.prec:
        prec = {"fp64": 0, "fp32": 1, "fp32fast": 2}[args.prec]
        label += " [precision %s]" % args.prec
    torch.cuda.set_device(0)
    lat = L.Lattices(cases, prec)
    lat.seed()
    tuned = None
    if args.launch:
        cfg = [int(x) for x in args.launch.split(",")]
        lat.set_launch(*cfg)
    elif args.autotune:
        tuned = lat.autotune(steps_per_trial=args.tune_steps)
    launch = lat.get_launch()
    # timed runs replay the step graph: its length fits inside the run, and
    # its two instances (one per buffer parity) are built here, untimed
    kg = max(2, min(64, (args.steps - 1) // 2 * 2))
    lat.set_graph_steps(kg)
    for _ in range(2):
        lat.step(kg + 1)
    lat.step(args.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    stream = lat.stream
    torch.cuda.synchronize()
    ev0.record(stream)
    lat.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    ms_step = ms / args.steps
    nodes = lat.nodes
    mlups = nodes * args.steps / (ms / 1e3) / 1e6
    bpu = bytes_per_update(cases[0], prec)
    algo = bpu * nodes  # bytes per launch of the step kernel (one per time step)
    algo_step = algo
    step_gbs = algo_step / (ms_step / 1e3) / 1e9
    # the step kernel's own duration: HIP events around each of its launches
    # on the handle's stream, over a second stretch of real steps
    lat.set_profiling(True)
    lat.step(args.kernel_steps)
    k_ms, k_n = lat.kernel_time()
    lat.set_profiling(False)
    k_avg_ms = k_ms / max(k_n, 1)
    achieved = algo / (k_avg_ms / 1e3) / 1e9
    tr = traffic_entry(args.workload, ",".join(str(int(x)) for x in launch))
    res = lat.residual()
    n_finite = int(sum(1 for r in res if r == r and r < 1e30))
    out = {
        "metric": "MLUPS (lattice node updates per second) and fraction of HBM peak",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == 2 else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": label,
                   "population_storage": "f64" if prec == 0 else "f32",
                   "lattices": len(cases),
                   "nodes": nodes, "bytes_per_update": bpu,
                   "bytes_per_update_f_only_convention": 144 if prec == 0 else 72,
                   "launch": {"tile_z": launch[0], "tile_r": launch[1], "grid": launch[2],
                              "xcd_aware": launch[3], "nt_store": launch[4],
                              "autotuned": tuned is not None}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": tr,
                     "kernel": "k_step (fused pull-stream + collide)",
                     "kernel_avg_ms": round(k_avg_ms, 5), "kernel_launches_timed": k_n,
                     "algorithmic_bytes_per_launch": algo,
                     "whole_step_gbs": round(step_gbs, 1)},
        "lattices_finite": n_finite,
    }
    if args.workload == "batch256" and args.tts_melts > 0:
        lat.close()
        out["time_to_steady"] = time_to_steady_leg(args.tts_melts)
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(cases, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

"""Learned warm start of the batched melt solver.

A U-Net (liblbnn.so, BF16 MFMA kernels) maps the geometry and parameters of a
rotating crystal / crucible melt (the Wheeler configuration of Sec. IV C,
extended with Boussinesq buoyancy) to its steady fields (rho, u_z, u_r,
u_theta, T).  The prediction seeds the populations at equilibrium (Eq. 6 with
half the Eq. (12) source, Eq. 54), and the plain lattice Boltzmann run then continues
until the Eq. (57) residual reaches the tolerance.  The run, not the network,
decides when a field is steady: a poor prediction costs steps, never
accuracy.  The network is trained on steady fields that the batched solver
itself produces from rest.

Every step of the pipeline runs in the two HIP libraries; this module builds
the input channels on the host and marshals tensors between the calls.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time
from dataclasses import dataclass

import numpy as np

from . import lbaxi as L
from . import lbnn as N
from . import workloads as W
from .steady import Solve, solve  # noqa: F401  (re-exported for callers)

C_IN, C_OUT = 8, 5
WIDTHS = (32, 64, 128, 256)
FIELDS = ("rho", "uz", "ur", "uth", "T")  # network output channels, in order


# ---- inputs and targets -----------------------------------------------------

def features(cases) -> np.ndarray:
    """Input channels [B, nr, nz, 8] (float32), one row per r, z fastest:
    r / R_c, z / H, Re_c / 1000, Re_x / 1000, log10 Gr - 4, the column under
    the crystal (r <= r_split), and the rigid-rotation speeds of the crucible
    and of the crystal column (Re r / (1000 R_c))."""
    out = []
    for c in cases:
        nr, nz = int(c["nr"]), int(c["nz"])
        wet = bool(c.get("wet"))
        Rc = nr - (1.0 if wet else 0.5)   # wall through / half a spacing beyond the last row
        one = np.ones((nr, nz))
        r = np.arange(nr)[:, None] / Rc * one
        zc = np.arange(nz)[None, :] / (nz - 1.0) if wet else (np.arange(nz)[None, :] + 0.5) / nz
        z = zc * one
        rs = float(c["east"].get("r_split", -1.0))
        crystal = (np.arange(nr)[:, None] <= rs) * one
        rec, rex = c["Re_c"] / 1000.0, c["Re_x"] / 1000.0
        lg = math.log10(c["Gr"]) - 4.0
        out.append(np.stack([r, z, rec * one, rex * one, lg * one, crystal, rec * r,
                             rex * r * crystal], -1))
    return np.asarray(out, dtype=np.float32)


@dataclass
class Scales:
    """Target channel k is (field_k - off[k]) / s[k]: the density and the
    temperature are taken relative to rho0 and T_ref (the pressure carries the
    centrifugal balance of the swirl, so a seed without it would start an
    acoustic transient that decays only on the viscous time scale)."""
    s: np.ndarray
    off: np.ndarray

    @staticmethod
    def fit(fields: dict, rho0: float, T_ref: float) -> "Scales":
        off = np.array([rho0 if k == "rho" else T_ref if k == "T" else 0.0 for k in FIELDS])
        s = [float(np.sqrt(np.mean(np.square(fields[k] - off[i])))) or 1.0
             for i, k in enumerate(FIELDS)]
        return Scales(np.asarray(s, np.float64), off)


def targets(fields: dict, sc: Scales, shape) -> np.ndarray:
    """Packed solver fields (numpy, [nodes]) -> [B, nr, nz, C_OUT] float32."""
    B, nr, nz = shape
    ch = [(fields[k] - sc.off[i]) / sc.s[i] for i, k in enumerate(FIELDS)]
    return np.stack([c.reshape(B, nr, nz) for c in ch], -1).astype(np.float32)


# ---- solver runs: see steady.py ---------------------------------------------

# ---- network ------------------------------------------------------------------

def make_net(nr, nz, max_batch=8, seed=0):
    """U-Net of widths 32-64-128-256 with He-normal weights and zero biases."""
    net = N.Net(nr, nz, C_IN, C_OUT, WIDTHS, max_batch=max_batch)
    rng = np.random.default_rng(seed)
    cins = [C_IN, WIDTHS[0], WIDTHS[0], WIDTHS[1], WIDTHS[1], WIDTHS[2], WIDTHS[2], WIDTHS[3],
            WIDTHS[3] + WIDTHS[2], WIDTHS[2], WIDTHS[2] + WIDTHS[1], WIDTHS[1],
            WIDTHS[1] + WIDTHS[0], WIDTHS[0]]
    couts = [WIDTHS[0], WIDTHS[0], WIDTHS[1], WIDTHS[1], WIDTHS[2], WIDTHS[2], WIDTHS[3], WIDTHS[3],
             WIDTHS[2], WIDTHS[2], WIDTHS[1], WIDTHS[1], WIDTHS[0], WIDTHS[0]]
    parts = []
    for ci, co in zip(cins, couts):
        parts.append(rng.standard_normal(9 * ci * co) * math.sqrt(2.0 / (9 * ci)))
        parts.append(np.zeros(co))
    parts.append(rng.standard_normal(WIDTHS[0] * C_OUT) * math.sqrt(1.0 / WIDTHS[0]))
    parts.append(np.zeros(C_OUT))
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == net.nparam
    net.set_params(flat)
    return net


def train(net, X, Y, steps, batch, lr, log=None, seed=0, budget_s=None):
    """Adam on the MSE loss with a cosine learning-rate decay; X, Y device
    tensors [n, nr, nz, C].  Returns the per-step losses."""
    import torch
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    losses = []
    t0 = time.perf_counter()
    perm = rng.permutation(n)
    pos = 0
    for s in range(steps):
        if pos + batch > n:
            perm, pos = rng.permutation(n), 0
        idx = torch.as_tensor(perm[pos:pos + batch], device=X.device)
        pos += batch
        lr_s = 0.5 * lr * (1.0 + math.cos(math.pi * s / steps))
        losses.append(net.train_step(X.index_select(0, idx), Y.index_select(0, idx), lr_s))
        if log and (s % 200 == 0 or s == steps - 1):
            log("train step %d/%d loss %.4e  %.1fs" % (s, steps, losses[-1], time.perf_counter() - t0))
        if budget_s is not None and time.perf_counter() - t0 > budget_s:
            if log:
                log("train: time budget reached at step %d" % s)
            break
    return losses


def predict(net, X, sc: Scales, smooth=True) -> dict:
    """Network prediction for every row of X -> packed float32 device fields
    (rho, u_z, u_r, u_theta, T) in the solver's layout, low-passed by the
    (1, 2, 1)/4 filter when smooth (a checkerboard in a seed would sit in the
    lattice's weakly damped staggered modes)."""
    import torch
    B, nr, nz, _ = X.shape
    hw = nr * nz
    outs = {k: torch.empty(B * hw, dtype=torch.float32, device=X.device) for k in FIELDS}
    for b0 in range(0, B, net.max_batch):
        bs = min(net.max_batch, B - b0)
        y = net.forward(X[b0:b0 + bs])
        net.to_fields(y, sc.s, sc.off, [outs[k][b0 * hw:(b0 + bs) * hw] for k in FIELDS],
                      smooth=smooth)
    return outs


def save_model(path, net, sc: Scales, meta: dict):
    """Trained parameters (FP32 masters, flat), target scales and offsets,
    and a JSON description of how the model was made (no pickled objects)."""
    p = net.get_params().cpu().numpy()
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    np.savez(path, params=p, scales=sc.s, offsets=sc.off, meta=json.dumps(meta))


def load_model(path, max_batch=8):
    z = np.load(path, allow_pickle=False)
    meta = json.loads(str(z["meta"]))
    net = N.Net(meta["nr"], meta["nz"], C_IN, C_OUT, WIDTHS, max_batch=max_batch)
    net.set_params(z["params"])
    return net, Scales(np.asarray(z["scales"]), np.asarray(z["offsets"])), meta


# ---- the experiment ---------------------------------------------------------

def rel_field_error(a: dict, b: dict, shape) -> np.ndarray:
    """Per instance: max over nodes of |a - b| of the three velocity fields,
    divided by the instance's max speed in b."""
    B, nr, nz = shape
    err = np.zeros(B)
    for i in range(B):
        sl = slice(i * nr * nz, (i + 1) * nr * nz)
        umax = max(np.abs(b[k][sl]).max() for k in ("uz", "ur", "uth"))
        err[i] = max(np.abs(a[k][sl] - b[k][sl]).max() for k in ("uz", "ur", "uth")) / umax
    return err


def compare(z: Solve, w: Solve, t_inf: float, tols, errs=()) -> dict:
    """Time to each residual tolerance (and, when both runs tracked a
    reference, to each distance from it) from rest (z) and from the
    prediction (w): per-instance steps and the batch wall time until every
    instance that gets there in both runs has got there."""
    def one(cz, cw, key, val):
        both = (cz >= 0) & (cw >= 0)
        d = {key: val, "reached_zero": int((cz >= 0).sum()), "reached_nn": int((cw >= 0).sum()),
             "reached_both": int(both.sum())}
        if both.any():
            sz, sw = z.hist_steps[cz[both]], w.hist_steps[cw[both]]
            d.update(steps_zero=sz.tolist(), steps_nn=sw.tolist(),
                     steps_ratio_median=float(np.median(sz / sw)),
                     wall_zero_s=float(z.hist_wall[cz[both]].max()),
                     wall_nn_s=float(w.hist_wall[cw[both]].max() + t_inf))
            d["wall_ratio"] = d["wall_zero_s"] / d["wall_nn_s"]
        return d
    out = {"residual": [one(z.first_crossing(t), w.first_crossing(t), "tol", t) for t in tols]}
    if z.hist_err is not None and w.hist_err is not None:
        out["distance"] = [one(z.first_within(e), w.first_within(e), "err", e) for e in errs]
    return out


def experiment(n_train=256, n_eval=16, nr=128, nz=256, re_max=1000.0, tol=1e-8,
               gen_steps=1_200_000, eval_steps=3_000_000, train_steps=3000, batch=8, lr=1e-3,
               gen_budget_s=None, train_budget_s=None, eval_budget_s=None, check_every=1000,
               seed_train=2, seed_eval=1, tols=(1e-6, 3e-7, 1e-7, 3e-8, 1e-8),
               errs=(0.1, 0.03, 0.01, 0.003), out_dir=None, smooth_variants=(True,), wet=False,
               ref_tol=1e-10, ref_steps=2_000_000, ref_budget_s=None, log=print,
               load_model_path=None, save_model_path=None, gen_init_path=None):
    """Generate steady training fields with the batched solver, train the
    network on them, then solve held-out cases from rest and from the
    prediction and compare the time to each residual tolerance and to each
    distance from reference steady fields (an FP64 run to ref_tol), and the
    distance of each run's final field from that reference.  With
    load_model_path the generation and training are skipped (a model saved
    by save_model_path is used); with n_eval = 0 the evaluation is.  With
    gen_init_path the training melts are solved from that model's prediction
    rather than from rest."""
    import torch
    res = {"config": dict(n_train=n_train, n_eval=n_eval, nr=nr, nz=nz, re_max=re_max, tol=tol,
                          gen_steps=gen_steps, eval_steps=eval_steps, train_steps=train_steps,
                          batch=batch, lr=lr, check_every=check_every, seed_train=seed_train,
                          seed_eval=seed_eval, wet=wet, model=load_model_path)}
    ev = W.melt_set(n_eval, seed_eval, nr=nr, nz=nz, re_max=re_max, wet=wet) if n_eval else []
    if load_model_path:
        net, sc, meta = load_model(load_model_path, max_batch=batch)
        assert (meta["nr"], meta["nz"]) == (nr, nz), "model trained on another lattice size"
        res["train"] = dict(meta.get("train", {}), loaded_from=load_model_path)
        res["generate"] = meta.get("generate", {})
    else:
        net, sc = _generate_and_train(res, n_train, nr, nz, re_max, tol, gen_steps, train_steps,
                                      batch, lr, gen_budget_s, train_budget_s, check_every,
                                      seed_train, wet, log, gen_init_path)
        if save_model_path:
            save_model(save_model_path, net, sc,
                       dict(nr=nr, nz=nz, re_max=re_max, wet=wet, seed_train=seed_train,
                            n_train=n_train, tol=tol, train=res["train"],
                            generate=res["generate"]))
    if not n_eval:
        return res
    return _evaluate(res, net, sc, ev, nr, nz, tol, eval_steps, check_every, eval_budget_s,
                     tols, errs, smooth_variants, ref_tol, ref_steps, ref_budget_s, out_dir, log,
                     re_max)


def _generate_and_train(res, n_train, nr, nz, re_max, tol, gen_steps, train_steps, batch, lr,
                        gen_budget_s, train_budget_s, check_every, seed_train, wet, log,
                        gen_init_path=None):
    import torch
    tr = W.melt_set(n_train, seed_train, nr=nr, nz=nz, re_max=re_max, wet=wet)
    rho0, T_ref = tr[0]["rho0"], tr[0]["T_ref"]

    # the training fields are steady states of the solver; with gen_init_path
    # the solver starts from an earlier model's prediction instead of rest
    # (it still runs every melt to the residual tol, so the fields are its
    # own steady states, reached in fewer steps)
    init = None
    if gen_init_path:
        net0, sc0, meta0 = load_model(gen_init_path, max_batch=batch)
        assert (meta0["nr"], meta0["nz"]) == (nr, nz), "model trained on another lattice size"
        init = predict(net0, torch.tensor(features(tr), device="cuda"), sc0, smooth=True)
        del net0
    g = solve(tr, init=init, tol=tol, max_steps=gen_steps, check_every=check_every,
              budget_s=gen_budget_s, log=log, tag="gen")
    del init
    keep = np.flatnonzero(g.status != L.DIVERGED)
    res["generate"] = dict(wall_s=g.wall_s, converged=int((g.status == L.CONVERGED).sum()),
                           capped=int((g.status == L.CAPPED).sum()),
                           diverged=int((g.status == L.DIVERGED).sum()),
                           steps_median=float(np.median(g.steps)),
                           residual_median_kept=float(np.nanmedian(g.residual[keep])),
                           residual_max_kept=float(np.nanmax(g.residual[keep])),
                           node_steps=float(g.steps.sum()) * nr * nz, init_model=gen_init_path)
    hw = nr * nz
    sc = Scales.fit({k: np.concatenate([g.fields[k][i * hw:(i + 1) * hw] for i in keep])
                     for k in FIELDS}, rho0, T_ref)
    Yall = targets(g.fields, sc, (n_train, nr, nz))[keep]
    X = torch.tensor(features([tr[i] for i in keep]), device="cuda")
    Y = torch.tensor(Yall, device="cuda")

    net = make_net(nr, nz, max_batch=batch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = train(net, X, Y, train_steps, batch, lr, log=log, budget_s=train_budget_s)
    torch.cuda.synchronize()
    res["train"] = dict(wall_s=time.perf_counter() - t0, steps=len(losses), samples=int(len(keep)),
                        loss_first=losses[0], loss_last=float(np.mean(losses[-20:])),
                        params=net.nparam, scales=sc.s.tolist())
    del X, Y
    return net, sc


def _evaluate(res, net, sc, ev, nr, nz, tol, eval_steps, check_every, eval_budget_s, tols, errs,
              smooth_variants, ref_tol, ref_steps, ref_budget_s, out_dir, log, re_max):
    import torch
    n_eval = len(ev)

    # reference steady fields: FP64 from rest to a residual far below tol
    ref_run = solve(ev, tol=ref_tol, max_steps=ref_steps, check_every=check_every,
                    budget_s=ref_budget_s, prec=L.FP64, log=log, tag="reference")
    ref = {k: torch.tensor(ref_run.fields[k], device="cuda") for k in ("uz", "ur", "uth")}
    shape = (n_eval, nr, nz)
    res["reference"] = dict(wall_s=ref_run.wall_s, status=ref_run.status.tolist(),
                            steps=ref_run.steps.tolist(), residual=ref_run.residual.tolist(),
                            prec="f64", tol=ref_tol)
    # from rest and from the prediction, with the distance to the reference
    # recorded at every check (the same macros pass in both runs)
    z = solve(ev, tol=tol, max_steps=eval_steps, check_every=check_every,
              budget_s=eval_budget_s, log=log, tag="zero", ref=ref)
    dz = rel_field_error(z.fields, ref_run.fields, shape)
    res["eval"] = dict(cases=[c["name"] for c in ev],
                       zero=dict(wall_s=z.wall_s, steps=z.steps.tolist(), status=z.status.tolist(),
                                 residual=z.residual.tolist(), final_error=dz.tolist()))
    for smooth in smooth_variants:
        tag = "nn_smooth" if smooth else "nn_raw"
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Xe = torch.tensor(features(ev), device="cuda")
        init = predict(net, Xe, sc, smooth=smooth)
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t0
        pred = {k: v.double().cpu().numpy() for k, v in init.items()}
        w = solve(ev, init=init, tol=tol, max_steps=eval_steps, check_every=check_every,
                  budget_s=eval_budget_s, log=log, tag=tag, ref=ref)
        dw = rel_field_error(w.fields, ref_run.fields, shape)
        cmp = compare(z, w, t_inf, tols, errs)
        res["eval"][tag] = dict(
            wall_s=w.wall_s + t_inf, inference_s=t_inf, steps=w.steps.tolist(),
            status=w.status.tolist(), residual=w.residual.tolist(),
            by_tol=cmp["residual"], by_distance=cmp.get("distance", []),
            prediction_error=rel_field_error(pred, ref_run.fields, shape).tolist(),
            final_error=dw.tolist(),
            final_difference=rel_field_error(w.fields, z.fields, shape).tolist())
    if out_dir:
        os.makedirs(out_dir, exist_ok=True)
        save_model(os.path.join(out_dir, "melt_unet_%dx%d.npz" % (nz, nr)), net, sc,
                   dict(nr=nr, nz=nz, re_max=re_max))
        with open(os.path.join(out_dir, "warmstart_%dx%d.json" % (nz, nr)), "w") as f:
            json.dump(res, f, indent=1)
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description="learned warm start of the batched melt solver")
    ap.add_argument("--n-train", type=int, default=256)
    ap.add_argument("--n-eval", type=int, default=16)
    ap.add_argument("--nr", type=int, default=128)
    ap.add_argument("--nz", type=int, default=256)
    ap.add_argument("--re-max", type=float, default=1000.0)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--gen-steps", type=int, default=1_200_000)
    ap.add_argument("--eval-steps", type=int, default=3_000_000)
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--gen-budget", type=float, default=None)
    ap.add_argument("--train-budget", type=float, default=None)
    ap.add_argument("--eval-budget", type=float, default=None)
    ap.add_argument("--check-every", type=int, default=1000)
    ap.add_argument("--ref-tol", type=float, default=1e-10)
    ap.add_argument("--ref-steps", type=int, default=2_000_000)
    ap.add_argument("--ref-budget", type=float, default=None)
    ap.add_argument("--out", default=None)
    ap.add_argument("--variants", default="smooth", help="comma list of smooth,raw")
    ap.add_argument("--wet", action="store_true", help="wet-node walls (the paper's treatment)")
    ap.add_argument("--save-model", default=None, help="write the trained model (.npz) here")
    ap.add_argument("--load-model", default=None,
                    help="skip generation and training: evaluate this saved model")
    ap.add_argument("--gen-init-model", default=None,
                    help="solve the training melts from this saved model's prediction")
    a = ap.parse_args(argv)
    variants = tuple(v == "smooth" for v in a.variants.split(","))
    r = experiment(a.n_train, a.n_eval, a.nr, a.nz, a.re_max, a.tol, a.gen_steps, a.eval_steps,
                   a.train_steps, a.batch, a.lr, a.gen_budget, a.train_budget, a.eval_budget,
                   check_every=a.check_every, out_dir=a.out, smooth_variants=variants, wet=a.wet,
                   ref_tol=a.ref_tol, ref_steps=a.ref_steps, ref_budget_s=a.ref_budget,
                   log=lambda s: print(s, flush=True), load_model_path=a.load_model,
                   save_model_path=a.save_model, gen_init_path=a.gen_init_model)
    print(json.dumps({k: r[k] for k in ("generate", "train")}))
    if a.out and "eval" not in r:
        os.makedirs(a.out, exist_ok=True)
        with open(os.path.join(a.out, "train_%dx%d.json" % (a.nz, a.nr)), "w") as f:
            json.dump(r, f, indent=1)
    for tag in ("nn_smooth", "nn_raw"):
        if tag not in r.get("eval", {}):
            continue
        e = r["eval"][tag]
        print(tag, "prediction error median %.3f" % float(np.median(e["prediction_error"])),
              "final error vs reference: nn median %.2e max %.2e, zero median %.2e max %.2e" % (
                  np.median(e["final_error"]), np.max(e["final_error"]),
                  np.median(r["eval"]["zero"]["final_error"]), np.max(r["eval"]["zero"]["final_error"])))
        for d in e["by_tol"] + e["by_distance"]:
            print(tag, json.dumps({k: v for k, v in d.items()
                                   if not k.startswith("steps_") or k == "steps_ratio_median"}))


if __name__ == "__main__":
    main()

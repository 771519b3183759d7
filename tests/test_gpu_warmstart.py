"""The learned warm start end to end on small melts (32 x 64 nodes, wet-node
walls as in the paper's rotating flows), with the network trained on the GPU
by the library's own kernels on steady fields the batched solver generates.
Every held-out melt with a steady state reaches the Eq. (57) residual 1e-8
both from rest and from the prediction; the warm-started batch gets there in
less wall time, inference included, and ends at least as close to reference steady fields
(FP64, residual 1e-10) as the batch started from rest.  Training is
deterministic (fixed-order reductions), so its loss drop is a fixed number."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_warm_start_reaches_the_steady_field_sooner():
    from paper_1003_0282_amd import warmstart as WS
    r = WS.experiment(n_train=96, n_eval=8, nr=32, nz=64, re_max=250.0, tol=1e-8,
                      gen_steps=200_000, eval_steps=400_000, train_steps=800, batch=8, lr=1e-3,
                      check_every=1000, tols=(1e-6, 1e-8), errs=(0.1, 0.03), wet=True,
                      ref_tol=1e-10, ref_steps=400_000, log=None)
    e = r["eval"]["nn_smooth"]
    print({k: r[k] for k in ("generate", "train")})
    for tag in ("zero", "nn_smooth"):
        print(tag, "status", r["eval"][tag]["status"], "steps", r["eval"][tag]["steps"],
              "residual", ["%.2e" % x for x in r["eval"][tag]["residual"]])
    for d in e["by_distance"] + e["by_tol"]:
        print({k: v for k, v in d.items() if not k.startswith("steps_") or "median" in k})
    assert r["train"]["loss_last"] < 0.2 * r["train"]["loss_first"]
    n = len(r["eval"]["cases"])
    print("reference status", r["reference"]["status"],
          "residual", ["%.2e" % x for x in r["reference"]["residual"]])
    # the paper's criterion, residual 1e-8: every melt that has a steady state
    # (its FP64 reference run, aimed at 1e-10, gets below 1e-8) gets there both
    # ways; a melt whose flow never settles is excluded and counted (at most
    # one here)
    steady = [k for k in range(n) if r["reference"]["residual"][k] <= 1e-8]
    assert len(steady) >= n - 1
    for tag in ("zero", "nn_smooth"):
        st = r["eval"][tag]["status"]
        assert all(st[k] == 1 for k in steady), (tag, st)
    # and the warm-started batch gets there sooner in wall time (inference
    # included), over the melts that reach it in both runs
    r8 = {d["tol"]: d for d in e["by_tol"]}[1e-8]
    assert r8["reached_both"] >= len(steady)
    assert r8["wall_nn_s"] < r8["wall_zero_s"], r8
    assert r8["steps_ratio_median"] > 1.0
    # equal final accuracy: against the FP64 reference the warm-started runs
    # end no farther away than the runs from rest (median and worst case)
    z_err = np.asarray(r["eval"]["zero"]["final_error"])[steady]
    n_err = np.asarray(e["final_error"])[steady]
    print("final distance to the reference: warm start median %.3e max %.3e, "
          "from rest median %.3e max %.3e" % (np.median(n_err), n_err.max(),
                                               np.median(z_err), z_err.max()))
    assert np.median(n_err) <= np.median(z_err)
    assert n_err.max() <= z_err.max()

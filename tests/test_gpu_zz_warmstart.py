"""The learned warm start end to end on small melts (32 x 64 nodes, wet-node
walls as in the paper's rotating flows), with the network trained on the GPU
by the library's own kernels on steady fields the batched solver generates:
the warm-started runs come within 10 % of reference steady fields (FP64,
residual 1e-10) and reach the Eq. (57) residual 1e-6 in fewer steps than the
runs from rest, and stop as close to the reference as they do."""
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
                      gen_steps=200_000, eval_steps=150_000, train_steps=800, batch=8, lr=1e-3,
                      check_every=1000, tols=(1e-6, 1e-8), errs=(0.1, 0.03), wet=True,
                      ref_tol=1e-10, ref_steps=400_000, log=None)
    e = r["eval"]["nn_smooth"]
    print({k: r[k] for k in ("generate", "train")})
    for d in e["by_distance"] + e["by_tol"]:
        print({k: v for k, v in d.items() if not k.startswith("steps_") or "median" in k})
    # training does not repeat bit for bit (its reductions use atomics), so
    # the loss drop is asked with margin: about 0.2 x is typical, 0.3 x required
    assert r["train"]["loss_last"] < 0.3 * r["train"]["loss_first"]
    d10 = {d["err"]: d for d in e["by_distance"]}[0.1]
    assert d10["reached_both"] >= 6
    assert d10["steps_ratio_median"] > 2.0
    r6 = {d["tol"]: d for d in e["by_tol"]}[1e-6]
    assert r6["reached_both"] >= 6
    assert r6["steps_ratio_median"] > 1.1
    # at the same Eq. (57) tolerance both starts end as close to the
    # reference steady field (FP64, residual 1e-10) as each other
    z_err = np.asarray(r["eval"]["zero"]["final_error"])
    n_err = np.asarray(e["final_error"])
    assert np.median(n_err) < 2.0 * np.median(z_err) + 1e-3

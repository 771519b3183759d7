"""GPU parity over long runs: FP32 and FP64 handles against the CPU oracle
after as many steps as the configured workloads take.

The steady workloads run 1e5 - 1e6 steps in FP32 storage, the Womersley pipe
ten periods of 4000 steps.  Here the same lengths are run on lattices the
oracle finishes in seconds: a 37 x 70 rotating-lid cylinder and a 29 x 75
crystal / crucible melt (swirl and temperature), both with wet-node walls and
1e5 steps from rest (near their steady states), and the 64 x 128 Womersley
pipe for its full 40 000 steps.  Every node of u_z, u_r, u_theta (and T) is
compared: max |u_gpu - u_oracle| / u_max <= 1e-10 in FP64 and <= 1e-5 in FP32
storage, the same bar as the short runs.
"""
import time

import numpy as np
import pytest

from paper_1003_0282_amd import workloads as W
from _parity import assert_parity, errors, gpu_run, oracle_run, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


LONG = {
    "cavity_wet_37x70": (lambda: W.cavity(37, 70, 400.0, wet=True), 100_000),
    "melt_wet_29x75": (lambda: W.melt(-300.0, 500.0, 2e4, nr=29, nz=75, wet=True), 100_000),
    "womersley_64x128": (lambda: W.womersley(), 40_000),
}


@pytest.mark.parametrize("name", sorted(LONG))
def test_long_run_parity(name):
    make, steps = LONG[name]
    case = make()
    t0 = time.perf_counter()
    o = oracle_run(case, steps)
    om = o.macros()
    print("%s: oracle %d steps in %.1f s, residual %.2e" % (name, steps, time.perf_counter() - t0,
                                                           o.residual()), flush=True)
    shape = (case["nr"], case["nz"])
    for prec in (0, 1):
        lat = gpu_run([case], steps, prec)
        assert lat.time() == steps
        gm = {k: v.reshape(shape) for k, v in to_np(lat.macros()).items()}
        e, u_max = errors(case, gm, om)
        print("%s prec %d: u_max %.3e errors %s" % (name, prec, u_max,
                                                    {k: "%.2e" % v for k, v in e.items()}),
              flush=True)
        assert_parity(case, gm, om, prec, "%s %d steps" % (name, steps))
        lat.close()

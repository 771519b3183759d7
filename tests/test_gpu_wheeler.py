"""Wheeler's Czochralski benchmark (Sec. IV B, Table 1) on the GPU.

Parity: the 100 x 100 crystal/crucible case with wet-node walls, a rotating
crystal disk and a free surface on the top, from seeded random fields for
300 steps against the oracle (FP64 <= 1e-10, FP32 storage <= 1e-5 of u_max;
BGK and MRT).  Physics: both Table 1 cases run from rest to the Eq. (57)
residual 1e-9 in one batched FP64 handle; the extrema of the stream
function, in units of nu R_c, must fall within 10 % of the spread of the
three sets of values Table 1 lists (the paper's, its Refs. 26 and 50).
Table 1's column labels are taken as given (Re_x = 10^2, Re_c = -25 and
Re_x = 10^3, Re_c = -250).  The first case runs on the paper's 100 x 100
grid; the second on 200 x 200: on 100 x 100 it does not settle below a
residual of about 7e-10 and its extrema drift by some 10 % after passing
1e-8, while at 200 x 200 it converges (about 200 000 steps)."""
import numpy as np
import pytest

from paper_1003_0282_amd import workloads as W
from _parity import assert_parity, gpu_run, oracle_run, to_np

pytestmark = pytest.mark.gpu

def _table1():
    """(Re_x, Re_c) -> (psi_min values, psi_max values) of the three references."""
    import json
    import os
    p = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table1_wheeler.json")
    with open(p) as f:
        g = json.load(f)
    return {(c["Re_x"], c["Re_c"]): (tuple(c["psi_min"].values()), tuple(c["psi_max"].values()))
            for c in g["cases"]}


TABLE1 = _table1()


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("mrt", [False, True])
def test_wheeler_parity(prec, mrt):
    case = dict(W.wheeler(1000.0, -250.0), mrt=mrt)
    fields = W.random_fields(case, 21)
    fields.pop("T")
    o = oracle_run(case, 300, fields)
    lat = gpu_run([case], 300, prec, [fields])
    gm = {k: v.reshape(case["nr"], case["nz"]) for k, v in to_np(lat.macros()).items()}
    e = assert_parity(case, gm, o.macros(), prec, "wheeler")
    print("wheeler prec %d mrt %d" % (prec, mrt), e)


def _band(vals, slack=0.1):
    lo, hi = min(vals), max(vals)
    pad = slack * max(abs(lo), abs(hi))
    return lo - pad, hi + pad


def test_wheeler_table1():
    from paper_1003_0282_amd import lbaxi as L
    from paper_1003_0282_amd import steady as ST
    from paper_1003_0282_amd import streamfn as SF
    cases = [W.wheeler(100.0, -25.0), W.wheeler(1000.0, -250.0, n=200)]
    r = ST.solve(cases, tol=1e-9, max_steps=1_000_000, check_every=2000, prec=L.FP64)
    assert (r.status == L.CONVERGED).all(), r.status
    off = 0
    for k, c in enumerate(cases):
        n = c["nr"] * c["nz"]
        uz = r.fields["uz"][off:off + n]
        off += n
        lo, hi = SF.wheeler_extrema(c, uz)
        mins, maxs = TABLE1[(c["Re_x"], c["Re_c"])]
        print(c["name"], "steps %d psi_min %.4f psi_max %.4f (Table 1: %s, %s)"
              % (r.steps[k], lo, hi, mins, maxs))
        a, b = _band(mins)
        assert a <= lo <= b, (lo, mins)
        a, b = _band(maxs)
        assert a <= hi <= b, (hi, maxs)

"""Parity at the benchmark's full sizes, in the launch shapes bench.py times.

The whole workload runs on the GPU in one handle (256 cavities, 56.3 M nodes,
with BGK and with MRT collision; 512 melts of 128 x 256; the 16384 x 2048
pipe with halfway walls, with Zou-He walls and under the original scheme)
from seeded random states; the oracle recomputes a sample of the lattices
(the largest, the smallest and a few seeded picks) in full for the same
number of steps, and every node of those lattices is compared.  Graph replay is part of the run (graph length 8,
20 steps: two replays and four direct steps).  The other lattices must stay
finite.  Tolerance: FP32 storage 1e-5 of u_max, FP64 1e-10, as elsewhere.
"""
import numpy as np
import pytest

from _parity import TOL, errors, oracle_run
from paper_1003_0282_amd import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 20


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _packed_fields(lat, cases, sampled, seed):
    """Packed seed fields on the device: numpy random_fields for the sampled
    lattices (so the oracle sees the same values), torch random values of the
    same ranges elsewhere."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    keys = ["uz", "ur", "rho"]
    if all(c.get("swirl") for c in cases):
        keys.append("uth")
    if all(c.get("thermal") for c in cases):
        keys.append("T")
    out, per = {}, {}
    for k in keys:
        t = torch.rand(lat.nodes, generator=g, device="cuda", dtype=torch.float32)
        if k == "rho":
            t = 1.0 + 0.01 * (2 * t - 1)
        elif k == "T":
            t = cases[0].get("T_ref", 0.0) + 0.5 * (2 * t - 1)
        else:
            t = 0.02 * (2 * t - 1)
        out[k] = t.to(lat.dtype)
    for i in sampled:
        f = W.random_fields(cases[i], 1000 + i)
        per[i] = {k: f[k] for k in keys}
        for k in keys:
            out[k][lat.offsets[i]:lat.offsets[i + 1]] = torch.as_tensor(
                f[k].reshape(-1), dtype=lat.dtype, device="cuda")
    return out, per


def _run_and_compare(cases, prec, launch, sampled, seed):
    import torch
    from paper_1003_0282_amd import lbaxi as L
    lat = L.Lattices(cases, prec)
    lat.set_launch(*launch)
    lat.set_graph_steps(8)
    fields, per = _packed_fields(lat, cases, sampled, seed)
    lat.seed(**fields)
    del fields
    lat.step(STEPS)
    m = lat.macros()
    finite = bool(torch.isfinite(m["uz"]).all()) and bool(torch.isfinite(m["rho"]).all())
    assert finite, "non-finite values in the batch"
    worst = 0.0
    for i in sampled:
        c = cases[i]
        o = oracle_run(c, STEPS, per[i])
        sl = slice(lat.offsets[i], lat.offsets[i + 1])
        gm = {k: v[sl].double().cpu().numpy().reshape(c["nr"], c["nz"]) for k, v in m.items()}
        e, _ = errors(c, gm, o.macros())
        worst = max(worst, max(e.values()))
        assert max(e.values()) < TOL[prec], (c["name"], launch, e)
    lat.close()
    print("worst relative error", worst)


def _sample(cases, extra, seed):
    sizes = [c["nz"] * c["nr"] for c in cases]
    rng = np.random.default_rng(seed)
    pick = {int(np.argmax(sizes)), int(np.argmin(sizes))}
    pick.update(int(k) for k in rng.choice(len(cases), size=extra, replace=False))
    return sorted(pick)


@pytest.mark.parametrize("launch", [(128, 1, 0, 0, 1), (256, 1, 0, 0, 1)])
def test_batch256_full_size(launch):
    """The default bench workload, FP32 storage, in the two shapes the
    autotuner picks for it."""
    cases = W.batch_cavities(256, seed=0)
    _run_and_compare(cases, 1, launch, _sample(cases, 3, 5), seed=11)


def test_melt512_full_size():
    cases = W.melt_set(512, seed=1)
    _run_and_compare(cases, 1, (256, 1, 0, 0, 1), _sample(cases, 2, 6), seed=12)


def test_roofline_pipe_full_size_fp64():
    """16384 x 2048 body-force pipe in FP64, every node compared."""
    _run_and_compare([W.roofline_pipe()], 0, (256, 1, 0, 0, 1), [0], seed=13)


def test_batch256_mrt_full_size():
    """The 256 cavities with the MRT collision (bench workload batch256_mrt)."""
    cases = [dict(c, mrt=True) for c in W.batch_cavities(256, seed=0)]
    _run_and_compare(cases, 1, (128, 1, 0, 0, 1), _sample(cases, 2, 7), seed=14)


def test_pipe_original_full_size_fp64():
    """The pipe under the original scheme (bench workload pipe_fp64_original),
    in the autotuner's shape for it, every node compared."""
    _run_and_compare([dict(W.roofline_pipe(), original=True)], 0, (512, 1, 0, 0, 0), [0],
                     seed=15)


def test_pipe_zou_he_full_size_fp64():
    """The pipe with wet-node Zou-He walls (bench workload pipe_fp64_zou_he)."""
    _run_and_compare([dict(W.roofline_pipe(), wet=True, zou_he=True)], 0, (256, 2, 0, 0, 1), [0],
                     seed=16)

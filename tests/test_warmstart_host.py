"""Host-side logic of the learned warm start: input channels, target
scaling, and the time-to-tolerance bookkeeping (no GPU needed)."""
import numpy as np

from paper_1003_0282_amd import warmstart as WS
from paper_1003_0282_amd import workloads as W


def test_features_layout():
    cases = W.melt_set(3, seed=4, nr=16, nz=32, re_max=250.0)
    x = WS.features(cases)
    assert x.shape == (3, 16, 32, WS.C_IN) and x.dtype == np.float32
    c = cases[1]
    # r / R_c grows along r, z / H along z
    assert x[1, 0, 5, 0] == 0.0 and np.isclose(x[1, 15, 5, 0], 15 / 15.5)
    assert np.isclose(x[1, 3, 31, 1], 31.5 / 32)
    assert np.allclose(x[1, ..., 2], c["Re_c"] / 1000) and np.allclose(x[1, ..., 3], c["Re_x"] / 1000)
    # crystal column: rows with r <= beta R_c
    rs = c["east"]["r_split"]
    assert (x[1, :, 0, 5] == (np.arange(16) <= rs)).all()
    assert np.allclose(x[1, ..., 6], x[1, ..., 2] * x[1, ..., 0])


def test_targets_roundtrip():
    rng = np.random.default_rng(0)
    B, nr, nz = 2, 4, 8
    f = {k: rng.standard_normal(B * nr * nz) for k in WS.FIELDS}
    f["T"] += 0.5
    f["rho"] = 1.0 + 0.01 * f["rho"]
    sc = WS.Scales.fit(f, 1.0, 0.5)
    y = WS.targets(f, sc, (B, nr, nz))
    assert y.shape == (B, nr, nz, WS.C_OUT) and WS.FIELDS[0] == "rho"
    for i, k in enumerate(WS.FIELDS):
        back = y[..., i].reshape(-1) * sc.s[i] + {"rho": 1.0, "T": 0.5}.get(k, 0.0)
        assert np.allclose(back, f[k], atol=1e-6)
        assert np.isclose(np.sqrt(np.mean(y[..., i].astype(np.float64) ** 2)), 1.0, rtol=1e-5)


def _solve(hist, wall):
    h = np.asarray(hist, dtype=float)
    return WS.Solve(np.zeros(h.shape[1], np.int32), np.zeros(h.shape[1], np.int64),
                    h[-1], wall[-1], {}, np.arange(1, len(h) + 1) * 1000, np.asarray(wall), h)


def test_time_to_tolerance_bookkeeping():
    nan = np.nan
    z = _solve([[1e-5, 1e-5, 1e-5], [1e-7, 1e-6, 1e-5], [5e-9, 2e-7, 1e-5], [nan, 5e-9, 1e-5]],
               [1.0, 2.0, 3.0, 4.0])
    w = _solve([[1e-6, 1e-5, 1e-5], [5e-9, 5e-9, 1e-5], [nan, nan, 1e-5], [nan, nan, 1e-5]],
               [1.5, 2.5, 3.5, 4.5])
    assert z.first_crossing(1e-8).tolist() == [2, 3, -1]
    assert w.first_crossing(1e-6).tolist() == [0, 1, -1]
    d6, d8 = WS.compare(z, w, 0.25, (1e-6, 1e-8))["residual"]
    assert d6["reached_both"] == 2 and d6["steps_zero"] == [2000, 2000] and d6["steps_nn"] == [1000, 2000]
    assert d8["reached_zero"] == 2 and d8["reached_nn"] == 2
    assert d8["steps_zero"] == [3000, 4000] and d8["steps_nn"] == [2000, 2000]
    assert np.isclose(d8["wall_zero_s"], 4.0) and np.isclose(d8["wall_nn_s"], 2.5 + 0.25)


def test_first_within_requires_staying_below():
    s = _solve([[1e-5, 1e-5], [1e-6, 1e-6], [1e-7, 1e-7]], [1.0, 2.0, 3.0])
    s.hist_err = np.array([[0.5, 0.5], [0.005, 0.2], [0.02, 0.004]])
    # instance 0 dips below 1% at check 1 but leaves again; instance 1 stays from check 2
    assert s.first_within(0.01).tolist() == [-1, 2]
    assert s.first_within(0.03).tolist() == [1, 2]
    assert s.first_within(1.0).tolist() == [0, 0]

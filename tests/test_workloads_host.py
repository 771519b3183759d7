"""The seeded benchmark workloads match their stated recipes."""
import numpy as np

from paper_1003_0282_amd import workloads as W


def test_batch_cavities_recipe():
    """256 cavities: Nr in [64, 512], H/R in [1, 3], Re in [500, 2500], the
    lid Reynolds number exact (Omega R^2 / nu = Re), tau_s >= 0.52, lid speed
    0.1 unless that would put tau_s lower, node count of seed 0."""
    cases = W.batch_cavities(256, seed=0)
    assert len(cases) == 256
    assert W.node_count(cases) == 56270414
    lifted = 0
    for c in cases:
        nr, nz = c["nr"], c["nz"]
        R = nr - 0.5
        assert 64 <= nr <= 512
        assert 1.0 - 1e-9 <= nz / R <= 3.0 + 1.0 / R
        assert 500.0 <= c["Re"] <= 2500.0
        nu = (c["tau"] - 0.5) / 3.0
        u_lid = c["east"]["omega"] * R
        assert abs(u_lid * R / nu - c["Re"]) < 1e-6 * c["Re"]
        assert c["tau"] >= 0.52 - 1e-12
        if u_lid > 0.1 + 1e-12:
            lifted += 1
            assert abs(c["tau"] - 0.52) < 1e-12
        else:
            assert abs(u_lid - 0.1) < 1e-12
    assert 0 < lifted < 64


def test_melt_set_recipe():
    cases = W.melt_set(64, seed=1)
    for c in cases:
        assert (c["nr"], c["nz"]) == (128, 256)
        assert 0.0 <= c["Re_c"] <= 1000.0 and 0.0 <= c["Re_x"] <= 1000.0
        assert 1e3 <= c["Gr"] <= 1e5
        assert c.get("swirl") and c.get("thermal")
    assert len({round(c["Gr"], 6) for c in cases}) == 64  # seeded, all distinct

"""The seeded input generators (no GPU): the geometry and case recipes that
both the oracle and the HIP library consume.  They hold none of the method's
arithmetic; these checks pin the recipes to their stated properties."""
import numpy as np
import pytest

import lbr_inputs as LI


def _area(xy):
    x, y = xy[:, 0], xy[:, 1]
    return 0.5 * np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y)


@pytest.mark.parametrize("seed", [0, 1, 7])
def test_airfoil_polyline_recipe(seed):
    xy = LI.airfoil_polyline(seed, n_side=512)
    assert xy.shape == (1024, 2)
    assert _area(xy) > 0                                       # counter-clockwise
    assert np.isclose(xy[:, 0].min(), 0.0, atol=1e-4) and np.isclose(xy[:, 0].max(), 1.0)
    thick = np.max(xy[:512, 1]) - np.min(xy[512:, 1])
    assert abs(thick - 0.12) < 2e-3                            # 12 % thick
    assert np.allclose(xy[0], (1.0, 0.0), atol=1e-12)          # sharp trailing edge
    # the same seed gives the same body, another seed another body
    assert np.array_equal(xy, LI.airfoil_polyline(seed, n_side=512))
    assert not np.allclose(xy, LI.airfoil_polyline(seed + 1, n_side=512))


def test_rotation_by_alpha_about_quarter_chord():
    xy = LI.airfoil_polyline(0, n_side=256)
    r = LI.rotate(xy, 10.0)
    assert np.allclose(np.linalg.norm(r - (0.25, 0.0), axis=1), np.linalg.norm(xy - (0.25, 0.0), axis=1))
    te = r[0]                                                  # nose up: trailing edge goes down
    assert te[1] < 0 and np.isclose(np.arctan2(-te[1], te[0] - 0.25), np.radians(10.0))


def test_three_element_bodies_keep_their_gaps():
    bodies = LI.three_element_polylines(0, n_side=256)
    assert len(bodies) == 3 and all(_area(b) > 0 for b in bodies)
    for i in range(3):
        for j in range(i + 1, 3):
            assert LI._min_distance(bodies[i], bodies[j]) >= 0.01


def test_sweep_cases_follow_the_recipe():
    alphas, levels = [], []
    for k in range(16):
        c = LI.case_sweep(k)
        alphas.append(c["alpha_deg"])
        levels.append(c["n_levels"])
        assert c["dx0"] * 2 ** -(c["n_levels"] - 1) == pytest.approx(1.0 / 512)   # finest c/512
        S = c["nx0"] * c["dx0"]
        assert 8.0 - 1e-9 <= S <= 20.0 + 1e-9 and 0.25 <= c["bands"][-1] <= 1.0
        assert 0.5e6 <= c["target_cells"] <= 4e6
        est = LI._estimate_cells(S, c["bands"][-1], c["n_levels"], 512)
        assert est == pytest.approx(c["cells_estimate"], rel=1e-9)
        # the target is met within 10 % unless it lies outside what the feasible
        # domains and bands give (three levels: an 8c domain at c/128 alone is
        # 1.27M cells; five levels: the level-1 band of a 20c domain caps it)
        lo, hi = c["feasible_cells"]
        if lo <= c["target_cells"] <= hi:
            assert abs(est / c["target_cells"] - 1) <= 0.10
        else:
            assert est == pytest.approx(lo if c["target_cells"] < lo else hi, rel=1e-9)
    assert np.allclose(alphas, [-4 + 4 * k / 3 for k in range(16)])
    assert levels == [3 + k % 3 for k in range(16)]

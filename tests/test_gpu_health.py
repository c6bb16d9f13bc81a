"""Health check of lbr_advance and the convergence status of a run to steady
state (needs an MI355X)."""
import numpy as np
import pytest

import lbr_inputs as LI
import paper_2601_18443_amd as P
from tests import parity_util as U

pytestmark = pytest.mark.gpu


def _fields(s, n_levels):
    return [s.field(l, f) for l in range(n_levels) for f in (0, 1, 2, 3)]


def test_scans_leave_the_state_untouched():
    """With a scan after every fifth coarse step the fields are bit-identical to a
    run without scans, and a healthy run reports no failure."""
    case = LI.case_airfoil_small()
    a = U.gpu_solver(case, "f32")
    b = U.gpu_solver(dict(case, health_every=5), "f32")
    for s in (a, b):
        s.use_graph(True)
        s.advance(7)
        s.advance(6)
    for x, y in zip(_fields(a, case["n_levels"]), _fields(b, case["n_levels"])):
        assert np.array_equal(x, y, equal_nan=True)


def test_a_non_finite_cell_is_reported_as_divergence():
    """A NaN density planted at one level-0 cell through the initial state is found
    by the first scan: LBR_ERR_DIVERGED, with the level in the message."""
    case = dict(LI.case_airfoil_small(), health_every=1)
    g = U.gpu_solver(case, "f64")
    inf = g.level_info(0)
    rho = np.ones((inf["ny"], inf["nx"]))
    types = g.field(0, P.FIELD_TYPE)
    j, i = np.argwhere(types == 1)[len(np.argwhere(types == 1)) // 3]
    rho[j, i] = np.nan
    g.init(0, rho=rho)
    with pytest.raises(P.LbrError) as e:
        g.advance(1)
    assert "error -5" in str(e.value) and "health check" in str(e.value) and "level 0" in str(e.value)


def test_run_to_steady_reports_a_run_that_did_not_converge():
    """A tolerance the run cannot reach within its step limit gives
    LBR_ERR_NOT_CONVERGED (not raised by the binding): the steps and the last
    residual are still returned; a reachable tolerance converges."""
    case = LI.case_airfoil_small()
    g = U.gpu_solver(case, "f32")
    steps, r = g.run_to_steady(1e-30, 40, 20)
    assert steps == 40 and r > 1e-30 and not g.converged
    steps, r = g.run_to_steady(1.0, 40, 20)
    assert steps == 20 and r < 1.0 and g.converged

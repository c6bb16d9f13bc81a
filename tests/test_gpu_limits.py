"""Size edge cases on the GPU (needs an MI355X).

lbr_build refuses a level whose storage box is too large for the 32-bit
buffer addressing of the step kernels (about 29.8M cells).  The largest box it
accepts must step like a small one: a channel that is uniform in x advances
every column alike, so a 28M-cell channel is compared, column by column, with
a 64-column channel of the same height, which is itself compared with the
oracle.
"""
import numpy as np
import pytest

import lbr_inputs as LI
import oracle
import paper_2601_18443_amd as P
from tests import parity_util as U

pytestmark = pytest.mark.gpu

NY = 3500           # with 8000 columns: a storage box of 8064 x 3504 = 28.3M cells


def _laminar(case):
    """The channel's laminar start without its noise: uniform in x."""
    ny, nx = case["ny0"], case["nx0"]
    h = 0.5 * ny
    y = np.arange(ny) + 0.5
    prof = 1.5 * case["u_ref"] * (1.0 - ((y - h) / h) ** 2)
    ux = np.ascontiguousarray(np.tile(prof[:, None], (1, nx)))
    return dict(rho=np.ones_like(ux), ux=ux, uy=np.zeros_like(ux), chi=np.full_like(ux, case["chi_init"]))


def _run(sim, case, steps):
    sim.init(0, **_laminar(case))
    sim.advance(steps)
    return [sim.field(0, f) for f in range(4)]


def test_largest_level_box_steps_like_a_narrow_one():
    steps = 3
    narrow, wide = LI.case_channel(nx=64, ny=NY), LI.case_channel(nx=8000, ny=NY)
    o = oracle.Sim(narrow)
    ref = _run(o, narrow, steps)
    g = U.gpu_solver(narrow, "f32")
    small = _run(g, narrow, steps)
    g.close()
    # the narrow channel against the oracle, cell by cell (FP32 bounds: u within
    # 1e-5 U, chi within 1e-5 of its largest value, rho within 1e-6)
    assert np.array_equal(np.isfinite(small[1]), np.isfinite(ref[1]))
    m = np.isfinite(ref[1])
    assert np.max(np.abs(small[1][m] - ref[1][m])) < 1e-5 * narrow["u_ref"]
    assert np.max(np.abs(small[3][m] - ref[3][m])) < 1e-5 * np.max(np.abs(ref[3][m]))
    assert np.max(np.abs(small[0][m] - ref[0][m])) < 1e-6
    w = U.gpu_solver(wide, "f32")
    assert w.level_info(0)["nx"] == 8000
    big = _run(w, wide, steps)
    w.close()
    # every column of both channels equals the first column of the narrow one
    for f in range(4):
        col = small[f][:, :1]
        assert np.all(np.isfinite(col)), f
        np.testing.assert_allclose(small[f], np.broadcast_to(col, small[f].shape), rtol=1e-6, atol=1e-12)
        np.testing.assert_allclose(big[f], np.broadcast_to(col, big[f].shape), rtol=1e-6, atol=1e-12)


def test_level_box_past_the_addressing_limit_is_refused():
    with pytest.raises(P.LbrError, match="per-array limit"):
        U.gpu_solver(LI.case_channel(nx=8192, ny=4096), "f32")


def test_level_box_past_the_tile_index_range_is_refused():
    """4.5M cells, well inside the byte limit, but 70,004 rows: more 2-row tile
    rows than a 15-bit index holds."""
    with pytest.raises(P.LbrError, match="tile index range"):
        U.gpu_solver(LI.case_channel(nx=64, ny=70000), "f32")

"""Precomputed cut-link input of the HIP library against the oracle (needs an
MI355X).  Section 2.1 has the preprocessor hand over the geometry and the
cut-link list; Section 2.3 defines the link-wise wall data each boundary node
carries (IW, the normal, d_WB, q per cut link).  A seeded perturbation of the
oracle's own lists stands in for another preprocessor's output: both codes read
the same cut-link file, and the library must use it exactly as the oracle does
(element-wise FP64 bounds of the parity tests), and a list it reads back from
itself must reproduce its generated run bit for bit."""
import numpy as np
import pytest

import lbr_inputs as LI
import oracle
from tests import parity_util as U

pytestmark = pytest.mark.gpu

TOL64, RHO64 = 1e-10, 1e-12
CUT_COLS = (0, 1, 2, 3, 4, 5, 6, 15) + tuple(range(19, 27))


def _check64(g, o, case, level):
    U.assert_fields_match(g, o, case, TOL64, RHO64)
    U.assert_walls_match(g, o, level, 1e-10, RHO64, U.reference_speed(case))


def _perturbed_file(tmp_path, case, level, seed):
    rec = LI.perturbed_cut_links(LI.cut_link_records(oracle.Sim(case).wall(level)), seed=seed)
    path = tmp_path / f"{case['name']}_{level}.cut"
    LI.write_cut_links(path, {level: rec}, comment=f"seeded perturbation {seed} of the generated list")
    return path, rec


def test_perturbed_list_on_the_airfoil_fp64(tmp_path):
    """Small airfoil (3 levels, finest c/64): the finest level's nodes from a
    perturbed list.  Structure and wall records as supplied; fields, wall
    records, surface and forces after one and after four coarse steps within
    the FP64 bounds."""
    case = LI.case_airfoil_small()
    lf = case["n_levels"] - 1
    path, rec = _perturbed_file(tmp_path, case, lf, seed=3)
    o = oracle.Sim(case, cut_links=path)
    g = U.gpu_solver_links(case, "f64", path)
    assert U.structure_mismatch(g, o, case["n_levels"]) == []
    np.testing.assert_array_equal(g.wall(lf)[:, CUT_COLS], rec)
    for steps in (1, 3):
        o.advance(steps)
        g.advance(steps)
        _check64(g, o, case, lf)
        np.testing.assert_allclose(g.forces(), o.forces(), rtol=1e-9, atol=1e-12)
        U.assert_surface_match(g, o, 0, 1e-9, 1e-9)


def test_perturbed_list_on_the_channel_walls_fp64(tmp_path):
    """Plane channel with the VN wall model: the level-0 nodes of both channel
    walls (bodies -1 and -2) from a perturbed list; fields and wall records
    after 20 steps within the FP64 bounds."""
    case = LI.case_channel(nx=64, ny=32)
    path, rec = _perturbed_file(tmp_path, case, 0, seed=11)
    assert set(np.unique(rec[:, 7])) == {-1.0, -2.0}
    o = oracle.Sim(case, cut_links=path)
    g = U.gpu_solver_links(case, "f64", path)
    assert U.structure_mismatch(g, o, 1) == []
    U.channel_init(case, (o, g))
    o.advance(20)
    g.advance(20)
    _check64(g, o, case, 0)


def test_list_read_back_from_the_library_is_bit_identical_fp32():
    """The library's own finest-level records handed back through
    lbr_set_cut_links (arrays, no file) give the same grid and, three coarse
    steps later, bit-identical FP32 fields and wall records."""
    case = LI.case_airfoil_small()
    lf = case["n_levels"] - 1
    a = U.gpu_solver(case, "f32")
    rec = LI.cut_link_records(a.wall(lf))
    b = U.gpu_solver_links(case, "f32", {lf: rec})
    for l in range(case["n_levels"]):
        assert a.level_info(l) == b.level_info(l)
    a.advance(3)
    b.advance(3)
    for l in range(case["n_levels"]):
        for f in range(4):
            np.testing.assert_array_equal(a.field(l, f), b.field(l, f))
    np.testing.assert_array_equal(a.wall(lf), b.wall(lf))


def test_build_refuses_lists_that_do_not_fit_the_grid():
    """lbr_build checks a list against the level's cells: a node on a solid
    cell, a body index that names no body, and a link into a solid cell that
    the list leaves uncut are refused with LBR_ERR_GEOMETRY; a list given
    after lbr_build is refused with LBR_ERR_STATE."""
    import paper_2601_18443_amd as P
    case = LI.case_airfoil_small()
    lf = case["n_levels"] - 1
    ref = U.gpu_solver(case, "f32")
    rec = LI.cut_link_records(ref.wall(lf))
    t = ref.field(lf, 5)
    inf = ref.level_info(lf)
    solid = np.argwhere(t == P.CELL_SOLID)[0]
    on_solid = rec.copy()
    on_solid[0, 0], on_solid[0, 1] = solid[1] + inf["gx0"], solid[0] + inf["gy0"]
    no_body = rec.copy()
    no_body[0, 7] = 5
    for bad, word in ((on_solid, "not an owned fluid cell"), (no_body, "names no body"),
                      (rec[1:], "not a cut link of the list")):
        with pytest.raises(P.LbrError, match=word):
            U.gpu_solver_links(case, "f32", {lf: bad})
    r = np.ascontiguousarray(rec)
    assert P.lib().lbr_set_cut_links(ref.h, lf, len(r), U.dptr(r)) == P.ERR_STATE

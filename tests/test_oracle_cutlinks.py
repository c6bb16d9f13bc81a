"""Pins of the oracle's precomputed cut-link input (Section 2.1: the preprocessor
hands the solver the geometry and the cut-link list; Section 2.3: per boundary
node B the wall point IW, the normal, d_WB and the wall fraction q of every cut
link): a list takes the place of the polyline intersections and is used as
given."""
import numpy as np
import pytest

import lbr_inputs as LI
import oracle

WALL_COLS = (0, 1, 2, 3, 4, 5, 6, 15) + tuple(range(19, 27))


def _channel(ny, **kw):
    c = LI.case_channel(nx=4, ny=ny)
    c.update(wall_model=LI.WALL_NOSLIP, sa_mode=LI.SA_FROZEN, chi_init=0.0, nu0=0.1,
             force=(1e-6, 0.0), u_ref=0.0, bb_mode=LI.BB_YU)
    c.update(kw)
    return c


def _steady_u(sim, ny, steps):
    sim.init(0, rho=np.ones((ny, 4)), ux=np.zeros((ny, 4)), uy=np.zeros((ny, 4)),
             chi=np.zeros((ny, 4)))
    sim.advance(steps)
    return sim.field(0, oracle.F_UX)[:, 0]


def test_generated_list_read_back_reproduces_the_run(tmp_path):
    """The oracle's own boundary nodes of the finest level, written to a cut-link
    file and read back in place of the polylines' intersections, give the same
    wall records and, two coarse steps later, the same fields bit for bit."""
    case = LI.case_airfoil_small()
    lf = case["n_levels"] - 1
    a = oracle.Sim(case)
    rec = LI.cut_link_records(a.wall(lf))
    assert len(rec) > 100
    path = tmp_path / "airfoil.cut"
    LI.write_cut_links(path, {lf: rec}, comment="finest-level nodes of the small airfoil")
    b = oracle.Sim(case, cut_links=path)
    for l in range(case["n_levels"]):
        assert a.level_info(l) == b.level_info(l)
    np.testing.assert_array_equal(b.wall(lf)[:, WALL_COLS], rec)
    a.advance(2)
    b.advance(2)
    for l in range(case["n_levels"]):
        for f in (oracle.F_RHO, oracle.F_UX, oracle.F_UY, oracle.F_CHI):
            np.testing.assert_array_equal(a.field(l, f), b.field(l, f))
    np.testing.assert_array_equal(a.wall(lf), b.wall(lf))


def test_supplied_records_are_used_as_given(tmp_path):
    """A perturbed list (another preprocessor's q, IW, normal and d_WB) is echoed
    unchanged in the wall records, and it changes the flow next to the wall."""
    case = LI.case_airfoil_small()
    lf = case["n_levels"] - 1
    a = oracle.Sim(case)
    rec = LI.perturbed_cut_links(LI.cut_link_records(a.wall(lf)), seed=3)
    path = tmp_path / "perturbed.cut"
    LI.write_cut_links(path, {lf: rec})
    b = oracle.Sim(case, cut_links=path)
    np.testing.assert_array_equal(b.wall(lf)[:, WALL_COLS], rec)
    assert b.level_info(lf)["n_cut"] == int((rec[:, 8:] >= 0).sum())
    a.advance(1)
    b.advance(1)
    d = np.nanmax(np.abs(a.field(lf, oracle.F_UX) - b.field(lf, oracle.F_UX)))
    assert d > 1e-6


@pytest.mark.parametrize("q_lo,q_hi", [(0.3, 0.8), (0.9, 0.15)])
def test_list_that_moves_the_walls_gives_that_poiseuille_profile(tmp_path, q_lo, q_hi):
    """Channel generated with its walls half a cell from the first and last cell
    centres (q = 1/2), run with a list whose q place the walls at
    y_lo = 1/2 - q_lo and y_hi = ny - 1/2 + q_hi instead: the steady profile is
    the parabola between those walls, F (y - y_lo)(y_hi - y) / (2 nu), within the
    error of Yu's interpolated bounce-back at ny = 16, and it is the profile of
    the channel generated with the walls there."""
    ny, nu, F = 16, 0.1, 1e-6
    base = _channel(ny, wall_y=(0.0, float(ny)))
    rec = LI.cut_link_records(oracle.Sim(base).wall(0))
    assert len(rec) == 8 and np.all(rec[:, 8:][rec[:, 8:] >= 0] == 0.5)
    q = rec[:, 8:]
    lower = rec[:, 1] == 0
    for o in (4, 6, 7):                  # links with c_y = -1 cross the lower wall
        q[lower & (q[:, o - 1] >= 0), o - 1] = q_lo
    for o in (3, 5, 8):                  # c_y = +1: the upper wall
        q[~lower & (q[:, o - 1] >= 0), o - 1] = q_hi
    path = tmp_path / "channel.cut"
    LI.write_cut_links(path, {0: rec})
    steps = int(60 * ny * ny)
    u = _steady_u(oracle.Sim(base, cut_links=path), ny, steps)
    y = np.arange(ny) + 0.5
    ylo, yhi = 0.5 - q_lo, ny - 0.5 + q_hi
    exact = F / (2 * nu) * (y - ylo) * (yhi - y)
    assert np.sqrt(np.mean((u - exact) ** 2)) / exact.max() < 0.02
    u_gen = _steady_u(oracle.Sim(_channel(ny, wall_y=(ylo, yhi))), ny, steps)
    np.testing.assert_allclose(u, u_gen, rtol=1e-9, atol=1e-12 * exact.max())


def _refused(case, path, match):
    with pytest.raises(RuntimeError, match=match):
        oracle.Sim(case, cut_links=path)


def test_lists_that_leave_a_wall_link_open_are_refused(tmp_path):
    case = LI.case_airfoil_small()
    lf = case["n_levels"] - 1
    sim = oracle.Sim(case)
    rec = LI.cut_link_records(sim.wall(lf))
    t = sim.field(lf, oracle.F_TYPE)
    inf = sim.level_info(lf)
    # a node whose cut link ends in a solid cell loses that link
    cx = [0, 1, -1, 0, 0, 1, -1, 1, -1]
    cy = [0, 0, 0, 1, -1, 1, -1, -1, 1]
    bad = rec.copy()
    done = False
    for r in range(len(bad)):
        i, j = int(bad[r, 0]) - inf["gx0"], int(bad[r, 1]) - inf["gy0"]
        for o in range(1, 9):
            if bad[r, 7 + o] >= 0 and t[j + cy[o], i + cx[o]] == oracle.T_SOLID and (bad[r, 8:] >= 0).sum() > 1:
                bad[r, 7 + o] = -1.0
                done = True
                break
        if done:
            break
    assert done
    p = tmp_path / "open.cut"
    LI.write_cut_links(p, {lf: bad})
    _refused(case, p, "not listed")
    # a node dropped altogether
    p = tmp_path / "dropped.cut"
    LI.write_cut_links(p, {lf: rec[1:]})
    _refused(case, p, "not listed")


def test_malformed_lists_are_refused(tmp_path):
    case = LI.case_airfoil_small()
    lf = case["n_levels"] - 1
    rec = LI.cut_link_records(oracle.Sim(case).wall(lf))
    cases = (
        ("twice", np.concatenate([rec, rec[:1]]), "listed twice"),
        ("q_range", _with(rec, 0, 8 + int(np.argmax(rec[0, 8:] >= 0)), 1.5), r"outside \(0, 1\]"),
        ("no_cut", _with(rec, 0, slice(8, 16), -1.0), "no cut link"),
        ("not_unit", _with(rec, 0, 4, 2.0), "normal"),
        ("solid_cell", _with(rec, 0, 0, rec[0, 0] + 200), "not a fluid cell"),
    )
    for name, r, match in cases:
        p = tmp_path / (name + ".cut")
        LI.write_cut_links(p, {lf: r})
        _refused(case, p, match)
    p = tmp_path / "truncated.cut"
    LI.write_cut_links(p, {lf: rec})
    text = open(p).read()
    open(p, "w").write(text[: len(text) // 2])
    _refused(case, p, "truncated")
    p = tmp_path / "header.cut"
    open(p, "w").write("cut-links 1\n")
    _refused(case, p, "not a cut-link file")
    _refused(case, tmp_path / "missing.cut", "cannot open")


def _with(rec, row, col, value):
    r = rec.copy()
    r[row, col] = value
    return r

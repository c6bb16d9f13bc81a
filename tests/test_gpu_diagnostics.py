"""Output diagnostics of the HIP library against the FP64 oracle's state (needs
an MI355X): the y+ of the R, B and V points of every wall node (Section 3.1.3,
Figure 6) and rakes of velocity and eddy-viscosity ratio (Section 3.1.4,
Figure 10).

Both are defined from quantities the oracle reports: y+ = u_tau y / nu with
u_tau from the oracle's wall records, y the wall distance of the point and
nu = nu_0 2^l (nu_0 = U c / Re in level-0 lattice units); a rake point takes
the values of the owned fluid cell of the finest level that contains it,
evaluated here on the oracle's fields.  FP64 storage; after five coarse steps
the two states agree to about 1e-12, hence the 1e-9 bounds.
"""
import math

import numpy as np
import pytest

import lbr_inputs as LI
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pair():
    import paper_2601_18443_amd as P
    case = LI.case_airfoil_small()
    g = P.Solver(case, storage="f64")
    o = oracle.Sim(case)
    g.advance(5)
    o.advance(5)
    return case, g, o


def test_wall_yplus_of_r_b_and_v(pair):
    case, g, o = pair
    U = case["mach"] / math.sqrt(3.0)
    nu0 = U * (case["ref_length"] / case["dx0"]) / case["reynolds"]
    seen = 0
    for lvl in range(case["n_levels"]):
        wo = o.wall(lvl)
        y = g.wall_yplus(lvl)
        assert y.shape == (len(wo), 3)
        if len(wo) == 0:
            continue
        seen += len(wo)
        nu = nu0 * 2 ** lvl
        utau, dwb = wo[:, 8], wo[:, 6]
        expect = np.stack([utau * case["d_wr"] / nu, utau * dwb / nu, utau * case["d_wv"] / nu], axis=1)
        assert np.allclose(y, expect, rtol=1e-9, atol=1e-12)
        # B lies between the wall and R (d_WB < d_WR), V nearer the wall than R
        assert np.all(y[:, 1] <= y[:, 0] + 1e-12) and np.all(y[:, 2] <= y[:, 0])
    assert seen > 0


def test_surface_yplus_of_v_at_the_segment_centroids(pair):
    """lbr_surface_yplus: y+ of V along the surface (Section 3.1.3, Figure 6) at
    the segment centroids, interpolated as Cp and Cf are after eq (30): from the
    two wall nodes nearest to the centroid, weighted by inverse squared distance
    (a node on the centroid alone).  Rebuilt here from the oracle's wall records
    (u_tau, IW, body) and the body's polyline."""
    case, g, o = pair
    lf = case["n_levels"] - 1
    U = case["mach"] / math.sqrt(3.0)
    nu = U * (case["ref_length"] / case["dx0"]) / case["reynolds"] * 2 ** lf
    wo = o.wall(lf)
    mine = wo[wo[:, 15] == 0]                       # column 15: the body
    yv_node = mine[:, 8] * case["d_wv"] / nu
    dx = case["dx0"] / 2 ** lf
    xy = (np.asarray(case["bodies"][0]) - np.asarray(case["origin"])) / dx
    mid = 0.5 * (xy + np.roll(xy, -1, axis=0))
    expect = np.empty(len(mid))
    for k, (mx, my) in enumerate(mid):
        d2 = (mine[:, 2] - mx) ** 2 + (mine[:, 3] - my) ** 2
        a, b = np.argsort(d2, kind="stable")[:2]
        if d2[a] < 1e-24:
            expect[k] = yv_node[a]
        else:
            expect[k] = (yv_node[a] / d2[a] + yv_node[b] / d2[b]) / (1.0 / d2[a] + 1.0 / d2[b])
    got = g.surface_yplus(0)
    assert got.shape == expect.shape
    np.testing.assert_allclose(got, expect, rtol=1e-9, atol=1e-12)
    assert np.all(got > 0)


def _oracle_rake(case, o, p0, p1, n):
    out = np.full((n, 5), np.nan)
    out[:, 0] = -1
    ox, oy = case["origin"]
    fields = {lvl: [o.field(lvl, f) for f in (oracle.F_RHO, oracle.F_UX, oracle.F_UY, oracle.F_CHI)]
              for lvl in range(case["n_levels"])}
    info = {lvl: o.level_info(lvl) for lvl in range(case["n_levels"])}
    U = case["mach"] / math.sqrt(3.0)
    for k in range(n):
        t = k / (n - 1)
        x, y = p0[0] + t * (p1[0] - p0[0]), p0[1] + t * (p1[1] - p0[1])
        for lvl in reversed(range(case["n_levels"])):
            dx = case["dx0"] / 2 ** lvl
            i, j = math.floor((x - ox) / dx), math.floor((y - oy) / dx)
            li = info[lvl]
            a, b = i - li["gx0"], j - li["gy0"]
            if not (0 <= a < li["nx"] and 0 <= b < li["ny"]):
                continue
            rho, ux, uy, chi = (f[b, a] for f in fields[lvl])
            if not np.isfinite(ux):                      # not an owned fluid cell of this level
                continue
            nut = chi ** 4 / (chi ** 3 + 7.1 ** 3) if chi > 0 else 0.0
            out[k] = (lvl, ux / U, uy / U, nut, rho)
            break
    return out


def test_rake_through_the_body_and_its_boundary_layer(pair):
    case, g, o = pair
    p0, p1, n = (0.5, -0.4), (0.5, 0.9), 261          # crosses the body at mid-chord
    r = g.rake(p0, p1, n)
    ref = _oracle_rake(case, o, p0, p1, n)
    assert np.array_equal(r[:, 0], ref[:, 0])              # same level (or solid) per point
    inside = r[:, 0] < 0
    assert inside.any() and (~inside).any()
    assert np.all(np.isnan(r[inside, 1:]))
    assert np.allclose(r[~inside, 1:], ref[~inside, 1:], rtol=1e-9, atol=1e-12)
    # several levels are crossed, the finest next to the body
    assert len(set(r[~inside, 0])) >= 2

"""Helpers that drive the oracle and the HIP library on identical seeded inputs."""
import numpy as np

import lbr_inputs as LI
import oracle

FIELDS = {"rho": (oracle.F_RHO, 0), "ux": (oracle.F_UX, 1), "uy": (oracle.F_UY, 2),
          "chi": (oracle.F_CHI, 3)}


def gpu_solver(case, storage):
    import paper_2601_18443_amd as P
    return P.Solver(case, storage=storage)


def gpu_solver_links(case, storage, cut_links):
    """A library context whose cut links come from a file path or {level: records}."""
    import paper_2601_18443_amd as P
    return P.Solver(case, storage=storage, cut_links=cut_links)


def dptr(a):
    import ctypes as C
    return a.ctypes.data_as(C.POINTER(C.c_double))


def channel_init(case, sims):
    ux, uy = LI.channel_initial_velocity(case)
    rho = np.ones_like(ux)
    chi = np.full_like(ux, case["chi_init"])
    for s in sims:
        s.init(0, rho=rho, ux=ux, uy=uy, chi=chi)


def rel_l2(a, b):
    m = np.isfinite(a) & np.isfinite(b)
    assert np.array_equal(np.isfinite(a), np.isfinite(b)), "different fluid masks"
    den = np.sqrt(np.sum(b[m] ** 2))
    return np.sqrt(np.sum((a[m] - b[m]) ** 2)) / (den if den > 0 else 1.0)


def field_errors(g, o, n_levels, names=("rho", "ux", "uy", "chi")):
    out = {}
    for l in range(n_levels):
        for name in names:
            fo, fg = FIELDS[name]
            a = g.field(l, fg)
            b = o.field(l, fo)
            if name == "rho":
                a, b = a - 1.0, b - 1.0          # compare the density deviation
            out[(l, name)] = rel_l2(a, b)
    return out


def density_error(g, o, n_levels):
    """Largest absolute density difference over all levels."""
    worst = 0.0
    for l in range(n_levels):
        a, b = g.field(l, 0), o.field(l, oracle.F_RHO)
        m = np.isfinite(b)
        assert np.array_equal(np.isfinite(a), m), "different fluid masks"
        worst = max(worst, float(np.max(np.abs(a[m] - b[m]))))
    return worst


def reference_speed(case):
    """The case's reference velocity in lattice units (the same on every level under
    acoustic scaling): the scale of the element-wise velocity bounds."""
    u = case.get("u_ref", 0.0)
    return u if u > 0 else case["mach"] / np.sqrt(3.0)


def level_errors(g, o, n_levels, u_scale):
    """Per level, the largest element-wise differences over the owned fluid cells:
    |du_x| / U and |du_y| / U (U the reference speed; u itself may vanish),
    |dchi| / max(|chi|, 1) per cell ("chi") and |dchi| / max |chi| of the level
    ("chi_level"; chi = nu~ / nu is of order 1 in the free stream and grows to
    1e2-1e3 in boundary layers and wakes), and |drho| (rho is about 1)."""
    out = {}
    for l in range(n_levels):
        e = {}
        for name in ("ux", "uy", "chi", "rho"):
            fo, fg = FIELDS[name]
            a, b = g.field(l, fg), o.field(l, fo)
            m = np.isfinite(b)
            assert np.array_equal(np.isfinite(a), m), ("different fluid masks", l, name)
            if not m.any():
                e[name] = 0.0
                if name == "chi":
                    e["chi_level"] = 0.0
                continue
            d = np.abs(a[m] - b[m])
            if name in ("ux", "uy"):
                d = d / u_scale
            elif name == "chi":
                e["chi_level"] = float(d.max() / max(float(np.abs(b[m]).max()), 1.0))
                d = d / np.maximum(np.abs(b[m]), 1.0)
            e[name] = float(d.max())
        out[l] = e
    return out


def assert_fields_match(g, o, case, tol, rho_tol, chi_scale="cell"):
    """Every owned fluid cell of every level: velocity within tol x U, density
    within rho_tol, chi within tol x max(|chi|, 1) of the cell (chi_scale "cell")
    or within tol x the level's largest |chi| (chi_scale "level"); returns the
    errors."""
    L = case["n_levels"]
    errs = level_errors(g, o, L, reference_speed(case))
    skip = "chi" if chi_scale == "level" else "chi_level"
    bad = {(l, k): v for l, e in errs.items() for k, v in e.items()
           if k != skip and (v > (rho_tol if k == "rho" else tol) or not np.isfinite(v))}
    assert not bad, f"element-wise bounds exceeded (tol {tol}, rho {rho_tol}): {bad}; all: {errs}"
    return errs


def assert_walls_match(g, o, level, rtol, rho_tol, u_scale):
    """Wall records of one level node by node: u_tau relative, the slip velocity
    against U, and rho_W absolute."""
    wo, wg = o.wall(level), g.wall(level)
    assert len(wo) == len(wg)
    assert np.array_equal(wo[:, :2], wg[:, :2])
    np.testing.assert_allclose(wg[:, 8], wo[:, 8], rtol=rtol, atol=rtol * 1e-3 * u_scale)   # u_tau
    np.testing.assert_allclose(wg[:, 9:11] / u_scale, wo[:, 9:11] / u_scale, rtol=0, atol=rtol)  # u_W
    np.testing.assert_allclose(wg[:, 11], wo[:, 11], rtol=0, atol=rho_tol)         # rho_W


def assert_surface_match(g, o, body, cp_tol, cf_tol):
    """Segment by segment: Cp within cp_tol, Cf within cf_tol x max |Cf| of the body."""
    (cpg, cfg), (cpo, cfo) = g.surface(body), o.surface(body)
    np.testing.assert_allclose(cpg, cpo, rtol=0, atol=cp_tol)
    np.testing.assert_allclose(cfg, cfo, rtol=0, atol=cf_tol * np.max(np.abs(cfo)))


def velocity_error(g, o, n_levels):
    """Relative L2 error of the velocity vector over all levels (area weighted);
    a summary figure only: the bounds are element-wise (assert_fields_match)."""
    num = den = 0.0
    for l in range(n_levels):
        w = 4.0 ** -l
        for fo, fg in ((oracle.F_UX, 1), (oracle.F_UY, 2)):
            a, b = g.field(l, fg), o.field(l, fo)
            m = np.isfinite(b)
            num += w * np.sum((a[m] - b[m]) ** 2)
            den += w * np.sum(b[m] ** 2)
    return np.sqrt(num / den)


def structure_mismatch(g, o, n_levels, nx0=None):
    """Returns a list of differences in the grid and wall data built independently by both.

    Integers must agree exactly.  Positions, distances and link fractions are FP64
    values computed from lattice coordinates of up to the level's domain size L
    cells, so both codes round them at about L * 2^-52; they must agree within
    16 of those units (and 1e-11 at least).
    """
    bad = []
    for l in range(n_levels):
        size = (nx0 or 0) << l
        tol = max(1e-11, 16 * size * 2.0**-52)
        gi, oi = g.level_info(l), o.level_info(l)
        for k, gk in (("gx0", "gx0"), ("gy0", "gy0"), ("nx", "nx"), ("ny", "ny"),
                      ("n_fluid", "n_fluid"), ("n_bnodes", "n_wall_nodes"),
                      ("n_cut", "n_cut_links"), ("n_ghost", "n_ghost")):
            if oi[k] != gi[gk]:
                bad.append((l, k, oi[k], gi[gk]))
        if bad:
            continue
        to = o.field(l, oracle.F_TYPE)
        to = np.where(to == 5, 0, to)
        tg = g.field(l, 5)
        if not np.array_equal(to, tg):
            bad.append((l, "type", int(np.sum(to != tg))))
        do, dg = o.field(l, oracle.F_DIST), g.field(l, 6)
        m = np.isfinite(do) & (do < 1e200)
        if not np.allclose(do[m], dg[m], rtol=1e-12, atol=tol):
            bad.append((l, "dist", float(np.max(np.abs(do[m] - dg[m])))))
        wo, wg = o.wall(l), g.wall(l)
        if len(wo) != len(wg):
            bad.append((l, "wall count", len(wo), len(wg)))
            continue
        if len(wo):
            if not np.array_equal(wo[:, :2], wg[:, :2]):
                bad.append((l, "wall cells"))
            for cols, name in (((2, 3), "IW"), ((4, 5), "normal"), ((6,), "d_WB")):
                if not np.allclose(wo[:, cols], wg[:, cols], rtol=1e-11, atol=tol):
                    bad.append((l, name, float(np.max(np.abs(wo[:, cols] - wg[:, cols])))))
            if not np.array_equal(wo[:, 19:27] < 0, wg[:, 19:27] < 0):
                bad.append((l, "cut links"))
            elif not np.allclose(wo[:, 19:27], wg[:, 19:27], rtol=1e-11, atol=tol):
                bad.append((l, "q", float(np.max(np.abs(wo[:, 19:27] - wg[:, 19:27])))))
    return bad

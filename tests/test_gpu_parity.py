"""HIP library vs. the FP64 oracle on the same seeded inputs (needs an MI355X).

Every comparison is element by element, per level, over the owned fluid cells
(tests/parity_util.py): |du_x| and |du_y| against the reference speed U,
|dchi| against max(|chi|, 1), |drho| absolute; wall records node by node and
surface Cp, Cf segment by segment.

Tolerances:
  * FP64 storage and arithmetic: 1e-10 on u / U and chi, 1e-12 on rho.  The two
    codes differ by rounding order only (the GPU uses a closed-form
    central-moment collision in shifted variables, the oracle solves with the
    transfer matrix of eq. (6)): about 1e-16 per operation, amplified by at most
    1 / (tau - 1/2) ~ 1e4 where the relaxation is slowest, over a few thousand
    steps.
  * FP32 (spec bound): 1e-5 of the field's scale: u against U, chi
    against the level's largest |chi|; rho within 1e-6, u_tau to 1e-5 relative,
    Cp to (2 c_s^2 / U^2) 1e-6 and Cf to 3e-5 max |Cf| (both follow from the rho_W
    and u_tau bounds through eq. (29)).  Chi is measured against its field scale,
    not cell by cell, because every step adds the velocity's rounding error times
    the chi gradient through the convection term, and next to the wall that
    gradient is of the order of the wall value chi_B = kappa y_B+ per cell: with
    an FP32 velocity error of about 1e-7 (1e-6 U) and chi_B ~ 1e2, two coarse
    steps (256 steps of the finest level) leave absolute chi errors of a few
    1e-4 where chi itself is of order 1 (measured: 3e-4 on the benchmark
    airfoil, one to three cells off the wall; the wall values themselves agree
    to 1e-6), i.e. about 1e-6 of the level's largest chi.
  * Grid, cut links and wall records are built independently by both sides
    and must agree exactly (integers) or to 1e-11 (positions, q).
"""
import numpy as np
import pytest

import lbr_inputs as LI
import oracle
from tests import parity_util as U

pytestmark = pytest.mark.gpu

TOL64, RHO64 = 1e-10, 1e-12
TOL32, RHO32 = 1e-5, 1e-6


def _pair(case, storage):
    o = oracle.Sim(case)
    g = U.gpu_solver(case, storage)
    return o, g


def _check64(g, o, case, walls=True, surfaces=True):
    U.assert_fields_match(g, o, case, TOL64, RHO64)
    lf = case["n_levels"] - 1
    us = U.reference_speed(case)
    if walls:
        U.assert_walls_match(g, o, lf, 1e-10, RHO64, us)
    if surfaces:
        np.testing.assert_allclose(g.forces(), o.forces(), rtol=1e-9, atol=1e-12)
        for body in range(len(case.get("bodies", []))):
            U.assert_surface_match(g, o, body, 1e-9, 1e-9)


def _check32(g, o, case):
    U.assert_fields_match(g, o, case, TOL32, RHO32, chi_scale="level")
    us = U.reference_speed(case)
    U.assert_walls_match(g, o, case["n_levels"] - 1, TOL32, RHO32, us)
    cp_tol = (2.0 / 3.0) * RHO32 / us**2
    for body in range(len(case["bodies"])):
        U.assert_surface_match(g, o, body, cp_tol, 3e-5)
    np.testing.assert_allclose(g.forces()[:4], o.forces()[:4], rtol=1e-4)


def test_channel_structure():
    case = LI.case_channel()
    o, g = _pair(case, "f64")
    assert U.structure_mismatch(g, o, 1) == []


def test_airfoil_small_structure():
    case = LI.case_airfoil_small()
    o, g = _pair(case, "f64")
    assert U.structure_mismatch(g, o, case["n_levels"]) == []


@pytest.mark.parametrize("steps", [1, 10])
def test_channel_fp64_short(steps):
    case = LI.case_channel()
    o, g = _pair(case, "f64")
    U.channel_init(case, [o, g])
    o.advance(steps)
    g.advance(steps)
    _check64(g, o, case, surfaces=False)


def test_channel_fp64_full_run():
    """2000 steps of the Re_tau = 2000 channel: every cell's u and chi within 1e-10,
    rho within 1e-12, every wall node's u_tau and slip within 1e-10."""
    case = LI.case_channel()
    o, g = _pair(case, "f64")
    U.channel_init(case, [o, g])
    o.advance(case["steps"])
    g.advance(case["steps"])
    _check64(g, o, case, surfaces=False)


def test_airfoil_small_fp64():
    case = LI.case_airfoil_small()
    o, g = _pair(case, "f64")
    for steps in (1, 4):
        o.advance(steps)
        g.advance(steps)
        _check64(g, o, case)


def test_angle_of_attack_from_the_config_fp64():
    """Incidence set in the configuration (alpha 10 degrees about the quarter
    chord; Section 3.1.1) on an unturned body: the library turns the body as the
    oracle does (same grid, fields, wall records, surface data and forces after
    one and four coarse steps within the FP64 bounds), and its result is that of
    the recipe's turned body bit for bit (FP32)."""
    flat = LI.case_airfoil_small(alpha_deg=0.0)
    flat.update(config_alpha_deg=10.0, config_alpha_pivot=(0.25, 0.0))
    o, g = _pair(flat, "f64")
    assert U.structure_mismatch(g, o, flat["n_levels"]) == []
    for steps in (1, 3):
        o.advance(steps)
        g.advance(steps)
        _check64(g, o, flat)
    a = U.gpu_solver(LI.case_airfoil_small(alpha_deg=10.0), "f32")
    b = U.gpu_solver(flat, "f32")
    a.advance(2)
    b.advance(2)
    for l in range(flat["n_levels"]):
        assert a.level_info(l) == b.level_info(l)
        for f in range(4):
            np.testing.assert_array_equal(a.field(l, f), b.field(l, f))
    np.testing.assert_array_equal(a.forces(), b.forces())


@pytest.mark.parametrize("levels", [1, 2])
def test_airfoil_with_one_or_two_levels_fp64(levels):
    """Degenerate depths of the recursion: one level (wall nodes, domain edges
    and the absorbing layer on the same level, no transfers) and two levels (a
    refinement, but no level deep enough to merge), direct launches and graph
    replay, against the oracle."""
    case = LI.case_airfoil(seed=5, finest_cells_per_chord=64, n_levels=levels, domain_chords=8.0,
                           band_finest=0.25, n_side=128)
    o, g = _pair(case, "f64")
    h = U.gpu_solver(case, "f64")
    h.use_graph(True)
    o.advance(4)
    g.advance(4)
    h.advance(1)
    h.advance(3)
    _check64(g, o, case)
    for l in range(levels):
        for f in (0, 1, 2, 3):
            x, y = h.field(l, f), g.field(l, f)
            assert np.array_equal(np.isnan(x), np.isnan(y))
            m = ~np.isnan(x)
            assert np.array_equal(x[m], y[m]), (l, f)


def test_airfoil_small_fp32_window():
    case = LI.case_airfoil_small()
    o, g = _pair(case, "f32")
    o.advance(3)
    g.advance(3)
    _check32(g, o, case)


def _edge_state(case, sims, seed=7, body=0):
    """Seeded random state on every level: chi of both signs, a nearly uniform
    velocity (wave amplitude 1e-4, so the vorticity is small next to S-bar near
    the walls), and a still disc around one point of the upper surface of a body."""
    pts = case["bodies"][body]
    centre = pts[len(pts) // 4]                    # a quarter of the way round: upper surface
    for l in range(case["n_levels"]):
        inf = sims[0].level_info(l)
        fields = LI.seeded_level_state(case, l, inf["gx0"], inf["gy0"], inf["nx"], inf["ny"], seed,
                                       still_centre=centre, still_radius=0.08, wave=1e-4)
        for s in sims:
            s.init(l, *fields)


def _branch_census(case, o):
    """Cells of the finest level whose state takes each rarely taken branch of
    the SA-neg update (eqs (14), (15), (17)), from the oracle's own source terms
    on the state itself, the vorticity by the interior least-squares gradient."""
    lf = case["n_levels"] - 1
    chi = o.field(lf, oracle.F_CHI)
    ux, uy = o.field(lf, oracle.F_UX), o.field(lf, oracle.F_UY)
    d = o.field(lf, oracle.F_DIST)
    # lattice viscosity of the finest level: U (c / dx) / Re with dx that level's cell
    nu = U.reference_speed(case) * (case["ref_length"] / (case["dx0"] / 2 ** lf)) / case["reynolds"]
    c = np.s_[1:-1, 1:-1]
    ok = np.isfinite(chi[c])
    for a in (chi, ux, uy):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                ok &= np.isfinite(np.roll(np.roll(a, -dy, 0), -dx, 1)[c])

    def sh(a, dx, dy):
        return np.roll(np.roll(a, -dy, 0), -dx, 1)[c]
    dudy = ((sh(ux, -1, 1) - sh(ux, -1, -1)) + (sh(ux, 0, 1) - sh(ux, 0, -1)) + (sh(ux, 1, 1) - sh(ux, 1, -1))) / 6
    dvdx = ((sh(uy, 1, -1) - sh(uy, -1, -1)) + (sh(uy, 1, 0) - sh(uy, -1, 0)) + (sh(uy, 1, 1) - sh(uy, -1, 1))) / 6
    omega = np.abs(dvdx - dudy)[ok]
    nt = (chi[c] * nu)[ok]
    dist = d[c][ok]
    counts = dict(negative=0, second_branch=0, r_clip=0)
    for k in range(len(nt)):
        if nt[k] < 0:
            counts["negative"] += 1
            continue
        src = oracle.sa_source(nt[k], nu, omega[k], dist[k])
        x = nt[k] / nu
        fv1 = x**3 / (x**3 + 7.1**3)
        sbar = nt[k] * (1 - x / (1 + x * fv1)) / (0.41**2 * dist[k] ** 2)
        if sbar < -0.7 * omega[k] * 1.01:
            counts["second_branch"] += 1
        if src["r"] == 10.0:
            counts["r_clip"] += 1
    return counts


def _fallback_links(g, level):
    """Cut links whose next node along the link (F2 = B + c_i, i the missing
    direction) is not fluid: there the interpolated rule of eq. (27) has no second
    point and eq. (24) applies."""
    cx = [0, 1, -1, 0, 0, 1, -1, 1, -1]
    cy = [0, 0, 0, 1, -1, 1, -1, -1, 1]
    opp = [0, 2, 1, 4, 3, 6, 5, 8, 7]
    t = g.field(level, 5)
    inf = g.level_info(level)
    n = 0
    for rec in g.wall(level):
        gi, gj = int(rec[0]), int(rec[1])
        for i in range(1, 9):
            if rec[19 + opp[i] - 1] < 0:
                continue                            # population i is not missing
            fx, fy = gi + cx[i] - inf["gx0"], gj + cy[i] - inf["gy0"]
            if not (0 <= fx < inf["nx"] and 0 <= fy < inf["ny"]) or t[fy, fx] != 1:
                n += 1
    return n


def test_rarely_taken_branches_fp64():
    """A seeded random state on every level of a small three-element case (3
    levels to c/64, so that the 2 % gaps are one or two cells wide; chi uniform
    in [-5, 40], a nearly uniform velocity, a still disc on the main element)
    drives the branches that smooth runs from the free stream never reach:
    negative nu~ (eqs (16)-(17)), S-bar < -c_v2 Omega (second branch of eq. (14)),
    r at its limit (eq. (15)), wall nodes with U_t = 0 (step 3 of the VN
    procedure: u_tau = 0, no slip) and cut links whose next node is solid (eq. (24)
    in place of eq. (27)).  The census of each is taken on the state itself; one
    and four FP64 steps then match the oracle element by element."""
    case = LI.case_three_element(finest_cells_per_chord=64, n_levels=3, domain_chords=8.0,
                                 band_finest=0.3, n_side=256)
    case.update(ramp_steps=0.0, ramp_start=0.0)
    o, g = _pair(case, "f64")
    _edge_state(case, [o, g], body=1)
    lf = case["n_levels"] - 1
    census = _branch_census(case, o)
    assert census["negative"] > 100 and census["second_branch"] > 100 and census["r_clip"] > 100, census
    w0 = o.wall(lf)
    assert np.sum(w0[:, 12] == 0.0) >= 3                # U_t = 0 at the still wall nodes
    assert _fallback_links(g, lf) > 0
    for steps in (1, 3):
        o.advance(steps)
        g.advance(steps)
        _check64(g, o, case)


def test_sa_face_limit_never_binds_on_the_channel_and_the_small_airfoil():
    """The optional SA face-diffusivity limit (0.2 sigma) changes nothing, bit for
    bit, on the channel over its 2000 steps and on the small airfoil over 300
    coarse steps: the face diffusivities of those flows stay below it."""
    for case, steps in ((LI.case_channel(), 2000), (LI.case_airfoil_small(), 300)):
        a = U.gpu_solver(case, "f64")
        b = U.gpu_solver(dict(case, sa_mu_cap=0.2 * (2.0 / 3.0)), "f64")
        if case["name"] == "channel":
            U.channel_init(case, [a, b])
        a.advance(steps)
        b.advance(steps)
        for l in range(case["n_levels"]):
            for f in (0, 1, 2, 3):
                x, y = a.field(l, f), b.field(l, f)
                m = ~np.isnan(x)
                assert np.array_equal(np.isnan(x), np.isnan(y)) and np.array_equal(x[m], y[m]), (case["name"], l, f)


def test_sa_face_limit_never_binds_on_the_benchmark_airfoil():
    """The same on the 8-level benchmark airfoil in FP32 over 3000 coarse steps
    (about 33 convective times, where its residual falls below 1e-6)."""
    case = LI.case_airfoil_2M()
    a = U.gpu_solver(case, "f32")
    b = U.gpu_solver(dict(case, sa_mu_cap=0.2 * (2.0 / 3.0)), "f32")
    for s in (a, b):
        s.use_graph(True)
        s.advance(3000)
    for l in range(case["n_levels"]):
        for f in (1, 2, 3):
            x, y = a.field(l, f), b.field(l, f)
            m = ~np.isnan(x)
            assert np.array_equal(np.isnan(x), np.isnan(y)) and np.array_equal(x[m], y[m]), (l, f)
    assert np.array_equal(a.forces(), b.forces())


def test_refined_box_conserves_mass_on_gpu():
    case = LI.case_airfoil_small(alpha_deg=0.0)
    case.update(bc=(LI.BC_PERIODIC,) * 4, body_mode=LI.BODY_REFINE, sa_mode=LI.SA_FROZEN,
                chi_init=0.0, u_ref=0.05, nu0=0.002)
    g = U.gpu_solver(case, "f64")
    rng = np.random.default_rng(11)
    for l in range(case["n_levels"]):
        inf = g.level_info(l)
        sh = (inf["ny"], inf["nx"])
        g.init(l, rho=1 + 0.01 * rng.uniform(-1, 1, sh), ux=0.05 + 0.01 * rng.uniform(-1, 1, sh),
               uy=0.01 * rng.uniform(-1, 1, sh), chi=np.zeros(sh))

    def mass():
        return sum(np.nansum(g.field(l, 0)) * 4.0**-l for l in range(case["n_levels"]))
    m0 = mass()
    g.advance(6)
    assert abs(mass() - m0) / m0 < 1e-14


@pytest.mark.parametrize("storage,levels", [("f64", 3), ("f32", 3), ("f32", 6), ("f16", 6), ("mixeds", 6)])
def test_graph_replay_matches_direct_launches(storage, levels):
    """The merged schedule (coarse sub-steps inside the launches of finer ones),
    replayed from a graph with odd numbers of steps in between, and launched
    directly under timing, gives the same fields, bit for bit, as the direct
    recursive cycle."""
    case = (LI.case_airfoil_small() if levels == 3 else
            LI.case_airfoil(seed=3, finest_cells_per_chord=256, n_levels=levels, domain_chords=8.0,
                            band_finest=0.0625, n_side=256))
    a = U.gpu_solver(case, storage)
    b = U.gpu_solver(case, storage)
    c = U.gpu_solver(case, storage)
    a.use_graph(True)
    for n in (1, 3, 2, 1, 5, 4):
        a.advance(n)
        a.synchronize()
        a.field(case["n_levels"] - 1, 1)       # eager work between replays
    b.advance(16)
    c.profile(True)
    c.advance(7)
    c.advance(9)
    kt = c.profile(False)
    full = 2 ** levels - 1
    assert kt[3] < full if levels >= 3 else kt[3] == full   # merged launches per coarse step
    for s in (a, c):
        for l in range(case["n_levels"]):
            for f in (0, 1, 2, 3):
                x, y = s.field(l, f), b.field(l, f)
                assert np.array_equal(np.isnan(x), np.isnan(y))
                m = ~np.isnan(x)
                assert np.array_equal(x[m], y[m]), (l, f)
        assert np.array_equal(s.forces(), b.forces())


@pytest.mark.parametrize("variant", [
    dict(sa_mode=LI.SA_UPWIND1),                 # first-order upwind SA convection (Section 3.3)
    dict(wall_model=LI.WALL_NISHIMURA),          # eq (31) with d_WR = 1.75 (Section 3.1.5)
    dict(bb_mode=LI.BB_HALFWAY),                 # eq (24) at every cut link
    dict(outlet=LI.OUTLET_EXTRAP1),
    dict(outlet=LI.OUTLET_PRESSURE),
    dict(sponge_width=0.0),
    dict(ramp_steps=3.0),                        # start-up ramp over the first 3 steps
])
def test_airfoil_small_variants_fp64(variant):
    """Each variant of the method against the oracle, FP64.  From rest (start-up
    ramp) the flow needs ~100 coarse steps to reach the body; until then the
    velocity at R is round-off noise (about 1e-17 U), u_tau of order the square
    root of that noise (sqrt(nu U_t / d_WR), about 1e-12) and the wall value
    chi_B = kappa u_tau d_WB / nu noise-sized too (about 1e-7), and the two codes'
    different noise stays in chi near the wall after the flow arrives.  So the
    ramped comparison waits 150 steps and bounds chi by that noise (1e-6 of
    max(|chi|, 1)); every other bound is the FP64 one."""
    case = LI.case_airfoil_small()
    case.update(variant)
    o, g = _pair(case, "f64")
    ramped = "ramp_steps" in variant
    steps = 150 if ramped else 4
    o.advance(steps)
    g.advance(steps)
    if ramped:
        errs = U.level_errors(g, o, case["n_levels"], U.reference_speed(case))
        for l, e in errs.items():
            assert e["ux"] < TOL64 and e["uy"] < TOL64 and e["rho"] < RHO64 and e["chi"] < 1e-6, (l, e)
        np.testing.assert_allclose(g.forces(), o.forces(), rtol=1e-9, atol=1e-12)
    else:
        _check64(g, o, case)


def test_three_element_small_fp64():
    """Three bodies with narrow gaps (slat, main element, flap; 4 levels to
    c/256): grids, cut links and wall records built independently must agree,
    then four FP64 coarse steps match the oracle in every cell of every level,
    in every wall node and in the forces and surface data of each body."""
    case = LI.case_three_element(finest_cells_per_chord=256, n_levels=4, domain_chords=8.0,
                                 band_finest=0.1, n_side=256)
    case.update(ramp_steps=0.0, ramp_start=0.0)
    o, g = _pair(case, "f64")
    L = case["n_levels"]
    assert U.structure_mismatch(g, o, L, case["nx0"]) == []
    o.advance(4)
    g.advance(4)
    _check64(g, o, case)
    for body in (0, 1, 2, -1):
        np.testing.assert_allclose(g.forces(body), o.forces(body), rtol=1e-9, atol=1e-12)


def test_full_size_airfoil_fp32_against_oracle():
    """The benchmark workload itself (8 levels, ~2.0M cells, FP32, graph replay as
    timed by the benchmark) against the FP64 oracle after two coarse steps (510
    k_step launches, 2.5e8 cell updates): every owned cell of every level within
    the FP32 bounds (u 1e-5 U, chi 1e-5 of the level's largest chi, rho 1e-6),
    every wall node's u_tau, slip and rho_W, every segment's Cp and Cf, and the
    forces within 1e-4."""
    case = LI.case_airfoil_2M()
    o, g = _pair(case, "f32")
    assert U.structure_mismatch(g, o, case["n_levels"], case["nx0"]) == []
    g.use_graph(True)
    o.advance(2)
    g.advance(2)
    _check32(g, o, case)


@pytest.mark.slow
def test_full_size_three_element_fp32_against_oracle():
    """The three-element case at its full size (19.4M cells, 8 levels to c/4096,
    three bodies): grids, cut links and wall records built independently by both
    codes agree exactly, and after one coarse step (1.35e9 cell updates) the FP32
    library matches the FP64 oracle within the FP32 bounds in every cell, wall
    node and surface segment of every body."""
    case = LI.case_three_element()
    o, g = _pair(case, "f32")
    assert U.structure_mismatch(g, o, case["n_levels"], case["nx0"]) == []
    o.advance(1)
    g.advance(1)
    _check32(g, o, case)

"""Pins of the oracle's SA-neg terms (Section 2.2) and its interpolation helpers."""
import numpy as np
import pytest

import oracle
from tests.golden.load import constants

SA = constants("sa_constants.txt")
K = SA["kappa"]


def cw1():
    return SA["c_b1"] / K**2 + (1.0 + SA["c_b2"]) / SA["sigma"]


def fv1(chi):
    return chi**3 / (chi**3 + SA["c_v1"] ** 3)


@pytest.mark.parametrize("yplus", [2.0, 5.0, 10.0, 30.0, 100.0, 1000.0, 1e4])
def test_log_layer_solution(yplus):
    """eq. (20): chi = kappa y+ with the eq. (19) gradient gives S~ = u_tau^2/(nu kappa y+), r = 1."""
    nu, utau = 1.5e-5, 4e-3
    y = yplus * nu / utau
    nt = K * utau * y
    chi = nt / nu
    omega = utau**2 / (nu * (1.0 + chi * fv1(chi)))       # (nu + nu_t) du/dy = u_tau^2
    src = oracle.sa_source(nt, nu, omega, y)
    assert src["S_tilde"] == pytest.approx(utau**2 / (nu * K * yplus), rel=1e-12)
    assert src["r"] == pytest.approx(1.0, rel=1e-12)
    assert src["f_w"] == pytest.approx(1.0, rel=1e-12)
    # budget: P - D + (1/sigma)[d/dy((nu + nt) dnt/dy) + c_b2 (dnt/dy)^2] = 0 because
    # c_w1 = c_b1/kappa^2 + (1 + c_b2)/sigma
    diffusion = (K * utau) ** 2 * (1.0 + SA["c_b2"]) / SA["sigma"]
    assert (src["P"] - src["D"] + diffusion) / diffusion == pytest.approx(0.0, abs=1e-12)


def test_cw1_value():
    assert cw1() == pytest.approx(3.2390678167757, rel=1e-12)


def test_modified_vorticity_is_continuous_at_branch_switch():
    # at S-bar = -c_v2 Omega both branches of eq. (14) give (1 - c_v2) Omega
    nu, omega, d = 1e-5, 3e-3, 0.02
    chi = 3.0                                     # f_v2 < 0 here
    nt = chi * nu
    fv2 = 1 - chi / (1 + chi * fv1(chi))
    d_switch = np.sqrt(nt * fv2 / (-SA["c_v2"] * omega * K**2))
    for eps in (1e-9, -1e-9):
        st = oracle.sa_source(nt, nu, omega, d_switch * (1 + eps))["S_tilde"]
        assert st == pytest.approx((1 - SA["c_v2"]) * omega, rel=1e-6)


def test_modified_vorticity_stays_bounded_on_the_second_branch():
    """Below S-bar = -c_v2 Omega, eq. (14) must keep S-tilde between
    (1 - c_v3) Omega (S-bar -> -inf) and (1 - c_v2) Omega (the switch), with no
    pole: sweep S-bar over five decades through the branch."""
    nu, omega = 1e-5, 2e-3
    chi = 10.0                                    # f_v2 < 0: S-bar < 0
    nt = chi * nu
    fv2 = 1 - chi / (1 + chi * fv1(chi))
    assert fv2 < 0
    lo, hi = (1 - SA["c_v3"]) * omega, (1 - SA["c_v2"]) * omega
    prev = None
    for ratio in np.logspace(np.log10(0.71), 4, 400):          # |S-bar| / Omega
        d = np.sqrt(nt * fv2 / (-ratio * omega * K**2))
        st = oracle.sa_source(nt, nu, omega, d)["S_tilde"]
        assert lo <= st <= hi * (1 + 1e-12), (ratio, st)
        if prev is not None:
            assert st <= prev * (1 + 1e-12)                    # decreasing in |S-bar|
        prev = st
    assert prev == pytest.approx(lo, rel=1e-3)


@pytest.mark.parametrize("chi", [-0.5, -2.0, -10.0])
def test_negative_branch(chi):
    nu, omega, d = 1e-5, 2e-3, 0.01
    nt = chi * nu
    src = oracle.sa_source(nt, nu, omega, d)
    assert src["nu_t"] == 0.0                         # eq. (11)
    assert src["P"] - src["D"] > 0.0                  # both terms drive nt back towards zero
    assert src["P"] > 0.0 and -src["D"] > 0.0
    # continuity of the diffusivity at nt = 0
    assert oracle.sa_source(-1e-14 * nu, nu, omega, d)["mu"] == pytest.approx(nu, rel=1e-12)
    assert oracle.sa_source(1e-14 * nu, nu, omega, d)["mu"] == pytest.approx(nu, rel=1e-12)


def test_destruction_vanishes_far_from_walls():
    src = oracle.sa_source(3e-5, 1e-5, 1e-4, 1e12)
    assert src["D"] < 1e-30


def _stencil(fun):
    return np.array([[fun(dx, dy) for dx in (-1, 0, 1)] for dy in (-1, 0, 1)])


@pytest.mark.parametrize("mode", [1, 2])
def test_cell_update_exact_for_linear_fields(mode):
    """Linear nt and uniform u: every discrete operator is exact, so the update equals
    -u.grad nt + P - D + (1/sigma)(1 + c_b2)|grad nt|^2 from the continuous equation."""
    nu, d = 1e-5, 0.5
    a, bx, by = 4e-4, 3e-6, -2e-6
    u, v = 0.04, -0.015
    nt = _stencil(lambda dx, dy: a + bx * dx + by * dy)
    ux = _stencil(lambda dx, dy: u)
    uy = _stencil(lambda dx, dy: v)
    got = oracle.sa_cell(nt, ux, uy, nu, d, mode)
    src = oracle.sa_source(a, nu, 0.0, d)
    expect = a - (u * bx + v * by) + src["P"] - src["D"] + (1 + SA["c_b2"]) * (bx**2 + by**2) / SA["sigma"]
    assert got == pytest.approx(expect, rel=1e-12)


def test_vorticity_from_least_squares_gradients():
    """A linear shear u = (g y, 0) has vorticity |g| exactly; it enters through S~ = Omega + S-bar."""
    nu, d, g = 1e-5, 1e9, 2e-3
    nt0 = 3e-5
    nt = _stencil(lambda dx, dy: nt0)
    ux = _stencil(lambda dx, dy: g * dy)
    uy = _stencil(lambda dx, dy: 0.0)
    got = oracle.sa_cell(nt, ux, uy, nu, d, 1)
    src = oracle.sa_source(nt0, nu, g, d)
    assert got == pytest.approx(nt0 + src["P"] - src["D"], rel=1e-12)
    assert src["S_tilde"] == pytest.approx(g, rel=1e-6)


def test_lax_wendroff_advects_quadratics_exactly():
    """For nt = c x^2 with uniform u, Lax-Wendroff gives c (x - u)^2 at x = 0 (exact advection);
    the diffusion of the quadratic is removed by taking the difference of two velocities."""
    nu, d, c = 1e-5, 1e12, 1e-4
    nt = _stencil(lambda dx, dy: 1e-3 + c * dx * dx)
    zero = _stencil(lambda dx, dy: 0.0)
    for u in (0.03, -0.07):
        ux = _stencil(lambda dx, dy: u)
        diff = oracle.sa_cell(nt, ux, zero, nu, d, 1) - oracle.sa_cell(nt, zero, zero, nu, d, 1)
        assert diff == pytest.approx(c * u * u, rel=1e-9)


def test_lsq_exact_for_linear_fields():
    rng = np.random.default_rng(0)
    for n in (3, 4, 9, 16):
        px, py = rng.uniform(-2, 2, n), rng.uniform(-2, 2, n)
        v = 0.3 + 1.7 * px - 0.4 * py
        x, y = 0.37, -0.61
        assert oracle.lsq_point(px, py, v, x, y) == pytest.approx(0.3 + 1.7 * x - 0.4 * y, rel=1e-12)
    assert np.isnan(oracle.lsq_point([0, 1, 2], [0, 1, 2], [1, 2, 3], 0.5, 0.5))  # collinear


def test_idw_exact_for_constants_and_at_nodes():
    rng = np.random.default_rng(1)
    px, py = rng.uniform(-1, 1, 5), rng.uniform(-1, 1, 5)
    assert oracle.idw_point(px, py, np.full(5, 2.5), 0.1, 0.2) == pytest.approx(2.5, rel=1e-15)
    v = rng.uniform(0, 1, 5)
    assert oracle.idw_point(px, py, v, px[2], py[2]) == v[2]
    got = oracle.idw_point(px, py, v, 0.1, 0.2)
    assert v.min() <= got <= v.max()


@pytest.mark.parametrize("chi", [10.0, 1e3, 1e5, 1e7])
def test_limited_face_diffusivity_keeps_the_update_within_the_stencil(chi):
    """With the optional face-diffusivity limit of 0.2 sigma, pure diffusion (no
    velocity, wall far away) of a centre value below its four face neighbours
    never overshoots them, whatever the eddy viscosity."""
    nu, d = 1e-4, 1e12
    hi = chi * nu
    nt = np.full(9, hi)
    nt[4] = 0.5 * hi
    new = oracle.sa_cell(nt, np.zeros(9), np.zeros(9), nu, d, 1, mu_cap=0.2 * SA["sigma"])
    assert 0.5 * hi < new <= hi


@pytest.mark.parametrize("chi", [10.0, 1e3, 1e5])
def test_unlimited_face_diffusivity_is_the_printed_scheme(chi):
    """Without the limit (the default), the centred diffusion of eq. (12) uses the
    mean of the two nodal diffusivities nu + nt at every face.  A centre value C
    whose four face neighbours hold 2C (no velocity, wall far away, so the sources
    vanish and the centred gradient, hence the c_b2 term, is zero) gains
    (1/sigma) 4 ((nu + C) + (nu + 2C)) / 2 C.  A limit above every face value
    changes nothing, bit for bit."""
    nu, d = 1e-4, 1e12
    C = 0.5 * chi * nu
    nt = np.full(9, C)
    nt[[1, 3, 5, 7]] = 2 * C
    expect = C + 4 * (0.5 * ((nu + C) + (nu + 2 * C))) * C / SA["sigma"]
    got = oracle.sa_cell(nt, np.zeros(9), np.zeros(9), nu, d, 1)
    assert got == pytest.approx(expect, rel=1e-12)
    assert oracle.sa_cell(nt, np.zeros(9), np.zeros(9), nu, d, 1, mu_cap=10 * (nu + 2 * C)) == got


def _fw_sweep():
    """(r, f_w) over a sweep of the vorticity at fixed nt and d: r = nt / (S~ kappa^2 d^2)
    runs from far below 1 up to its limit r_lim."""
    nu, d = 1e-5, 0.05
    nt = 0.95 * nu                                 # 0 < f_v2 < 0.1: r -> 1 / f_v2 > r_lim as Omega -> 0
    out = []
    for omega in np.logspace(-12, 2, 300):
        src = oracle.sa_source(nt, nu, omega, d)
        out.append((src["r"], src["f_w"], src["D"], nt, d))
    return out


def test_destruction_function_limits():
    """eq. (15): for r -> 0, g -> (1 - c_w2) r and f_w / r -> (1 - c_w2) ((1 + c_w3^6) / c_w3^6)^(1/6);
    at the clip r = r_lim, g = r_lim + c_w2 (r_lim^6 - r_lim) is about 3e5 and f_w equals
    (1 + c_w3^6)^(1/6) to 1e-12; f_w = 1 at r = 1 (see the log-layer test)."""
    cw2, cw3 = SA["c_w2"], SA["c_w3"]
    sweep = _fw_sweep()
    r_small, fw_small = min(sweep)[:2]
    assert r_small < 1e-3
    assert fw_small / r_small == pytest.approx((1 - cw2) * ((1 + cw3**6) / cw3**6) ** (1 / 6), rel=1e-9)
    r_big, fw_big = max(sweep)[:2]
    assert r_big == SA["r_lim"]
    assert fw_big == pytest.approx((1 + cw3**6) ** (1 / 6), rel=1e-12)


def test_destruction_function_is_increasing_and_enters_the_destruction_term():
    """f_w never decreases with r, increases strictly until it saturates at
    (1 + c_w3^6)^(1/6) (g ~ 1e3 from r ~ 4 on, where the difference drops below
    FP64 resolution), and D = c_w1 f_w (nt / d)^2 (eq. (13))."""
    sweep = sorted(_fw_sweep())
    rs = np.array([x[0] for x in sweep])
    fws = np.array([x[1] for x in sweep])
    assert np.all(np.diff(fws) >= -4e-16 * fws[1:])               # rounding of pow() at saturation
    rising = fws < 0.999 * (1 + SA["c_w3"] ** 6) ** (1 / 6)
    assert rising.sum() > 50 and np.all(np.diff(fws[rising]) > 0)
    for r, fw, D, nt, d in sweep[::37]:
        assert D == pytest.approx(3.2390678167757 * fw * (nt / d) ** 2, rel=1e-12)


@pytest.mark.parametrize("chi,fn,mu_over_nu", [(-1.0, 15.0 / 17.0, 2.0 / 17.0), (-2.0, 1.0 / 3.0, 1.0 / 3.0)])
def test_negative_branch_hand_values(chi, fn, mu_over_nu):
    """eqs. (16)-(17) at chi = -1 and -2 with c_n1 = 16: f_n = (16 + chi^3) / (16 - chi^3)
    is 15/17 and 1/3, so the nodal diffusivity nu + nt f_n is 2 nu / 17 and nu / 3.
    With nu = 1e-5, Omega = 2e-3 and d = 0.01, worked by hand from the printed
    constants: P_n = c_b1 (1 - c_t3) Omega nt = -5.42e-5 nt (5.42e-10 and 1.084e-9),
    D_n = -c_w1 (nt / d)^2 (-c_w1 1e-6 and -c_w1 4e-6), and nu_t = 0 (eq. (11))."""
    nu, omega, d = 1e-5, 2e-3, 0.01
    nt = chi * nu
    src = oracle.sa_source(nt, nu, omega, d)
    assert src["mu"] / nu == pytest.approx(mu_over_nu, rel=1e-13)
    assert (src["mu"] - nu) / nt == pytest.approx(fn, rel=1e-13)
    expect_P = {-1.0: 5.42e-10, -2.0: 1.084e-9}[chi]            # -0.0271 * 2e-3 * nt
    expect_D = {-1.0: -3.2390678167757e-6, -2.0: -1.29562712671028e-5}[chi]   # -c_w1 (nt/d)^2
    assert src["P"] == pytest.approx(expect_P, rel=1e-12)
    assert src["D"] == pytest.approx(expect_D, rel=1e-12)
    assert src["nu_t"] == 0.0


def test_lax_wendroff_cross_term_advects_a_bilinear_field_exactly():
    """nt = b + c x y is advected by a uniform (u, v) to b + c (x - u)(y - v); at the
    centre after one step the increment is c u v, which only the corner cross term
    delta_xy of the unsplit scheme produces (the first and second centred differences
    of x y vanish at the centre).  A dropped factor 2 or a wrong sign fails."""
    nu, d, b, c = 1e-5, 1e12, 1e-3, 2e-4
    nt = _stencil(lambda dx, dy: b + c * dx * dy)
    zero = _stencil(lambda dx, dy: 0.0)
    for u, v in ((0.03, 0.05), (-0.07, 0.02), (0.04, -0.06)):
        ux = _stencil(lambda dx, dy: u)
        uy = _stencil(lambda dx, dy: v)
        diff = oracle.sa_cell(nt, ux, uy, nu, d, 1) - oracle.sa_cell(nt, zero, zero, nu, d, 1)
        assert diff == pytest.approx(c * u * v, rel=1e-9)

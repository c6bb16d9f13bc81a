"""Pins of the oracle's wall function, Newton solve and slip velocity.

Each test checks the oracle against something the paper or mathematics fixes
independently of the oracle's own formula: eq. (22) must integrate eq. (21),
its constants must be the roots of the denominator of eq. (21), its log-law
asymptote must be 1/kappa, and so on.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import oracle
from tests.golden.load import constants

WF = constants("wall_function_constants.txt")
SA = constants("sa_constants.txt")
KAPPA, CV1 = SA["kappa"], SA["c_v1"]


def eq21(y):
    """du+/dy+ of Section 2.2, eq. (21), written out from the paper."""
    ky = KAPPA * y
    return (CV1**3 + ky**3) / (CV1**3 + ky**3 * (1.0 + ky))


@pytest.mark.parametrize("y", np.logspace(-3, 5, 41))
def test_derivative_of_eq22_is_eq21(y):
    h = 1e-4 * max(y, 1.0)
    fd = (oracle.uplus(y + h) - oracle.uplus(y - h)) / (2 * h) if y > h else \
        (oracle.uplus(y + h) - oracle.uplus(y)) / h
    assert fd == pytest.approx(eq21(y), rel=2e-6, abs=1e-8)


@pytest.mark.parametrize("y", [0.5, 3.0, 6.9287, 7.5, 30.0, 300.0, 5000.0])
def test_eq22_is_the_integral_of_eq21(y):
    # the continuous branch: no jump at y+ = -a2 = 6.9287 (principal arctan would jump by pi c4)
    integral = quad(eq21, 0.0, y, limit=400, epsabs=1e-13, epsrel=1e-12)[0]
    assert oracle.uplus(y) - oracle.uplus(0.0) == pytest.approx(integral, rel=1e-10, abs=1e-11)


def test_constants_are_roots_of_eq21_denominator():
    # kappa^4 y^4 + kappa^3 y^3 + c_v1^3 = 0 has roots -a_j +- i b_j
    roots = np.roots([KAPPA**4, KAPPA**3, 0.0, 0.0, CV1**3])
    expect = [complex(-WF["a1"], WF["b1"]), complex(-WF["a1"], -WF["b1"]),
              complex(-WF["a2"], WF["b2"]), complex(-WF["a2"], -WF["b2"])]
    for e in expect:
        assert min(abs(r - e) for r in roots) < 1e-9


def test_log_law_asymptote():
    # u+ - ln(y+)/kappa -> B_bar as y+ -> infinity (the arctangents vanish)
    y = 1e9
    assert oracle.uplus(y) - math.log(y) / KAPPA == pytest.approx(WF["B_bar"], abs=1e-6)
    assert 2 * (WF["c1"] - WF["c2"]) == pytest.approx(1.0 / KAPPA, rel=1e-12)


def test_viscous_sublayer():
    for y in (1e-3, 1e-2, 0.1):
        assert oracle.uplus(y) - oracle.uplus(0.0) == pytest.approx(y, rel=1e-3)
    assert abs(oracle.uplus(0.0)) < 1e-3


@pytest.mark.parametrize("yplus", np.logspace(0, 5, 26))
def test_newton_round_trip(yplus):
    nu, dwr = 1.5e-5, 2.0
    utau = yplus * nu / dwr
    ut = utau * oracle.uplus(yplus)
    for guess in (0.0, 0.3 * utau, 3.0 * utau):
        got = oracle.solve_utau(ut, dwr, nu, guess)
        assert got == pytest.approx(utau, rel=1e-13)


def test_newton_zero_velocity():
    assert oracle.solve_utau(0.0, 2.0, 1e-5, 0.0) == 0.0


@pytest.mark.parametrize("yv", [1.0, 10.0, 30.0, 100.0, 400.0])
def test_slip_velocity_closed_form(yv):
    # eq. (28) with (nu_t)_V = nu kappa y_V+:  u_W / u_tau = u+(y_V+) - y_V+ / (1 + kappa y_V+)
    nu, dwv = 2e-5, 1.0
    utau = yv * nu / dwv
    uw = oracle.slip(utau, dwv, nu)
    assert uw / utau == pytest.approx(oracle.uplus(yv) - yv / (1.0 + KAPPA * yv), rel=1e-13)
    assert 0.0 < uw < utau * oracle.uplus(yv)


@pytest.mark.parametrize("yv", [0.5, 10.0, 30.0, 50.0, 100.0, 200.0, 400.0, 3000.0])
def test_slip_velocity_from_the_integrated_wall_law(yv):
    """Steps 4-5 of the VN procedure built from independent pieces: u_V comes from
    integrating eq. (21) numerically from the wall (plus the wall value of eq. (22),
    pinned above), and the slip is the wall intercept of the straight line through
    (d_WV, u_V) whose slope is the wall shear stress u_tau^2 divided by the total
    viscosity nu + (nu_t)_V at V, with (nu_t)_V = nu kappa y_V+ (eq. (28))."""
    nu, dwv = 2e-5, 1.0
    utau = yv * nu / dwv
    u_v = utau * (oracle.uplus(0.0) + quad(eq21, 0.0, yv, limit=400, epsabs=1e-13, epsrel=1e-12)[0])
    slope = utau**2 / (nu + nu * KAPPA * yv)
    assert oracle.slip(utau, dwv, nu) == pytest.approx(u_v - slope * dwv, rel=1e-10)


def test_slip_velocity_limits():
    """Deep in the viscous sublayer the line through V hits the wall at the wall value
    of eq. (22) plus a second-order remainder (u_W / u_tau ~ u+(0) + kappa y_V+^2); in
    the log layer the slip tends to u_V - u_tau / kappa."""
    nu, dwv = 2e-5, 1.0
    for yv in (1e-3, 1e-2):
        utau = yv * nu / dwv
        rest = oracle.slip(utau, dwv, nu) / utau - oracle.uplus(0.0)
        assert rest == pytest.approx(KAPPA * yv * yv, rel=2e-2)
    yv = 1e7
    utau = yv * nu / dwv
    assert oracle.slip(utau, dwv, nu) / utau == pytest.approx(oracle.uplus(yv) - 1.0 / KAPPA, abs=1e-6)

"""Pins of the oracle's equilibrium and central-moment collision (Section 2.1)."""
import numpy as np
import pytest

import oracle

CX = np.array([0, 1, -1, 0, 0, 1, -1, 1, -1], dtype=float)
CY = np.array([0, 0, 0, 1, -1, 1, -1, -1, 1], dtype=float)
CS2 = 1.0 / 3.0


def central(f, ux, uy, p, q):
    """Central moment of order (p, q), by its definition."""
    return float(np.sum((CX - ux) ** p * (CY - uy) ** q * f))


def product_form(rho, ux, uy):
    """Factorised D2Q9 equilibrium rho psi(c_x, u_x) psi(c_y, u_y) (an independent closed form)."""
    def psi(c, u):
        return np.where(c == 0, 1.0 - (CS2 + u * u), 0.5 * (CS2 + u * u + c * u))
    return rho * psi(CX, ux) * psi(CY, uy)


CASES = [(1.0, 0.0, 0.0), (1.03, 0.08, -0.05), (0.97, -0.12, 0.07), (1.2, 0.2, 0.15)]


@pytest.mark.parametrize("rho,ux,uy", CASES)
def test_equilibrium_is_the_product_form(rho, ux, uy):
    np.testing.assert_allclose(oracle.feq(rho, ux, uy), product_form(rho, ux, uy), atol=1e-15)


@pytest.mark.parametrize("rho,ux,uy", CASES)
def test_equilibrium_central_moments(rho, ux, uy):
    f = oracle.feq(rho, ux, uy)
    assert np.sum(f) == pytest.approx(rho, rel=1e-14)
    assert np.sum(CX * f) == pytest.approx(rho * ux, abs=1e-15)
    assert np.sum(CY * f) == pytest.approx(rho * uy, abs=1e-15)
    assert central(f, ux, uy, 2, 0) == pytest.approx(rho * CS2, rel=1e-13)
    assert central(f, ux, uy, 0, 2) == pytest.approx(rho * CS2, rel=1e-13)
    assert abs(central(f, ux, uy, 1, 1)) < 1e-15
    assert abs(central(f, ux, uy, 2, 1)) < 1e-15
    assert abs(central(f, ux, uy, 1, 2)) < 1e-15
    assert central(f, ux, uy, 2, 2) == pytest.approx(rho * CS2**2, rel=1e-13)


def test_transfer_matrix_rows_are_eq6():
    rng = np.random.default_rng(3)
    f = rng.uniform(0.01, 0.5, 9)
    ux, uy = 0.07, -0.04
    k = oracle.central_moments(f, ux, uy)
    expect = [central(f, ux, uy, 0, 0), central(f, ux, uy, 1, 0), central(f, ux, uy, 0, 1),
              central(f, ux, uy, 2, 0) + central(f, ux, uy, 0, 2),
              central(f, ux, uy, 2, 0) - central(f, ux, uy, 0, 2),
              central(f, ux, uy, 1, 1), central(f, ux, uy, 2, 1), central(f, ux, uy, 1, 2),
              central(f, ux, uy, 2, 2)]
    np.testing.assert_allclose(k, expect, atol=1e-15)


def _state(seed):
    rng = np.random.default_rng(seed)
    rho, ux, uy = 1.0 + 0.05 * rng.uniform(-1, 1), 0.1 * rng.uniform(-1, 1), 0.1 * rng.uniform(-1, 1)
    return product_form(rho, ux, uy) * (1.0 + 0.05 * rng.uniform(-1, 1, 9))


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("nu", [1e-6, 1e-3, 0.05, 0.3])
def test_collision_conserves_mass_and_momentum(seed, nu):
    f = _state(seed)
    F = np.array([2e-5, -1e-5])
    fs = oracle.collide(f, nu, 1.0, F)
    assert np.sum(fs) == pytest.approx(np.sum(f), rel=1e-14)
    assert np.sum(CX * fs) == pytest.approx(np.sum(CX * f) + F[0], abs=1e-15)
    assert np.sum(CY * fs) == pytest.approx(np.sum(CY * f) + F[1], abs=1e-15)


@pytest.mark.parametrize("seed", range(5))
def test_full_relaxation_gives_equilibrium(seed):
    # K = I (omega_nu = omega_b = 1, i.e. nu = c_s^2 / 2): f* = f_eq(rho, u)
    f = _state(seed)
    rho = np.sum(f)
    ux, uy = np.sum(CX * f) / rho, np.sum(CY * f) / rho
    np.testing.assert_allclose(oracle.collide(f, CS2 / 2, 1.0), product_form(rho, ux, uy), atol=1e-15)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("nu,omega_b", [(1e-5, 1.0), (0.02, 1.0), (0.02, 1.4)])
def test_central_moment_relaxation(seed, nu, omega_b):
    f = _state(seed)
    F = np.array([3e-5, 1e-5])
    rho = np.sum(f)
    ux = (np.sum(CX * f) + F[0] / 2) / rho
    uy = (np.sum(CY * f) + F[1] / 2) / rho
    fs = oracle.collide(f, nu, omega_b, F)
    w = 1.0 / (nu / CS2 + 0.5)                                    # eq. (9)
    d0 = central(f, ux, uy, 2, 0) - central(f, ux, uy, 0, 2)
    t0 = central(f, ux, uy, 2, 0) + central(f, ux, uy, 0, 2)
    d1 = central(fs, ux, uy, 2, 0) - central(fs, ux, uy, 0, 2)
    t1 = central(fs, ux, uy, 2, 0) + central(fs, ux, uy, 0, 2)
    assert d1 == pytest.approx((1 - w) * d0, abs=1e-15)
    assert central(fs, ux, uy, 1, 1) == pytest.approx((1 - w) * central(f, ux, uy, 1, 1), abs=1e-15)
    assert t1 == pytest.approx((1 - omega_b) * t0 + omega_b * 2 * rho * CS2, abs=1e-14)
    assert central(fs, ux, uy, 1, 0) == pytest.approx(F[0] / 2, abs=1e-15)
    assert central(fs, ux, uy, 0, 1) == pytest.approx(F[1] / 2, abs=1e-15)
    assert abs(central(fs, ux, uy, 2, 1)) < 1e-15
    assert abs(central(fs, ux, uy, 1, 2)) < 1e-15
    assert central(fs, ux, uy, 2, 2) == pytest.approx(rho * CS2**2, abs=1e-15)

"""Pins of the semi-analytic reference solutions themselves (App. C, App. D)
against closed forms and independent finite-difference solutions."""
import math

import numpy as np
import pytest

from oracle import analytic as A


def fd_transient(H, rho1, rho2, eta1, eta2, u0, T, n=800):
    """Crank-Nicolson finite volumes for rho u_t = (eta u_x)_x, u(0) = u(H) = 0."""
    dx = H / n
    x = (np.arange(n) + 0.5) * dx
    rho = np.where(x < H / 2, rho1, rho2)
    eta_c = np.where(x < H / 2, eta1, eta2)
    eta_f = np.empty(n + 1)
    eta_f[1:-1] = 2 * eta_c[:-1] * eta_c[1:] / (eta_c[:-1] + eta_c[1:])
    eta_f[0], eta_f[-1] = eta_c[0], eta_c[-1]
    Lm = np.zeros((n, n))
    for i in range(n):
        wl = eta_f[i] / dx ** 2 * (2 if i == 0 else 1)
        wr = eta_f[i + 1] / dx ** 2 * (2 if i == n - 1 else 1)
        Lm[i, i] = -(wl + wr) / rho[i]
        if i > 0:
            Lm[i, i - 1] = wl / rho[i]
        if i < n - 1:
            Lm[i, i + 1] = wr / rho[i]
    u = np.where(x < H / 2, u0, -u0).astype(float)
    dt = 0.05
    I = np.eye(n)
    step = np.linalg.solve(I - 0.5 * dt * Lm, I + 0.5 * dt * Lm)
    for _ in range(int(round(T / dt))):
        u = step @ u
    return x, u


@pytest.mark.parametrize("rho2", [0.1, 0.5])
def test_flat_transient_matches_finite_differences(rho2):
    H, eta, u0, T = 20.0, 1.0 / 6.0, 1.0, 40.0
    x, ufd = fd_transient(H, 1.0, rho2, eta, eta, u0, T)
    ua = A.flat_transient(x, T, H, 1.0, rho2, eta, eta, u0, n_modes=300)
    assert np.max(np.abs(ua - ufd)) < 2e-3 * u0


def test_eigenfunctions_are_orthonormal_with_weight_rho():
    H, rho1, rho2, eta = 10.0, 1.0, 0.2, 0.3
    cs, A1, A2 = A.flat_modes(H, rho1, rho2, eta, eta, 6)
    x = np.linspace(0, H, 200001)
    rho = np.where(x < H / 2, rho1, rho2)
    phis = [A.flat_phi(x, c, a1, a2, H, rho1, rho2, eta, eta) for c, a1, a2 in zip(cs, A1, A2)]
    for i in range(6):
        for j in range(6):
            v = np.trapezoid(rho * phis[i] * phis[j], x)
            assert abs(v - (1.0 if i == j else 0.0)) < 1e-4


def test_two_layer_steady_reduces_to_poiseuille_and_matches_traction():
    H, eta, G = 12.0, 0.4, 1e-3
    x = np.linspace(0, H, 101)
    u = A.two_layer_steady(x, H, eta, eta, G)
    assert np.max(np.abs(u - G * x * (H - x) / (2 * eta))) < 1e-15
    u2 = A.two_layer_steady(np.array([H / 2 - 1e-7, H / 2 + 1e-7]), H, 0.4, 4.0, G)
    assert abs(u2[0] - u2[1]) < 1e-9
    h = 1e-6
    d1 = (A.two_layer_steady(H / 2 - h, H, 0.4, 4.0, G) - A.two_layer_steady(H / 2 - 2 * h, H, 0.4, 4.0, G)) / h
    d2 = (A.two_layer_steady(H / 2 + 2 * h, H, 0.4, 4.0, G) - A.two_layer_steady(H / 2 + h, H, 0.4, 4.0, G)) / h
    assert abs(0.4 * d1 - 4.0 * d2) < 1e-6


def test_startup_transient_limits():
    H, rho1, rho2, eta1, eta2, G = 16.0, 1.0, 0.5, 0.2, 0.6, 1e-4
    x = np.linspace(0.5, H - 0.5, 16)
    u0 = A.startup_transient(x, 0.0, H, rho1, rho2, eta1, eta2, G, n_modes=300)
    assert np.max(np.abs(u0)) < 2e-2 * np.max(A.two_layer_steady(x, H, eta1, eta2, G))
    uinf = A.startup_transient(x, 1e6, H, rho1, rho2, eta1, eta2, G)
    assert np.max(np.abs(uinf - A.two_layer_steady(x, H, eta1, eta2, G))) < 1e-15


def test_stratified_steady_uniform_density_is_poiseuille():
    """App. D with constant density reduces to the parabola G x (H - x)/(2 nu rho)."""
    H, nu, G = 20.0, 0.3, 1e-4
    x = np.linspace(0, H, 41)
    u = A.stratified_steady(x, H, nu, G, lambda a: 0.7 + 0 * a)
    assert np.max(np.abs(u - G * x * (H - x) / (2 * nu * 0.7))) < 1e-12


def test_laplace_and_error_measure():
    assert A.laplace_pressure(0.01, 20.0) == 0.0005
    u = np.array([1.0, 2.0, 4.0])
    assert A.transient_error(u, u) == 0.0
    assert abs(A.transient_error(np.array([1.0, 2.0]), np.array([1.0, 1.0])) - 0.125) < 1e-15


# ----------------------------------------------------------------------------
# App. D, curved interfaces: azimuthal transient in a circular container
# ----------------------------------------------------------------------------

def fd_radial(R0, R, rho1, rho2, eta, omega, T, n=600):
    """Crank-Nicolson finite volumes for rho r u_t = eta [(r u_r)_r - u/r],
    u(0) = u(R) = 0, from u = omega r (r < R0), 0 beyond."""
    dr = R / n
    r = (np.arange(n) + 0.5) * dr
    rf = np.arange(n + 1) * dr
    rho = np.where(r < R0, rho1, rho2)
    L = np.zeros((n, n))
    for i in range(n):
        m = rho[i] * r[i] * dr
        wr = eta * rf[i + 1] / dr * (2 if i == n - 1 else 1)   # wall at R: u = 0 half a cell away
        wl = eta * rf[i] / dr
        L[i, i] = -(wl + wr + eta * dr / r[i]) / m
        if i > 0:
            L[i, i - 1] = wl / m
        if i < n - 1:
            L[i, i + 1] = wr / m
    u = np.where(r < R0, omega * r, 0.0)
    dt = 0.05
    I = np.eye(n)
    step = np.linalg.solve(I - 0.5 * dt * L, I + 0.5 * dt * L)
    for _ in range(int(round(T / dt))):
        u = step @ u
    return r, u


def test_radial_equal_densities_give_bessel_zeros():
    """One fluid: the container's modes are J1(c r / sqrt(nu)) with
    c R / sqrt(nu) the zeros of J1."""
    from scipy.special import jn_zeros
    R0, R, eta = 12.0, 36.0, 0.333
    cs = A.radial_eigenvalues(R0, R, eta, eta, 8)
    assert np.max(np.abs(cs * R / math.sqrt(eta) / jn_zeros(1, 8) - 1.0)) < 1e-12


def test_radial_modes_orthonormal_and_matched():
    R0, R, rho1, rho2, eta = 12.0, 36.0, 1.0, 0.2, 0.333
    cs, a, b = A.radial_modes(R0, R, rho1, rho2, eta, 6)
    r = np.linspace(0, R, 400001)
    rho = np.where(r < R0, rho1, rho2)
    phis = [A.radial_phi(r, c, an, bn, R0, R, rho1, rho2, eta) for c, an, bn in zip(cs, a, b)]
    for i in range(6):
        for j in range(6):
            v = np.trapezoid(rho * r * phis[i] * phis[j], r)
            assert abs(v - (1.0 if i == j else 0.0)) < 1e-5
    # value and slope continuous at R0, zero at the wall
    h = 1e-6
    for c, an, bn in zip(cs, a, b):
        f = lambda x: float(A.radial_phi(x, c, an, bn, R0, R, rho1, rho2, eta))
        assert abs(f(R0 - h) - f(R0 + h)) < 1e-5 * abs(an)
        s_in = (f(R0 - h) - f(R0 - 2 * h)) / h
        s_out = (f(R0 + 2 * h) - f(R0 + h)) / h
        assert abs(s_in - s_out) < 1e-3 * max(abs(s_in), 1e-12)
        assert abs(f(R)) < 1e-12


@pytest.mark.parametrize("rho2", [1.0, 0.2])
def test_radial_transient_matches_finite_differences(rho2):
    R0, R, eta, omega, T = 12.0, 36.0, 0.333, 1e-3, 60.0
    r, ufd = fd_radial(R0, R, 1.0, rho2, eta, omega, T)
    ua = A.radial_transient(r, T, R0, R, 1.0, rho2, eta, omega, n_modes=150)
    assert np.max(np.abs(ua - ufd)) < 2e-5 * omega * R0   # measured 2.4e-6

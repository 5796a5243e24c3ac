"""Semi-analytic reference flows used to pin the oracle (test infrastructure only).

* ``flat_transient``    App. C: decay of a sheared two-layer flow between
                         no-slip walls, Sturm-Liouville eigen-expansion.
* ``stratified_steady`` App. D: steady force-driven flow with a continuous
                         transverse density profile, Simpson quadrature.
* ``radial_transient``  App. D (curved interfaces): decay of an azimuthal flow
                         in a circular container with a dense core,
                         Bessel-function eigen-expansion.
* ``laplace_pressure``  Laplace's law for a 2D drop, Delta p = sigma / R
                         (Sec. IV, curved interfaces).
* ``transient_error``   the error measure epsilon(t) of Sec. IV.
"""
import functools
import math
import numpy as np


# ----------------------------------------------------------------------------
# App. C: flat-interface transient
# ----------------------------------------------------------------------------

def _char(c, H, rho1, rho2, eta1, eta2):
    """Matching condition of the two sine pieces at x = H/2 (kinematic + traction).

    With equal shear viscosities this is App. C's
        sqrt(rho2) tan(c H / (2 sqrt(nu1))) + sqrt(rho1) tan(c H / (2 sqrt(nu2))) = 0;
    for unequal ones the traction condition eta1 phi1' = eta2 phi2' turns it into
        sqrt(eta2 rho2) tan(a) + sqrt(eta1 rho1) tan(b) = 0,
    a = c H/(2 sqrt(nu1)), b = c H/(2 sqrt(nu2)).  Written here in the
    pole-free form sqrt(eta2 rho2) sin a cos b + sqrt(eta1 rho1) cos a sin b.
    """
    nu1, nu2 = eta1 / rho1, eta2 / rho2
    a = c * H / (2.0 * math.sqrt(nu1))
    b = c * H / (2.0 * math.sqrt(nu2))
    return math.sqrt(eta2 * rho2) * math.sin(a) * math.cos(b) + \
        math.sqrt(eta1 * rho1) * math.cos(a) * math.sin(b)


def eigenvalues(H, rho1, rho2, eta1, eta2, n_modes):
    """First n_modes positive roots c_n of the matching condition.

    App. C solves it by Newton iteration; here roots are bracketed on a fine
    grid and refined by bisection followed by Newton polishing.
    """
    nu1, nu2 = eta1 / rho1, eta2 / rho2
    cmax_step = math.pi / (H / (2.0 * math.sqrt(min(nu1, nu2)))) / 64.0
    roots = []
    c = cmax_step * 1e-3
    f_prev = _char(c, H, rho1, rho2, eta1, eta2)
    while len(roots) < n_modes:
        c_next = c + cmax_step
        f_next = _char(c_next, H, rho1, rho2, eta1, eta2)
        if f_prev == 0.0 or f_prev * f_next < 0.0:
            lo, hi = c, c_next
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                fm = _char(mid, H, rho1, rho2, eta1, eta2)
                if (fm < 0) == (_char(lo, H, rho1, rho2, eta1, eta2) < 0):
                    lo = mid
                else:
                    hi = mid
            roots.append(0.5 * (lo + hi))
        c, f_prev = c_next, f_next
    return np.array(roots)


def flat_modes(H, rho1, rho2, eta1, eta2, n_modes):
    """Eigen-pairs (c_n, A1_n, A2_n) of App. C (normalised: int rho phi_n^2 = 1)."""
    nu1, nu2 = eta1 / rho1, eta2 / rho2
    cs = eigenvalues(H, rho1, rho2, eta1, eta2, n_modes)
    A1, A2 = [], []
    for c in cs:
        a = c * H / (2.0 * math.sqrt(nu1))
        b = c * H / (2.0 * math.sqrt(nu2))
        ratio = math.sin(a) / math.sin(b)
        norm = rho1 * (H - math.sqrt(nu1) / c * math.sin(c * H / math.sqrt(nu1))) + \
            ratio ** 2 * rho2 * (H - math.sqrt(nu2) / c * math.sin(c * H / math.sqrt(nu2)))
        a1 = 2.0 / math.sqrt(norm)
        A1.append(a1)
        A2.append(-a1 * ratio)
    return cs, np.array(A1), np.array(A2)


def flat_phi(x, c, a1, a2, H, rho1, rho2, eta1, eta2):
    """Eigenfunction phi_n(x): A1 sin(c x/sqrt(nu1)) on [0, H/2), A2 sin(c (x-H)/sqrt(nu2)) beyond."""
    nu1, nu2 = eta1 / rho1, eta2 / rho2
    x = np.asarray(x, dtype=float)
    return np.where(x < H / 2.0, a1 * np.sin(c * x / math.sqrt(nu1)),
                    a2 * np.sin(c * (x - H) / math.sqrt(nu2)))


def flat_transient(x, t, H, rho1, rho2, eta1, eta2, u0, n_modes=200):
    """u(x, t) for the initial profile u = +u0 on [0, H/2), -u0 on [H/2, H] (App. C).

    sigma_n follows App. C's closed form (projection of the step initial
    condition with weight rho).
    """
    nu1, nu2 = eta1 / rho1, eta2 / rho2
    cs, A1, A2 = flat_modes(H, rho1, rho2, eta1, eta2, n_modes)
    u = np.zeros_like(np.asarray(x, dtype=float))
    for c, a1, a2 in zip(cs, A1, A2):
        a = c * H / (2.0 * math.sqrt(nu1))
        b = c * H / (2.0 * math.sqrt(nu2))
        sig = a1 * u0 / c * (rho1 * math.sqrt(nu1) * (1.0 - math.cos(a))
                             - rho2 * math.sqrt(nu2) * math.sin(a) / math.sin(b) * (1.0 - math.cos(b)))
        u = u + sig * math.exp(-c * c * t) * flat_phi(x, c, a1, a2, H, rho1, rho2, eta1, eta2)
    return u


def two_layer_steady(x, H, eta1, eta2, G):
    """Steady two-layer channel flow under body-force density G along the
    walls (layer 1 on [0, H/2), layer 2 on [H/2, H]): piecewise parabolas
    joined by continuity of u and of the shear stress eta u'."""
    h = H / 2.0
    # u1 = -G x^2/(2 eta1) + a1 x ; u2 = -G (x-H)^2/(2 eta2) + a2 (x - H)
    A = np.array([[h, h], [eta1, -eta2]], dtype=float)
    rhs = np.array([G * h * h / (2 * eta1) - G * h * h / (2 * eta2), 2 * G * h])
    a1, a2 = np.linalg.solve(A, rhs)
    x = np.asarray(x, dtype=float)
    return np.where(x < h, -G * x * x / (2 * eta1) + a1 * x,
                    -G * (x - H) ** 2 / (2 * eta2) + a2 * (x - H))


def startup_transient(x, t, H, rho1, rho2, eta1, eta2, G, n_modes=200, nquad=4001):
    """Flow started from rest under body force G: u_ss(x) - sum_n s_n e^{-c_n^2 t} phi_n(x),
    s_n = int rho u_ss phi_n dx (orthonormality of App. C's eigenfunctions)."""
    cs, A1, A2 = flat_modes(H, rho1, rho2, eta1, eta2, n_modes)
    xq = np.linspace(0.0, H, nquad)
    rq = np.where(xq < H / 2.0, rho1, rho2)
    uss_q = two_layer_steady(xq, H, eta1, eta2, G)
    u = two_layer_steady(x, H, eta1, eta2, G)
    for c, a1, a2 in zip(cs, A1, A2):
        ph = flat_phi(xq, c, a1, a2, H, rho1, rho2, eta1, eta2)
        s = np.trapezoid(rq * uss_q * ph, xq)
        u = u - s * math.exp(-c * c * t) * flat_phi(x, c, a1, a2, H, rho1, rho2, eta1, eta2)
    return u


# ----------------------------------------------------------------------------
# App. D: steady flow with continuous stratification
# ----------------------------------------------------------------------------

def ba_density(x, H, rho0R, rho0B, beta):
    """Symmetric transverse stratification of App. D: rho0B at the walls,
    rho0R in the core, tanh interfaces of width 1/beta centred at H/4 and 3H/4."""
    x = np.asarray(x, dtype=float)
    lower = np.tanh(beta * (x - H / 4.0))
    upper = np.tanh(beta * (3.0 * H / 4.0 - x))
    th = np.where(x < H / 2.0, lower, upper)
    return 0.5 * (rho0R + rho0B) + 0.5 * (rho0R - rho0B) * th


def _simpson(fx, h):
    """Composite Simpson rule on an odd number of equally spaced samples."""
    n = len(fx) - 1
    assert n % 2 == 0
    return h / 3.0 * (fx[0] + fx[-1] + 4.0 * fx[1:-1:2].sum() + 2.0 * fx[2:-1:2].sum())


def stratified_steady(x, H, nu, G, density, nsub=400):
    """u(x) = G/(2 nu) int_0^x (H - 2a)/rho(a) da for x <= H/2, mirrored above (App. D).

    App. D writes the balance as d/dx(eta du/dx) = G for a pressure gradient
    -G; for a body force density G along the flow the balance is
    d/dx(eta du/dx) = -G, which flips the integrand's sign to (H - 2a).
    Evaluated with Simpson's rule as in App. D; ``density`` is a callable.
    """
    out = []
    for xv in np.atleast_1d(np.asarray(x, dtype=float)):
        xs = xv if xv <= H / 2.0 else H - xv
        if xs <= 0.0:
            out.append(0.0)
            continue
        a = np.linspace(0.0, xs, 2 * nsub + 1)
        fx = (H - 2.0 * a) / density(a)
        out.append(G / (2.0 * nu) * _simpson(fx, xs / (2 * nsub)))
    return np.array(out)


# ----------------------------------------------------------------------------
# App. D, curved interfaces: azimuthal transient in a circular container
# ----------------------------------------------------------------------------
# rho(r) du/dt = (1/r^2) d/dr (r^3 eta d/dr (u/r)), u(R) = 0, fluid 1 (density
# rho1) for r < R0, fluid 2 beyond, one shear viscosity eta.  In each region
# u = e^{-c^2 t} phi(r) with phi'' + phi'/r - phi/r^2 = -(c^2/nu) phi (Bessel's
# equation of order 1 in k r, k = c/sqrt(nu)): phi = a J1(k1 r) inside (regular
# at 0) and b Z(r) outside, Z(r) = J1(k2 r) Y1(k2 R) - Y1(k2 r) J1(k2 R)
# (zero at the wall).  Continuity of u and of the traction eta r d/dr(u/r)
# (with one eta: of phi and phi') at R0 fixes c.  The modes are orthogonal
# with weight rho r (the paper writes the same weight as r/nu = r rho/eta).

def _radial_parts(c, R0, R, nu1, nu2):
    """(J1(k1 R0), k1 J1'(k1 R0), Z(R0), Z'(R0), k1, k2)."""
    from scipy.special import j1, y1, jvp, yvp
    k1, k2 = c / math.sqrt(nu1), c / math.sqrt(nu2)
    jR, yR = j1(k2 * R), y1(k2 * R)
    Z = j1(k2 * R0) * yR - y1(k2 * R0) * jR
    dZ = k2 * (jvp(1, k2 * R0) * yR - yvp(1, k2 * R0) * jR)
    return j1(k1 * R0), k1 * jvp(1, k1 * R0), Z, dZ, k1, k2


def _radial_char(c, R0, R, nu1, nu2):
    """Matching determinant: zero when a J1 and b Z join with equal value and slope."""
    J, dJ, Z, dZ, _, _ = _radial_parts(c, R0, R, nu1, nu2)
    return J * dZ - dJ * Z


def radial_eigenvalues(R0, R, nu1, nu2, n_modes):
    """First n_modes positive roots c_n of the matching determinant (the paper
    uses Newton iteration; here a fine scan brackets each root and Brent's
    method refines it)."""
    from scipy.optimize import brentq
    step = math.pi * math.sqrt(min(nu1, nu2)) / R / 64.0
    roots = []
    c = step * 1e-3
    f_prev = _radial_char(c, R0, R, nu1, nu2)
    while len(roots) < n_modes:
        c_next = c + step
        f_next = _radial_char(c_next, R0, R, nu1, nu2)
        if f_prev * f_next < 0.0:
            roots.append(brentq(_radial_char, c, c_next, args=(R0, R, nu1, nu2), xtol=1e-15, rtol=1e-15))
        c, f_prev = c_next, f_next
    return np.array(roots)


def _lommel(C, dC, k, r):
    """int_0^r s C(k s)^2 ds for a cylinder function C of order 1 (Lommel's
    integral): r^2/2 [C'(k r)^2 + (1 - 1/(k r)^2) C(k r)^2], minus its value at
    the lower end (zero for J1 at 0)."""
    x = k * r
    return 0.5 * r * r * (dC(x) ** 2 + (1.0 - 1.0 / (x * x)) * C(x) ** 2)


@functools.lru_cache(maxsize=32)
def radial_modes(R0, R, rho1, rho2, eta, n_modes):
    """Eigen-pairs: c_n and the coefficients (a_n, b_n) of phi_n = a_n J1(k1 r)
    inside, b_n Z(r) outside, normalised so that int_0^R rho r phi_n^2 dr = 1."""
    from scipy.special import j1, y1, jvp, yvp
    nu1, nu2 = eta / rho1, eta / rho2
    cs = radial_eigenvalues(R0, R, nu1, nu2, n_modes)
    a, b = [], []
    for c in cs:
        J, dJ, Z, dZ, k1, k2 = _radial_parts(c, R0, R, nu1, nu2)
        # b Z(R0) = a J1(k1 R0): take a = 1, then b from whichever is larger
        bb = J / Z if abs(Z) > abs(dZ) / k2 else dJ / dZ
        jR, yR = j1(k2 * R), y1(k2 * R)
        Cz = lambda x: j1(x) * yR - y1(x) * jR
        dCz = lambda x: jvp(1, x) * yR - yvp(1, x) * jR
        inner = _lommel(j1, lambda x: jvp(1, x), k1, R0)
        outer = _lommel(Cz, dCz, k2, R) - _lommel(Cz, dCz, k2, R0)
        norm = rho1 * inner + rho2 * bb * bb * outer
        s = 1.0 / math.sqrt(norm)
        a.append(s)
        b.append(s * bb)
    return cs, np.array(a), np.array(b)


def radial_phi(r, c, a, b, R0, R, rho1, rho2, eta):
    """phi_n(r) of the container transient."""
    from scipy.special import j1, y1
    nu1, nu2 = eta / rho1, eta / rho2
    k1, k2 = c / math.sqrt(nu1), c / math.sqrt(nu2)
    r = np.asarray(r, dtype=float)
    Z = j1(k2 * r) * y1(k2 * R) - y1(k2 * r) * j1(k2 * R)
    return np.where(r < R0, a * j1(k1 * r), b * Z)


def radial_transient(r, t, R0, R, rho1, rho2, eta, omega, n_modes=200):
    """u_phi(r, t) from rigid rotation u_phi = omega r of the core (r < R0),
    fluid 2 at rest: sigma_n = int rho r u_phi(r, 0) phi_n dr
    = rho1 a_n omega R0^2 J2(k1 R0) / k1 (int_0^R0 r^2 J1(k r) dr = R0^2 J2(k R0)/k)."""
    from scipy.special import jv
    nu1 = eta / rho1
    cs, a, b = radial_modes(R0, R, rho1, rho2, eta, n_modes)
    u = np.zeros_like(np.asarray(r, dtype=float))
    for c, an, bn in zip(cs, a, b):
        k1 = c / math.sqrt(nu1)
        sig = rho1 * an * omega * R0 * R0 * jv(2, k1 * R0) / k1
        u = u + sig * math.exp(-c * c * t) * radial_phi(r, c, an, bn, R0, R, rho1, rho2, eta)
    return u


# ----------------------------------------------------------------------------
# Sec. IV: Laplace law and the transient error measure
# ----------------------------------------------------------------------------

def laplace_pressure(sigma, R):
    """Pressure step across a 2D (cylindrical) interface of radius R: sigma / R."""
    return sigma / R


def transient_error(u_sim, u_theory):
    """epsilon(t) of Sec. IV: sum_i |u - u*|^2 / max(u*)^2 over the transverse
    lattice points, divided by their number (the text calls it a domain average)."""
    u_sim = np.asarray(u_sim, dtype=float)
    u_theory = np.asarray(u_theory, dtype=float)
    return float(np.sum((u_theory - u_sim) ** 2) / np.max(np.abs(u_sim)) ** 2 / len(u_sim))

"""Physics pins of the oracle (each tens of seconds on the CPU):

* Laplace's law for a static drop (Sec. IV, curved interfaces);
* single-phase Poiseuille flow between half-way bounce-back walls;
* App. C flat-interface transient, error epsilon(t) below the paper's 1 % bound;
* App. D steady stratified ("Ba") flow, same bound;
* width of a flat interface at rest (Sec. II re-colour with unit link
  vectors) and its position at density ratios 10 and 100 (colour index).

Inputs follow the paper's set-ups at reduced size; the flat-interface and
stratified runs start from the relaxed tanh colour profile (Sec. II,
kinematic solution) rather than a step, to keep the start-up transient of a
sharp density jump out of the comparison.
"""
import math

import numpy as np
import pytest
import torch

from oracle import analytic as A
from oracle import chromo as O
from oracle.lattice import C
from paper_2005_04642_amd import workloads as Wk

torch.set_default_dtype(torch.float64)

pytestmark = pytest.mark.slow


def test_laplace_law_static_drop():
    """Delta p = p(centre) - p(far field) = sigma / R_eff within 5 % for two
    tensions (p is the isotropic equilibrium pressure of App. A,
    R_eff from the red area)."""
    n, R = 48, 12.0
    for sigma in (0.0025, 0.01):
        d = Wk.base_params(Lambda=10.0, sigma=sigma)
        p = O.Params(nx=n, ny=n, **d)
        o = O.Oracle(p).init(Wk.static_drop(n, n, R))
        o.step(2000)
        f = o.fields()
        P = O.isotropic_pressure(f["rhoR"], f["rhoB"], p)
        c = n // 2
        dp = float(P[c - 1:c + 1, c - 1:c + 1].mean() - P[0:2, 0:2].mean())
        Reff = math.sqrt(float(((1 + f["rhoN"]) / 2).sum()) / math.pi)
        ratio = dp / A.laplace_pressure(sigma, Reff)
        assert abs(ratio - 1.0) < 0.05, (sigma, ratio)


def test_single_phase_poiseuille():
    """Pure red fluid, body force g between walls at y = 1/2 and H + 1/2:
    u(y) = g y (H - y) / (2 eta) within 1e-3 relative L2."""
    H = 16
    d = Wk.base_params(Lambda=10.0)
    d.update(walls=True, gx=1e-6)
    p = O.Params(nx=4, ny=H + 2, **d)
    o = O.Oracle(p).init(np.ones((H + 2, 4)))
    o.step(1500)
    u = o.fields()["ux"][1:-1, 0].numpy()
    y = np.arange(H) + 0.5
    ua = 1e-6 * y * (H - y) / (2 * d["nu_R"] * d["rho0_R"])
    assert np.linalg.norm(u - ua) / np.linalg.norm(ua) < 1e-3


@pytest.mark.parametrize("Lam", [2.0, 10.0])
def test_flat_interface_transient(Lam):
    """App. C: red (dense) half moving +u0, blue half -u0, equal shear
    viscosity eta = 1/6, beta = 0.5; epsilon(t) against the Sturm-Liouville
    solution stays below the paper's 1 % bound (Table 3 text)."""
    H, eta, beta, u0 = 64, 1.0 / 6.0, 0.5, 1e-2
    d = Wk.base_params(Lambda=Lam, beta=beta)
    d.update(walls=True, nu_R=eta / 1.0, nu_B=eta * Lam)
    p = O.Params(nx=4, ny=H + 2, **d)
    yy = (np.arange(H + 2) - 0.5)[:, None] * np.ones((1, 4))
    rn = np.tanh(0.9 * beta * (H / 2 - yy))
    o = O.Oracle(p).init_moving(rn, u0 * rn, np.zeros_like(rn))
    y = np.arange(H) + 0.5
    done = 0
    for T in (250, 1000):
        o.step(T - done)
        done = T
        u = o.fields()["ux"][1:-1, 0].numpy()
        ua = A.flat_transient(y, T, H, 1.0, 1.0 / Lam, eta, eta, u0, n_modes=400)
        eps = A.transient_error(u, ua)
        assert eps < 0.01, (T, eps)


def test_stratified_steady_flow_ba():
    """App. D / Sec. IV A: a_B = 0.2, a_R = 0.9 (Lambda = 8), nu = 0.333, blue
    against the walls and red in the core; the steady profile matches the
    Simpson-rule semi-analytic solution built from the run's own density
    profile, epsilon < 1 %.  This flow exercises the density-contrast source
    F_1 (C_xy = -(1 - l3/2) u_x d_y Phi' is non-zero across the interfaces)."""
    H, beta, G = 32, 0.67, 2e-6
    d = Wk.base_params(Lambda=8.0, beta=beta)
    d.update(walls=True, alpha_R=0.9, alpha_B=0.2, nu_R=0.333, nu_B=0.333, gx=G)
    p = O.Params(nx=4, ny=H + 2, **d)
    yy = (np.arange(H + 2) - 0.5)[:, None] * np.ones((1, 4))
    rn = np.where(yy < H / 2, np.tanh(0.9 * beta * (yy - H / 4)), np.tanh(0.9 * beta * (3 * H / 4 - yy)))
    o = O.Oracle(p).init(rn)
    o.step(4500)
    f = o.fields()
    u = f["ux"][1:-1, 0].numpy()
    rho = f["rho"][1:-1, 0].numpy()
    y = np.arange(H) + 0.5
    ua = A.stratified_steady(y, H, 0.333, G, lambda a: np.interp(a, y, rho))
    assert A.transient_error(u, ua) < 0.01


# ---------------------------------------------------------------------------
# Width and position of a flat interface at rest (Sec. II re-colour equation
# and the modified equation that follows it).
#
# At rest with sigma = 0 the steady colour profile balances two fluxes of the
# red density.  The pull gather expanded to second order (the modified
# equation of Sec. II) gives the diffusive flux (1/2) d/dy sum_i c_iy^2 R_i++
# = (3/10) d/dy (mu rho_R), with mu rho = (1 - a_R) rho_R + (1 - a_B) rho_B
# (the second moment of the proportional split is (rho_R/rho) P and P = 3/5 mu
# rho).  The re-colour adds the segregation flux sum_i c_iy t_i
# = beta (rho_R rho_B / rho) (9/5) mu S, with S = sum_i w_i c_iy (m . c_hat_i)
# = (2 + 1/sqrt 2)/9 for the unit link vectors c_hat_i that the re-colour
# equation prints (axis links 2/9, diagonal links 4/(36 sqrt 2)).  A flat
# interface has no curvature, so P is uniform and mu rho is constant; the
# balance then gives, for the mass fraction phi = rho_R / rho,
#     d phi / dy = 2 k beta phi (1 - phi),  k = 9 S / 3 = (2 + 1/sqrt 2)/3,
# i.e. 2 phi - 1 = tanh(k beta (y - y0)), k = 0.9024.  The modified equation
# as printed carries the coefficient k_phi c_s^2 = (9/5)(1/3), which is what
# the plain link vectors c_i give in place of c_hat_i (sum_i w_i c_iy c_iy =
# 1/3): k = 1, the tanh(beta n.r) of eq. equ_rhoN.  The width tells the two
# readings apart (the oracle follows the printed re-colour equation).
# ---------------------------------------------------------------------------

K_UNIT_LINKS = (2.0 + 1.0 / math.sqrt(2.0)) / 3.0


def _flat_slab(Lam, beta, ny, steps, k0):
    """Periodic red slab between y = ny/4 and 3 ny/4 (one column), sigma = 0,
    started from tanh(k0 beta y) profiles and stepped to steady state."""
    d = Wk.base_params(Lambda=Lam, beta=beta, sigma=0.0)
    p = O.Params(nx=1, ny=ny, **d)
    y = np.arange(ny)[:, None].astype(float)
    rn = np.tanh(k0 * beta * (y - ny / 4)) * -np.tanh(k0 * beta * (y - 3 * ny / 4))
    o = O.Oracle(p).init(rn).step(steps)
    return p, o.fields()


def _tanh_width(profile, beta):
    """k of a fit of profile(y) = tanh(k beta (y - y0)) across the lower
    interface (points with |profile| < 0.8)."""
    v = np.asarray(profile)[:, 0]
    y = np.arange(len(v))
    sel = (np.abs(v) < 0.8) & (y < len(v) / 2)
    return float(np.polyfit(y[sel], np.arctanh(v[sel]), 1)[0] / beta)


@pytest.mark.parametrize("beta,ny,steps,k0", [(0.1, 240, 2500, 0.95), (0.2, 120, 1500, 1.0)])
def test_flat_interface_width_of_the_recolour(beta, ny, steps, k0):
    """Lambda = 1: rho^N = 2 phi - 1 = tanh(k beta y) with k = (2 + 1/sqrt 2)/3
    within 1 % (the O(beta^2) lattice corrections measure 0.1-0.2 % here)."""
    _, f = _flat_slab(1.0, beta, ny, steps, k0)
    k = _tanh_width(f["rhoN"].numpy(), beta)
    assert abs(k / K_UNIT_LINKS - 1.0) < 0.01, k


def test_flat_interface_width_separates_the_link_vector_readings(monkeypatch):
    """The same slab with the plain link vectors c_i in the re-colour settles
    at k = 1 (measured 0.997), outside the 1 % band of the pin above: the pin
    decides between the two readings of Sec. II."""
    monkeypatch.setattr(O, "CHAT", tuple((float(cx), float(cy)) for cx, cy in C))
    _, f = _flat_slab(1.0, 0.2, 120, 1000, 0.9)
    k = _tanh_width(f["rhoN"].numpy(), 0.2)
    assert k > 0.98, k
    assert abs(k / K_UNIT_LINKS - 1.0) > 0.05


@pytest.mark.parametrize("Lam", [10.0, 100.0])
def test_flat_interface_at_density_ratio(Lam):
    """Lambda = 10, 100: the steady mass fraction follows 2 phi - 1 = tanh(k beta y)
    (same k, within 1 %); the isotropic pressure P of App. A is uniform across
    the flat interface (mechanical equilibrium, 2e-4); uniform P means
    rho_R/rho_0R + rho_B/rho_0B = 1, so the colour index of Sec. II is
    2 rho_R/rho_0R - 1 there (measured within 3e-5 and 7e-5).  A colour index
    without the 1/rho_0C normalisation, (rho_R - rho_B)/rho, misses that by
    O(1) at these density ratios."""
    beta = 0.2
    p, f = _flat_slab(Lam, beta, 120, 2000, 0.9)
    rR, rB = f["rhoR"].numpy(), f["rhoB"].numpy()
    phi = rR / (rR + rB)
    k = _tanh_width(2.0 * phi - 1.0, beta)
    assert abs(k / K_UNIT_LINKS - 1.0) < 0.01, k
    P = O.isotropic_pressure(f["rhoR"], f["rhoB"], p).numpy()
    assert (P.max() - P.min()) / P.mean() < 2e-4
    a = rR / p.rho0_R
    assert np.max(np.abs(f["rhoN"].numpy() - (2.0 * a - 1.0))) < 2e-4
    assert np.max(np.abs((rR - rB) / (rR + rB) - (2.0 * a - 1.0))) > 0.5

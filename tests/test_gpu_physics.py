"""Physics of the GPU path itself (not only its agreement with the oracle):
Laplace's law for a static drop (Sec. IV, curved interfaces: the pressure
step across a drop follows sigma / R), in FP32 on the static-drop workload's
lattice, for two tensions and two radii."""
import math

import numpy as np
import pytest
import torch

from oracle import analytic as A
from oracle import chromo as O
from paper_2005_04642_amd import lbm, workloads as Wk

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def colour_densities(rho, rhoN, p):
    """rho_R, rho_B from rho and rho^N = (a - b)/(a + b), a = rho_R/rho0_R, b = rho_B/rho0_B."""
    s = 2.0 * rho / (p["rho0_R"] * (1.0 + rhoN) + p["rho0_B"] * (1.0 - rhoN))
    return p["rho0_R"] * (1.0 + rhoN) * s / 2.0, p["rho0_B"] * (1.0 - rhoN) * s / 2.0


@pytest.mark.parametrize("sigma,R", [(0.0025, 16.0), (0.01, 16.0), (0.01, 12.0)])
def test_laplace_law(sigma, R):
    """Delta p = p(centre) - p(far field) = sigma / R_eff within 5 % after 2000
    steps (p the isotropic equilibrium pressure of App. A, R_eff from the red
    area), Lambda = 10, 64x64 periodic."""
    n = 64
    d = Wk.base_params(Lambda=10.0, sigma=sigma)
    sim = lbm.Simulation(n, n, d, Wk.static_drop(n, n, R), storage="f32", device=DEV)
    sim.step(2000)
    f = {k: v.double().cpu().numpy() for k, v in sim.fields().items()}
    sim.close()
    rR, rB = colour_densities(f["rho"], f["rhoN"], d)
    P = O.isotropic_pressure(rR, rB, O.Params(nx=n, ny=n, **d))
    c = n // 2
    dp = float(P[c - 1:c + 1, c - 1:c + 1].mean() - P[0:2, 0:2].mean())
    Reff = math.sqrt(float(((1 + f["rhoN"]) / 2).sum()) / math.pi)
    ratio = dp / A.laplace_pressure(sigma, Reff)
    print("Laplace sigma %g R %g: dp / (sigma / R_eff) = %.4f" % (sigma, R, ratio))
    assert abs(ratio - 1.0) < 0.05

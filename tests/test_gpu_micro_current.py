"""Inter-facial micro-current of a static drop against Tables 1 and 2 of the
paper (Sec. IV, inter-facial micro-current): a red drop of radius 60 on a
200 x 200 periodic lattice, with the curvature computed (Table 2) or fixed at
K = 1/R (Table 1), alpha from the density ratio as in the tables.

The paper prints neither sigma, beta, nu nor the run length, so the printed
magnitudes are only comparable where the micro-current does not depend on
them.  The paper attributes the large-Lambda micro-current to the density
contrast (both tables give the same values there); these runs use this
build's readings (sigma 0.01, beta 0.67, nu 1/6, 40000 steps from a tanh
profile of width 2, steady by then) and check:
* Lambda = 1000: max|u| within a factor 2 of the printed 7.8e-5;
* Lambda = 100: within an order of magnitude of the printed 1.8e-5;
* Lambda >= 100: fixed and computed curvature give the same max|u| (10 %);
* Lambda = 10: fixed curvature lowers it (Table 1 against Table 2).
Measured: 7.1e-5 / 6.9e-5 (Lambda 1000, computed / fixed), 4.8e-5 / 4.7e-5
(Lambda 100), 2.5e-6 / 7.4e-7 (Lambda 10; the paper's 1.8e-7 / 1.3e-9 there
are interface-force dominated and so depend on the unprinted sigma)."""
import json
import os

import numpy as np
import pytest
import torch

from paper_2005_04642_amd import lbm, workloads as Wk

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))["micro_current_tables"]
STEPS = 40000


def printed(table, Lam):
    return dict((row[0], row[1] * 1e-5) for row in GOLD[table])[Lam]


def umax(Lam, fixed):
    n, R = GOLD["n"], float(GOLD["R"])
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    c = (n - 1) / 2.0
    rn = np.tanh((R - np.hypot(x - c, y - c)) / 2.0)
    p = Wk.base_params(Lambda=Lam, sigma=0.01)
    if fixed:
        p["fixed_K"] = 1.0 / R
    sim = lbm.Simulation(n, n, p, rn, storage="f64", device=DEV)
    sim.step(STEPS)
    f = sim.fields()
    u = float(torch.sqrt(f["ux"] ** 2 + f["uy"] ** 2).max())
    m = sim.masses()
    sim.close()
    assert np.isfinite(u) and all(np.isfinite(m))
    print("micro-current Lambda %g %s K: max|u| = %.3e" % (Lam, "fixed" if fixed else "computed", u))
    return u


@pytest.fixture(scope="module")
def runs():
    return {(Lam, fixed): umax(Lam, fixed) for Lam in (10.0, 100.0, 1000.0) for fixed in (False, True)}


def test_large_density_ratio_matches_printed_magnitude(runs):
    for fixed, table in ((False, "computed_K"), (True, "fixed_K")):
        r1000 = runs[(1000.0, fixed)] / printed(table, 1000)
        r100 = runs[(100.0, fixed)] / printed(table, 100)
        assert 0.5 < r1000 < 2.0, (table, r1000)
        assert 0.1 < r100 < 10.0, (table, r100)


def test_curvature_choice_irrelevant_at_large_density_ratio(runs):
    for Lam in (100.0, 1000.0):
        assert abs(runs[(Lam, True)] / runs[(Lam, False)] - 1.0) < 0.1, Lam


def test_fixed_curvature_lowers_micro_current_at_Lambda_10(runs):
    assert printed("fixed_K", 10) < printed("computed_K", 10)
    assert runs[(10.0, True)] < 0.5 * runs[(10.0, False)]

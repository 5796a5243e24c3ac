"""Pins of the oracle's constants against the paper's printed values and the
lattice identities it states (App. A, App. B), in exact rational arithmetic."""
import json
import os
from fractions import Fraction
from itertools import product

import pytest

from oracle import lattice as L

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def frac(pair):
    return Fraction(pair[0], pair[1])


def test_weights_and_ghost_match_print():
    g = GOLD["d2q9_weights"]
    assert L.W_EXACT[0] == frac(g["w0"])
    for i in range(1, 9):
        assert L.W_EXACT[i] == (frac(g["w_odd"]) if i % 2 else frac(g["w_even"]))
    gv = GOLD["ghost_vector"]
    assert L.G_EXACT[0] == gv["g0"]
    for i in range(1, 9):
        assert L.G_EXACT[i] == (gv["g_odd"] if i % 2 else gv["g_even"])
    # odd links are the long ones (Fig. A1 caption)
    for i in range(1, 9):
        assert (abs(L.C[i][0]) + abs(L.C[i][1]) == 2) == (i % 2 == 1)
    assert Fraction(L.K_PHI).limit_denominator(10) == frac(GOLD["rest_fraction_k"]["k"])


def test_lattice_isotropy_identities():
    """App. A: sum w = 1, odd moments vanish, sum w c c = delta/3,
    sum w c c c c = (dd + dd + dd)/9."""
    w, c = L.W_EXACT, L.C
    assert sum(w) == 1
    for a in range(2):
        for p in range(4):
            assert sum(w[i] * c[i][a] ** (2 * p + 1) for i in range(9)) == 0
    d = lambda a, b: 1 if a == b else 0
    for a, b in product(range(2), repeat=2):
        assert sum(w[i] * c[i][a] * c[i][b] for i in range(9)) == Fraction(d(a, b), 3)
    for a, b, g, t in product(range(2), repeat=4):
        lhs = sum(w[i] * c[i][a] * c[i][b] * c[i][g] * c[i][t] for i in range(9))
        assert lhs == Fraction(d(a, b) * d(g, t) + d(a, g) * d(b, t) + d(a, t) * d(b, g), 9)


def test_opposites_and_unit_vectors():
    for i in range(9):
        j = L.OPP[i]
        assert L.C[j] == (-L.C[i][0], -L.C[i][1])
        assert L.OPP[j] == i
    for i in range(1, 9):
        assert abs(L.CHAT[i][0] ** 2 + L.CHAT[i][1] ** 2 - 1.0) < 1e-15


def test_projectors_and_printed_inverse_are_inverse():
    """h^(p) . k^(p') = delta_pp' (App. A, eq. for M^{-1}) with the unweighted
    rows; the w-weighted rows of Table A1 taken literally are not inverse to the
    printed k^(p) (this is why the unweighted reading is adopted)."""
    H = L.projector_rows_exact()
    K = L.inverse_columns_exact()
    for p in range(9):
        for q in range(9):
            dot = sum(H[p][i] * K[q][i] for i in range(9))
            assert dot == (1 if p == q else 0), (p, q, dot)
    weighted_ok = all(
        sum(L.W_EXACT[i] * H[p][i] * K[q][i] for i in range(9)) == (1 if p == q else 0)
        for p in range(9) for q in range(9))
    assert not weighted_ok


def test_high_order_stencil_solves_corrected_system():
    """App. B: the coefficient row b solves b . C = (3, 0, 0) with
    C_{Nj} = N^(2j-1)/(2j-1)!; the printed b matches the print, and the
    misprinted entry (2^3/5! in row 2) would not give it."""
    from math import factorial
    b = [frac(v) for v in GOLD["high_order_stencil"]["b"]]
    assert tuple(b) == L.high_order_stencil_exact()

    def mat(typo):
        m = [[Fraction(N ** (2 * j - 1), factorial(2 * j - 1)) for j in (1, 2, 3)] for N in (1, 2, 3)]
        if typo:
            m[1][2] = Fraction(2 ** 3, factorial(5))
        return m

    for typo, ok in ((False, True), (True, False)):
        m = mat(typo)
        # d f/dx = sum_N b_N S_N with S_N = (N/3) f' + ... so b . column_0 = 3 and b . other columns = 0
        cols = [sum(b[N] * m[N][j] for N in range(3)) for j in range(3)]
        assert (cols == [3, 0, 0]) == ok


def test_alpha_lambda_relation_holds_for_printed_tables():
    """Sec. II: Lambda = (1 - a_B)/(1 - a_R); every row of Tables 1-2 obeys it."""
    for lam, aB, aR in GOLD["micro_current_tables_alpha"]["rows"]:
        assert abs((1 - aB) / (1 - aR) - lam) <= 1e-9 * lam
    ba = GOLD["ba_test"]
    assert abs((1 - ba["alpha_B"]) / (1 - ba["alpha_R"]) - ba["Lambda"]) < 1e-12


def test_viscosity_rate_relation():
    """nu = (2/lambda_3 - 1)/6 (Sec. II / App. A): the oracle's lambda_3(rho^N)
    reproduces the printed pairs in a single-viscosity fluid."""
    import torch
    from oracle.chromo import Params, lambda3
    for nu, lam in GOLD["viscosity"]["pairs_nu_lambda3"]:
        p = Params(nx=1, ny=1, nu_R=nu, nu_B=nu)
        for rn in (-1.0, 0.0, 0.3, 1.0):
            assert abs(float(lambda3(torch.tensor(rn, dtype=torch.float64), p)) - lam) < 1e-15

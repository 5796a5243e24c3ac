"""D2Q9 lattice constants used by the oracle (test infrastructure only).

Indexing follows the paper's Fig. A1 convention that odd i are the long
(diagonal) links; the figure itself is not reproduced in the text, so the
angular order below (link i at angle i*45 degrees) is this oracle's reading.

* weights w_0 = 4/9, w_odd = 1/36, w_even = 1/9   (App. A, after the lattice
  isotropy identities, "Weightings w_i are those of Qian et al.")
* ghost vector g_0 = 1, g_odd = 4, g_even = -2    (App. A, Dellar ghost basis)
* lattice sound speed squared c_s^2 = 1/3          (isotropy identity
  sum_i w_i c_ia c_ib = delta_ab / 3, App. A)
* k = 9/5 in the rest-fraction weights phi_i      (Sec. II, eq. for phi_i)
"""
from fractions import Fraction
import math

Q = 9

# link vectors c_i, i = 0..8; odd i diagonal
C = ((0, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0))

W_EXACT = tuple(Fraction(4, 9) if i == 0 else (Fraction(1, 36) if i % 2 else Fraction(1, 9))
                for i in range(Q))
G_EXACT = tuple(1 if i == 0 else (4 if i % 2 else -2) for i in range(Q))

W = tuple(float(w) for w in W_EXACT)
GHOST = tuple(float(g) for g in G_EXACT)

CS2 = 1.0 / 3.0
K_PHI = 9.0 / 5.0


def opposite(i):
    """Index of the link pointing opposite to c_i."""
    cx, cy = C[i]
    return C.index((-cx, -cy))


OPP = tuple(opposite(i) for i in range(Q))

# unit link vectors c_i / |c_i| (c_0 -> 0); used by the recolour step (Sec. II)
CHAT = tuple((0.0, 0.0) if i == 0 else
             (C[i][0] / math.hypot(*C[i]), C[i][1] / math.hypot(*C[i])) for i in range(Q))


def projector_rows_exact():
    """Rows h^(p)_i of the projection matrix M (Table A1 and App. A).

    The table prints w-weighted definitions, but the projections the appendix
    then evaluates (h^(0).f = sum_i f_i = rho, h^(1).f = sum_i c_ix f_i, ...)
    use the unweighted polynomials; only the unweighted rows are the inverse of
    the printed k^(p) columns.  Reading adopted: unweighted rows
    (1, c_x, c_y, c_x^2, c_y^2, c_x c_y, g, g c_x, g c_y).
    """
    rows = []
    for p in range(Q):
        row = []
        for i in range(Q):
            cx, cy = C[i]
            g = G_EXACT[i]
            row.append(Fraction((1, cx, cy, cx * cx, cy * cy, cx * cy, g, g * cx, g * cy)[p]))
        rows.append(row)
    return rows


def inverse_columns_exact():
    """Columns k^(p)_i of M^{-1} exactly as printed in App. A (definitions of k^(p))."""
    cols = []
    for p in range(Q):
        col = []
        for i in range(Q):
            cx, cy = C[i]
            w = W_EXACT[i]
            g = G_EXACT[i]
            c2 = cx * cx + cy * cy
            val = (
                2 * w - Fraction(3, 2) * w * c2,                 # k^(0)
                3 * w * cx,                                      # k^(1)
                3 * w * cy,                                      # k^(2)
                Fraction(9, 2) * w * cx * cx - Fraction(3, 2) * w,  # k^(3)
                Fraction(9, 2) * w * cy * cy - Fraction(3, 2) * w,  # k^(4)
                9 * w * cx * cy,                                 # k^(5)
                Fraction(1, 4) * g * w,                          # k^(6)
                Fraction(3, 8) * g * w * cx,                     # k^(7)
                Fraction(3, 8) * g * w * cy,                     # k^(8)
            )[p]
            col.append(val)
        cols.append(col)
    return cols


def high_order_stencil_exact():
    """Coefficients b_N of the radius-3 first-derivative stencil (App. B).

    d f/dx = sum_{N=1..3} b_N sum_i w_i c_ix f(r + N c_i), with
    b = (9/2, -9/10, 1/10).  Obtained there by inverting the 3x3 matrix
    C_{Nj} = N^(2j-1)/(2j-1)!; the printed matrix carries a typo in row 2,
    column 3 (2^3/5! instead of 2^5/5!), and b matches the corrected matrix.
    """
    return (Fraction(9, 2), Fraction(-9, 10), Fraction(1, 10))


def compact_stencil_exact():
    """Radius-1 stencil d f/dx = 3 sum_i w_i c_ix f(r + c_i) (App. B with N = 1)."""
    return (Fraction(3),)


STENCIL_COEFFS = {1: tuple(float(b) for b in compact_stencil_exact()),
                  3: tuple(float(b) for b in high_order_stencil_exact())}

"""Pins of the App. B gradient stencils and of the wall mirror used with them."""
import math

import pytest
import torch

from oracle import brute
from oracle import chromo as O

torch.set_default_dtype(torch.float64)

N = 16


def grid():
    y, x = torch.meshgrid(torch.arange(N, dtype=torch.float64), torch.arange(N, dtype=torch.float64),
                          indexing="ij")
    return x - 7.3, y - 8.1


def monomials(deg):
    return [(a, deg - a) for a in range(deg + 1)]


@pytest.mark.parametrize("radius,exact_deg", [(1, 2), (3, 6)])
def test_stencil_exact_on_polynomials(radius, exact_deg):
    """App. B: the radius-3 stencil differentiates polynomials of degree <= 6
    exactly (the first surviving error term is E_7); the compact one degree <= 2."""
    X, Y = grid()
    inner = (slice(3, N - 3), slice(3, N - 3))   # stencil never crosses the periodic seam
    for deg in range(0, exact_deg + 2):
        worst = 0.0
        for a, b in monomials(deg):
            s = X ** a * Y ** b
            gx, gy = O.gradient(s, radius, walls=False)
            ex = a * X ** max(a - 1, 0) * Y ** b if a else torch.zeros_like(X)
            ey = b * X ** a * Y ** max(b - 1, 0) if b else torch.zeros_like(X)
            scale = float((X ** a * Y ** b).abs()[inner].max()) + 1.0
            worst = max(worst, float((gx - ex)[inner].abs().max()) / scale,
                        float((gy - ey)[inner].abs().max()) / scale)
        if deg <= exact_deg:
            assert worst < 1e-12, (deg, worst)
        else:
            assert worst > 1e-6, (deg, worst)


@pytest.mark.parametrize("radius,order", [(1, 2), (3, 6)])
def test_stencil_convergence_order(radius, order):
    """Observed order of accuracy on sin(k x) (error relative to the derivative
    amplitude, one wavelength per lattice) matches the design order."""
    errs = []
    for n in (32, 64):
        k = 2 * math.pi / n
        y, x = torch.meshgrid(torch.arange(4, dtype=torch.float64), torch.arange(n, dtype=torch.float64),
                              indexing="ij")
        s = torch.sin(k * x)
        gx, _ = O.gradient(s, radius, walls=False)
        errs.append(float((gx - k * torch.cos(k * x)).abs().max()) / k)   # relative to |d s/dx|
    observed = math.log2(errs[0] / errs[1])
    assert abs(observed - order) < 0.15, observed


def test_oracle_gradient_matches_per_site_stencil():
    g = torch.Generator().manual_seed(3)
    for walls in (False, True):
        nx, ny = 9, 11
        s_full = torch.rand(ny, nx, generator=g)
        rows = list(range(1, ny - 1)) if walls else list(range(ny))
        for radius in (1, 3):
            for odd in (False, True):
                gx, gy = O.gradient(s_full[rows], radius, walls, odd_y=odd)
                lst = s_full.tolist()
                for k, y in enumerate(rows):
                    for x in range(nx):
                        bx, by = brute.gradient_at(lst, x, y, nx, ny, radius, walls, odd_y=odd)
                        assert abs(bx - gx[k, x].item()) < 1e-15
                        assert abs(by - gy[k, x].item()) < 1e-15


def test_wall_mirror_even_and_odd_fields():
    """On a wall strip the stencil sees the mirror image about y = 1/2 (in
    full-lattice rows): an even quadratic about the wall and an odd linear
    function are both extended exactly, so their derivatives are exact right
    up to the wall (away from the far wall)."""
    nx, ny = 5, 40
    F = ny - 2
    k = torch.arange(F, dtype=torch.float64)[:, None].expand(F, nx)
    d = k + 0.5                          # distance from the bottom wall plane
    for radius in (1, 3):
        _, gy = O.gradient(d * d, radius, walls=True)
        assert float((gy[:10] - 2 * d[:10]).abs().max()) < 1e-12
        _, gy = O.gradient(d.clone(), radius, walls=True, odd_y=True)
        assert float((gy[:10] - 1.0).abs().max()) < 1e-12
        # the same odd field read as even sees a kink at the wall: derivative wrong there
        _, gy = O.gradient(d.clone(), radius, walls=True, odd_y=False)
        assert float((gy[0] - 1.0).abs().max()) > 0.1

"""Pins of the oracle's solid sites anywhere (a mask): half-way bounce-back at
every solid neighbour (the walls' rule, Sec. II kinetic equation) and the
zero-gradient continuation of the App. B stencils into the solid.

* an all-fluid mask is the periodic lattice, bit for bit;
* streaming with a mask against the per-site brute force (bit-exact, a
  permutation of the fluid sites' populations);
* stencils with a mask against the per-site brute force, zero on constants
  (to rounding), and unchanged wherever the footprint holds no solid site;
* a whole step against the per-site brute force on an 8x8 lattice;
* per-colour masses conserved around obstacles (FP64);
* a mask made of the two wall rows, single phase, x-independent flow: the
  same populations as the walls mode (its mirror image and the centre-value
  continuation give the same stencils there), so the mask inherits the
  walls' Poiseuille pin."""
import numpy as np
import pytest
import torch

from oracle import brute
from oracle import chromo as O
from oracle.lattice import C, Q
from paper_2005_04642_amd import workloads as Wk

torch.set_default_dtype(torch.float64)


def params(nx, ny, **kw):
    d = Wk.base_params(Lambda=10.0, sigma=0.02)
    d.update(kw)
    return O.Params(nx=nx, ny=ny, **d)


def perturbed(o, seed, scale=0.05):
    g = torch.Generator().manual_seed(seed)
    o.R = o.R * (1 + scale * torch.rand(o.R.shape, generator=g))
    o.B = o.B * (1 + scale * torch.rand(o.B.shape, generator=g))
    o._clear_solid()
    return o


def test_all_fluid_mask_is_the_periodic_lattice():
    n = 16
    rn = Wk.static_drop(n, n, 5.0)
    a = O.Oracle(params(n, n)).init(rn)
    b = O.Oracle(params(n, n, solid=np.zeros((n, n), bool))).init(rn)
    perturbed(a, 3)
    perturbed(b, 3)
    a.step(20)
    b.step(20)
    assert torch.equal(a.R, b.R) and torch.equal(a.B, b.B)


@pytest.mark.parametrize("shape,count,seed", [((6, 5), 4, 0), ((7, 7), 9, 1), ((5, 8), 1, 2)])
def test_streaming_with_mask_matches_brute_force_bit_exact(shape, count, seed):
    nx, ny = shape
    solid = Wk.random_solid_sites(nx, ny, count, seed)
    payload = [[[[float(((c * Q + i) * ny + y) * nx + x) for x in range(nx)] for y in range(ny)]
                for i in range(Q)] for c in range(2)]
    ref = brute.stream_site_by_site(payload, nx, ny, False, solid.tolist())
    P = torch.tensor(payload)
    m = torch.as_tensor(solid)
    for c in range(2):
        Pc = P[c].clone()
        Pc[:, m] = 0.0
        got = O.stream(Pc, False, m)
        for i in range(Q):
            for y in range(ny):
                for x in range(nx):
                    assert got[i, y, x].item() == ref[c][i][y][x], (c, i, x, y)
    # a permutation of the fluid sites' populations; solid sites hold 0
    fl = [(x, y) for y in range(ny) for x in range(nx) if not solid[y][x]]
    out = sorted(ref[c][i][y][x] for c in range(2) for i in range(Q) for (x, y) in fl)
    src = sorted(payload[c][i][y][x] for c in range(2) for i in range(Q) for (x, y) in fl)
    assert out == src
    assert all(ref[c][i][y][x] == 0.0 for c in range(2) for i in range(Q)
               for y in range(ny) for x in range(nx) if solid[y][x])


def test_brute_bounce_hand_case():
    """A link-8 (+x) population next to a solid site returns on link 4 at its
    own site; a link-1 (1,1) population whose target is fluid moves on."""
    nx = ny = 4
    solid = [[False] * nx for _ in range(ny)]
    solid[1][2] = True
    pops = [[[[0.0] * nx for _ in range(ny)] for _ in range(Q)] for _ in range(2)]
    pops[0][8][1][1] = 3.0
    pops[1][1][1][1] = 2.0
    out = brute.stream_site_by_site(pops, nx, ny, False, solid)
    assert out[0][4][1][1] == 3.0
    assert out[1][1][2][2] == 2.0


def test_gradient_with_mask_matches_brute_force_and_is_exact_on_constants():
    g = torch.Generator().manual_seed(5)
    nx, ny = 23, 19
    solid = Wk.random_solid_sites(nx, ny, 8, 7)
    m = torch.as_tensor(solid)
    s = torch.rand(ny, nx, generator=g)
    lst = s.tolist()
    for radius in (1, 3):
        gx, gy = O.gradient(s, radius, False, solid=m)
        for y in range(ny):
            for x in range(nx):
                if solid[y][x]:
                    continue
                bx, by = brute.gradient_at(lst, x, y, nx, ny, radius, False, solid=solid.tolist())
                assert abs(bx - gx[y, x].item()) < 1e-15 and abs(by - gy[y, x].item()) < 1e-15
        cx, cy = O.gradient(torch.full((ny, nx), 0.37), radius, False, solid=m)
        # zero up to the rounding of the link-by-link sum
        assert float(cx[~m].abs().max()) < 1e-16 and float(cy[~m].abs().max()) < 1e-16
        # away from the obstacles the stencil is the periodic one
        px, py = O.gradient(s, radius, False)
        clear = torch.ones(ny, nx, dtype=torch.bool)
        for dy in range(-radius, radius + 1):
            for dx in range(-radius, radius + 1):
                clear &= ~torch.roll(m, shifts=(dy, dx), dims=(0, 1))
        assert clear.any()
        assert torch.equal(gx[clear], px[clear]) and torch.equal(gy[clear], py[clear])


def test_whole_step_with_mask_matches_per_site_brute_force():
    for stencil in ((3, 3, 3, 3), (1, 1, 1, 1), (3, 1, 3, 1)):
        nx, ny = 9, 8
        solid = Wk.random_solid_sites(nx, ny, 6, 3)
        p = params(nx, ny, gx=2e-4, gy=-1e-4, stencil=stencil, solid=solid)
        g = torch.Generator().manual_seed(11)
        rn = 2 * torch.rand(ny, nx, generator=g) - 1
        o = perturbed(O.Oracle(p).init(rn), 12)
        pops = o.full_pops().tolist()
        o.step(1)
        ref = brute.full_step(pops, p)
        got = o.full_pops()
        err = max(abs(got[c, i, y, x].item() - ref[c][i][y][x])
                  for c in range(2) for i in range(Q) for y in range(ny) for x in range(nx))
        assert err < 1e-14, (stencil, err)


def test_masses_conserved_around_obstacles():
    n = 32
    solid = Wk.circular_wall(n, n, 14.0)
    for x, y in ((24, 9), (25, 9), (7, 22), (22, 23), (16, 5)):   # obstacles clear of the drop
        solid[y, x] = True
    yy, xx = np.mgrid[0:n, 0:n]
    rn = np.tanh((6.0 - np.hypot(xx - 14.0, yy - 16.5)) / 2.0)
    p = params(n, n, solid=solid, gx=1e-5, sigma=0.005)
    o = O.Oracle(p).init(rn)
    m0 = o.masses()
    o.step(200)
    m = o.masses()
    assert abs(m[0] - m0[0]) / m0[0] < 1e-13 and abs(m[1] - m0[1]) / m0[1] < 1e-13
    f = o.fields()
    assert bool(torch.isnan(f["rho"][torch.as_tensor(solid)]).all())
    assert bool(torch.isfinite(f["rho"][~torch.as_tensor(solid)]).all())


def test_wall_rows_as_mask_equal_walls_mode_for_channel_flow():
    """Single phase (rho^N = 1 everywhere, Lambda = 1, alpha = 4/9: Phi' = 0),
    body force along x, x-independent flow between solid rows 0 and ny-1: the
    mask and the walls mode give the same populations at every fluid site."""
    nx, ny = 6, 14
    d = Wk.base_params(Lambda=1.0)
    d.update(alpha_R=4.0 / 9.0, alpha_B=4.0 / 9.0, gx=1e-5)
    solid = np.zeros((ny, nx), bool)
    solid[0] = solid[-1] = True
    rn = np.ones((ny, nx))
    a = O.Oracle(O.Params(nx=nx, ny=ny, walls=True, **{k: v for k, v in d.items() if k != "walls"})).init(rn)
    b = O.Oracle(O.Params(nx=nx, ny=ny, solid=solid, **d)).init(rn)
    a.step(400)
    b.step(400)
    ra, rb = a.full_pops(), b.full_pops()
    scale = float(ra.abs().max())
    assert float((ra - rb).abs().max()) / scale < 1e-14
    ux = b.fields()["ux"][1:-1, 0]
    assert float(ux.abs().max()) > 1e-4

"""Pins of the oracle's local (per-site) algebra: equilibrium moments, source
moments, modal vs. distribution-space collision, recolour, streaming."""
import math

import pytest
import torch

from oracle import brute
from oracle import chromo as O
from oracle.lattice import C, W, GHOST, OPP, Q, CS2

torch.set_default_dtype(torch.float64)


def rand_sites(n=64, seed=0):
    g = torch.Generator().manual_seed(seed)
    rhoR = 0.05 + torch.rand(n, generator=g)
    rhoB = 0.05 + torch.rand(n, generator=g)
    ux = 0.05 * (torch.rand(n, generator=g) - 0.5)
    uy = 0.05 * (torch.rand(n, generator=g) - 0.5)
    return rhoR, rhoB, ux, uy, g


def moment(f, fn):
    return sum(f[i] * fn(i) for i in range(Q))


def test_equilibrium_moments():
    """App. A: sum f0 = rho, sum f0 c = rho u, sum f0 c c = P delta + rho u u
    with P = 3/5[(1-a_R) rho_R + (1-a_B) rho_B]; ghost projections of f0 are
    9/5(a_R rho_R + a_B rho_B) - 4/5 rho and 0, 0; sum phi = 1."""
    p = O.Params(nx=1, ny=1, alpha_R=0.9, alpha_B=0.35)
    rhoR, rhoB, ux, uy, _ = rand_sites()
    rho = rhoR + rhoB
    f0 = O.equilibrium(rhoR, rhoB, ux, uy, p)
    P = 0.6 * ((1 - p.alpha_R) * rhoR + (1 - p.alpha_B) * rhoB)
    tol = 1e-14
    assert torch.allclose(moment(f0, lambda i: 1.0), rho, atol=tol, rtol=0)
    assert torch.allclose(moment(f0, lambda i: C[i][0]), rho * ux, atol=tol, rtol=0)
    assert torch.allclose(moment(f0, lambda i: C[i][1]), rho * uy, atol=tol, rtol=0)
    assert torch.allclose(moment(f0, lambda i: C[i][0] ** 2), P + rho * ux * ux, atol=tol, rtol=0)
    assert torch.allclose(moment(f0, lambda i: C[i][1] ** 2), P + rho * uy * uy, atol=tol, rtol=0)
    assert torch.allclose(moment(f0, lambda i: C[i][0] * C[i][1]), rho * ux * uy, atol=tol, rtol=0)
    N0 = 1.8 * (p.alpha_R * rhoR + p.alpha_B * rhoB) - 0.8 * rho
    assert torch.allclose(moment(f0, lambda i: GHOST[i]), N0, atol=tol, rtol=0)
    assert torch.allclose(moment(f0, lambda i: GHOST[i] * C[i][0]), 0 * rho, atol=tol, rtol=0)
    assert torch.allclose(moment(f0, lambda i: GHOST[i] * C[i][1]), 0 * rho, atol=tol, rtol=0)
    phi = O.rest_fractions(rhoR, rhoB, p)
    assert torch.allclose(phi.sum(0), torch.ones_like(rho), atol=1e-15, rtol=0)
    # the sound speeds c_sC^2 = 3/5 (1 - a_C) of the pure phases
    assert abs(float(O.isotropic_pressure(torch.tensor(1.0), torch.tensor(0.0), p)) - 0.6 * (1 - p.alpha_R)) < 1e-16


def explicit_sources(ux, uy, Gx, Gy, dPx, dPy, theta, rho, lam3):
    """F1 (eq. source1 with T from eq. T_identity) and F2 (eq. source2), written
    directly from Sec. II / App. A in distribution space."""
    pre = (1.0 - lam3 / 2.0) / (2.0 * CS2 * CS2)
    udP = ux * dPx + uy * dPy
    u = (ux, uy)
    dP = (dPx, dPy)
    G = (Gx, Gy)
    T = [[None, None], [None, None]]
    for a in range(2):
        for b in range(2):
            T[a][b] = pre * ((rho * theta / 3.0 if a == b else 0.0)
                             - (u[a] * dP[b] + u[b] * dP[a] + (udP if a == b else 0.0)))
    F = []
    for i in range(Q):
        c = C[i]
        herm = lambda a, b: c[a] * c[b] - (CS2 if a == b else 0.0)
        f1 = W[i] * sum(T[a][b] * herm(a, b) for a in range(2) for b in range(2))
        f2 = W[i] * ((G[0] * c[0] + G[1] * c[1]) / CS2
                     + pre * sum((G[a] * u[b] + G[b] * u[a]) * herm(a, b)
                                 for a in range(2) for b in range(2)))
        F.append(f1 + f2)
    return torch.stack(F)


def test_source_moments_are_modal_sources():
    """Moments of F1 + F2: (0, G, C_ab, 0, 0, 0) with C_ab of eq. Correction;
    this fixes S^(3..5) = C and S^(6..8) = 0."""
    rhoR, rhoB, ux, uy, g = rand_sites(seed=1)
    rho = rhoR + rhoB
    n = rho.numel()
    Gx, Gy, dPx, dPy, theta = (1e-2 * (torch.rand(n, generator=g) - 0.5) for _ in range(5))
    lam3 = 0.4 + 1.2 * torch.rand(n, generator=g)
    F = explicit_sources(ux, uy, Gx, Gy, dPx, dPy, theta, rho, lam3)
    Cxx, Cyy, Cxy = O.correction_tensor(ux, uy, Gx, Gy, dPx, dPy, theta, rho, lam3)
    tol = 1e-16
    assert torch.allclose(moment(F, lambda i: 1.0), 0 * rho, atol=tol, rtol=0)
    assert torch.allclose(moment(F, lambda i: C[i][0]), Gx, atol=tol, rtol=0)
    assert torch.allclose(moment(F, lambda i: C[i][1]), Gy, atol=tol, rtol=0)
    assert torch.allclose(moment(F, lambda i: C[i][0] ** 2), Cxx, atol=tol, rtol=0)
    assert torch.allclose(moment(F, lambda i: C[i][1] ** 2), Cyy, atol=tol, rtol=0)
    assert torch.allclose(moment(F, lambda i: C[i][0] * C[i][1]), Cxy, atol=tol, rtol=0)
    for fn in (lambda i: GHOST[i], lambda i: GHOST[i] * C[i][0], lambda i: GHOST[i] * C[i][1]):
        assert torch.allclose(moment(F, fn), 0 * rho, atol=tol, rtol=0)


@pytest.mark.parametrize("l6,l7", [(1.4, 1.2), (1.0, 1.0), (0.7, 1.9)])
def test_modal_collision_equals_distribution_form(l6, l7):
    """Sec. II kinetic equation: f+ = f - A (f - f0) + F1 + F2 with
    A = M^{-1} diag(lambda) M (App. A, eq. Lambda = M A M^{-1}) equals the
    modal relaxation + reconstruction used by the oracle."""
    p = O.Params(nx=1, ny=1, alpha_R=0.95, alpha_B=0.5, lambda6=l6, lambda7=l7)
    rhoR, rhoB, ux, uy, g = rand_sites(seed=2)
    rho = rhoR + rhoB
    n = rho.numel()
    # an arbitrary non-equilibrium population set with these colour densities
    f0 = O.equilibrium(rhoR, rhoB, ux, uy, p)
    f = f0 + 1e-2 * (torch.rand(Q, n, generator=g) - 0.5)
    f = f - (f.sum(0) - rho) / Q          # keep sum f = rho
    jx = moment(f, lambda i: C[i][0])
    jy = moment(f, lambda i: C[i][1])
    Gx, Gy, dPx, dPy, theta = (1e-2 * (torch.rand(n, generator=g) - 0.5) for _ in range(5))
    ux = (jx + 0.5 * Gx) / rho
    uy = (jy + 0.5 * Gy) / rho
    lam3 = 0.4 + 1.2 * torch.rand(n, generator=g)
    Cxx, Cyy, Cxy = O.correction_tensor(ux, uy, Gx, Gy, dPx, dPy, theta, rho, lam3)
    modal = O.collide_modal(f, rhoR, rhoB, ux, uy, Gx, Gy, Cxx, Cyy, Cxy, lam3, p)

    M, Minv = O.projection_matrix()
    f0 = O.equilibrium(rhoR, rhoB, ux, uy, p)
    F = explicit_sources(ux, uy, Gx, Gy, dPx, dPy, theta, rho, lam3)
    out = torch.empty_like(f)
    for s in range(n):
        lam = torch.tensor([0, 0, 0, lam3[s], lam3[s], lam3[s], l6, l7, l7])
        A = Minv @ torch.diag(lam) @ M
        out[:, s] = f[:, s] - A @ (f[:, s] - f0[:, s]) + F[:, s]
    assert torch.allclose(modal, out, atol=2e-15, rtol=0)

    # the per-site closed form printed for f+ (second transcription) agrees too
    for s in range(0, n, 7):
        R = [float(f[i, s]) * float(rhoR[s] / rho[s]) for i in range(Q)]
        B = [float(f[i, s]) - R[i] for i in range(Q)]
        bf = brute.local_collide(R, B, float(Gx[s]), float(Gy[s]), float(ux[s]), float(uy[s]),
                                 float(Cxx[s]), float(Cyy[s]), float(Cxy[s]), float(lam3[s]), p)
        assert max(abs(bf[i] - float(modal[i, s])) for i in range(Q)) < 2e-15


def test_ghost_eq_literal_zero_breaks_fixed_point():
    """The literal N^(0) = 0 (modal evolution eqs.) is not a fixed point of f0
    unless a_R = a_B = 4/9; the projected N^(0) is (reading used by default)."""
    rhoR, rhoB, ux, uy, _ = rand_sites(seed=3)
    rho = rhoR + rhoB
    z = torch.zeros_like(rho)
    for ghost_eq, a_R, a_B, fixed in ((0, 0.95, 0.5, True), (1, 0.95, 0.5, False),
                                      (1, 4.0 / 9.0, 4.0 / 9.0, True)):
        p = O.Params(nx=1, ny=1, alpha_R=a_R, alpha_B=a_B, ghost_eq=ghost_eq)
        f0 = O.equilibrium(rhoR, rhoB, z, z, p)
        lam3 = torch.full_like(rho, 1.3)
        out = O.collide_modal(f0, rhoR, rhoB, z, z, z, z, z, z, z, lam3, p)
        assert torch.allclose(out, f0, atol=1e-15, rtol=0) == fixed


def test_recolour_conserves_colour_mass_and_splits_proportionally():
    """Sec. II re-colour: sum_i R++ = rho_R, sum_i B++ = rho_B (mass conserving),
    and with a zero director the split is purely proportional."""
    p = O.Params(nx=1, ny=1, beta=0.7)
    rhoR, rhoB, ux, uy, g = rand_sites(seed=4)
    rho = rhoR + rhoB
    fplus = O.equilibrium(rhoR, rhoB, ux, uy, p) + 1e-3 * torch.rand(Q, rho.numel(), generator=g)
    fplus = fplus - (fplus.sum(0) - rho) / Q
    ang = 2 * math.pi * torch.rand(rho.numel(), generator=g)
    Rpp, Bpp = O.recolour(fplus, rhoR, rhoB, torch.cos(ang), torch.sin(ang), p)
    assert torch.allclose(Rpp.sum(0), rhoR, atol=1e-15, rtol=0)
    assert torch.allclose(Bpp.sum(0), rhoB, atol=1e-15, rtol=0)
    z = torch.zeros_like(rho)
    Rpp, Bpp = O.recolour(fplus, rhoR, rhoB, z, z, p)
    assert torch.allclose(Rpp, rhoR / rho * fplus, atol=1e-16, rtol=0)
    # red is pushed along the director: the red flux along m exceeds the proportional share
    Rpp, _ = O.recolour(fplus, rhoR, rhoB, torch.ones_like(rho), z, p)
    flux = sum((Rpp[i] - fplus[i] * rhoR / rho) * C[i][0] for i in range(Q))
    assert bool((flux > 0).all())


def test_recolour_matches_per_site_brute_force():
    p = O.Params(nx=4, ny=4, beta=0.6)
    rhoR, rhoB, ux, uy, g = rand_sites(n=16, seed=5)
    fplus = O.equilibrium(rhoR, rhoB, ux, uy, p)
    mx, my = torch.rand(16, generator=g) - 0.5, torch.rand(16, generator=g) - 0.5
    Rpp, Bpp = O.recolour(fplus, rhoR, rhoB, mx, my, p)
    for s in range(16):
        r, b = brute.local_recolour([float(fplus[i, s]) for i in range(Q)], float(rhoR[s]),
                                    float(rhoB[s]), float(mx[s]), float(my[s]), p)
        assert max(abs(r[i] - float(Rpp[i, s])) for i in range(Q)) < 1e-16
        assert max(abs(b[i] - float(Bpp[i, s])) for i in range(Q)) < 1e-16


@pytest.mark.parametrize("Lam", [10.0, 100.0])
def test_colour_index_of_the_printed_profile_pair(Lam):
    """Sec. II prints the kinematic solution twice: as colour densities,
    rho_R = rho_0R (1 + t)/2 with the equivalent rho_B = rho_0B (1 - t)/2, and,
    substituted in the definition of the colour index, as rho^N = t (eq.
    equ_rhoN), t = tanh(beta n.(r - u t)).  So the colour index of that pair is
    t itself at every interior value, for any density ratio; the oracle's
    initial state (which writes that pair for a given rho^N) reads back the
    same through fields().  Without the 1/rho_0C normalisation of the
    definition the pair's index is (Lambda (1 + t) - (1 - t))/(Lambda (1 + t) + (1 - t)),
    off by O(1) for Lambda = 10, 100."""
    d = dict(rho0_R=1.0, rho0_B=1.0 / Lam, alpha_B=0.5, alpha_R=1.0 - 0.5 / Lam)
    p = O.Params(nx=7, ny=5, **d)
    t = torch.linspace(-0.999, 0.999, 35, dtype=torch.float64)
    rR = p.rho0_R * (1.0 + t) / 2.0
    rB = p.rho0_B * (1.0 - t) / 2.0
    assert float((O.colour_index(rR, rB, p) - t).abs().max()) < 4e-16
    f = O.Oracle(p).init(t.reshape(5, 7)).fields()
    assert float((f["rhoN"].reshape(-1) - t).abs().max()) < 1e-15  # through the summed populations
    unnormalised = (rR - rB) / (rR + rB)
    assert float((unnormalised - t).abs().max()) > 0.5


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("shape", [(4, 4), (5, 6), (4, 3)])
def test_streaming_matches_brute_force_bit_exact(walls, shape):
    """4x4-class lattices, payload = unique id per (colour, link, site)."""
    nx, ny = shape
    if walls and ny < 3:
        pytest.skip("needs a fluid row")
    payload = [[[[float(((c * Q + i) * ny + y) * nx + x) for x in range(nx)] for y in range(ny)]
                for i in range(Q)] for c in range(2)]
    ref = brute.stream_site_by_site(payload, nx, ny, walls)
    rows = list(range(1, ny - 1)) if walls else list(range(ny))
    P = torch.tensor(payload)
    for c in range(2):
        got = O.stream(P[c][:, rows], walls)
        for i in range(Q):
            for k, y in enumerate(rows):
                for x in range(nx):
                    assert got[i, k, x].item() == ref[c][i][y][x]
    # streaming is a permutation: every payload appears exactly once
    flat = sorted(ref[c][i][y][x] for c in range(2) for i in range(Q) for y in rows for x in range(nx))
    src = sorted(payload[c][i][y][x] for c in range(2) for i in range(Q) for y in rows for x in range(nx))
    assert flat == src


def test_brute_streaming_hand_case():
    """Hand check on a 4x4 periodic lattice: the population on link 1 (1,1) at
    (3, 3) wraps to (0, 0); with walls a link-2 (0,1) population at the top
    fluid row comes back on link 6 at the same site."""
    nx = ny = 4
    pops = [[[[0.0] * nx for _ in range(ny)] for _ in range(Q)] for _ in range(2)]
    pops[0][1][3][3] = 7.0
    out = brute.stream_site_by_site(pops, nx, ny, walls=False)
    assert out[0][1][0][0] == 7.0
    pops = [[[[0.0] * nx for _ in range(ny)] for _ in range(Q)] for _ in range(2)]
    pops[1][2][2][1] = 5.0   # top fluid row is y = 2 when rows 0 and 3 are solid
    out = brute.stream_site_by_site(pops, nx, ny, walls=True)
    assert out[1][6][2][1] == 5.0
    assert OPP[2] == 6


@pytest.mark.parametrize("walls", [False, True])
def test_whole_step_matches_per_site_brute_force(walls):
    """The vectorised sweep and the scalar per-site transcription agree on an
    8x8 lattice with random non-equilibrium populations, force and all stencils."""
    for stencil in ((3, 3, 3, 3), (1, 1, 1, 1), (3, 1, 3, 1)):
        p = O.Params(nx=8, ny=10 if walls else 8, walls=walls, gx=2e-4, gy=-1e-4,
                     stencil=stencil, sigma=0.02)
        g = torch.Generator().manual_seed(11)
        rn = 2 * torch.rand(p.ny, p.nx, generator=g) - 1
        o = O.Oracle(p).init(rn)
        o.R = o.R * (1 + 0.05 * torch.rand(o.R.shape, generator=g))
        o.B = o.B * (1 + 0.05 * torch.rand(o.B.shape, generator=g))
        pops = o.full_pops().tolist()
        o.step(1)
        ref = brute.full_step(pops, p)
        got = o.full_pops()
        rows = range(1, p.ny - 1) if walls else range(p.ny)
        err = max(abs(got[c, i, y, x].item() - ref[c][i][y][x])
                  for c in range(2) for i in range(Q) for y in rows for x in range(p.nx))
        assert err < 1e-14, (stencil, err)

"""Per-site scalar reference for tiny lattices (test infrastructure only).

A second, independent transcription of the local pieces of the scheme, in
plain Python floats and explicit index loops, so that whole-lattice sweeps in
``chromo`` (and the HIP path) can be checked against it on 4x4 to 8x8 lattices:

* streaming with periodic wrap and half-way bounce-back (Sec. II kinetic eq.),
  at wall rows or at the solid sites of a mask;
* the App. B gradient stencil, with explicit modular / mirrored indices (a
  tap on a solid site of a mask reads the centre value);
* the closed-form post-collision distribution printed in Sec. III / App. A
  (f+_i = w_i {[2 - 3/2 |c_i|^2] rho + 3 j+.c_i + 9/2 c_i.Pi+.c_i
  - 3/2 tr Pi+ + g_i N+/4 + 3/8 g_i J+.c_i}), fed by the modal evolution eqs.;
* the d'Ortona recolour (Sec. II).

Lattice state: nested lists pops[colour][i][y][x].
"""
import math

from .lattice import C, W, GHOST, OPP, Q, CHAT, K_PHI, STENCIL_COEFFS


def stream_site_by_site(pops, nx, ny, walls, solid=None):
    """Push each post-collision population along its link; a link that would
    enter a solid row (0 or ny-1 when ``walls``) or a solid site of the mask
    ``solid`` (nested [ny][nx] truth values) comes back reversed.  Solid sites
    end up holding 0."""
    out = [[[[None] * nx for _ in range(ny)] for _ in range(Q)] for _ in range(2)]
    rows = range(1, ny - 1) if walls else range(ny)
    for col in range(2):
        for y in rows:
            for x in range(nx):
                if solid is not None and solid[y][x]:
                    for i in range(Q):
                        out[col][i][y][x] = 0.0
                    continue
                for i in range(Q):
                    cx, cy = C[i]
                    xd = (x + cx) % nx
                    yd = y + cy
                    if walls and (yd <= 0 or yd >= ny - 1):
                        out[col][OPP[i]][y][x] = pops[col][i][y][x]
                    elif solid is not None and solid[yd % ny][xd]:
                        out[col][OPP[i]][y][x] = pops[col][i][y][x]
                    else:
                        out[col][i][yd % ny][xd] = pops[col][i][y][x]
    return out


def mirrored(y, ny, walls):
    """Row actually read for a (possibly out-of-lattice) row index y, and whether
    it is a mirror image (walls) or a periodic copy."""
    if not walls:
        return y % ny, False
    F = ny - 2
    t = (y - 1) % (2 * F)
    if t < F:
        return 1 + t, False
    return 1 + (2 * F - 1 - t), True


def gradient_at(field, x, y, nx, ny, radius, walls, odd_y=False, solid=None):
    """(d/dx, d/dy) of a scalar lattice field at one site with the App. B
    stencil; a tap on a solid site of ``solid`` reads the centre value."""
    gx = gy = 0.0
    for N, b in enumerate(STENCIL_COEFFS[radius], start=1):
        sx = sy = 0.0
        for i in range(1, Q):
            cx, cy = C[i]
            yy, refl = mirrored(y + N * cy, ny, walls)
            xx = (x + N * cx) % nx
            v = field[yy][xx]
            if solid is not None and solid[yy][xx]:
                v = field[y][x]
            if refl and odd_y:
                v = -v
            sx += W[i] * cx * v
            sy += W[i] * cy * v
        gx += b * sx
        gy += b * sy
    return gx, gy


def closed_form_fplus(rho, jx, jy, Pxx, Pyy, Pxy, N, Jx, Jy):
    """Post-collision f+_i from post-collision modes, closed form (App. A, after eq. for M^{-1})."""
    out = []
    tr = Pxx + Pyy
    for i in range(Q):
        cx, cy = C[i]
        c2 = cx * cx + cy * cy
        g = GHOST[i]
        out.append(W[i] * ((2.0 - 1.5 * c2) * rho
                           + 3.0 * (jx * cx + jy * cy)
                           + 4.5 * (Pxx * cx * cx + 2.0 * Pxy * cx * cy + Pyy * cy * cy)
                           - 1.5 * tr
                           + 0.25 * g * N + 0.375 * g * (Jx * cx + Jy * cy)))
    return out


def local_collide(R, B, Gx, Gy, ux, uy, Cxx, Cyy, Cxy, lam3, prm):
    """Collision at one site from its 9+9 populations; mode sums are written out
    term by term (Table A1 projectors, unweighted) and the modes are relaxed
    per the modal evolution equations of App. A."""
    f = [R[i] + B[i] for i in range(Q)]
    rhoR = sum(R)
    rhoB = sum(B)
    rho = rhoR + rhoB
    jx = sum(f[i] * C[i][0] for i in range(Q))
    jy = sum(f[i] * C[i][1] for i in range(Q))
    Pxx = sum(f[i] * C[i][0] ** 2 for i in range(Q))
    Pyy = sum(f[i] * C[i][1] ** 2 for i in range(Q))
    Pxy = sum(f[i] * C[i][0] * C[i][1] for i in range(Q))
    N = sum(f[i] * GHOST[i] for i in range(Q))
    Jx = sum(f[i] * GHOST[i] * C[i][0] for i in range(Q))
    Jy = sum(f[i] * GHOST[i] * C[i][1] for i in range(Q))
    P = 0.6 * ((1 - prm.alpha_R) * rhoR + (1 - prm.alpha_B) * rhoB)
    N0 = 1.8 * (prm.alpha_R * rhoR + prm.alpha_B * rhoB) - 0.8 * rho if prm.ghost_eq == 0 else 0.0
    Pxx_p = Pxx - lam3 * (Pxx - (P + rho * ux * ux)) + Cxx
    Pyy_p = Pyy - lam3 * (Pyy - (P + rho * uy * uy)) + Cyy
    Pxy_p = Pxy - lam3 * (Pxy - rho * ux * uy) + Cxy
    N_p = N - prm.lambda6 * (N - N0)
    Jx_p = Jx - prm.lambda7 * Jx
    Jy_p = Jy - prm.lambda7 * Jy
    return closed_form_fplus(rho, jx + Gx, jy + Gy, Pxx_p, Pyy_p, Pxy_p, N_p, Jx_p, Jy_p)


def local_recolour(fplus, rhoR, rhoB, mx, my, prm):
    """d'Ortona recolour at one site (Sec. II)."""
    rho = rhoR + rhoB
    moving = ((1 - prm.alpha_R) * rhoR + (1 - prm.alpha_B) * rhoB) / rho
    Rpp, Bpp = [], []
    for i in range(Q):
        phi = (prm.alpha_R * rhoR + prm.alpha_B * rhoB) / rho if i == 0 else K_PHI * W[i] * moving
        t = prm.beta * phi * rhoR * rhoB / rho * (mx * CHAT[i][0] + my * CHAT[i][1])
        if not prm.recolor:
            t = 0.0
        Rpp.append(rhoR / rho * fplus[i] + t)
        Bpp.append(rhoB / rho * fplus[i] - t)
    return Rpp, Bpp


def full_step(pops, prm, force=None):
    """One whole step, site by site, on a tiny lattice (pre-collision in, pre-collision out)."""
    nx, ny, walls = prm.nx, prm.ny, prm.walls
    solid = getattr(prm, 'solid', None)
    rows = list(range(1, ny - 1)) if walls else list(range(ny))
    sites = [(x, y) for y in rows for x in range(nx) if solid is None or not solid[y][x]]
    rg, rk, rphi, ru = prm.stencil
    nanrow = [float('nan')] * nx
    def blank():
        return [list(nanrow) for _ in range(ny)]
    rhoR, rhoB, rho, jx, jy, rhoN, lam3, Php = (blank() for _ in range(8))
    for x, y in sites:
        R = [pops[0][i][y][x] for i in range(Q)]
        B = [pops[1][i][y][x] for i in range(Q)]
        rR, rB = sum(R), sum(B)
        rhoR[y][x], rhoB[y][x] = rR, rB
        rho[y][x] = rR + rB
        jx[y][x] = sum((R[i] + B[i]) * C[i][0] for i in range(Q))
        jy[y][x] = sum((R[i] + B[i]) * C[i][1] for i in range(Q))
        a, b = rR / prm.rho0_R, rB / prm.rho0_B
        rn = (a - b) / (a + b)
        rhoN[y][x] = rn
        nu = prm.nu_R * (1 + rn) / 2 + prm.nu_B * (1 - rn) / 2
        lam3[y][x] = 2.0 / (6.0 * nu + 1.0)
        Php[y][x] = 0.6 * (1 - prm.alpha_R) * (rR + prm.rho0_R / prm.rho0_B * rB) - (rR + rB) / 3.0
    gnx, gny, mx, my = blank(), blank(), blank(), blank()
    for x, y in sites:
        gx, gy = gradient_at(rhoN, x, y, nx, ny, rg, walls, solid=solid)
        s = math.sqrt(gx * gx + gy * gy + prm.eps_n ** 2)
        gnx[y][x], gny[y][x] = gx, gy
        mx[y][x], my[y][x] = gx / s, gy / s
    nxf = [[-v for v in row] for row in mx]
    nyf = [[-v for v in row] for row in my]
    Gx, Gy, ux, uy = blank(), blank(), blank(), blank()
    for x, y in sites:
        if prm.fixed_K is None:
            K = gradient_at(nxf, x, y, nx, ny, rk, walls, solid=solid)[0] + \
                gradient_at(nyf, x, y, nx, ny, rk, walls, odd_y=True, solid=solid)[1]
        else:
            K = prm.fixed_K
        gx = 0.5 * prm.sigma * K * gnx[y][x] + prm.gx
        gy = 0.5 * prm.sigma * K * gny[y][x] + prm.gy
        if force is not None:
            gx += float(force[0][y][x])
            gy += float(force[1][y][x])
        Gx[y][x], Gy[y][x] = gx, gy
        ux[y][x] = (jx[y][x] + 0.5 * gx) / rho[y][x]
        uy[y][x] = (jy[y][x] + 0.5 * gy) / rho[y][x]
    post = [[[[0.0] * nx for _ in range(ny)] for _ in range(Q)] for _ in range(2)]
    for x, y in sites:
        dPx, dPy = gradient_at(Php, x, y, nx, ny, rphi, walls, solid=solid)
        theta = gradient_at(ux, x, y, nx, ny, ru, walls, solid=solid)[0] + \
            gradient_at(uy, x, y, nx, ny, ru, walls, odd_y=True, solid=solid)[1]
        l3 = lam3[y][x]
        k = 1 - l3 / 2
        u_x, u_y = ux[y][x], uy[y][x]
        iso = u_x * dPx + u_y * dPy - rho[y][x] * theta / 3
        Cxx = k * (2 * u_x * (Gx[y][x] - dPx) - iso)
        Cyy = k * (2 * u_y * (Gy[y][x] - dPy) - iso)
        Cxy = k * (u_x * (Gy[y][x] - dPy) + u_y * (Gx[y][x] - dPx))
        R = [pops[0][i][y][x] for i in range(Q)]
        B = [pops[1][i][y][x] for i in range(Q)]
        fp = local_collide(R, B, Gx[y][x], Gy[y][x], u_x, u_y, Cxx, Cyy, Cxy, l3, prm)
        Rpp, Bpp = local_recolour(fp, rhoR[y][x], rhoB[y][x], mx[y][x], my[y][x], prm)
        for i in range(Q):
            post[0][i][y][x] = Rpp[i]
            post[1][i][y][x] = Bpp[i]
    return stream_site_by_site(post, nx, ny, walls, solid)

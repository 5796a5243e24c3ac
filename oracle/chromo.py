"""Whole-lattice oracle of one chromodynamic MRT time step (test infrastructure).

Plain torch-CPU sweeps, float64 by default (float32 only to measure the
FP32 rounding floor).  Arrays are ``[9, ny, nx]`` per colour, x fastest; the
state handed between steps is the pair (R_i, B_i) of *pre-collision*
populations f_i(r, t) of the kinetic equation (Sec. II).

One step, in the paper's order (Sec. II and App. A):

 1. colour densities and raw momentum               (Sec. II, force-adjusted observables)
 2. colour index rho^N, rest fractions phi_i,        (Sec. II; App. A)
    isotropic pressure P, Phi', lambda_3
 3. grad rho^N by the App. B stencil, normal n = -grad rho^N/|grad rho^N|
 4. curvature K = div n, interface force             (Sec. II, Lishchuk/Brackbill force)
    G = sigma K grad rho^N / 2, velocity u = (j + G/2)/rho
 5. grad Phi', div u, correction tensor C            (App. A, eq. "Correction")
 6. modal relaxation m+ = m + Lambda (m^(0) - m) + S  (App. A, modal evolution eqs.)
    and reconstruction f+ = M^{-1} m+
 7. d'Ortona recolour                                (Sec. II, re-colour eq.)
 8. streaming f_i(r + c_i, t + 1) = f_i^{++}(r, t)    (Sec. II, kinetic equation LHS)

Readings of passages that are silent, ambiguous or inconsistent (each one is
a parameter or a constant here, and the HIP path takes the same reading):

* projector rows of M are the unweighted polynomials (see ``lattice``);
* the second-moment source is C_ab itself (symmetric), the ghost sources
  S^(6..8) are zero: these are the moments of the explicit F_1 + F_2 of Sec. II;
* ghost equilibrium N^(0) = h^(6).f^(0) = 9/5 (a_R rho_R + a_B rho_B) - 4/5 rho
  (App. A projections), ``ghost_eq=1`` gives the literal N^(0) = 0 of the
  modal evolution equations;
* recolour uses m = +grad rho^N/|.| (red grows along the director); the
  curvature uses the paper's n = -m, so K = +1/R for a red drop;
* |grad rho^N| is regularised as sqrt(|grad rho^N|^2 + eps^2);
* kinematic viscosity is linear in rho^N between nu_B (rho^N=-1) and nu_R (+1);
* all derivatives use fields of the current time step;
* walls (rows 0 and ny-1 solid) use half-way bounce-back, and every stencil
  sees a mirror image of the fluid about the wall planes (scalars and
  x-components even, y-components odd);
* solid sites anywhere (``Params.solid``, a staircase obstacle such as the
  circular no-slip wall of the curved-interface transient, Sec. IV and
  App. D) also use half-way bounce-back; a stencil tap that falls on a solid
  site reads the value of the field at the stencil's own centre (a
  zero-gradient continuation, so a uniform field has zero derivative next to
  any obstacle).  The mirror image of the walls has no unique form on a
  staircase; this continuation is the simplest that keeps the stencils exact
  on constants.
"""
from dataclasses import dataclass, field
import functools

import torch

from .lattice import C, W, GHOST, CHAT, OPP, Q, STENCIL_COEFFS, K_PHI, \
    projector_rows_exact, inverse_columns_exact


@dataclass
class Params:
    nx: int
    ny: int
    walls: bool = False            # True: rows 0 and ny-1 are solid
    rho0_R: float = 1.0            # bulk densities rho_0R, rho_0B (Sec. II)
    rho0_B: float = 0.1
    alpha_R: float = 0.95          # rest-mass parameters (Sec. II, eq. for phi_i)
    alpha_B: float = 0.5
    nu_R: float = 1.0 / 6.0        # kinematic viscosities of the bulk phases
    nu_B: float = 1.0 / 6.0
    sigma: float = 0.01            # interfacial tension
    beta: float = 0.67             # segregation parameter
    lambda6: float = 1.4           # ghost-mode rates (App. A)
    lambda7: float = 1.2
    gx: float = 0.0                # uniform external body force density
    gy: float = 0.0
    stencil: tuple = (3, 3, 3, 3)  # radii for grad rho^N, div n, grad Phi', div u
    ghost_eq: int = 0              # 0: projected N^(0); 1: N^(0) = 0
    fixed_K: float = None          # if set, K := fixed_K (Sec. IV, fixed curvature)
    recolor: bool = True
    eps_n: float = 1e-6
    solid: object = None           # optional [ny][nx] booleans: solid sites anywhere (needs walls=False)

    @property
    def Lambda(self):
        return self.rho0_R / self.rho0_B


def _tensor(vals, dtype):
    return torch.tensor(vals, dtype=dtype)


# ----------------------------------------------------------------------------
# lattice geometry
# ----------------------------------------------------------------------------

def solid_mask(p):
    """Solid sites as a bool tensor [ny, nx], or None when only the wall rows
    (or nothing) are solid."""
    if p.solid is None:
        return None
    if p.walls:
        raise ValueError("solid sites anywhere need walls=False (the mask may hold solid rows)")
    m = torch.as_tensor(p.solid).to(torch.bool)
    if tuple(m.shape) != (p.ny, p.nx):
        raise ValueError("solid mask must have shape (ny, nx)")
    return m


def fluid_rows(p):
    """Row indices of fluid sites (all rows when y is periodic)."""
    return list(range(1, p.ny - 1)) if p.walls else list(range(p.ny))


def _fold(v, F):
    """Mirror-extended row index on a fluid strip of F rows: (row, reflected?)."""
    t = v % (2 * F)
    return (t, False) if t < F else (2 * F - 1 - t, True)


def shift(s, dx, dy, walls, odd_y=False):
    """Field s evaluated at r + (dx, dy) for every fluid site r.

    ``s`` has shape [..., F, nx] (fluid rows only).  x is periodic; y is
    periodic, or mirrored about the two wall planes when ``walls``.  With
    ``odd_y`` the mirrored copy changes sign (y-component of a vector).
    """
    out = torch.roll(s, shifts=-dx, dims=-1)
    if not walls:
        return torch.roll(out, shifts=-dy, dims=-2)
    idx, sign = _mirror_map(s.shape[-2], dy)
    out = out[..., idx, :]
    if odd_y:
        out = out * sign.to(s.dtype)[:, None]
    return out


_MIRROR_CACHE = {}


def _mirror_map(F, dy):
    """Row index read for each fluid row shifted by dy, and the sign (-1 where
    the read row is a mirror image) -- built once per (F, dy)."""
    key = (F, dy)
    if key not in _MIRROR_CACHE:
        idx, sign = [], []
        for y in range(F):
            r, refl = _fold(y + dy, F)
            idx.append(r)
            sign.append(-1.0 if refl else 1.0)
        _MIRROR_CACHE[key] = (torch.tensor(idx), torch.tensor(sign, dtype=torch.float64))
    return _MIRROR_CACHE[key]


def gradient(s, radius, walls, odd_y=False, solid=None):
    """First-derivative stencil of App. B: d s/d alpha = sum_N b_N sum_i w_i c_ia s(r + N c_i).

    radius 1 gives the compact isotropic stencil (b = 3); radius 3 the
    sixth-order non-compact one (b = 9/2, -9/10, 1/10).  With a solid mask
    a tap on a solid site reads s at the centre r.
    """
    gx = torch.zeros_like(s)
    gy = torch.zeros_like(s)
    for N, b in enumerate(STENCIL_COEFFS[radius], start=1):
        sx = torch.zeros_like(s)
        sy = torch.zeros_like(s)
        for i in range(1, Q):
            cx, cy = C[i]
            v = shift(s, N * cx, N * cy, walls, odd_y)
            if solid is not None:
                v = torch.where(shift(solid, N * cx, N * cy, False), s, v)
            sx = sx + W[i] * cx * v
            sy = sy + W[i] * cy * v
        gx = gx + b * sx
        gy = gy + b * sy
    return gx, gy


def divergence(vx, vy, radius, walls, solid=None):
    """div v = d v_x/dx + d v_y/dy with the App. B stencil (v_y odd under the wall mirror)."""
    dxx, _ = gradient(vx, radius, walls, odd_y=False, solid=solid)
    _, dyy = gradient(vy, radius, walls, odd_y=True, solid=solid)
    return dxx + dyy


# ----------------------------------------------------------------------------
# local fields
# ----------------------------------------------------------------------------

def colour_densities(R, B):
    """rho_R = sum_i R_i, rho_B = sum_i B_i (Sec. II, force-adjusted observables)."""
    return R.sum(0), B.sum(0)


def raw_momentum(f):
    """j = sum_i f_i c_i (the first term of the force-adjusted velocity, Sec. II)."""
    cx = _tensor([c[0] for c in C], f.dtype)[:, None, None]
    cy = _tensor([c[1] for c in C], f.dtype)[:, None, None]
    return (f * cx).sum(0), (f * cy).sum(0)


def colour_index(rhoR, rhoB, p):
    """rho^N = (rho_R/rho_0R - rho_B/rho_0B)/(rho_R/rho_0R + rho_B/rho_0B) (Sec. II)."""
    a = rhoR / p.rho0_R
    b = rhoB / p.rho0_B
    return (a - b) / (a + b)


def rest_fractions(rhoR, rhoB, p):
    """phi_i of the density-contrast equilibrium (Sec. II, eq. for phi_i), shape [9, ...]."""
    rho = rhoR + rhoB
    phi0 = (p.alpha_R * rhoR + p.alpha_B * rhoB) / rho
    moving = ((1.0 - p.alpha_R) * rhoR + (1.0 - p.alpha_B) * rhoB) / rho
    return torch.stack([phi0] + [K_PHI * W[i] * moving for i in range(1, Q)])


def isotropic_pressure(rhoR, rhoB, p):
    """P = 3/5 [(1 - a_R) rho_R + (1 - a_B) rho_B], the isotropic part of the
    equilibrium second moment (App. A, after the equilibrium moment identities)."""
    return 0.6 * ((1.0 - p.alpha_R) * rhoR + (1.0 - p.alpha_B) * rhoB)


def phi_prime(rhoR, rhoB, p):
    """Phi' = 3/5 (1 - a_R)(rho_R + Lambda rho_B) - rho/3 (App. A, after eq. Pi_1)."""
    return 0.6 * (1.0 - p.alpha_R) * (rhoR + p.Lambda * rhoB) - (rhoR + rhoB) / 3.0


def lambda3(rhoN, p):
    """Shear rate lambda_3 from nu(rho^N) = (2/lambda_3 - 1)/6 (Sec. II; App. A
    after eq. Correction), with nu linear in rho^N between the bulk values."""
    nu = p.nu_R * (1.0 + rhoN) / 2.0 + p.nu_B * (1.0 - rhoN) / 2.0
    return 2.0 / (6.0 * nu + 1.0)


def equilibrium(rhoR, rhoB, ux, uy, p):
    """f^(0)_i = rho phi_i + w_i rho (3 u.c + 9/2 (u.c)^2 - 3/2 u^2) (Sec. II, App. A)."""
    rho = rhoR + rhoB
    phi = rest_fractions(rhoR, rhoB, p)
    out = []
    for i in range(Q):
        cu = C[i][0] * ux + C[i][1] * uy
        out.append(rho * phi[i] + W[i] * rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy)))
    return torch.stack(out)


# ----------------------------------------------------------------------------
# collision
# ----------------------------------------------------------------------------

@functools.lru_cache(maxsize=None)
def projection_matrix(dtype=torch.float64):
    """M with rows h^(p) (Table A1, unweighted reading) and M^{-1} with columns k^(p) (App. A)."""
    M = torch.tensor([[float(v) for v in row] for row in projector_rows_exact()], dtype=dtype)
    cols = inverse_columns_exact()
    Minv = torch.tensor([[float(cols[p][i]) for p in range(Q)] for i in range(Q)], dtype=dtype)
    return M, Minv


def correction_tensor(ux, uy, Gx, Gy, dPx, dPy, theta, rho, lam3):
    """C_ab = (1 - l3/2)[u_a (G_b - d_b Phi') + u_b (G_a - d_a Phi')
                         - (u.grad Phi' - rho div u / 3) delta_ab]   (App. A, eq. Correction)."""
    k = 1.0 - lam3 / 2.0
    iso = ux * dPx + uy * dPy - rho * theta / 3.0
    Cxx = k * (2.0 * ux * (Gx - dPx) - iso)
    Cyy = k * (2.0 * uy * (Gy - dPy) - iso)
    Cxy = k * (ux * (Gy - dPy) + uy * (Gx - dPx))
    return Cxx, Cyy, Cxy


def collide_modal(f, rhoR, rhoB, ux, uy, Gx, Gy, Cxx, Cyy, Cxy, lam3, p):
    """Forced modal relaxation and reconstruction (App. A, modal evolution eqs.).

    m = M f;  m+_p = m_p + lambda_p (m^(0)_p - m_p) + S^(p);  f+ = M^{-1} m+
    lambda = (0, 0, 0, l3, l3, l3, l6, l7, l7); equilibria are the projections
    of f^(0); sources S = (0, G_x, G_y, C_xx, C_yy, C_xy, 0, 0, 0).
    """
    M, Minv = projection_matrix(f.dtype)
    m = torch.einsum('pi,i...->p...', M, f)
    rho = rhoR + rhoB
    P = isotropic_pressure(rhoR, rhoB, p)
    zero = torch.zeros_like(rho)
    if p.ghost_eq == 0:
        N0 = 1.8 * (p.alpha_R * rhoR + p.alpha_B * rhoB) - 0.8 * rho
    else:
        N0 = zero
    meq = torch.stack([rho, rho * ux, rho * uy,
                       P + rho * ux * ux, P + rho * uy * uy, rho * ux * uy,
                       N0, zero, zero])
    S = torch.stack([zero, Gx, Gy, Cxx, Cyy, Cxy, zero, zero, zero])
    lam = torch.stack([zero, zero, zero, lam3, lam3, lam3,
                       torch.full_like(rho, p.lambda6), torch.full_like(rho, p.lambda7),
                       torch.full_like(rho, p.lambda7)])
    mplus = m + lam * (meq - m) + S
    return torch.einsum('ip,p...->i...', Minv, mplus)


def recolour(fplus, rhoR, rhoB, mx, my, p):
    """d'Ortona segregation (Sec. II, re-colour eq.):
    R++ = (rho_R/rho) f+ + t_i,  B++ = (rho_B/rho) f+ - t_i,
    t_i = beta phi_i rho_R rho_B / rho (m . c_hat_i)."""
    rho = rhoR + rhoB
    phi = rest_fractions(rhoR, rhoB, p)
    Rpp, Bpp = [], []
    for i in range(Q):
        t = p.beta * phi[i] * rhoR * rhoB / rho * (mx * CHAT[i][0] + my * CHAT[i][1])
        if not p.recolor:
            t = torch.zeros_like(t)
        Rpp.append(rhoR / rho * fplus[i] + t)
        Bpp.append(rhoB / rho * fplus[i] - t)
    return torch.stack(Rpp), torch.stack(Bpp)


def stream(S, walls, solid=None):
    """f_i(r + c_i, t + 1) = S_i(r, t); a link that would enter a wall returns
    to its own site reversed (half-way bounce-back, walls at y = 1/2 and F - 1/2
    on the fluid strip).  S has shape [9, F, nx] (fluid rows only).  With a
    solid mask (full lattice, periodic) a link whose target is a solid site
    returns the same way, and solid sites hold zero."""
    out = torch.empty_like(S)
    if solid is not None:
        for i in range(Q):
            cx, cy = C[i]
            moved = torch.roll(S[i], shifts=(cy, cx), dims=(-2, -1))            # S_i(r - c_i)
            from_solid = torch.roll(solid, shifts=(cy, cx), dims=(-2, -1))      # r - c_i solid?
            out[i] = torch.where(from_solid, S[OPP[i]], moved)
        out[:, solid] = 0.0
        return out
    F = S.shape[-2]
    for i in range(Q):
        cx, cy = C[i]
        moved = torch.roll(S[i], shifts=cx, dims=-1)
        if not walls:
            out[i] = torch.roll(moved, shifts=cy, dims=-2)
            continue
        if cy == 0:
            out[i] = moved
        elif cy == 1:
            out[i, 1:] = moved[:-1]
        else:
            out[i, :-1] = moved[1:]
    if walls:
        for i in range(Q):
            cy = C[i][1]
            if cy == 1:       # links leaving the top fluid row bounce back down
                out[OPP[i], F - 1] = S[i, F - 1]
            elif cy == -1:    # links leaving the bottom fluid row bounce back up
                out[OPP[i], 0] = S[i, 0]
    return out


# ----------------------------------------------------------------------------
# one step
# ----------------------------------------------------------------------------

def _force_field(force, p, F, dtype):
    if force is None:
        return None
    force = force.to(dtype)
    if p.walls:
        force = force[:, 1:p.ny - 1]
    return force


def interface_fields(R, B, p, force=None):
    """Steps 1-5 of the time step on the fluid strip; returns a dict of fields."""
    walls = p.walls
    solid = solid_mask(p)
    rg, rk, rphi, ru = p.stencil
    rhoR, rhoB = colour_densities(R, B)
    rho = rhoR + rhoB
    f = R + B
    jx, jy = raw_momentum(f)
    rhoN = colour_index(rhoR, rhoB, p)
    lam3 = lambda3(rhoN, p)
    Php = phi_prime(rhoR, rhoB, p)
    # colour gradient and director
    gnx, gny = gradient(rhoN, rg, walls, solid=solid)
    norm = torch.sqrt(gnx * gnx + gny * gny + p.eps_n * p.eps_n)
    mx, my = gnx / norm, gny / norm
    nx_, ny_ = -mx, -my                      # outward normal of a red drop (Sec. II)
    if p.fixed_K is None:
        K = divergence(nx_, ny_, rk, walls, solid)
    else:
        K = torch.full_like(rho, p.fixed_K)
    Gx = 0.5 * p.sigma * K * gnx + p.gx
    Gy = 0.5 * p.sigma * K * gny + p.gy
    ff = _force_field(force, p, R.shape[-2], R.dtype)
    if ff is not None:
        Gx = Gx + ff[0]
        Gy = Gy + ff[1]
    ux = (jx + 0.5 * Gx) / rho
    uy = (jy + 0.5 * Gy) / rho
    dPx, dPy = gradient(Php, rphi, walls, solid=solid)
    theta = divergence(ux, uy, ru, walls, solid)
    return dict(rhoR=rhoR, rhoB=rhoB, rho=rho, f=f, jx=jx, jy=jy, rhoN=rhoN, lam3=lam3,
                Phip=Php, gnx=gnx, gny=gny, mx=mx, my=my, K=K, Gx=Gx, Gy=Gy,
                ux=ux, uy=uy, dPx=dPx, dPy=dPy, theta=theta)


def collide_and_recolour(R, B, p, force=None):
    """Post-recolour populations R++, B++ at every fluid site (steps 1-7)."""
    d = interface_fields(R, B, p, force)
    Cxx, Cyy, Cxy = correction_tensor(d['ux'], d['uy'], d['Gx'], d['Gy'],
                                      d['dPx'], d['dPy'], d['theta'], d['rho'], d['lam3'])
    fplus = collide_modal(d['f'], d['rhoR'], d['rhoB'], d['ux'], d['uy'],
                          d['Gx'], d['Gy'], Cxx, Cyy, Cxy, d['lam3'], p)
    return recolour(fplus, d['rhoR'], d['rhoB'], d['mx'], d['my'], p)


class Oracle:
    """Time stepper holding the pre-collision populations of the fluid sites.

    ``R`` and ``B`` have shape [9, F, nx] with F = ny (periodic) or ny - 2 (walls).
    With a solid mask they cover the whole lattice and are zero at solid sites.
    """

    def __init__(self, p, dtype=torch.float64, force=None):
        self.p = p
        self.solid = solid_mask(p)
        self.dtype = dtype
        self.force = None if force is None else torch.as_tensor(force, dtype=dtype)
        self.t = 0
        self.R = None
        self.B = None

    # -- initial state -------------------------------------------------------
    def init(self, rhoN0):
        """rho_R = rho_0R (1 + rho^N)/2, rho_B = rho_0B (1 - rho^N)/2 at rest:
        C_i = rho_C phi_i = (rho_C/rho) f^(0)_i(rho, u = 0)."""
        p = self.p
        rn = torch.as_tensor(rhoN0, dtype=self.dtype)
        if p.walls:
            rn = rn[1:p.ny - 1]
        rhoR = p.rho0_R * (1.0 + rn) / 2.0
        rhoB = p.rho0_B * (1.0 - rn) / 2.0
        phi = rest_fractions(rhoR, rhoB, p)
        self.R = rhoR * phi
        self.B = rhoB * phi
        self._clear_solid()
        self.t = 0
        return self

    def _clear_solid(self):
        if self.solid is not None:
            self.R[:, self.solid] = 0.0
            self.B[:, self.solid] = 0.0

    def init_moving(self, rhoN0, ux, uy):
        """Initial state with a velocity field: C_i = (rho_C/rho) f^(0)_i(rho, u)
        (Sec. II equilibrium), used for the transient-flow pins."""
        p = self.p
        rn = torch.as_tensor(rhoN0, dtype=self.dtype)
        ux = torch.as_tensor(ux, dtype=self.dtype)
        uy = torch.as_tensor(uy, dtype=self.dtype)
        if p.walls:
            rn, ux, uy = rn[1:p.ny - 1], ux[1:p.ny - 1], uy[1:p.ny - 1]
        rhoR = p.rho0_R * (1.0 + rn) / 2.0
        rhoB = p.rho0_B * (1.0 - rn) / 2.0
        f0 = equilibrium(rhoR, rhoB, ux, uy, p)
        rho = rhoR + rhoB
        self.R = rhoR / rho * f0
        self.B = rhoB / rho * f0
        self._clear_solid()
        self.t = 0
        return self

    def set_state(self, R, B):
        self.R = torch.as_tensor(R, dtype=self.dtype).clone()
        self.B = torch.as_tensor(B, dtype=self.dtype).clone()
        return self

    # -- stepping -------------------------------------------------------------
    def post_collision(self):
        return collide_and_recolour(self.R, self.B, self.p, self.force)

    def step(self, n=1):
        for _ in range(n):
            Rpp, Bpp = self.post_collision()
            self.R = stream(Rpp, self.p.walls, self.solid)
            self.B = stream(Bpp, self.p.walls, self.solid)
            self.t += 1
        return self

    # -- observation ----------------------------------------------------------
    def fields(self):
        """rho, u (force-adjusted, Sec. II), rho^N on the full [ny, nx] lattice;
        solid rows and solid sites are NaN."""
        d = interface_fields(self.R, self.B, self.p, self.force)
        return {k: self._full(d[k]) for k in ('rho', 'ux', 'uy', 'rhoN', 'rhoR', 'rhoB')}

    def masses(self):
        return float(self.R.sum()), float(self.B.sum())

    def _full(self, a):
        if self.solid is not None:
            return torch.where(self.solid, torch.full_like(a, float('nan')), a)
        if not self.p.walls:
            return a
        out = torch.full((self.p.ny, self.p.nx), float('nan'), dtype=a.dtype)
        out[1:self.p.ny - 1] = a
        return out

    def full_pops(self, which=None):
        """Pre-collision populations on the full lattice [2, 9, ny, nx] (solid rows 0)."""
        p = self.p
        out = torch.zeros((2, Q, p.ny, p.nx), dtype=self.dtype)
        rows = slice(1, p.ny - 1) if p.walls else slice(0, p.ny)
        out[0, :, rows] = self.R
        out[1, :, rows] = self.B
        return out

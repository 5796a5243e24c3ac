"""Seeded synthetic inputs: initial colour-index fields, force fields and
parameter sets for the benchmark and test workloads.

This module holds no arithmetic of the scheme itself; it only builds the
geometry (drops, layers, emulsions) and the parameter dictionaries that both
the HIP path and the test oracle consume.  All randomness comes from
``numpy.random.default_rng(seed)``.

Workloads (the paper's own runs are synthetic drops and flat layers; these
take their structure):

* ``static_drop``      64x64 periodic, centred drop of radius 16, Lambda = 10
* ``layered_channel``  256x128, walls at rows 0 and 127, red below, blue above
* ``emulsion``         4096x4096 periodic, 50 non-overlapping drops, radii U[20, 80]
* ``ellipse_drop``     one axis-aligned elliptic drop per lattice (batched runs)
* ``gaussian_bumps``   smooth per-site body-force field
* ``circular_wall``    solid mask of a circular container (staircase wall)
* ``config_curved_transient``  rotating dense core inside a circular wall
* ``drop_to_ellipse``  the adjoint workload: a drop, an ellipse target, force bumps
"""
import math

import numpy as np

STENCIL_PAPER = (3, 3, 3, 3)     # high-order stencil for every derivative (App. B)
STENCIL_COMPACT = (1, 1, 1, 1)


def alphas_for_ratio(Lambda):
    """(alpha_R, alpha_B) for a density ratio Lambda = rho_0R / rho_0B.

    The lighter phase keeps alpha = 1/2 and the heavier one takes
    1 - 1/(2 Lambda) (resp. Lambda/2), the convention of the paper's
    micro-current tables, so that (1 - a_B) = Lambda (1 - a_R)."""
    if Lambda >= 1.0:
        return 1.0 - 0.5 / Lambda, 0.5
    return 0.5, 1.0 - 0.5 * Lambda


def base_params(Lambda=10.0, rho0_R=1.0, sigma=0.01, beta=0.67, nu=1.0 / 6.0,
                lambda6=1.4, lambda7=1.2, stencil=STENCIL_PAPER):
    aR, aB = alphas_for_ratio(Lambda)
    return dict(rho0_R=rho0_R, rho0_B=rho0_R / Lambda, alpha_R=aR, alpha_B=aB,
                nu_R=nu, nu_B=nu, sigma=sigma, beta=beta, lambda6=lambda6, lambda7=lambda7,
                gx=0.0, gy=0.0, stencil=tuple(stencil), walls=False, ghost_eq=0,
                fixed_K=None, eps_n=1e-6)


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------

def static_drop(nx=64, ny=64, radius=16.0, center=None):
    """+1 inside a circle (distance < radius), -1 outside; default centre
    ((nx-1)/2, (ny-1)/2) keeps the lattice problem D4-symmetric."""
    cx, cy = center if center is not None else ((nx - 1) / 2.0, (ny - 1) / 2.0)
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    return np.where((x - cx) ** 2 + (y - cy) ** 2 < radius * radius, 1.0, -1.0)


def layered_channel(nx=256, ny=128):
    """Red (+1) in fluid rows 1 .. ny/2 - 1, blue (-1) in ny/2 .. ny-2; rows 0
    and ny-1 are solid (value irrelevant, set to -1)."""
    out = -np.ones((ny, nx), dtype=np.float64)
    out[1:ny // 2] = 1.0
    return out


def emulsion_drops(nx=4096, ny=4096, ndrops=50, rmin=20.0, rmax=80.0, gap=6.0, seed=0,
                   max_tries=1_000_000):
    """Radii ~ U[rmin, rmax], centres ~ U[0, n)^2, accepted when every pair is
    separated (minimum image) by at least r_a + r_b + gap."""
    rng = np.random.default_rng(seed)
    radii = rng.uniform(rmin, rmax, size=ndrops)
    centres = []
    tries = 0
    for r in radii:
        while True:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("could not place drops")
            c = rng.uniform(0.0, 1.0, size=2) * (nx, ny)
            ok = True
            for (cx, cy), r2 in zip(centres, radii):
                dx = abs(c[0] - cx)
                dy = abs(c[1] - cy)
                dx = min(dx, nx - dx)
                dy = min(dy, ny - dy)
                if dx * dx + dy * dy < (r + r2 + gap) ** 2:
                    ok = False
                    break
            if ok:
                centres.append((float(c[0]), float(c[1])))
                break
    return np.array(centres), radii


def emulsion(nx=4096, ny=4096, ndrops=50, rmin=20.0, rmax=80.0, gap=6.0, seed=0):
    """+1 inside any drop (minimum-image distance < r), -1 elsewhere."""
    centres, radii = emulsion_drops(nx, ny, ndrops, rmin, rmax, gap, seed)
    out = -np.ones((ny, nx), dtype=np.float64)
    for (cx, cy), r in zip(centres, radii):
        x0, x1 = int(math.floor(cx - r)) - 1, int(math.ceil(cx + r)) + 2
        y0, y1 = int(math.floor(cy - r)) - 1, int(math.ceil(cy + r)) + 2
        xs = np.arange(x0, x1)
        ys = np.arange(y0, y1)
        X, Y = np.meshgrid(xs, ys)
        inside = (X - cx) ** 2 + (Y - cy) ** 2 < r * r
        out[Y[inside] % ny, X[inside] % nx] = 1.0
    return out


def ellipse_drop(n, aspect, center=None, width=None):
    """Axis-aligned ellipse with semi-axes (n/4) sqrt(AR) and (n/4)/sqrt(AR):
    rho^N = +1 inside, -1 outside, or, with ``width``, the smooth profile
    tanh(d / width) of the approximate signed distance d to the ellipse."""
    cx, cy = center if center is not None else ((n - 1) / 2.0, (n - 1) / 2.0)
    a = n / 4.0 * math.sqrt(aspect)
    b = n / 4.0 / math.sqrt(aspect)
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    q = np.sqrt(((x - cx) / a) ** 2 + ((y - cy) / b) ** 2)
    if width is None:
        return np.where(q < 1.0, 1.0, -1.0)
    return np.tanh((1.0 - q) * math.sqrt(a * b) / width)


def gaussian_bumps(nx, ny, nbumps=8, width=24.0, amplitude=1e-6, seed=2):
    """Per-site force field [2, ny, nx]: sum of Gaussian bumps with random
    centres and directions."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    out = np.zeros((2, ny, nx))
    for _ in range(nbumps):
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        ang = rng.uniform(0, 2 * math.pi)
        dx = np.minimum(abs(x - cx), nx - abs(x - cx))
        dy = np.minimum(abs(y - cy), ny - abs(y - cy))
        g = amplitude * np.exp(-(dx * dx + dy * dy) / (2 * width * width))
        out[0] += g * math.cos(ang)
        out[1] += g * math.sin(ang)
    return out


def circular_wall(nx, ny, radius, center=None):
    """Solid mask (True = solid) of a circular no-slip container: every site at
    distance >= radius from the centre (default ((nx-1)/2, (ny-1)/2)) is solid,
    a staircase approximation of the wall at r = radius."""
    cx, cy = center if center is not None else ((nx - 1) / 2.0, (ny - 1) / 2.0)
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    return (x - cx) ** 2 + (y - cy) ** 2 >= radius * radius


def random_solid_sites(nx, ny, count, seed):
    """Mask with ``count`` distinct solid sites drawn uniformly (parity tests)."""
    rng = np.random.default_rng(seed)
    m = np.zeros(ny * nx, dtype=bool)
    m[rng.choice(ny * nx, size=count, replace=False)] = True
    return m.reshape(ny, nx)


def random_state_perturbation(shape, scale, seed):
    """Multiplicative noise field (1 + scale U[-1, 1]) used by parity tests to
    drive the step away from equilibrium."""
    rng = np.random.default_rng(seed)
    return 1.0 + scale * (2.0 * rng.random(shape) - 1.0)


# ----------------------------------------------------------------------------
# named configurations
# ----------------------------------------------------------------------------

def config_static_drop():
    """64x64 periodic static drop, radius 16, Lambda = 10 (rho_R = 1, rho_B = 0.1),
    sigma = 0.01, beta = 0.67, nu = 1/6, ghost rates 1.4 / 1.2; 1000 steps."""
    p = base_params(Lambda=10.0, sigma=0.01)
    return dict(nx=64, ny=64, steps=1000, params=p, rhoN0=static_drop(64, 64, 16.0))


def config_layered_channel(width=2.0):
    """256x128 channel, walls at rows 0 and 127, Lambda = 100, dynamic
    viscosity ratio 10 (nu_B = 10 nu_R), body force density 1e-6 along x.
    Red below, blue above, joined by a tanh colour profile of the given width
    centred on the channel's mid-plane (width 0: the sharp +-1 step, which
    diverges within 500 steps at this density ratio)."""
    p = base_params(Lambda=100.0, sigma=0.01)
    p.update(nu_R=1.0 / 6.0, nu_B=10.0 / 6.0, gx=1e-6, walls=True)
    if width > 0:
        yy = (np.arange(128) - 0.5)[:, None] * np.ones((1, 256))
        rn = np.tanh((128 / 2.0 - yy) / width)
    else:
        rn = layered_channel(256, 128)
    return dict(nx=256, ny=128, steps=20000, params=p, rhoN0=rn)


def config_emulsion(nx=4096, ny=4096, seed=0):
    """4096^2 periodic emulsion: 50 drops, radii U[20, 80], Lambda = 10,
    sigma = 0.005, beta = 0.67, nu = 1/6; 1000 steps."""
    p = base_params(Lambda=10.0, sigma=0.005)
    return dict(nx=nx, ny=ny, steps=1000, params=p,
                rhoN0=emulsion(nx, ny, 50, 20.0, 80.0, 6.0, seed) if nx >= 1024 else None)


def config_curved_transient(Lambda, R0=120.0, R=360.0, eta=0.333, beta=0.3, sigma=0.001, u0=1e-3):
    """Decaying rotation of a dense red core inside a circular no-slip wall
    (Sec. IV, dynamics of curved interfaces; App. D): red for r < R0, blue
    out to the wall at r = R, equal shear viscosity eta (nu_C = eta / rho_0C),
    segregation beta = 0.3 and R0 = 120, R = 360 as in the paper.  The red
    core starts in rigid rotation with speed u0 at r = R0 (u_phi = u0 r / R0
    weighted by the red fraction (1 + rho^N)/2 of the tanh profile), the blue
    fluid at rest.  The paper prints neither sigma nor the speed: sigma = 1e-3,
    u0 = 1e-3.  Lattice: the smallest square with one solid ring outside r = R.
    Returns nx, ny, params, rhoN0, ux0, uy0, solid, centre."""
    n = int(2 * (math.ceil(R) + 2))
    c = (n - 1) / 2.0
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    r = np.hypot(x - c, y - c)
    rn = np.tanh(0.9 * beta * (R0 - r))
    red = 0.5 * (1.0 + rn)
    omega = u0 / R0
    ux0 = -omega * (y - c) * red
    uy0 = omega * (x - c) * red
    p = base_params(Lambda=Lambda, sigma=sigma, beta=beta)
    p.update(nu_R=eta / p["rho0_R"], nu_B=eta / p["rho0_B"])
    return n, n, p, rn, ux0, uy0, circular_wall(n, n, R, (c, c)), (c, c)


def emulsion_crop(n=512, ndrops=3, seed=0):
    """Smaller emulsion for parity runs: ``ndrops`` drops with the same radius law."""
    return emulsion(n, n, ndrops, 20.0, 80.0 if n >= 400 else n / 8.0, 6.0, seed)


def config_batch(nsim=256, seed=1, width=2.0):
    """Batch of independent periodic drops: side ~ U{64, 128, 256, 512},
    Lambda ~ U{1, 10, 100}, sigma = 10^U[-3, -1], an axis-aligned centred
    ellipse of aspect ratio ~ U[1, 1.5] with semi-axes (L/4) sqrt(AR) and
    (L/4)/sqrt(AR), given as tanh(d / width) of the distance to the ellipse
    (a sharp +-1 ellipse if width is None); beta = 0.67, nu = 1/6, ghost rates
    1.4 / 1.2.  At Lambda = 100 the scheme is unstable for sigma above about
    0.06 (these rates and viscosity), so sigma is redrawn there until it is at
    most 0.05.  Returns a list of (nx, ny, params, rhoN0)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nsim):
        L = int(rng.choice([64, 128, 256, 512]))
        Lam = float(rng.choice([1.0, 10.0, 100.0]))
        sigma = float(10.0 ** rng.uniform(-3.0, -1.0))
        while Lam >= 100.0 and sigma > 0.05:
            sigma = float(10.0 ** rng.uniform(-3.0, -1.0))
        ar = float(rng.uniform(1.0, 1.5))
        prm = base_params(Lambda=Lam, sigma=sigma)
        out.append((L, L, prm, ellipse_drop(L, ar, width=width)))
    return out


def drop_to_ellipse(n=512, width=2.0):
    """The adjoint workload: n^2 periodic, a centred drop of radius n/4 as the
    tanh profile tanh((n/4 - r)/width) (width None: the sharp +-1 circle), a
    seeded target ellipse of equal area (aspect ratio ~ U[1, 1.5], angle
    ~ U[0, pi), +-1), and 8 Gaussian force bumps of width 24, random direction,
    amplitude 1e-6; Lambda = 10, sigma = 0.01.  From the sharp circle the
    final-state loss is not a smooth function of sigma at working precision
    (FP64 central differences change sign between steps h of 1e-5 and 1e-8);
    from the tanh profile the FP64 adjoint equals them to 7 digits.  Returns
    (rhoN0, target, force [2, n, n], params)."""
    rng = np.random.default_rng(2)
    yy, xx = np.mgrid[0:n, 0:n]
    c = (n - 1) / 2.0
    r = np.hypot(xx - c, yy - c)
    rn0 = np.where(r < n / 4, 1.0, -1.0) if width is None else np.tanh((n / 4 - r) / width)
    ar = rng.uniform(1.0, 1.5)
    ang = rng.uniform(0, np.pi)
    xr = (xx - c) * np.cos(ang) + (yy - c) * np.sin(ang)
    yr = -(xx - c) * np.sin(ang) + (yy - c) * np.cos(ang)
    target = np.where(np.hypot(xr / np.sqrt(ar), yr * np.sqrt(ar)) < n / 4, 1.0, -1.0)
    force = np.zeros((2, n, n))
    for _ in range(8):
        bx, by = rng.uniform(0, n, 2)
        th = rng.uniform(0, 2 * np.pi)
        bump = 1e-6 * np.exp(-((xx - bx) ** 2 + (yy - by) ** 2) / (2 * 24.0 ** 2))
        force[0] += bump * np.cos(th)
        force[1] += bump * np.sin(th)
    return rn0, target, force, base_params(Lambda=10.0, sigma=0.01)

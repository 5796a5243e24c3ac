"""Shared helpers of the GPU parity tests (host side only)."""
import numpy as np
import torch

from oracle import chromo as O
from oracle.lattice import C, OPP, Q
from paper_2005_04642_amd import lbm

# FP32 bars of the parity tests: rho within 1e-5 relative; u within
# FP32_FLOOR_FACTOR times the error FP32 storage alone leaves on the same
# workload (the FP64 oracle with its state rounded to FP32 after every step).
# The FP32 path adds its arithmetic to that floor: measured 1.6 to 6.0 floors
# in u over the static drop, the channels, the emulsion crops and the batch
# members.
FP32_TOL_RHO = 1e-5
FP32_FLOOR_FACTOR = 8.0


def pull_gather(S, walls):
    """Pre-collision populations from a pull-layout buffer S [2, 9, ny, nx]:
    f_i(r) = S_i(r - c_i), or S_opp(i)(r) when r - c_i is a solid row.
    Returns the fluid rows only, [2, 9, F, nx]."""
    S = np.asarray(S)
    ny = S.shape[2]
    out = np.empty_like(S)
    for i in range(Q):
        cx, cy = C[i]
        out[:, i] = np.roll(np.roll(S[:, i], cx, axis=-1), cy, axis=-2)
    if walls:
        for i in range(Q):
            cy = C[i][1]
            if cy == 1:
                out[:, i, 1] = S[:, OPP[i], 1]
            elif cy == -1:
                out[:, i, ny - 2] = S[:, OPP[i], ny - 2]
        return out[:, :, 1:ny - 1]
    return out


def push_scatter(P, ny):
    """Inverse of pull_gather for walled lattices: the pull-layout buffer
    [2, 9, ny, nx] whose gather gives the fluid-row populations P [2, 9, ny-2, nx]
    (S_i(s) = P_i(s + c_i), or P_opp(i)(s) when s + c_i is a solid row)."""
    P = np.asarray(P)
    nx = P.shape[-1]
    Pf = np.zeros(P.shape[:2] + (ny, nx))
    Pf[:, :, 1:ny - 1] = P
    S = np.empty_like(Pf)
    for i in range(Q):
        cx, cy = C[i]
        S[:, i] = np.roll(np.roll(Pf[:, i], -cx, axis=-1), -cy, axis=-2)
    for i in range(Q):
        cy = C[i][1]
        if cy == -1:
            S[:, i, 1] = Pf[:, OPP[i], 1]
        elif cy == 1:
            S[:, i, ny - 2] = Pf[:, OPP[i], ny - 2]
    return S


def oracle_params(nx, ny, params):
    return O.Params(nx=nx, ny=ny, **params)


def oracle_post_collision(S, nx, ny, params, force=None):
    """Post-recolour populations the oracle computes from the pre-collision
    state encoded in the pull-layout buffer S (fluid rows, [2, 9, F, nx])."""
    p = oracle_params(nx, ny, params)
    P = pull_gather(S, p.walls)
    o = O.Oracle(p, force=force).set_state(torch.from_numpy(P[0]), torch.from_numpy(P[1]))
    R, B = o.post_collision()
    return np.stack([R.numpy(), B.numpy()])


def fluid(a, walls):
    return a[..., 1:-1, :] if walls else a


def perturbed_buffer(sim, scale, seed):
    """Multiply the live buffer by (1 + scale U[-1, 1]) (seeded, host-generated)."""
    from paper_2005_04642_amd import workloads as Wk
    buf = sim.live_pops()
    noise = Wk.random_state_perturbation(tuple(buf.shape), scale, seed)
    buf.mul_(torch.as_tensor(noise, dtype=buf.dtype, device=buf.device))
    return buf


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def pull_gather_masked(S, solid):
    """Pre-collision populations from a pull-layout buffer S [2, 9, ny, nx] on a
    lattice with a solid-site mask: f_i(r) = S_i(r - c_i), or S_opp(i)(r) when
    r - c_i is solid; zero at solid sites."""
    S = np.asarray(S)
    solid = np.asarray(solid, dtype=bool)
    out = np.empty_like(S)
    for i in range(Q):
        cx, cy = C[i]
        moved = np.roll(S[:, i], (cy, cx), axis=(-2, -1))
        src_solid = np.roll(solid, (cy, cx), axis=(-2, -1))
        out[:, i] = np.where(src_solid, S[:, OPP[i]], moved)
    out[:, :, solid] = 0.0
    return out


def push_scatter_masked(P, solid):
    """Inverse of pull_gather_masked: the buffer whose gather gives the
    populations P [2, 9, ny, nx] (S_i(s) = P_i(s + c_i), or P_opp(i)(s) when
    s + c_i is solid; zero at solid sites)."""
    P = np.asarray(P)
    solid = np.asarray(solid, dtype=bool)
    S = np.empty_like(P)
    for i in range(Q):
        cx, cy = C[i]
        moved = np.roll(P[:, i], (-cy, -cx), axis=(-2, -1))
        dst_solid = np.roll(solid, (-cy, -cx), axis=(-2, -1))
        S[:, i] = np.where(dst_solid, P[:, OPP[i]], moved)
    S[:, :, solid] = 0.0
    return S


def oracle_runs(nx, ny, params, rhoN0, steps, force=None):
    """Fields of the FP64 oracle after ``steps`` steps, and of the same oracle
    with its state rounded to FP32 after every step (FP64 arithmetic
    otherwise): the second is the error FP32 storage alone causes, the floor
    an FP32 path is measured against."""
    p = oracle_params(nx, ny, params)
    f = None if force is None else torch.as_tensor(force)
    exact = O.Oracle(p, force=f).init(rhoN0)
    rounded = O.Oracle(p, force=f).init(rhoN0)
    rounded.R, rounded.B = rounded.R.float().double(), rounded.B.float().double()
    for _ in range(steps):
        exact.step(1)
        rounded.step(1)
        rounded.R, rounded.B = rounded.R.float().double(), rounded.B.float().double()
    return ({k: v.numpy() for k, v in exact.fields().items()},
            {k: v.numpy() for k, v in rounded.fields().items()})


def field_errors(f, fo, walls=False):
    """e_rho = max |d rho| / rho and e_u = max |d u| / max |u| over fluid sites
    (NaN marks solid sites and is skipped)."""
    a = {k: fluid(np.asarray(v, dtype=np.float64), walls) for k, v in f.items()}
    b = {k: fluid(np.asarray(v, dtype=np.float64), walls) for k, v in fo.items()}
    e_rho = float(np.nanmax(np.abs(a["rho"] - b["rho"]) / b["rho"]))
    du = np.hypot(a["ux"] - b["ux"], a["uy"] - b["uy"])
    e_u = float(np.nanmax(du) / np.nanmax(np.hypot(b["ux"], b["uy"])))
    return e_rho, e_u

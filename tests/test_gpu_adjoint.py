"""The hand-written adjoint of the step (lbm_adjoint_step and the checkpointed
rollout built on it) against reverse-mode differentiation of the FP64 oracle
(torch autograd through its own operations) and against finite differences.

* one step, FP64: dL/dpops_t, dL/dsigma and dL/dG_ext for a random linear
  functional of the next state, every stencil profile and option;
* one step, FP32 against FP64 (the same state);
* colour-index and initial-state adjoints against autograd;
* multi-step rollout (32^2 drop, open and inside a circular wall with
  obstacles): gradients with respect to sigma, the force field and the
  initial colour index against central finite differences of the GPU forward,
  and checkpointing leaves them unchanged;
* walled lattices and masks of solid sites: one step against autograd.
"""
import numpy as np
import pytest
import torch

from oracle import chromo as O
from oracle.lattice import C, OPP
from paper_2005_04642_amd import adjoint, lbm, workloads as Wk

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def torch_pull(S):
    """Pre-collision populations of a periodic pull-layout buffer S [2, 9, ny, nx]:
    C_i(r) = S_i(r - c_i)."""
    return torch.stack([torch.roll(S[:, i], shifts=(C[i][1], C[i][0]), dims=(-2, -1)) for i in range(9)], dim=1)


def torch_pull_walls(S):
    """Fluid-row pre-collision populations of a walled pull-layout buffer S
    [2, 9, ny, nx]: C_i(r) = S_i(r - c_i), or S_opp(i)(r) when r - c_i is a
    solid row (half-way bounce-back); returns [2, 9, ny - 2, nx]."""
    ny = S.shape[-2]
    out = []
    for i in range(9):
        cx, cy = C[i]
        v = torch.roll(S[:, i], shifts=(cy, cx), dims=(-2, -1))
        if cy == 1:
            v = torch.cat([v[:, :1], S[:, OPP[i], 1:2], v[:, 2:]], dim=1)
        elif cy == -1:
            v = torch.cat([v[:, :ny - 2], S[:, OPP[i], ny - 2:ny - 1], v[:, ny - 1:]], dim=1)
        out.append(v)
    return torch.stack(out, dim=1)[:, :, 1:ny - 1]


def torch_pull_masked(S, solid, rest):
    """Pre-collision populations of a pull-layout buffer S on a lattice with a
    solid-site mask: C_i(r) = S_i(r - c_i), or S_opp(i)(r) when r - c_i is
    solid.  Solid sites take the constant state ``rest`` (finite, so that the
    oracle's arithmetic there, which nothing reads, stays finite under autograd)."""
    m = torch.as_tensor(solid)
    out = []
    for i in range(9):
        cx, cy = C[i]
        v = torch.roll(S[:, i], shifts=(cy, cx), dims=(-2, -1))
        src = torch.roll(m, shifts=(cy, cx), dims=(-2, -1))
        v = torch.where(src, S[:, OPP[i]], v)
        out.append(torch.where(m, rest[:, i], v))
    return torch.stack(out, dim=1)


def masked_container(nx, ny, seed):
    m = Wk.circular_wall(nx, ny, 0.5 * min(nx, ny) - 1.0)
    return m | Wk.random_solid_sites(nx, ny, max(3, nx * ny // 60), seed)


def state_and_params(nx, ny, seed, stencil=(3, 3, 3, 3), solid=None, **extra):
    params = Wk.base_params(Lambda=10.0, sigma=0.02, stencil=stencil)
    params.update(gx=3e-5, gy=-2e-5, nu_B=0.4)
    params.update(extra)
    rng = np.random.default_rng(seed)
    rn = np.clip(np.tanh(2.0 * rng.standard_normal((ny, nx))), -1, 1)
    sim = lbm.Simulation(nx, ny, params, rn, storage="f64", device=DEV)
    torch.cuda.synchronize()
    S = sim.live_pops().cpu().numpy()
    sim.close()
    S = S * Wk.random_state_perturbation(S.shape, 0.05, seed + 1)
    lam = rng.standard_normal(S.shape)
    force = 1e-4 * rng.standard_normal((2, ny, nx))
    if params.get("walls"):      # solid rows hold nothing
        for a in (S, lam):
            a[..., 0, :] = 0.0
            a[..., ny - 1, :] = 0.0
    if solid is not None:        # nor do solid sites
        S[:, :, solid] = 0.0
        lam[:, :, solid] = 0.0
    return params, rn, S, lam, force


def oracle_vjp(params, S, lam, force, solid=None):
    """Autograd of L = <lam, step(S)> through the oracle (FP64)."""
    ny, nx = S.shape[-2:]
    p = O.Params(nx=nx, ny=ny, solid=solid, **params)
    S_t = torch.tensor(S, dtype=torch.float64, requires_grad=True)
    sig = torch.tensor(float(params["sigma"]), dtype=torch.float64, requires_grad=True)
    p.sigma = sig
    F_t = None if force is None else torch.tensor(force, dtype=torch.float64, requires_grad=True)
    if solid is not None:
        rest = torch.full((2, 9, ny, nx), 0.05, dtype=torch.float64)
        P = torch_pull_masked(S_t, solid, rest)
    else:
        P = torch_pull_walls(S_t) if p.walls else torch_pull(S_t)
    R, B = O.collide_and_recolour(P[0], P[1], p, force=F_t)
    lam_t = torch.tensor(lam, dtype=torch.float64)
    if p.walls:
        lam_t = lam_t[..., 1:ny - 1, :]
    if solid is not None:        # solid sites store nothing
        m = torch.as_tensor(solid)
        R = torch.where(m, torch.zeros_like(R), R)
        B = torch.where(m, torch.zeros_like(B), B)
    L = (R * lam_t[0]).sum() + (B * lam_t[1]).sum()
    L.backward()
    return S_t.grad.numpy(), float(sig.grad), None if F_t is None else F_t.grad.numpy()


def gpu_vjp(params, rn, S, lam, force, storage="f64", solid=None):
    ny, nx = S.shape[-2:]
    sim = lbm.Simulation(nx, ny, params, rn, storage=storage, device=DEV, force=force, solid=solid)
    T = sim.dtype
    S_d = torch.tensor(S, dtype=T, device=DEV)
    lam_d = torch.tensor(lam, dtype=T, device=DEV)
    out = torch.empty_like(lam_d)
    dsig = torch.zeros(1, dtype=torch.float64, device=DEV)
    dforce = torch.zeros((2, ny, nx), dtype=T, device=DEV)
    sim.adjoint_step(S_d, lam_d, out, dsig, dforce)
    torch.cuda.synchronize()
    res = out.double().cpu().numpy(), float(dsig.item()), dforce.double().cpu().numpy()
    sim.close()
    return res


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


STENCILS = [(3, 3, 3, 3), (1, 1, 1, 1), (3, 1, 3, 1), (1, 3, 1, 3)]


@pytest.mark.parametrize("stencil", STENCILS)
@pytest.mark.parametrize("shape", [(12, 10), (40, 33)])
def test_adjoint_one_step_f64_matches_oracle_autograd(stencil, shape):
    nx, ny = shape
    params, rn, S, lam, force = state_and_params(nx, ny, seed=nx + ny, stencil=stencil)
    gS, gsig, gF = oracle_vjp(params, S, lam, force)
    aS, asig, aF = gpu_vjp(params, rn, S, lam, force)
    e = (rel(aS, gS), abs(asig - gsig) / abs(gsig), rel(aF, gF))
    print("adjoint f64 %s %s: pops %.2e sigma %.2e force %.2e" % (shape, stencil, *e))
    assert e[0] < 1e-11 and e[1] < 1e-10 and e[2] < 1e-11


@pytest.mark.parametrize("stencil", [(3, 3, 3, 3), (1, 1, 1, 1), (3, 1, 1, 3)])
@pytest.mark.parametrize("shape", [(12, 10), (33, 40)])
def test_adjoint_one_step_walls_f64_matches_oracle_autograd(stencil, shape):
    """Walls at rows 0 and ny - 1: the stencils' mirror images and the
    bounce-back transposed."""
    nx, ny = shape
    params, rn, S, lam, force = state_and_params(nx, ny, seed=3 * nx + ny, stencil=stencil, walls=True)
    gS, gsig, gF = oracle_vjp(params, S, lam, force)
    aS, asig, aF = gpu_vjp(params, rn, S, lam, force)
    e = (rel(aS, gS), abs(asig - gsig) / abs(gsig), rel(aF, gF))
    print("adjoint walls f64 %s %s: pops %.2e sigma %.2e force %.2e" % (shape, stencil, *e))
    assert e[0] < 1e-11 and e[1] < 1e-10 and e[2] < 1e-11


@pytest.mark.parametrize("stencil", [(3, 3, 3, 3), (3, 1, 3, 1), (1, 1, 1, 1)])
@pytest.mark.parametrize("shape", [(14, 12), (41, 34)])
def test_adjoint_one_step_mask_f64_matches_oracle_autograd(stencil, shape):
    """A mask of solid sites (a staircase circle and scattered obstacles): the
    transposed centre-value continuation of the stencils and the bounce-back."""
    nx, ny = shape
    solid = masked_container(nx, ny, nx)
    params, rn, S, lam, force = state_and_params(nx, ny, seed=5 * nx + ny, stencil=stencil, solid=solid)
    gS, gsig, gF = oracle_vjp(params, S, lam, force, solid=solid)
    aS, asig, aF = gpu_vjp(params, rn, S, lam, force, solid=solid)
    e = (rel(aS, gS), abs(asig - gsig) / abs(gsig), rel(aF, gF))
    print("adjoint mask f64 %s %s: pops %.2e sigma %.2e force %.2e" % (shape, stencil, *e))
    assert e[0] < 1e-11 and e[1] < 1e-10 and e[2] < 1e-11
    assert np.all(aS[:, :, solid] == 0.0)


def test_adjoint_with_mask_rejects_other_stencil_profiles():
    nx, ny = 20, 16
    solid = masked_container(nx, ny, 1)
    params, rn, S, lam, force = state_and_params(nx, ny, seed=2, stencil=(1, 3, 1, 3), solid=solid)
    with pytest.raises(lbm.LbmError) as e:
        gpu_vjp(params, rn, S, lam, force, solid=solid)
    assert e.value.code == lbm.LBM_ENOTIMPL


@pytest.mark.parametrize("extra", [dict(ghost_eq=1), dict(fixed_K=0.05), dict(recolor=False)])
def test_adjoint_one_step_options_f64(extra):
    nx, ny = 24, 20
    params, rn, S, lam, force = state_and_params(nx, ny, seed=5, **extra)
    gS, gsig, gF = oracle_vjp(params, S, lam, force)
    aS, asig, aF = gpu_vjp(params, rn, S, lam, force)
    e = (rel(aS, gS), abs(asig - gsig) / max(abs(gsig), 1e-300), rel(aF, gF))
    print("adjoint f64 %s: pops %.2e sigma %.2e force %.2e" % (extra, *e))
    assert e[0] < 1e-11 and e[2] < 1e-11
    assert e[1] < 1e-10 or abs(asig - gsig) < 1e-14


def test_adjoint_one_step_f32_against_f64():
    nx, ny = 40, 33
    params, rn, S, lam, force = state_and_params(nx, ny, seed=9)
    S32 = S.astype(np.float32).astype(np.float64)
    a64 = gpu_vjp(params, rn, S32, lam, force, "f64")
    a32 = gpu_vjp(params, rn, S32, lam, force, "f32")
    e = (rel(a32[0], a64[0]), abs(a32[1] - a64[1]) / abs(a64[1]), rel(a32[2], a64[2]))
    print("adjoint f32 vs f64: pops %.2e sigma %.2e force %.2e" % e)
    assert e[0] < 1e-4 and e[1] < 1e-4 and e[2] < 1e-4


@pytest.mark.parametrize("walls", [False, True])
def test_rhoN_and_init_adjoints_match_autograd(walls):
    nx, ny = 20, 16
    params, rn, S, lam, force = state_and_params(nx, ny, seed=3, walls=walls)
    rng = np.random.default_rng(4)
    w = rng.standard_normal((ny, nx))
    # colour index of the pre-collision state of S
    S_t = torch.tensor(S, requires_grad=True)
    P = torch_pull_walls(S_t) if walls else torch_pull(S_t)
    p = O.Params(nx=nx, ny=ny, **params)
    rhoN = O.colour_index(P[0].sum(0), P[1].sum(0), p)
    (rhoN * torch.tensor(w[1:ny - 1] if walls else w)).sum().backward()
    sim = lbm.Simulation(nx, ny, params, rn, storage="f64", device=DEV)
    out = torch.empty((2, 9, ny, nx), dtype=torch.float64, device=DEV)
    sim.rhoN_adjoint(torch.tensor(S, device=DEV), torch.tensor(w, device=DEV), out)
    torch.cuda.synchronize()
    e1 = rel(out.cpu().numpy(), S_t.grad.numpy())
    # initial rest state (un-streamed) as a function of rho^N_0
    rn_t = torch.tensor(rn, requires_grad=True)
    rhoR = p.rho0_R * (1.0 + rn_t) / 2.0
    rhoB = p.rho0_B * (1.0 - rn_t) / 2.0
    phi = O.rest_fractions(rhoR, rhoB, p)
    pre = torch.stack([rhoR * phi, rhoB * phi])               # pre-collision at each site
    buf = torch.stack([torch.roll(pre[:, i], shifts=(-C[i][1], -C[i][0]), dims=(-2, -1)) for i in range(9)], dim=1)
    if walls:   # word i at s next to a solid row holds link opp(i) of s; solid rows hold nothing
        rows = []
        for y in range(ny):
            if y in (0, ny - 1):
                rows.append(torch.zeros_like(buf[:, :, y]))
                continue
            links = []
            for i in range(9):
                ys = y + C[i][1]
                links.append(pre[:, OPP[i], y] if ys in (0, ny - 1) else buf[:, i, y])
            rows.append(torch.stack(links, dim=1))
        buf = torch.stack(rows, dim=2)
    (buf * torch.tensor(lam)).sum().backward()
    g0 = torch.zeros((ny, nx), dtype=torch.float64, device=DEV)
    sim.init_adjoint(torch.tensor(lam, device=DEV), g0)
    torch.cuda.synchronize()
    e2 = rel(g0.cpu().numpy(), rn_t.grad.numpy())
    sim.close()
    print("rhoN adjoint %.2e, init adjoint %.2e" % (e1, e2))
    assert e1 < 1e-12 and e2 < 1e-12


def test_rhoN_and_init_adjoints_with_mask_match_autograd():
    nx, ny = 22, 18
    solid = masked_container(nx, ny, 3)
    m = torch.as_tensor(solid)
    params, rn, S, lam, force = state_and_params(nx, ny, seed=6, solid=solid)
    rng = np.random.default_rng(8)
    w = rng.standard_normal((ny, nx))
    w[solid] = 0.0
    S_t = torch.tensor(S, requires_grad=True)
    P = torch_pull_masked(S_t, solid, torch.full((2, 9, ny, nx), 0.05, dtype=torch.float64))
    p = O.Params(nx=nx, ny=ny, **params)
    rhoN = O.colour_index(P[0].sum(0), P[1].sum(0), p)
    (rhoN * torch.tensor(w)).sum().backward()
    sim = lbm.Simulation(nx, ny, params, rn, storage="f64", device=DEV, solid=solid)
    out = torch.empty((2, 9, ny, nx), dtype=torch.float64, device=DEV)
    sim.rhoN_adjoint(torch.tensor(S, device=DEV), torch.tensor(w, device=DEV), out)
    torch.cuda.synchronize()
    e1 = rel(out.cpu().numpy(), S_t.grad.numpy())
    # the rest state after lbm_set_solid: word i at a fluid s holds link i's
    # rest population of s + c_i, or link opp(i)'s of s itself when s + c_i is
    # solid; solid sites hold nothing
    rn_t = torch.tensor(rn, requires_grad=True)
    rhoR = p.rho0_R * (1.0 + rn_t) / 2.0
    rhoB = p.rho0_B * (1.0 - rn_t) / 2.0
    phi = O.rest_fractions(rhoR, rhoB, p)
    pre = torch.stack([rhoR * phi, rhoB * phi])
    words = []
    for i in range(9):
        cx, cy = C[i]
        moved = torch.roll(pre[:, i], shifts=(-cy, -cx), dims=(-2, -1))
        dst_solid = torch.roll(m, shifts=(-cy, -cx), dims=(-2, -1))
        v = torch.where(dst_solid, pre[:, OPP[i]], moved)
        words.append(torch.where(m, torch.zeros_like(v), v))
    buf = torch.stack(words, dim=1)
    (buf * torch.tensor(lam)).sum().backward()
    g0 = torch.zeros((ny, nx), dtype=torch.float64, device=DEV)
    sim.init_adjoint(torch.tensor(lam, device=DEV), g0)
    torch.cuda.synchronize()
    grad = rn_t.grad.numpy().copy()
    grad[solid] = 0.0
    e2 = rel(g0.cpu().numpy(), grad)
    sim.close()
    print("mask: rhoN adjoint %.2e, init adjoint %.2e" % (e1, e2))
    assert e1 < 1e-12 and e2 < 1e-12


# (dL/dpops, dL/dsigma, dL/dG_ext) bounds of the full-size check
FULL_SIZE_TOL = {"f64": (1e-10, 1e-10, 1e-12), "f32": (2e-2, 1e-4, 1e-6)}


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_full_size_adjoint_sampled_sites(storage):
    """The rollout workload's lattice (512^2, drop of radius 128, eight force
    bumps) after 100 steps: the adjoint step of the full lattice for a
    functional supported on a 17 x 17 square around a sampled site, against
    autograd of the FP64 oracle on a 49 x 49 window (which holds the whole
    dependency cone of that functional): dL/dpops on the square, dL/dsigma,
    dL/dG_ext at the centre.

    Measured: FP64 3e-12..8e-12, 1e-13, 5e-16; FP32 1.7e-3..5.3e-3, 5e-5,
    2e-7.  Both are set by the director m = g / sqrt(|g|^2 + eps^2) in the
    tails of the interface, where |g| = |grad rho^N| is of the order of
    eps = 1e-6: there its derivative grows like 1/eps, and the recolour's
    weight rho_R rho_B / rho, which keeps the forward step insensitive to m in
    the tails, is only ~1e-6 -- so the adjoint carries O(1) terms built from
    a g that FP32 arithmetic resolves to ~1e-7 (FP64: ~1e-16).  The oracle
    itself, run in FP32 arithmetic on a 128^2 version of this state, differs
    from its FP64 adjoint by 2.2e-3..2.5e-3 at interface sites: the FP32
    figure is the conditioning of the regularised director, not an error of
    the kernels.  The small lattices' random states never come near
    |g| ~ eps, hence their 1e-15 (FP64) and 3e-7 (FP32 against FP64)
    agreement."""
    n, half, sup = 512, 24, 8
    params = Wk.base_params(Lambda=10.0, sigma=0.01)
    yy, xx = np.mgrid[0:n, 0:n]
    c = (n - 1) / 2.0
    rn = np.where(np.hypot(xx - c, yy - c) < n / 4, 1.0, -1.0)
    force = Wk.gaussian_bumps(n, n, nbumps=8, width=24.0, amplitude=1e-6, seed=2)
    sim = lbm.Simulation(n, n, params, rn, storage=storage, device=DEV,
                         force=torch.tensor(force, dtype=torch.float64 if storage == "f64" else torch.float32))
    sim.step(100)
    S_d = sim.pops_like()
    S_d.copy_(sim.live_pops())
    S = S_d.double().cpu().numpy()
    rng = np.random.default_rng(17)
    # sites on the interface (where every term of the step is active) and one in the bulk
    r = np.hypot(xx - c, yy - c)
    ring = np.argwhere(np.abs(r - n / 4) < 1.0)
    picks = [tuple(ring[k]) for k in rng.choice(len(ring), 3, replace=False)] + [(100, 400)]
    worst = [0.0, 0.0, 0.0]
    for (y, x) in picks:
        lam = np.zeros((2, 9, n, n))
        ys = np.arange(y - sup, y + sup + 1) % n
        xs = np.arange(x - sup, x + sup + 1) % n
        lam[:, :, ys[:, None], xs[None, :]] = rng.standard_normal((2, 9, 2 * sup + 1, 2 * sup + 1))
        T = sim.dtype
        out = sim.pops_like()
        dsig = torch.zeros(1, dtype=torch.float64, device=DEV)
        dfor = torch.zeros((2, n, n), dtype=T, device=DEV)
        sim.adjoint_step(S_d, torch.tensor(lam, dtype=T, device=DEV), out, dsig, dfor)
        torch.cuda.synchronize()
        wy = np.arange(y - half, y + half + 1) % n
        wx = np.arange(x - half, x + half + 1) % n
        Sw = S[:, :, wy[:, None], wx[None, :]]
        lw = lam[:, :, wy[:, None], wx[None, :]]
        fw = force[:, wy[:, None], wx[None, :]]
        gS, gsig, gF = oracle_vjp(params, Sw, lw, fw)
        a_sq = out.double().cpu().numpy()[:, :, ys[:, None], xs[None, :]]
        g_sq = gS[:, :, half - sup:half + sup + 1, half - sup:half + sup + 1]
        e = (rel(a_sq, g_sq), abs(float(dsig.item()) - gsig) / max(abs(gsig), 1e-6),
             rel(dfor.double().cpu().numpy()[:, y, x], gF[:, half, half]))
        print("  site (%d, %d): pops %.2e sigma %.2e (%.3e vs %.3e) force %.2e, max|dL/dpops| %.2e"
              % (x, y, e[0], e[1], float(dsig.item()), gsig, e[2], np.max(np.abs(g_sq))))
        worst = [max(w, v) for w, v in zip(worst, e)]
    sim.close()
    print("full-size adjoint %s: pops %.2e sigma %.2e force %.2e" % (storage, *worst))
    assert all(w < t for w, t in zip(worst, FULL_SIZE_TOL[storage])), worst


# ---------------------------------------------------------------------------
# multi-step rollout: finite differences and checkpointing
# ---------------------------------------------------------------------------

def fd_case():
    n, R, steps = 32, 8.0, 24
    params = Wk.base_params(Lambda=10.0, sigma=0.01)
    yy, xx = np.mgrid[0:n, 0:n]
    d = np.hypot(xx - 15.5, yy - 15.5)
    rn0 = np.tanh(0.8 * (R - d))
    target = np.tanh(0.8 * (R - np.hypot((xx - 15.5) / 1.2, (yy - 15.5) * 1.2)))
    rng = np.random.default_rng(2)
    force = np.zeros((2, n, n))
    for _ in range(3):
        cx, cy = rng.uniform(0, n, 2)
        ang = rng.uniform(0, 2 * np.pi)
        bump = 1e-3 * np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2 * 4.0 ** 2))
        force[0] += bump * np.cos(ang)
        force[1] += bump * np.sin(ang)
    return n, steps, params, rn0, target, force


def loss_of(rn0, sigma, force, params, steps, target, checkpoint=100):
    out = adjoint.rollout(rn0, sigma, force, params, steps, checkpoint=checkpoint, storage="f64", device=DEV)
    return ((out - target) ** 2).sum()


def test_rollout_gradients_match_finite_differences():
    n, steps, params, rn0, target, force = fd_case()
    tgt = torch.tensor(target, device=DEV)
    rn_t = torch.tensor(rn0, device=DEV, requires_grad=True)
    sig_t = torch.tensor(0.01, dtype=torch.float64, requires_grad=True)
    f_t = torch.tensor(force, device=DEV, requires_grad=True)
    L = loss_of(rn_t, sig_t, f_t, params, steps, tgt, checkpoint=7)
    L.backward()

    def L_at(rn=rn0, sigma=0.01, frc=force):
        with torch.no_grad():
            return float(loss_of(torch.tensor(rn, device=DEV), sigma, torch.tensor(frc, device=DEV), params,
                                 steps, tgt))

    h = 1e-5
    fd_sig = (L_at(sigma=0.01 + h) - L_at(sigma=0.01 - h)) / (2 * h)
    e_sig = abs(float(sig_t.grad) - fd_sig) / abs(fd_sig)
    errs = []
    for (y, x) in [(15, 23), (8, 16), (20, 10)]:
        hr = 1e-6
        a = rn0.copy(); a[y, x] += hr
        b = rn0.copy(); b[y, x] -= hr
        fd = (L_at(rn=a) - L_at(rn=b)) / (2 * hr)
        errs.append(abs(float(rn_t.grad[y, x]) - fd) / max(abs(fd), 1e-12))
    for (c, y, x) in [(0, 15, 24), (1, 9, 15)]:
        hf = 1e-5
        a = force.copy(); a[c, y, x] += hf
        b = force.copy(); b[c, y, x] -= hf
        fd = (L_at(frc=a) - L_at(frc=b)) / (2 * hf)
        errs.append(abs(float(f_t.grad[c, y, x]) - fd) / max(abs(fd), 1e-12))
    print("rollout FD: sigma %.2e (grad %.6e fd %.6e); rhoN0/force %s" % (e_sig, float(sig_t.grad), fd_sig,
                                                                          ["%.2e" % v for v in errs]))
    assert e_sig < 1e-5
    assert max(errs) < 1e-4


def test_rollout_with_mask_gradients_match_finite_differences():
    """The checkpointed rollout inside a circular wall with two obstacles."""
    n, steps, params, rn0, target, force = fd_case()
    solid = Wk.circular_wall(n, n, 15.0)
    solid[6, 20] = solid[25, 9] = True
    params = dict(params, solid=solid)
    m = torch.as_tensor(solid, device=DEV)
    tgt = torch.tensor(target, device=DEV)

    def loss(rn, sigma, frc, checkpoint=100):
        # solid sites read as NaN: the loss covers the fluid only
        out = adjoint.rollout(rn, sigma, frc, params, steps, checkpoint=checkpoint, storage="f64", device=DEV)
        d = torch.where(m, torch.zeros_like(out), out - tgt)
        return (d ** 2).sum()

    rn_t = torch.tensor(rn0, device=DEV, requires_grad=True)
    sig_t = torch.tensor(0.01, dtype=torch.float64, requires_grad=True)
    f_t = torch.tensor(force, device=DEV, requires_grad=True)
    L = loss(rn_t, sig_t, f_t, checkpoint=5)
    L.backward()

    def L_at(rn=rn0, sigma=0.01, frc=force):
        with torch.no_grad():
            return float(loss(torch.tensor(rn, device=DEV), sigma, torch.tensor(frc, device=DEV)))

    # central differences at h and h/2, Richardson-extrapolated (the loss is
    # more strongly curved in sigma here than on the open lattice)
    h = 1e-5
    fd1 = (L_at(sigma=0.01 + h) - L_at(sigma=0.01 - h)) / (2 * h)
    fd2 = (L_at(sigma=0.01 + h / 2) - L_at(sigma=0.01 - h / 2)) / h
    fd_sig = (4 * fd2 - fd1) / 3
    e_sig = abs(float(sig_t.grad) - fd_sig) / abs(fd_sig)
    errs = []
    for (y, x) in [(15, 23), (8, 16), (20, 10)]:
        hr = 1e-6
        a = rn0.copy(); a[y, x] += hr
        b = rn0.copy(); b[y, x] -= hr
        fd = (L_at(rn=a) - L_at(rn=b)) / (2 * hr)
        errs.append(abs(float(rn_t.grad[y, x]) - fd) / max(abs(fd), 1e-12))
    for (c, y, x) in [(0, 15, 24), (1, 9, 15)]:
        hf = 1e-5
        a = force.copy(); a[c, y, x] += hf
        b = force.copy(); b[c, y, x] -= hf
        fd = (L_at(frc=a) - L_at(frc=b)) / (2 * hf)
        errs.append(abs(float(f_t.grad[c, y, x]) - fd) / max(abs(fd), 1e-12))
    print("masked rollout FD: sigma %.2e (plain central difference %.2e); rhoN0/force %s"
          % (e_sig, abs(float(sig_t.grad) - fd1) / abs(fd1), ["%.2e" % v for v in errs]))
    assert e_sig < 1e-6          # measured 4.4e-8 (9.3e-6 before extrapolation)
    assert max(errs) < 1e-4
    assert float(rn_t.grad[torch.as_tensor(solid, device=DEV)].abs().max()) == 0.0


def test_checkpointing_does_not_change_gradients():
    n, steps, params, rn0, target, force = fd_case()
    tgt = torch.tensor(target, device=DEV)
    grads = []
    for ck in (1, 5, 100):
        rn_t = torch.tensor(rn0, device=DEV, requires_grad=True)
        sig_t = torch.tensor(0.01, dtype=torch.float64, requires_grad=True)
        f_t = torch.tensor(force, device=DEV, requires_grad=True)
        loss_of(rn_t, sig_t, f_t, params, steps, tgt, checkpoint=ck).backward()
        grads.append((rn_t.grad.cpu().numpy(), float(sig_t.grad), f_t.grad.cpu().numpy()))
    for g in grads[1:]:
        assert np.array_equal(grads[0][0], g[0])
        assert grads[0][1] == g[1]
        assert np.array_equal(grads[0][2], g[2])


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_recompute_overlap_does_not_change_gradients(storage):
    """The backward pass with the next segment recomputed on a second stream,
    unconfined or with the two streams on disjoint CUs (64 for the recompute,
    the rest for the adjoint), gives bit-identical gradients to the one-stream
    backward (5 segments, the last one shorter)."""
    n, steps, params, rn0, target, force = fd_case()
    T = torch.float64 if storage == "f64" else torch.float32
    tgt = torch.tensor(target, dtype=T, device=DEV)
    grads = []
    for ov, rc in ((False, 0), (True, 0), (True, 64), (None, None)):
        rn_t = torch.tensor(rn0, dtype=T, device=DEV, requires_grad=True)
        sig_t = torch.tensor(0.01, dtype=torch.float64, requires_grad=True)
        f_t = torch.tensor(force, dtype=T, device=DEV, requires_grad=True)
        out = adjoint.rollout(rn_t, sig_t, f_t, params, steps, checkpoint=5, storage=storage, device=DEV,
                              overlap=ov, recompute_cus=rc)
        ((out - tgt) ** 2).sum().backward()
        grads.append((rn_t.grad.cpu().numpy(), float(sig_t.grad), f_t.grad.cpu().numpy()))
    for g in grads[1:]:
        assert np.array_equal(grads[0][0], g[0])
        assert grads[0][1] == g[1]
        assert np.array_equal(grads[0][2], g[2])


@pytest.mark.parametrize("kind", ["periodic", "walls", "mask"])
def test_trajectory_calls_equal_single_steps(kind):
    """lbm_step_into (a trajectory into separate buffers, one call) equals
    lbm_step one step at a time, and lbm_adjoint_steps (backwards through it,
    one call) equals lbm_adjoint_step per step: states, adjoints and
    dL/dsigma bit for bit, for an even and an odd number of steps, on a
    periodic, a walled and a masked lattice."""
    n = 48
    params = Wk.base_params(Lambda=10.0, sigma=0.01)
    solid = None
    if kind == "walls":
        params = dict(params, walls=True)
    elif kind == "mask":
        solid = Wk.circular_wall(n, n, 22.0)
    rn0 = Wk.static_drop(n, n, 12.0)
    for steps in (6, 7):
        sim = lbm.Simulation(n, n, params, rn0, storage="f64", device=DEV, solid=solid)
        sim.step(5)
        S0 = sim.live_pops().clone()
        states = [S0] + [sim.pops_like() for _ in range(steps - 1)]
        lbm.lbm_step_into(sim.h, S0.data_ptr(), [t.data_ptr() for t in states[1:]], sim.stream())
        live, nxt = S0.clone(), sim.pops_like()
        sim.set_pops(live, nxt)
        ref = [S0]
        for _ in range(steps - 1):
            sim.step(1)
            ref.append(sim.live_pops().clone())
        rows = slice(1, n - 1) if kind == "walls" else slice(0, n)   # (wall rows hold no state: never written)
        for a, b in zip(states, ref):
            assert torch.equal(a[:, :, rows], b[:, :, rows])
        g = torch.Generator(device=DEV).manual_seed(5)
        lam0 = 1e-3 * torch.randn((2, 9, n, n), generator=g, device=DEV, dtype=torch.float64)
        ws = sim.adjoint_workspace()
        # one call
        A, B = sim.pops_like(), sim.pops_like()
        A.copy_(lam0)
        ds1 = torch.zeros(1, dtype=torch.float64, device=DEV)
        df1 = torch.zeros((2, n, n), dtype=torch.float64, device=DEV)
        lbm.lbm_adjoint_steps(sim.h, [t.data_ptr() for t in states], A.data_ptr(), B.data_ptr(), ws.data_ptr(),
                              ws.numel(), ds1.data_ptr(), df1.data_ptr(), sim.stream())
        got = A if steps % 2 == 0 else B
        # step by step
        cur, nxt = sim.pops_like(), sim.pops_like()
        cur.copy_(lam0)
        ds2 = torch.zeros(1, dtype=torch.float64, device=DEV)
        df2 = torch.zeros((2, n, n), dtype=torch.float64, device=DEV)
        for t in reversed(states):
            sim.adjoint_step(t, cur, nxt, ds2, df2)
            cur, nxt = nxt, cur
        assert torch.equal(got, cur)
        assert float(ds1) == float(ds2)
        assert torch.equal(df1, df2)
        sim.close()


def test_step_into_hands_the_last_two_states_to_the_handle():
    """After lbm_step_into the handle steps on from states[-1] and writes its
    next step into states[-2] (its other buffer), as the header states."""
    n = 40
    params = Wk.base_params(Lambda=10.0, sigma=0.01)
    sim = lbm.Simulation(n, n, params, Wk.static_drop(n, n, 10.0), storage="f64", device=DEV)
    sim.step(3)
    S0 = sim.live_pops().clone()
    states = [sim.pops_like() for _ in range(3)]
    lbm.lbm_step_into(sim.h, S0.data_ptr(), [t.data_ptr() for t in states], sim.stream())
    first, last = states[0].clone(), states[2].clone()
    sim.step(1)                             # from states[-1] into the handle's other buffer
    ref = sim.pops_like()
    lbm.lbm_step_into(sim.h, last.data_ptr(), [ref.data_ptr()], sim.stream())   # the same step, into ref
    torch.cuda.synchronize()
    assert torch.equal(states[1], ref)      # it was states[-2]
    assert torch.equal(states[2], last)     # read, not written
    assert torch.equal(states[0], first)    # the rest of the trajectory untouched
    sim.close()


def test_partition_stream_range_beyond_the_device():
    """A CU range past the device's CUs is refused (LBM_EINVAL) before any
    stream is created; a whole-device range is accepted."""
    ncu = torch.cuda.get_device_properties(0).multi_processor_count // 8 * 8
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_partition_stream(ncu - 8, 16)
    assert e.value.code == lbm.LBM_EINVAL
    assert lbm.lbm_partition_stream(0, ncu)


def test_cu_budget_does_not_change_results():
    """Tiles planned for fewer CUs (lbm_set_cu_budget), run on a stream
    confined to them (lbm_partition_stream): the same states and adjoints, bit
    for bit."""
    n = 160
    params = Wk.base_params(Lambda=10.0, sigma=0.01)
    rn0 = Wk.static_drop(n, n, 40.0)
    ref = lbm.Simulation(n, n, params, rn0, storage="f32", device=DEV)
    ref.step(30)
    S = ref.live_pops().clone()
    g = torch.Generator(device=DEV).manual_seed(3)
    lam = ref.pops_like()
    lam.copy_(1e-3 * torch.randn((2, 9, n, n), generator=g, device=DEV))
    outs = []
    for budget, cus in ((0, None), (64, (0, 64)), (192, (64, 192))):
        sim = lbm.Simulation(n, n, params, rn0, storage="f32", device=DEV)
        sim.set_cu_budget(budget, budget)
        # (the rollout's own confined streams, created once per process)
        strm = adjoint._partition(DEV, *cus) if cus else torch.cuda.current_stream()
        strm.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(strm):
            sim.step(30)
            out = sim.pops_like()
            ds = torch.zeros(1, dtype=torch.float64, device=DEV)
            sim.adjoint_step(S, lam, out, ds)
        torch.cuda.current_stream().wait_stream(strm)
        torch.cuda.synchronize()
        outs.append((sim.live_pops().clone(), out, float(ds)))
        sim.close()
    for o in outs[1:]:
        assert torch.equal(outs[0][0], o[0])
        assert torch.equal(outs[0][1], o[1])
        assert outs[0][2] == o[2]
    ref.close()


def test_adjoint_workload_gradient_against_finite_differences():
    """The 512^2 adjoint workload (a drop of radius 128, tanh profile of width 2,
    to a seeded ellipse; 8 force bumps), 200 steps, a checkpoint every 100:
    FP64 dL/dsigma against central differences of the FP64 forward to 1e-6
    (measured 7 digits at h = 1e-5 .. 1e-8); FP32 against FP64: dL/dsigma 1e-4,
    dL/dG_ext 1e-4, dL/drho^N_0 5e-2 relative to its largest value (measured 5e-6,
    2e-6, 2.4e-2: the initial colour index's adjoint passes through the
    regularised director of the interface tails, which FP32 resolves poorly)."""
    rn0, target, force, params = Wk.drop_to_ellipse(512)
    steps = 200
    tgt = {T: torch.tensor(target, dtype=T, device=DEV) for T in (torch.float64, torch.float32)}

    def run(storage, sigma, grad=True):
        T = torch.float64 if storage == "f64" else torch.float32
        rn = torch.tensor(rn0, dtype=T, device=DEV, requires_grad=grad)
        f = torch.tensor(force, dtype=T, device=DEV, requires_grad=grad)
        sig = torch.tensor(sigma, dtype=torch.float64, requires_grad=grad)
        out = adjoint.rollout(rn, sig, f, params, steps, checkpoint=100, storage=storage, device=DEV)
        loss = ((out - tgt[T]) ** 2).sum()
        if not grad:
            return float(loss)
        loss.backward()
        return float(sig.grad), rn.grad.double().cpu().numpy(), f.grad.double().cpu().numpy()

    s64, rn64, f64 = run("f64", 0.01)
    s32, rn32, f32 = run("f32", 0.01)
    h = 1e-6
    fd = (run("f64", 0.01 + h, False) - run("f64", 0.01 - h, False)) / (2 * h)
    print("adjoint workload 512^2, %d steps: dL/dsigma f64 %.8e fd %.8e f32 %.8e; f32 vs f64 rhoN0 %.2e force %.2e"
          % (steps, s64, fd, s32, rel(rn32, rn64), rel(f32, f64)))
    assert abs(s64 - fd) <= 1e-6 * abs(fd)
    assert abs(s32 - s64) <= 1e-4 * abs(s64)
    assert rel(f32, f64) < 1e-4
    assert rel(rn32, rn64) < 5e-2


# ---------------------------------------------------------------------------
# lattices past 2^31 / 21 sites
# ---------------------------------------------------------------------------

def test_adjoint_on_a_lattice_of_105m_sites():
    """The adjoint addresses its workspace ([ny][39][nx], 16.4 GB here) with
    64-bit row offsets.  A 10240^2 FP32 lattice (104.9 M sites) whose state and
    adjoint input tile a 512^2 lattice's 20 x 20 times has, site by site, the
    tiled adjoint of the 512^2 lattice: the step does the same arithmetic at
    every site, so dL/dpops and dL/dG_ext are bit-identical; dL/dsigma is 400
    times the small lattice's up to the order of its FP64 sum."""
    n, reps = 512, 20
    N = n * reps
    params = Wk.base_params(Lambda=10.0, sigma=0.01)
    rn0 = Wk.emulsion_crop(n, ndrops=3, seed=4)
    small = lbm.Simulation(n, n, params, rn0, storage="f32", device=DEV)
    big = lbm.Simulation(N, N, params, np.tile(rn0, (reps, reps)), storage="f32", device=DEV)
    small.step(3)
    big.step(3)
    Ss, Sb = small.live_pops(), big.live_pops()
    assert torch.equal(Sb, Ss.repeat(1, 1, reps, reps))
    g = torch.Generator(device=DEV).manual_seed(11)
    lam_s = small.pops_like()
    lam_s.copy_(1e-3 * torch.randn((2, 9, n, n), generator=g, device=DEV))
    lam_b = big.pops_like()
    lam_b.copy_(lam_s.repeat(1, 1, reps, reps))
    out_s, out_b = small.pops_like(), big.pops_like()
    ds_s = torch.zeros(1, dtype=torch.float64, device=DEV)
    ds_b = torch.zeros(1, dtype=torch.float64, device=DEV)
    df_s = torch.zeros((2, n, n), dtype=torch.float32, device=DEV)
    df_b = torch.zeros((2, N, N), dtype=torch.float32, device=DEV)
    print("adjoint 512^2 and tiled 10240^2, FP32", flush=True)
    small.adjoint_step(Ss, lam_s, out_s, ds_s, df_s)
    big.adjoint_step(Sb, lam_b, out_b, ds_b, df_b)
    torch.cuda.synchronize()
    assert torch.equal(out_b, out_s.repeat(1, 1, reps, reps))
    assert torch.equal(df_b, df_s.repeat(1, reps, reps))
    a, b = float(ds_b), reps * reps * float(ds_s)
    print("dL/dsigma 10240^2 %.12e, 400 x 512^2 %.12e" % (a, b))
    assert abs(a - b) <= 1e-9 * abs(b)
    small.close()
    big.close()

"""Solid sites anywhere (lbm_set_solid) on the GPU against the oracle.

* an all-fluid mask reproduces the fused step kernel bit for bit (same
  arithmetic, same stencil sums) over 20 steps, FP64 and FP32;
* set_solid keeps the pre-collision populations of every fluid site (the
  rest state of the oracle with the same mask) and zeroes solid sites;
* one step from random non-equilibrium states inside a staircase circle with
  scattered obstacles, every stencil profile, with a force field: FP64 to
  1e-13 of the largest population, FP32 to 2e-6;
* a drop beside obstacles in a circular container for 300 steps: FP64 fields
  to 1e-11, masses conserved;
* the fused step kernel's mask variant against the four passes, bit for bit;
* the benchmark's masked workload at full size (4096^2, FP32): sampled sites
  against the oracle on windows (measured 1.3e-7), the whole lattice against
  the four passes;
* argument errors of the entry point.
"""
import numpy as np
import pytest
import torch

from oracle import chromo as O
from paper_2005_04642_amd import lbm, workloads as Wk

from gpu_helpers import oracle_params, pull_gather_masked, push_scatter_masked, rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def container(nx, ny, seed, radius=None, nobst=6):
    """Circular wall plus a few scattered solid sites inside it."""
    r = radius if radius is not None else 0.5 * min(nx, ny) - 1.5
    m = Wk.circular_wall(nx, ny, r)
    m |= Wk.random_solid_sites(nx, ny, nobst, seed)
    return m


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_all_fluid_mask_reproduces_fused_step(storage):
    nx, ny = 70, 52
    params = Wk.base_params(Lambda=10.0, sigma=0.02)
    params.update(gx=2e-5, nu_B=0.4)
    rng = np.random.default_rng(4)
    rn = np.clip(np.tanh(2.0 * rng.standard_normal((ny, nx))), -1, 1)
    a = lbm.Simulation(nx, ny, params, rn, storage=storage, device=DEV)
    b = lbm.Simulation(nx, ny, params, rn, storage=storage, device=DEV, solid=np.zeros((ny, nx), bool))
    a.step(20)
    b.step(20)
    pa, pb = host(a.live_pops()), host(b.live_pops())
    fa, fb = a.fields(), b.fields()
    assert np.array_equal(pa, pb), float(np.max(np.abs(pa - pb)))
    for k in ("rho", "ux", "uy", "rhoN"):
        assert torch.equal(fa[k], fb[k]), k
    a.close()
    b.close()


def test_set_solid_keeps_fluid_state_and_clears_solid():
    nx, ny = 40, 36
    solid = container(nx, ny, 1)
    params = Wk.base_params(Lambda=10.0)
    rn = Wk.static_drop(nx, ny, 7.0)
    sim = lbm.Simulation(nx, ny, params, rn, storage="f64", device=DEV, solid=solid)
    S = host(sim.live_pops())
    assert np.all(S[:, :, solid] == 0.0)
    o = O.Oracle(oracle_params(nx, ny, dict(params, solid=solid))).init(rn)
    ref = np.stack([o.R.numpy(), o.B.numpy()])
    got = pull_gather_masked(S, solid)
    assert np.max(np.abs(got - ref)) < 1e-15
    sim.close()


STENCILS = [(3, 3, 3, 3), (1, 1, 1, 1), (3, 1, 3, 1), (1, 3, 1, 3)]


@pytest.mark.parametrize("stencil", STENCILS)
@pytest.mark.parametrize("storage,tol", [("f64", 1e-13), ("f32", 2e-6)])
@pytest.mark.parametrize("shape", [(40, 36), (97, 61)])
def test_one_step_random_state_with_mask(stencil, storage, tol, shape):
    nx, ny = shape
    solid = container(nx, ny, 2, nobst=12)
    params = Wk.base_params(Lambda=10.0, sigma=0.02, stencil=stencil)
    params.update(gx=3e-5, gy=-2e-5, nu_B=0.4)
    rng = np.random.default_rng(7)
    rn = np.clip(np.tanh(2.0 * rng.standard_normal((ny, nx))), -1, 1)
    force = Wk.gaussian_bumps(nx, ny, nbumps=3, width=6.0, amplitude=1e-4, seed=5)
    sim = lbm.Simulation(nx, ny, params, rn, storage=storage, device=DEV, force=force, solid=solid)
    # a random non-equilibrium state, handed over in the pull layout
    o0 = O.Oracle(oracle_params(nx, ny, dict(params, solid=solid))).init(rn)
    P = np.stack([o0.R.numpy(), o0.B.numpy()]) * Wk.random_state_perturbation((2, 9, ny, nx), 0.05, 3)
    P[:, :, solid] = 0.0
    if storage == "f32":
        P = P.astype(np.float32).astype(np.float64)
    sim.live_pops().copy_(torch.from_numpy(push_scatter_masked(P, solid)))
    o = O.Oracle(oracle_params(nx, ny, dict(params, solid=solid)), force=force)
    o.set_state(torch.from_numpy(P[0]), torch.from_numpy(P[1]))
    R, B = o.post_collision()
    ref = np.stack([R.numpy(), B.numpy()])
    sim.step(1)
    got = host(sim.live_pops()).astype(np.float64)
    fl = ~solid
    err = np.max(np.abs(got[:, :, fl] - ref[:, :, fl])) / np.max(np.abs(ref[:, :, fl]))
    print("mask one step %s %s %s: %.3e" % (shape, storage, stencil, err))
    assert err < tol, err
    assert np.all(got[:, :, solid] == 0.0)
    sim.close()


def test_drop_in_container_300_steps_f64():
    n = 64
    solid = Wk.circular_wall(n, n, 30.0)
    for x, y in ((50, 20), (51, 20), (14, 44), (40, 48), (32, 10)):
        solid[y, x] = True
    yy, xx = np.mgrid[0:n, 0:n]
    rn = np.tanh((11.0 - np.hypot(xx - 29.0, yy - 33.5)) / 2.0)
    params = Wk.base_params(Lambda=10.0, sigma=0.005)
    params.update(gx=1e-5)
    sim = lbm.Simulation(n, n, params, rn, storage="f64", device=DEV, solid=solid)
    m0 = sim.masses()
    sim.step(300)
    f = {k: host(v) for k, v in sim.fields().items()}
    m = sim.masses()
    sim.close()
    o = O.Oracle(oracle_params(n, n, dict(params, solid=solid))).init(rn).step(300)
    fo = {k: v.numpy() for k, v in o.fields().items()}
    fl = ~solid
    assert np.all(np.isnan(f["rho"][solid])) and np.all(np.isfinite(f["rho"][fl]))
    e_rho = rel_err(f["rho"][fl], fo["rho"][fl])
    umax = np.max(np.hypot(fo["ux"][fl], fo["uy"][fl]))
    e_u = np.max(np.hypot(f["ux"][fl] - fo["ux"][fl], f["uy"][fl] - fo["uy"][fl])) / umax
    print("drop in container, 300 steps FP64: e_rho %.2e e_u %.2e (max|u| %.2e)" % (e_rho, e_u, umax))
    assert e_rho < 1e-11 and e_u < 1e-11
    assert abs(m[0] - m0[0]) / m0[0] < 1e-13 and abs(m[1] - m0[1]) / m0[1] < 1e-13


def test_set_solid_argument_errors():
    nx, ny = 32, 24
    params = Wk.base_params(Lambda=10.0)
    rn = Wk.static_drop(nx, ny, 5.0)
    solid = Wk.circular_wall(nx, ny, 11.0)
    sim = lbm.Simulation(nx, ny, params, rn, storage="f32", device=DEV, solid=solid)
    with pytest.raises(lbm.LbmError) as e:
        sim.set_solid(solid)            # one mask per handle
    assert e.value.code == lbm.LBM_EINVAL
    sim.close()
    pw = dict(params, walls=True)
    sw = lbm.Simulation(nx, ny, pw, rn, storage="f32", device=DEV)
    m = torch.zeros((ny, nx), dtype=torch.uint8, device=DEV)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device=DEV)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_set_solid(sw.h, m.data_ptr(), ws.data_ptr(), ws.numel(), sw.stream())
    assert e.value.code == lbm.LBM_EINVAL
    sw.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("stencil", [(3, 3, 3, 3), (3, 1, 3, 1), (1, 1, 1, 1)])
@pytest.mark.parametrize("shape", [(97, 61), (300, 90)])
def test_fused_masked_step_equals_four_passes(storage, stencil, shape):
    """The fused step kernel's mask variant and the four-pass kernels give the
    same populations bit for bit (30 steps, obstacles in and across strips,
    force field)."""
    nx, ny = shape
    solid = container(nx, ny, 3, nobst=25)
    params = Wk.base_params(Lambda=10.0, sigma=0.01, stencil=stencil)
    params.update(gx=3e-5, gy=-2e-5, nu_B=0.4)
    # smooth drops (a noise field blows up within ten steps beside obstacles,
    # in the oracle as well)
    rng = np.random.default_rng(9)
    yy, xx = np.mgrid[0:ny, 0:nx]
    rn = -np.ones((ny, nx))
    for _ in range(4):
        cx, cy, r = rng.uniform(0.3 * nx, 0.7 * nx), rng.uniform(0.3 * ny, 0.7 * ny), rng.uniform(5, 9)
        rn = np.maximum(rn, np.tanh((r - np.hypot(xx - cx, yy - cy)) / 2.0))
    force = Wk.gaussian_bumps(nx, ny, nbumps=3, width=6.0, amplitude=1e-5, seed=5)
    out = []
    for flags in (0, lbm.LBM_FLAG_MASK_PASSES):
        sim = lbm.Simulation(nx, ny, params, rn, storage=storage, device=DEV, force=force, solid=solid,
                             flags=flags)
        sim.step(30)
        out.append(host(sim.live_pops()))
        m = sim.masses()
        sim.close()
        assert all(np.isfinite(m))
    d = float(np.max(np.abs(out[0] - out[1])))
    print("fused vs four passes %s %s %s: max |diff| %.3e" % (shape, storage, stencil, d))
    assert np.array_equal(out[0], out[1]), d


def test_full_size_masked_emulsion_sampled_sites():
    """The benchmark lattice inside a circular wall (the bench's masked leg):
    4096^2 emulsion, FP32, solid outside r = 2046.  After 20 steps, one step of
    the fused mask variant at sampled sites (beside the wall, on drop
    interfaces, anywhere) against the oracle on windows of the state, and the
    whole lattice against the four-pass kernels, bit for bit."""
    cfg = Wk.config_emulsion()
    n = cfg["nx"]
    params = cfg["params"]
    solid = Wk.circular_wall(n, n, n / 2.0 - 2.0)
    sims = [lbm.Simulation(n, n, params, cfg["rhoN0"], storage="f32", device=DEV, solid=solid, flags=f)
            for f in (0, lbm.LBM_FLAG_MASK_PASSES)]
    for sim in sims:
        sim.step(20)
    before = sims[0].live_pops().clone()
    for sim in sims:
        sim.step(1)
    after = sims[0].live_pops()
    assert torch.equal(after, sims[1].live_pops())
    rng = np.random.default_rng(321)
    fl = ~solid
    yy, xx = np.mgrid[0:n, 0:n]
    r = np.hypot(xx - (n - 1) / 2.0, yy - (n - 1) / 2.0)
    near_wall = np.argwhere(fl & (r > n / 2.0 - 6.0))
    rn = cfg["rhoN0"]
    edge = np.argwhere(fl & (np.abs(np.roll(rn, 1, 0) - rn) + np.abs(np.roll(rn, 1, 1) - rn) > 0))
    anywhere = np.argwhere(fl)
    picks = [tuple(near_wall[k]) for k in rng.choice(len(near_wall), 8, replace=False)]
    picks += [tuple(edge[k]) for k in rng.choice(len(edge), 6, replace=False)]
    picks += [tuple(anywhere[k]) for k in rng.choice(len(anywhere), 4, replace=False)]
    half = 16
    worst = 0.0
    m_dev = torch.as_tensor(solid, device=DEV)
    for (y, x) in picks:
        ys = torch.arange(y - half, y + half + 1, device=DEV) % n
        xs = torch.arange(x - half, x + half + 1, device=DEV) % n
        S = before[:, :, ys][:, :, :, xs].double().cpu().numpy()
        msk = m_dev[ys][:, xs].cpu().numpy()
        w = 2 * half + 1
        o = O.Oracle(oracle_params(w, w, dict(params, solid=msk)))
        P = pull_gather_masked(S, msk)
        o.set_state(torch.from_numpy(P[0]), torch.from_numpy(P[1]))
        R, B = o.post_collision()
        ref = np.stack([R.numpy(), B.numpy()])[:, :, half, half]
        got = after[:, :, y, x].double().cpu().numpy()
        worst = max(worst, float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))
    print("masked emulsion 4096^2 sampled sites: max rel err %.3e" % worst)
    assert worst < 2e-5
    for sim in sims:
        sim.close()


@pytest.mark.parametrize("stencil", [(3, 3, 3, 3), (1, 3, 1, 3)])
def test_one_step_options_with_mask_f64(stencil):
    """Fixed curvature, literal ghost equilibrium and no recolour on a masked
    lattice (the fused mask variant for 3333, the four passes for 1313)."""
    nx, ny = 44, 38
    solid = container(nx, ny, 6, nobst=10)
    rng = np.random.default_rng(12)
    rn = np.clip(np.tanh(2.0 * rng.standard_normal((ny, nx))), -1, 1)
    for extra in (dict(fixed_K=0.05), dict(ghost_eq=1), dict(recolor=False)):
        params = Wk.base_params(Lambda=4.0, sigma=0.02, stencil=stencil)
        params.update(**extra)
        sim = lbm.Simulation(nx, ny, params, rn, storage="f64", device=DEV, solid=solid)
        o0 = O.Oracle(oracle_params(nx, ny, dict(params, solid=solid))).init(rn)
        P = np.stack([o0.R.numpy(), o0.B.numpy()]) * Wk.random_state_perturbation((2, 9, ny, nx), 0.05, 7)
        P[:, :, solid] = 0.0
        sim.live_pops().copy_(torch.from_numpy(push_scatter_masked(P, solid)))
        o = O.Oracle(oracle_params(nx, ny, dict(params, solid=solid)))
        o.set_state(torch.from_numpy(P[0]), torch.from_numpy(P[1]))
        R, B = o.post_collision()
        ref = np.stack([R.numpy(), B.numpy()])
        sim.step(1)
        got = host(sim.live_pops())
        fl = ~solid
        err = np.max(np.abs(got[:, :, fl] - ref[:, :, fl])) / np.max(np.abs(ref[:, :, fl]))
        assert err < 1e-13, (extra, err)
        sim.close()


def test_drop_in_container_1000_steps_f32():
    """FP32 storage and arithmetic, 1000 steps of the container drop against the
    FP64 oracle: rho within 1e-5 relative; u, a micro-current of ~3e-5 here
    (ten times smaller than the open static drop's, so one FP32 ulp of a
    population is a larger part of it), within FP32_FLOOR_FACTOR times the
    storage floor (the FP64 oracle with its state rounded to FP32 every
    step)."""
    from gpu_helpers import FP32_FLOOR_FACTOR, FP32_TOL_RHO, field_errors, oracle_runs
    n = 64
    solid = Wk.circular_wall(n, n, 30.0)
    for x, y in ((50, 20), (51, 20), (14, 44), (40, 48), (32, 10)):
        solid[y, x] = True
    yy, xx = np.mgrid[0:n, 0:n]
    rn = np.tanh((11.0 - np.hypot(xx - 29.0, yy - 33.5)) / 2.0)
    params = Wk.base_params(Lambda=10.0, sigma=0.005)
    sim = lbm.Simulation(n, n, params, rn, storage="f32", device=DEV, solid=solid)
    sim.step(1000)
    f = {k: host(v).astype(np.float64) for k, v in sim.fields().items()}
    sim.close()
    fo, fr = oracle_runs(n, n, dict(params, solid=solid), rn, 1000)
    e_rho, e_u = field_errors(f, fo)
    floor = field_errors(fr, fo)
    umax = np.nanmax(np.hypot(fo["ux"], fo["uy"]))
    print("drop in container, 1000 steps FP32: e_rho %.2e e_u %.2e (max|u| %.2e; fp32 storage floor %.2e %.2e)"
          % (e_rho, e_u, umax, *floor))
    assert e_rho < FP32_TOL_RHO and e_u < FP32_FLOOR_FACTOR * floor[1]

"""Batched launch (lbm_batch_*): every lattice of a batch evolves exactly as it
does alone under lbm_step, before and after the autotuner picks a tile shape,
and the autotuner leaves the state unchanged."""
import numpy as np
import pytest
import torch

from paper_2005_04642_amd import lbm, workloads as Wk

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def lattices(walls=False, stencil=(3, 3, 3, 3)):
    rng = np.random.default_rng(0)
    out = []
    for (nx, ny, Lam, sigma) in [(5, 7, 10.0, 0.005), (64, 64, 1.0, 0.001), (100, 60, 100.0, 0.01),
                                 (130, 40, 10.0, 0.01), (200, 200, 10.0, 0.005), (37, 300, 2.0, 0.02)]:
        prm = Wk.base_params(Lambda=Lam, sigma=sigma, stencil=stencil)
        prm["walls"] = walls
        y, x = np.mgrid[0:ny, 0:nx]
        d = np.hypot((x - (nx - 1) / 2.0) / 1.15, (y - (ny - 1) / 2.0) * 1.15)
        rn = 0.3 * np.tanh(rng.standard_normal((ny, nx))) if nx < 10 else np.tanh((min(nx, ny) / 4.0 - d) / 2.0)
        out.append((nx, ny, prm, rn))
    return out


def singles(lats, storage, steps):
    res = []
    for nx, ny, prm, rn in lats:
        s = lbm.Simulation(nx, ny, prm, rn, storage=storage, device=DEV)
        s.step(steps)
        torch.cuda.synchronize()
        raw = s.pops[lbm.lbm_current_pops(s.h)].cpu().numpy().copy()  # memory order
        res.append((raw, s.masses(), s.live_words().cpu().numpy().copy()))
        s.close()
    return res


@pytest.mark.parametrize("storage", ["f32", "f64", "f16"])
def test_batch_matches_single_lattices(storage):
    lats = lattices()
    b = lbm.Batch(lats, storage=storage, device=DEV)
    info = b.plan_info()
    assert info["items"] >= len(lats)
    b.step(12)
    ref = singles(lats, storage, 12)
    live = lambda k: b.pops[b.lib.lbm_batch_current_pops(b.h)]
    for k, (nx, ny, _, _) in enumerate(lats):
        words = lbm.WORDS_PER_SITE[storage] * nx * ny
        esz = 8 if storage == "f64" else 4
        got = live(k)[b.offsets[k]:b.offsets[k] + words * esz].cpu().numpy()
        want = ref[k][0].reshape(-1).view(np.uint8)
        assert np.array_equal(got, want), k
        m = b.masses(k)
        assert m == ref[k][1], k
    b.close()


def test_autotune_keeps_state_and_results():
    lats = lattices()
    b = lbm.Batch(lats, storage="f32", device=DEV)
    b.step(3)
    torch.cuda.synchronize()
    before = b.pops[b.lib.lbm_batch_current_pops(b.h)].clone()
    chosen = b.autotune(steps_per_trial=2)
    assert chosen[0] in (128, 192)
    torch.cuda.synchronize()
    after = b.pops[b.lib.lbm_batch_current_pops(b.h)]
    assert torch.equal(before, after) and b.steps == 3
    b.step(9)
    ref = singles(lats, "f32", 12)
    for k in range(len(lats)):
        got = b.state(k).cpu().numpy()
        assert np.array_equal(got, ref[k][2].reshape(got.shape)), k
    f = b.fields(2)
    assert torch.isfinite(f["rho"]).all()
    b.close()


def test_batch_of_the_benchmark_workload_runs():
    """The benchmark's batch (256 drops of side 64..512) in the launch
    configuration the benchmark times (3 steps, autotune, more steps): every
    lattice finite, and sampled lattices of each size bit for bit as alone."""
    lats = Wk.config_batch(nsim=256, seed=1)
    b = lbm.Batch(lats, storage="f32", device=DEV)
    b.step(3)
    b.autotune(2)
    b.step(17)
    for k in range(len(lats)):
        m = b.masses(k)
        assert np.isfinite(m).all()
    picks = {}
    for k, (nx, ny, _, _) in enumerate(lats):
        picks.setdefault(nx, k)
    for k in sorted(picks.values()):
        nx, ny, prm, rn = lats[k]
        s = lbm.Simulation(nx, ny, prm, rn, storage="f32", device=DEV)
        s.step(20)
        torch.cuda.synchronize()
        assert torch.equal(b.state(k), s.live_pops()), (k, nx)
        s.close()
    b.close()


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_batch_with_force_fields_matches_single_lattices(storage):
    """Per-lattice force fields (lbm_batch_set_force) on some lattices of the
    batch, set before and changed after the autotuner: each lattice evolves as
    a single Simulation with the same force, bit for bit."""
    lats = lattices()
    forces = {k: Wk.gaussian_bumps(nx, ny, nbumps=2, width=max(3.0, min(nx, ny) / 6.0), amplitude=2e-5, seed=k)
              for k, (nx, ny, _, _) in enumerate(lats) if k in (1, 2, 4)}
    b = lbm.Batch(lats, storage=storage, device=DEV)
    for k, f in forces.items():
        b.set_force(k, f)
    b.step(6)
    b.autotune(steps_per_trial=2)
    b.set_force(2, None)            # lattice 2 runs on without its force
    b.step(6)
    for k, (nx, ny, prm, rn) in enumerate(lats):
        s = lbm.Simulation(nx, ny, prm, rn, storage=storage, device=DEV, force=forces.get(k))
        s.step(6)
        if k == 2:
            # continue without the force from the same state
            state = s.live_pops().clone()
            s.close()
            s = lbm.Simulation(nx, ny, prm, rn, storage=storage, device=DEV)
            s.live_pops().copy_(state)
        s.step(6)
        torch.cuda.synchronize()
        assert torch.equal(b.state(k), s.live_pops()), k
        s.close()
    b.close()


@pytest.mark.parametrize("storage", ["f32", "f64", "f16"])
@pytest.mark.parametrize("stencil", [(3, 3, 3, 3), (3, 1, 3, 1)])
def test_batch_of_walled_lattices_matches_single_lattices(storage, stencil):
    """A batch of walled lattices (rows 0 and ny-1 solid), with a force field
    on one of them: each evolves as it does alone, bit for bit, before and
    after the autotuner."""
    lats = lattices(walls=True, stencil=stencil)
    b = lbm.Batch(lats, storage=storage, device=DEV)
    nx3, ny3 = lats[3][0], lats[3][1]
    f3 = Wk.gaussian_bumps(nx3, ny3, nbumps=2, width=6.0, amplitude=2e-5, seed=3)
    b.set_force(3, f3)
    b.step(6)
    chosen = b.autotune(steps_per_trial=2)
    if storage != "f64":      # 192-wide walled batch kernels spill registers: 128 only
        assert chosen[0] == 128 and b.plan_info()["ntx"] == 128
    b.step(6)
    for k, (nx, ny, prm, rn) in enumerate(lats):
        s = lbm.Simulation(nx, ny, prm, rn, storage=storage, device=DEV, force=f3 if k == 3 else None)
        s.step(12)
        torch.cuda.synchronize()
        got = b.pops[b.lib.lbm_batch_current_pops(b.h)]
        words = lbm.WORDS_PER_SITE[storage] * nx * ny
        esz = 8 if storage == "f64" else 4
        raw = s.pops[lbm.lbm_current_pops(s.h)].cpu().numpy().reshape(-1).view(np.uint8)
        assert np.array_equal(got[b.offsets[k]:b.offsets[k] + words * esz].cpu().numpy(), raw), k
        m = b.masses(k)
        assert m == s.masses(), k
        s.close()
    b.close()


@pytest.mark.parametrize("storage", ["f32", "f64", "f16"])
@pytest.mark.parametrize("stencil", [(3, 3, 3, 3), (3, 1, 3, 1)])
def test_batch_with_masks_matches_single_lattices(storage, stencil):
    """Solid-site masks on two lattices of a periodic batch (one also forced):
    every lattice evolves as alone, bit for bit, before and after the
    autotuner; fields read NaN at the solid sites."""
    lats = lattices(stencil=stencil)
    masks = {4: Wk.circular_wall(200, 200, 97.0) | Wk.random_solid_sites(200, 200, 30, 4),
             2: Wk.random_solid_sites(100, 60, 25, 2)}
    f2 = Wk.gaussian_bumps(100, 60, nbumps=2, width=6.0, amplitude=2e-5, seed=2)
    b = lbm.Batch(lats, storage=storage, device=DEV)
    for k, m in masks.items():
        b.set_solid(k, m)
    if storage != "f64":      # a masked batch is re-planned at 128-wide strips (192 spills registers)
        assert b.plan_info()["ntx"] == 128
    b.set_force(2, f2)
    b.step(6)
    chosen = b.autotune(steps_per_trial=2)
    if storage != "f64":
        assert chosen[0] == 128
    b.step(6)
    for k, (nx, ny, prm, rn) in enumerate(lats):
        s = lbm.Simulation(nx, ny, prm, rn, storage=storage, device=DEV, force=f2 if k == 2 else None,
                           solid=masks.get(k))
        s.step(12)
        torch.cuda.synchronize()
        got = b.pops[b.lib.lbm_batch_current_pops(b.h)]
        words = lbm.WORDS_PER_SITE[storage] * nx * ny
        esz = 8 if storage == "f64" else 4
        raw = s.pops[lbm.lbm_current_pops(s.h)].cpu().numpy().reshape(-1).view(np.uint8)
        assert np.array_equal(got[b.offsets[k]:b.offsets[k] + words * esz].cpu().numpy(), raw), k
        assert b.masses(k) == s.masses(), k
        s.close()
    rho = b.fields(4)["rho"].cpu().numpy()
    assert np.all(np.isnan(rho[masks[4]])) and np.all(np.isfinite(rho[~masks[4]]))
    b.close()


# ---------------------------------------------------------------------------
# every member of a batch against the oracle (FP64 and FP32): density ratios
# 1, 10 and 100 on lattices of sides 64 and 128, and one ragged lattice whose
# 203 columns split into two uneven strips
# ---------------------------------------------------------------------------

ORACLE_STEPS = 200


def ellipse(nx, ny, aspect, width=2.0):
    """Centred axis-aligned elliptic drop, tanh(d / width) of its approximate
    signed distance, semi-axes (min(nx, ny)/4) sqrt(AR) and .../sqrt(AR)."""
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    r0 = min(nx, ny) / 4.0
    a, b = r0 * np.sqrt(aspect), r0 / np.sqrt(aspect)
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    q = np.sqrt(((x - cx) / a) ** 2 + ((y - cy) / b) ** 2)
    return np.tanh((1.0 - q) * np.sqrt(a * b) / width)


def oracle_lattices():
    out = []
    for (nx, ny, Lam, sigma, ar) in [(64, 64, 1.0, 0.02, 1.3), (64, 64, 10.0, 0.005, 1.1),
                                     (64, 64, 100.0, 0.01, 1.45), (128, 128, 1.0, 0.001, 1.2),
                                     (128, 128, 10.0, 0.05, 1.5), (128, 128, 100.0, 0.003, 1.0),
                                     (203, 77, 10.0, 0.01, 1.4)]:
        out.append((nx, ny, Wk.base_params(Lambda=Lam, sigma=sigma), ellipse(nx, ny, ar)))
    return out


@pytest.fixture(scope="module")
def batch_oracle():
    from gpu_helpers import oracle_runs
    lats = oracle_lattices()
    return lats, [oracle_runs(nx, ny, prm, rn, ORACLE_STEPS) for nx, ny, prm, rn in lats]


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_batch_members_against_oracle(storage, batch_oracle):
    """After 200 steps of one batch, each member's fields against the FP64
    oracle run on that lattice alone: FP64 within 1e-11 (u: of max |u|, or 1e-14
    absolute); FP32 rho within 1e-5 and u within FP32_FLOOR_FACTOR times the
    member's FP32 storage floor."""
    from gpu_helpers import field_errors
    from gpu_helpers import FP32_TOL_RHO, FP32_FLOOR_FACTOR
    lats, runs = batch_oracle
    b = lbm.Batch(lats, storage=storage, device=DEV)
    b.step(ORACLE_STEPS)
    for k, ((nx, ny, prm, _), (fo, fr)) in enumerate(zip(lats, runs)):
        f = {key: v.detach().cpu().numpy() for key, v in b.fields(k).items()}
        e_rho, e_u = field_errors(f, fo)
        floor = field_errors(fr, fo)
        umax = float(np.max(np.hypot(fo["ux"], fo["uy"])))
        print("batch member %d (%dx%d, Lambda %g, sigma %g) %s: e_rho %.3e e_u %.3e (fp32 storage floor %.3e %.3e; "
              "max|u| %.3e)" % (k, nx, ny, prm["rho0_R"] / prm["rho0_B"], prm["sigma"], storage, e_rho, e_u,
                                floor[0], floor[1], umax))
        if storage == "f64":
            # u relative to max |u|, or absolute: a drop with sigma = 0.001 has a
            # micro-current of 5e-5, carried by populations of order one whose
            # FP64 ulp is 2e-16, so 1e-11 of it is a few ulps (measured 7e-16)
            assert e_rho < 1e-11 and (e_u < 1e-11 or e_u * umax < 1e-14), k
        else:
            assert e_rho < FP32_TOL_RHO, k
            assert e_u < FP32_FLOOR_FACTOR * floor[1], (k, e_u, floor[1])
    b.close()

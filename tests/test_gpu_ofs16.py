"""Parity of the 16-bit offset storage formats (LBM_STORAGE_F16_OFS and
LBM_STORAGE_BF16_OFS, FP32 arithmetic) with the FP64 oracle, through the C ABI.

* streaming and boundary indexing of the packed words: bit-exact;
* initial state and one step from random states: every population within the
  format's rounding of the oracle's value plus FP32 arithmetic;
* static drop (1000 steps) and layered channel: errors against the FP64 oracle
  below the stated tolerances, which sit above the format's own rounding floor
  (test_ofs16_floor.py); the layered-channel workload at density ratio 100
  (1000 steps) against a floor computed in the test;
* full-size 4096^2 emulsion: sampled sites of a step, recomputed by the oracle;
* masses and NaN reporting with packed words.
"""
import numpy as np
import pytest
import torch

import ofs16
from oracle import chromo as O
from paper_2005_04642_amd import lbm, workloads as Wk
from test_ofs16_floor import CHANNEL_TOL, OFS16_TOL, channel_case, round_through_format

from gpu_helpers import FP32_FLOOR_FACTOR, field_errors, fluid, oracle_params, oracle_post_collision, pull_gather

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
FMTS = ["f16", "bf16"]
# FP32 arithmetic of one step relative to the largest population (the FP32
# path meets 2e-5 on the full-size emulsion; the one-step states here are
# gentler)
ARITH = 2e-6


def sim_for(nx, ny, params, rn, storage, **kw):
    return lbm.Simulation(nx, ny, params, rn, storage=storage, device=DEV, **kw)


def host_words(sim):
    torch.cuda.synchronize()
    return sim.live_words().cpu().numpy().view(np.uint32)


def upload_words(sim, W):
    sim.live_words().copy_(torch.from_numpy(np.ascontiguousarray(W).view(np.int32)).to(DEV))


def perturbed_rest_state(nx, ny, params, seed, scale=0.05):
    """Pull-layout populations [2, 9, ny, nx] as float32: the initial state of a
    white-noise colour field written by the FP32 path's lbm_init, each
    population scaled by (1 + scale U[-1, 1]) (the FP32 one-step test's recipe)."""
    rng = np.random.default_rng(seed)
    rn = np.clip(np.tanh(2.0 * rng.standard_normal((ny, nx))), -1, 1)
    sim = sim_for(nx, ny, params, rn, "f32")
    torch.cuda.synchronize()
    S = sim.live_pops().cpu().numpy().astype(np.float64)
    sim.close()
    return (S * Wk.random_state_perturbation(S.shape, scale, seed + 1)).astype(np.float32)


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("shape", [(4, 4), (5, 7), (300, 9), (64, 64)])
def test_ofs16_stream_only_bit_exact(fmt, walls, shape):
    nx, ny = shape
    params = Wk.base_params()
    params["walls"] = walls
    sim = sim_for(nx, ny, params, -np.ones((ny, nx)), fmt, flags=lbm.LBM_FLAG_STREAM_ONLY)
    rng = np.random.default_rng(nx * 131 + ny)
    W = rng.integers(0, 2 ** 32, size=(10, ny, nx), dtype=np.uint64).astype(np.uint32)
    upload_words(sim, W)
    for _ in range(3):
        sim.step(1)
        W = ofs16.pull_words(W, walls)
        got = host_words(sim)
        assert np.array_equal(fluid(got, walls), fluid(W, walls))
    sim.close()


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("walls", [False, True])
def test_ofs16_initial_state(fmt, walls):
    nx, ny = 37, 23
    params = Wk.base_params(Lambda=10.0)
    params["walls"] = walls
    rn = np.tanh(0.4 * (np.arange(nx)[None, :] - 15.0)) * np.ones((ny, 1))
    sim = sim_for(nx, ny, params, rn, fmt)
    S = ofs16.decode_pair(host_words(sim), params, fmt)
    P = pull_gather(S, walls)
    o = O.Oracle(oracle_params(nx, ny, params)).init(rn)
    ref = np.stack([o.R.numpy(), o.B.numpy()])
    tol = ofs16.rounding_bound(ref, params, fmt) + ARITH * np.max(np.abs(ref))
    assert np.all(np.abs(P - ref) <= tol)
    sim.close()


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("stencil", [(3, 3, 3, 3), (1, 1, 1, 1)])
@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("shape", [(8, 8), (47, 29), (100, 60)])
def test_ofs16_one_step_random_state(fmt, stencil, walls, shape):
    nx, ny = shape
    params = Wk.base_params(Lambda=10.0, sigma=0.02, stencil=stencil)
    params.update(walls=walls, gx=3e-5, gy=-2e-5, nu_B=0.4)
    sim = sim_for(nx, ny, params, -np.ones((ny, nx)), fmt)
    W = ofs16.encode(*perturbed_rest_state(nx, ny, params, seed=nx + ny), params, fmt)
    upload_words(sim, W)
    S = ofs16.decode_pair(W, params, fmt)            # the state the device starts from
    ref = oracle_post_collision(S, nx, ny, params)  # FP64, fluid rows
    sim.step(1)
    got = fluid(ofs16.decode_pair(host_words(sim), params, fmt), walls)
    tol = ofs16.rounding_bound(ref, params, fmt) + ARITH * np.max(np.abs(ref))
    excess = np.abs(got - ref) / tol
    print("%s one step %s walls=%s %s: max err/tol %.3f" % (fmt, shape, walls, stencil, excess.max()))
    assert np.all(excess <= 1.0)
    sim.close()


@pytest.fixture(scope="module")
def static_drop_oracle():
    cfg = Wk.config_static_drop()
    o = O.Oracle(oracle_params(64, 64, cfg["params"])).init(cfg["rhoN0"]).step(1000)
    return {k: v.numpy() for k, v in o.fields().items()}, o.masses()


@pytest.mark.parametrize("fmt", FMTS)
def test_ofs16_static_drop_1000_steps(fmt, static_drop_oracle):
    fo, mo = static_drop_oracle
    cfg = Wk.config_static_drop()
    sim = sim_for(64, 64, cfg["params"], cfg["rhoN0"], fmt)
    sim.step(1000)
    f = {k: v.cpu().numpy().astype(np.float64) for k, v in sim.fields().items()}
    m = sim.masses()
    sim.close()
    e = dict(rho=float(np.max(np.abs(f["rho"] - fo["rho"]) / fo["rho"])),
             u=float(np.max(np.hypot(f["ux"] - fo["ux"], f["uy"] - fo["uy"])) / np.max(np.hypot(fo["ux"], fo["uy"]))),
             rhoN=float(np.max(np.abs(f["rhoN"] - fo["rhoN"]))),
             mass=max(abs(m[0] - mo[0]) / mo[0], abs(m[1] - mo[1]) / mo[1]))
    print("static drop %s: " % fmt + " ".join("e_%s %.3e" % kv for kv in e.items()))
    for k, tol in OFS16_TOL[fmt].items():
        assert e[k] < tol, (k, e[k])


@pytest.mark.parametrize("fmt", FMTS)
def test_ofs16_layered_channel(fmt):
    nx, ny, steps, params, rn = channel_case()
    sim = sim_for(nx, ny, params, rn, fmt)
    sim.step(steps)
    f = {k: fluid(v.cpu().numpy().astype(np.float64), True) for k, v in sim.fields().items()}
    sim.close()
    o = O.Oracle(oracle_params(nx, ny, params)).init(rn).step(steps)
    fo = {k: fluid(v.numpy(), True) for k, v in o.fields().items()}
    e_rho = float(np.max(np.abs(f["rho"] - fo["rho"]) / fo["rho"]))
    e_u = float(np.max(np.hypot(f["ux"] - fo["ux"], f["uy"] - fo["uy"])) / np.max(np.hypot(fo["ux"], fo["uy"])))
    print("channel %s: e_rho %.3e e_u %.3e" % (fmt, e_rho, e_u))
    assert e_rho < CHANNEL_TOL[fmt]["rho"] and e_u < CHANNEL_TOL[fmt]["u"]


@pytest.fixture(scope="module")
def channel_workload_oracle():
    """The layered-channel workload (256 x 128 between walls, Lambda = 100,
    nu_B = 10 nu_R, g = 1e-6 along x, tanh start): the FP64 oracle's fields
    after 1000 steps, and those of the same oracle with its state passed
    through each 16-bit format's words after every step (the format's rounding
    floor; the initial state is rounded as lbm_init writes it)."""
    cfg = Wk.config_layered_channel()
    nx, ny, p = cfg["nx"], cfg["ny"], cfg["params"]
    op = oracle_params(nx, ny, p)
    exact = O.Oracle(op).init(cfg["rhoN0"])
    rounded = {fmt: O.Oracle(op).init(cfg["rhoN0"]) for fmt in FMTS}
    m0 = {}
    for fmt, o in rounded.items():
        round_through_format(o, p, fmt)
        m0[fmt] = o.masses()
    for _ in range(1000):
        exact.step(1)
        for fmt, o in rounded.items():
            o.step(1)
            round_through_format(o, p, fmt)
    fo = {k: v.numpy() for k, v in exact.fields().items()}
    fr = {fmt: {k: v.numpy() for k, v in o.fields().items()} for fmt, o in rounded.items()}
    dm = {fmt: max(abs(o.masses()[c] - m0[fmt][c]) / m0[fmt][c] for c in (0, 1)) for fmt, o in rounded.items()}
    return cfg, fo, fr, dm


@pytest.mark.parametrize("fmt", FMTS)
def test_ofs16_layered_channel_workload_1000_steps(fmt, channel_workload_oracle):
    """The 16-bit formats at density ratio 100 (the moving populations of both
    pure phases rest at the same fref, so the offsets stay small in either
    phase): rho, u and the drift of the colour masses within FP32_FLOOR_FACTOR
    times what the format's rounding alone does to the oracle on this
    workload (measured: F16 e_rho 8.5e-5 / floor 3.4e-4, e_u 1.3e-2 / 1.3e-2,
    drift 5.9e-5 / 6.8e-5; BF16 3.8e-3 / 8.5e-4, 0.157 / 0.160, 1.6e-4 /
    2.4e-4: at g = 1e-6 the flow is slow against the populations' rounding)."""
    cfg, fo, fr, dm_floor = channel_workload_oracle
    nx, ny = cfg["nx"], cfg["ny"]
    sim = sim_for(nx, ny, cfg["params"], cfg["rhoN0"], fmt)
    m0 = sim.masses()
    sim.step(1000)
    f = {k: v.cpu().numpy().astype(np.float64) for k, v in sim.fields().items()}
    m1 = sim.masses()
    sim.close()
    e_rho, e_u = field_errors(f, fo, walls=True)
    floor = field_errors(fr[fmt], fo, walls=True)
    dm = max(abs(m1[0] - m0[0]) / m0[0], abs(m1[1] - m0[1]) / m0[1])
    print("layered channel 256x128 %s, 1000 steps: e_rho %.3e e_u %.3e (format floor %.3e %.3e), mass drift %.2e "
          "(floor %.2e)" % (fmt, e_rho, e_u, floor[0], floor[1], dm, dm_floor[fmt]))
    assert e_rho < FP32_FLOOR_FACTOR * floor[0], (e_rho, floor[0])
    assert e_u < FP32_FLOOR_FACTOR * floor[1], (e_u, floor[1])
    assert dm < FP32_FLOOR_FACTOR * dm_floor[fmt], (dm, dm_floor[fmt])


def test_ofs16_full_size_emulsion_sampled_sites():
    """4096^2 emulsion in F16_OFS, the launch configuration of the benchmark:
    one step from the device state after 20 steps, at sampled interface and
    random sites, recomputed by the oracle from the decoded words of a window."""
    fmt = "f16"
    cfg = Wk.config_emulsion()
    n = cfg["nx"]
    params = cfg["params"]
    sim = sim_for(n, n, params, cfg["rhoN0"], fmt)
    sim.step(20)
    before = sim.live_words().clone()
    sim.step(1)
    after = sim.live_words()
    rng = np.random.default_rng(321)
    rn = cfg["rhoN0"]
    edge = np.argwhere(np.abs(np.roll(rn, 1, 0) - rn) + np.abs(np.roll(rn, 1, 1) - rn) > 0)
    picks = [tuple(edge[k]) for k in rng.choice(len(edge), 12, replace=False)]
    picks += [tuple(rng.integers(0, n, 2)) for _ in range(4)]
    half = 16
    worst = 0.0
    for (y, x) in picks:
        ys = torch.arange(y - half, y + half + 1, device=DEV) % n
        xs = torch.arange(x - half, x + half + 1, device=DEV) % n
        Wwin = before[:, ys][:, :, xs].cpu().numpy().view(np.uint32)
        S = ofs16.decode_pair(Wwin, params, fmt)
        ref = oracle_post_collision(S, 2 * half + 1, 2 * half + 1, params)[:, :, half, half]
        got = ofs16.decode_pair(after[:, y:y + 1, x:x + 1].cpu().numpy().view(np.uint32), params, fmt)[:, :, 0, 0]
        tol = ofs16.rounding_bound(ref[:, :, None], params, fmt)[:, :, 0] + 2e-5 * np.max(np.abs(ref))
        worst = max(worst, float(np.max(np.abs(got - ref) / tol)))
    print("emulsion 4096^2 f16 sampled sites: max err/tol %.3f" % worst)
    assert worst <= 1.0
    sim.close()


@pytest.mark.parametrize("fmt", FMTS)
def test_ofs16_masses_and_nan(fmt):
    cfg = Wk.config_static_drop()
    sim = sim_for(64, 64, cfg["params"], cfg["rhoN0"], fmt)
    sim.step(5, with_mass=True)
    torch.cuda.synchronize()
    dev = sim.mass.cpu().numpy()
    S = ofs16.decode_pair(host_words(sim), cfg["params"], fmt)
    assert abs(dev[0] - S[0].sum()) < 1e-9 * S[0].sum() and abs(dev[1] - S[1].sum()) < 1e-9 * S[1].sum()
    W = host_words(sim).copy()
    W[0, 10, 10] = np.float32(np.nan).view(np.uint32)   # rest-link red population
    upload_words(sim, W)
    sim.step(1)
    with pytest.raises(lbm.LbmError) as ei:
        sim.masses()
    assert ei.value.code == lbm.LBM_ENONFINITE
    sim.close()


@pytest.mark.parametrize("fmt", FMTS)
def test_ofs16_largest_lattice_class_streaming(fmt):
    """11264^2 in a 16-bit offset format: 5.08 GB per buffer (past the 4 GiB one
    32-bit buffer offset spans; rows are addressed through resources of their
    own); the packed words stream bit-exactly at sites in the first and last
    rows and columns."""
    from oracle.lattice import C
    n = 11264
    params = Wk.base_params(Lambda=10.0)
    sim = sim_for(n, n, params, Wk.emulsion(n, n, 12, 20.0, 80.0, 6.0, 4), fmt, flags=lbm.LBM_FLAG_STREAM_ONLY)
    sim.step(2)
    before = sim.live_words().clone()
    sim.step(1)
    after = sim.live_words()
    rng = np.random.default_rng(9)
    picks = [(0, 0), (n - 1, n - 1), (n - 1, 0), (0, n - 1)] + [tuple(rng.integers(0, n, 2)) for _ in range(3)]
    for (y, x) in picks:
        for q in range(10):
            i = 0 if q < 2 else q - 1        # word q carries link i (words 0, 1: the rest link)
            cx, cy = C[i]
            assert torch.equal(after[q, y, x], before[q, (y - cy) % n, (x - cx) % n]), (y, x, q)
    sim.close()


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("stencil", [(3, 3, 3, 3), (1, 1, 1, 1), (3, 1, 3, 1)])
@pytest.mark.parametrize("shape", [(47, 29), (100, 60)])
def test_ofs16_one_step_with_mask(fmt, stencil, shape):
    """A mask of solid sites (circular wall and scattered obstacles) with the
    16-bit formats: one step from a random state within the format's rounding
    plus the arithmetic allowance of the FP64 oracle; solid sites keep the
    encoding of zero populations."""
    from gpu_helpers import pull_gather_masked, push_scatter_masked
    nx, ny = shape
    solid = Wk.circular_wall(nx, ny, 0.5 * min(nx, ny) - 1.5) | Wk.random_solid_sites(nx, ny, 10, nx)
    params = Wk.base_params(Lambda=10.0, sigma=0.02, stencil=stencil)
    params.update(gx=3e-5, gy=-2e-5, nu_B=0.4)
    P = pull_gather(perturbed_rest_state(nx, ny, params, seed=nx + ny).astype(np.float64), False)
    P[:, :, solid] = 0.0
    W = ofs16.encode(*push_scatter_masked(P, solid).astype(np.float32), params, fmt)
    sim = sim_for(nx, ny, params, -np.ones((ny, nx)), fmt, solid=solid)
    upload_words(sim, W)
    S = pull_gather_masked(ofs16.decode_pair(W, params, fmt), solid)   # the state the device starts from
    o = O.Oracle(oracle_params(nx, ny, dict(params, solid=solid))).set_state(torch.from_numpy(S[0]),
                                                                            torch.from_numpy(S[1]))
    R, B = o.post_collision()
    ref = np.stack([R.numpy(), B.numpy()])
    sim.step(1)
    got = ofs16.decode_pair(host_words(sim), params, fmt)
    fl = ~solid
    tol = ofs16.rounding_bound(ref[:, :, fl], params, fmt) + ARITH * np.max(np.abs(ref[:, :, fl]))
    excess = np.abs(got[:, :, fl] - ref[:, :, fl]) / tol
    print("%s mask one step %s %s: max err/tol %.3f" % (fmt, shape, stencil, excess.max()))
    assert np.all(excess <= 1.0)
    assert np.all(got[:, :, solid] == 0.0)
    sim.close()


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("stencil", [(3, 3, 3, 3), (1, 1, 1, 1)])
def test_ofs16_fused_masked_step_equals_four_passes(fmt, stencil):
    nx, ny = 130, 70
    solid = Wk.circular_wall(nx, ny, 0.5 * ny - 1.5) | Wk.random_solid_sites(nx, ny, 20, 4)
    params = Wk.base_params(Lambda=10.0, sigma=0.01, stencil=stencil)
    params.update(gx=3e-5, nu_B=0.4)
    yy, xx = np.mgrid[0:ny, 0:nx]
    rn = np.maximum(np.tanh((9.0 - np.hypot(xx - 60.0, yy - 35.0)) / 2.0),
                    np.tanh((7.0 - np.hypot(xx - 75.0, yy - 30.0)) / 2.0))
    out = []
    for flags in (0, lbm.LBM_FLAG_MASK_PASSES):
        sim = sim_for(nx, ny, params, rn, fmt, solid=solid, flags=flags)
        sim.step(25)
        out.append(host_words(sim))
        m = sim.masses()
        assert all(np.isfinite(m))
        f = {k: v.cpu().numpy() for k, v in sim.fields().items()}
        assert np.all(np.isnan(f["rho"][solid])) and np.all(np.isfinite(f["rho"][~solid]))
        assert np.all(np.isfinite(f["ux"][~solid])) and np.all(np.abs(f["rhoN"][~solid]) <= 1.0)
        sim.close()
    assert np.array_equal(out[0], out[1])

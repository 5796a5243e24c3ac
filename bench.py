"""Benchmark: D2Q9 chromodynamic MRT step on the 4096x4096 emulsion (FP32).

python bench.py [--gpus 1] [--steps K] [--warmup W] [--stencil 3333]
                [--storage f32|f16|bf16] [--no-cpu]

Prints one JSON line: MLUPS of the whole step (all stages: gather, fields,
stencils, force, collision, recolour, store) with the populations resident in
HBM, the roofline of the step kernel (HBM bound: algorithmic bytes per lattice
update = read + write of one site's population words: 144 B for FP32 storage,
80 B for the 16-bit offset formats), the CPU oracle timed on a bounded
sample of the same workload, and the adjoint: one lbm_adjoint_step against one
forward step on the same lattice, the gradient of an interface-shape loss
over a checkpointed 512^2 rollout of 2000 steps (forward vs backward time),
one eighth of the lattice as a slab of rows with and without halo rows (the
share of one GPU if the lattice were split over eight), and a batch of 256
uneven lattices in one launch per step.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, 8 TB/s
BYTES_PER_LU = {"f32": 144, "f64": 288, "f16": 80, "bf16": 80}
# 18 populations of 16 bits read and written: the bytes of a pure 16-bit
# storage, against which the offset formats (which keep the two rest
# populations in FP32, 80 B per update) are also reported
BYTES_16BIT_POPS = 72
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2005_04642_amd", "csrc", f)
                  for f in ("chromo_kernels.hpp", "chromo_launch.hpp", "chromo_host.hpp", "chromo_api.hip")]


STORAGE_NAME = {"f32": "FP32", "f16": "FP16-offset (16-bit words, FP32 arithmetic)",
                "bf16": "BF16-offset (16-bit words, FP32 arithmetic)"}


def traffic_file(storage):
    return os.path.join(ROOT, "profiles", "traffic_step_emulsion4096_%s.json" % storage)


def kernel_hash():
    """Hash of the kernel sources' code: comments and blank space are dropped,
    so a counter run stays matched to the code it measured across comment
    edits."""
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        src = open(f).read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(storage):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on the current kernel source (else None)."""
    try:
        d = json.load(open(traffic_file(storage)))
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_threads():
    """Threads the oracle may use: the CPUs this process may run on, capped by
    OMP_NUM_THREADS when that is set (the host's share of a shared machine)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_baseline(warmup=1, steps=3, drop_steps=1000):
    """The oracle (torch-CPU float64, untuned) on the host: the full 4096^2
    emulsion workload for `steps` steps after `warmup` (the benchmark's own
    lattice, the value reported), and the 64^2 static drop for `drop_steps`."""
    import torch
    from oracle import chromo as O
    from paper_2005_04642_amd import workloads as Wk
    torch.set_num_threads(cpu_threads())
    threads = torch.get_num_threads()
    cfg = Wk.config_emulsion()
    n = cfg["nx"]
    o = O.Oracle(O.Params(nx=n, ny=n, **cfg["params"])).init(cfg["rhoN0"])
    o.step(warmup)
    t0 = time.time()
    o.step(steps)
    dt = time.time() - t0
    del o
    c1 = Wk.config_static_drop()
    o = O.Oracle(O.Params(nx=c1["nx"], ny=c1["ny"], **c1["params"])).init(c1["rhoN0"])
    t1 = time.time()
    o.step(drop_steps)
    dt1 = time.time() - t1
    return {"value": round(n * n * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": "%dx%d emulsion workload (50 drops, Lambda=10, sigma=0.005), %d steps after %d warm-up, "
                      "torch-CPU float64, %.1f s on %d threads" % (n, n, steps, warmup, dt, threads),
            "static_drop": {"value": round(c1["nx"] * c1["ny"] * drop_steps / dt1 / 1e6, 4), "unit": "MLUPS",
                            "sample": "%dx%d static drop, %d steps, %.1f s" % (c1["nx"], c1["ny"], drop_steps, dt1)}}


def copy_roof(n, params, rn, torch, storage, steps=200):
    """Same-bytes reference: the library's streaming-only step (gather of the
    site's words with the same pull offsets, store at the own site, no
    arithmetic) on the same lattice and storage format."""
    from paper_2005_04642_amd import lbm
    sim = lbm.Simulation(n, n, params, rn, storage=storage, device="cuda:0", flags=lbm.LBM_FLAG_STREAM_ONLY)
    sim.step(10)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    sim.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    sim.close()
    return {"kernel": "stream_only_kernel (gather + store, no arithmetic)", "ms_per_step": round(ms, 5),
            "GB_s": round(BYTES_PER_LU[storage] * n * n / (ms * 1e-3) / 1e9, 1)}


def adjoint_measure(n, params, rn, torch, steps=20, force=None):
    """Adjoint step (lbm_adjoint_step, FP32 storage, FP64 dL/dsigma) against the
    forward step on the same lattice and state."""
    from paper_2005_04642_amd import lbm
    sim = lbm.Simulation(n, n, params, rn, storage="f32", device="cuda:0", force=force)
    sim.step(20)
    S = sim.live_pops().clone()
    lam = torch.full_like(S, 1e-3)
    out = torch.empty_like(S)
    ds = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    df = torch.zeros((2, n, n), dtype=torch.float32, device="cuda:0")
    sim.adjoint_step(S, lam, out, ds, df)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        sim.adjoint_step(S, lam, out, ds, df)
    e1.record()
    torch.cuda.synchronize()
    ms_adj = e0.elapsed_time(e1) / steps
    e0.record()
    sim.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms_fwd = e0.elapsed_time(e1) / steps
    sim.close()
    return {"ms_forward": round(ms_fwd, 5), "ms_adjoint": round(ms_adj, 5),
            "MLUPS_forward": round(n * n / ms_fwd / 1e3, 1), "MLUPS_adjoint": round(n * n / ms_adj / 1e3, 1),
            "ratio": round(ms_fwd / ms_adj, 4)}


def storage16_measure(n, params, rn, torch, steps=200, warmup=20):
    """The 16-bit offset formats on the benchmark lattice: time per step, and the
    largest difference of rho (relative) and u (relative to max |u|) from the
    FP32 path after the same warmup + steps from the same initial state."""
    from paper_2005_04642_amd import lbm

    def run(storage, timed):
        sim = lbm.Simulation(n, n, params, rn, storage=storage, device="cuda:0")
        sim.step(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        sim.step(steps)
        e1.record()
        torch.cuda.synchronize()
        f = sim.fields()
        sim.close()
        return e0.elapsed_time(e1) / steps, f

    _, ref = run("f32", False)
    umax = float(torch.sqrt(ref["ux"] ** 2 + ref["uy"] ** 2).max())
    out = {"workload": "the benchmark lattice, %d + %d steps; differences from the FP32 path" % (warmup, steps)}
    for storage in ("f16", "bf16"):
        ms, f = run(storage, True)
        e_rho = float((torch.abs(f["rho"] - ref["rho"]) / ref["rho"]).max())
        e_u = float(torch.sqrt((f["ux"] - ref["ux"]) ** 2 + (f["uy"] - ref["uy"]) ** 2).max()) / umax
        gbs = BYTES_PER_LU[storage] * n * n / (ms * 1e-3) / 1e9
        gbs72 = BYTES_16BIT_POPS * n * n / (ms * 1e-3) / 1e9
        out[storage] = {"ms_per_step": round(ms, 5), "MLUPS": round(n * n / ms / 1e3, 1),
                        "GB_s": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                        "frac_of_hbm_peak_at_72B": round(gbs72 / HBM_PEAK_GBS, 4),
                        "max_rel_drho_vs_f32": float("%.3g" % e_rho), "max_du_over_umax_vs_f32": float("%.3g" % e_u)}
    return out


def solid_measure(n, params, rn, torch, ms_fused, steps=100, warmup=10):
    """Step with a solid-site mask (the fused kernel's mask variant; the four
    pass kernels timed beside it): the benchmark lattice inside a circular
    container wall of radius n/2 - 2 (FP32), and the curved-interface
    transient's 724^2 container at Lambda = 5 (FP64)."""
    import numpy as np
    from paper_2005_04642_amd import lbm, workloads as Wk

    def timed(sim, k):
        sim.step(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        sim.step(k)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    solid = Wk.circular_wall(n, n, n / 2.0 - 2.0)
    sim = lbm.Simulation(n, n, params, rn, storage="f32", device="cuda:0", solid=solid)
    ms = timed(sim, steps)
    sim.close()
    sim = lbm.Simulation(n, n, params, rn, storage="f32", device="cuda:0", solid=solid,
                         flags=lbm.LBM_FLAG_MASK_PASSES)
    ms4 = timed(sim, max(10, steps // 5))
    sim.close()
    fluid = int((~solid).sum())
    out = {"workload": "%dx%d emulsion inside a circular wall of radius %g (%.1f %% of sites solid), FP32, "
                       "%d steps" % (n, n, n / 2.0 - 2.0, 100.0 * (1 - fluid / (n * n)), steps),
           "ms_per_step": round(ms, 5), "MLUPS_all_sites": round(n * n / ms / 1e3, 1),
           "MLUPS_fluid_sites": round(fluid / ms / 1e3, 1),
           "vs_fused_step_without_mask": round(ms_fused / ms, 4),
           "four_pass_kernels_ms_per_step": round(ms4, 5)}
    nx, ny, p, rn2, _, _, solid2, _ = Wk.config_curved_transient(5.0)
    sim = lbm.Simulation(nx, ny, p, rn2, storage="f64", device="cuda:0", solid=solid2)
    ms2 = timed(sim, 200)
    sim.close()
    out["curved_transient"] = {"workload": "%dx%d container of the curved-interface transient, Lambda 5, FP64, "
                                           "200 steps" % (nx, ny),
                               "ms_per_step": round(ms2, 5), "MLUPS_all_sites": round(nx * ny / ms2 / 1e3, 1)}
    return out


def adjoint_rollout(torch, n=512, steps=2000, checkpoint=100):
    """Gradient of an interface-shape loss over a checkpointed rollout of the
    drop_to_ellipse workload; FP32 storage, FP64 dL/dsigma.  Returns forward
    and backward (recompute + adjoint) times: the backward as the rollout runs
    it (the next segment recomputed on a second stream during the current
    segment's adjoint steps, the two streams on disjoint CUs at this size)
    and, for context, with both streams on every CU and on one stream."""
    from paper_2005_04642_amd import adjoint, workloads as Wk
    rn0, target, force, params = Wk.drop_to_ellipse(n)
    dev = "cuda:0"
    rn_t = torch.tensor(rn0, dtype=torch.float32, device=dev, requires_grad=True)
    f_t = torch.tensor(force, dtype=torch.float32, device=dev, requires_grad=True)
    sig = torch.tensor(0.01, dtype=torch.float64, requires_grad=True)
    tgt = torch.tensor(target, dtype=torch.float32, device=dev)
    # untimed short rollout first: allocator pools, library load and first launches
    w = adjoint.rollout(rn_t, sig, f_t, params, 2 * checkpoint, checkpoint=checkpoint, storage="f32", device=dev)
    ((w - tgt) ** 2).sum().backward()

    def timed(overlap, recompute_cus=None):
        rn_t.grad = None
        f_t.grad = None
        sig.grad = None
        torch.cuda.synchronize()
        t0 = time.time()
        out = adjoint.rollout(rn_t, sig, f_t, params, steps, checkpoint=checkpoint, storage="f32", device=dev,
                              overlap=overlap, recompute_cus=recompute_cus)
        loss = ((out - tgt) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.time()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.time()
        return t1 - t0, t2 - t1, float(loss.detach()), float(sig.grad)

    fwd, bwd, loss, dsig = timed(None)
    lups = n * n * steps
    res = {"workload": "%d^2 periodic drop R=%d (tanh profile of width 2) to an ellipse target, %d steps, "
                       "checkpoint every %d, FP32" % (n, n // 4, steps, checkpoint),
           "forward_s": round(fwd, 3), "backward_s": round(bwd, 3),
           "MLUPS_forward": round(lups / fwd / 1e6, 1), "MLUPS_backward": round(lups / bwd / 1e6, 1),
           "ratio": round(fwd / bwd, 4), "loss": loss, "dL_dsigma": dsig}
    if checkpoint > 1:
        res["recompute_cus"] = adjoint.RECOMPUTE_CUS if n * n <= adjoint.PARTITION_MAX_SITES else 0
        # the same backward with both streams on every CU, and on one stream
        fwd2, bwd2, _, dsig2 = timed(True, 0)
        res["backward_s_two_streams_unconfined"] = round(bwd2, 3)
        fwd1, bwd1, _, dsig1 = timed(False)
        res["backward_s_one_stream"] = round(bwd1, 3)
        res["ratio_one_stream"] = round(fwd1 / bwd1, 4)
        res["same_dL_dsigma"] = dsig1 == dsig and dsig2 == dsig
    return res


def shard_measure(n, params, rn, torch, nslabs=8, halo=10, steps=200, warmup=20):
    """The step on one GPU's share of the benchmark lattice split into nslabs
    slabs of rows (the layout a halo exchange between GPUs would use): the
    slab alone, and the slab with the halo rows each GPU would march besides
    its own (halo = field-chain radius 9 + 1 for the gather, on either side),
    the periodic wrap standing in for the exchanged rows.  The initial colour
    index is the benchmark's, cut to the slab's rows; FP32."""
    import numpy as np
    from paper_2005_04642_amd import lbm
    rows = n // nslabs
    out = {"workload": "rows 0..%d of the %dx%d emulsion (one of %d slabs), FP32, %d steps after %d"
                       % (rows - 1, n, n, nslabs, steps, warmup),
           "halo_rows_per_side": halo, "halo_bytes_per_face": halo * n * 72}
    for label, ny in (("slab", rows), ("slab_with_halo", rows + 2 * halo)):
        sim = lbm.Simulation(n, ny, params, np.ascontiguousarray(rn[:ny]), storage="f32", device="cuda:0")
        sim.step(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        sim.step(steps)
        e1.record()
        torch.cuda.synchronize()
        sim.masses()
        sim.close()
        ms = e0.elapsed_time(e1) / steps
        out[label] = {"nx": n, "ny": ny, "ms_per_step": round(ms, 5), "MLUPS": round(n * ny / ms / 1e3, 1),
                      "GB_s": round(BYTES_PER_LU["f32"] * n * ny / ms / 1e6, 1)}
    # useful updates per second of a GPU that marches its slab and both halos
    out["MLUPS_own_rows_with_halo"] = round(n * rows / out["slab_with_halo"]["ms_per_step"] / 1e3, 1)
    return out


def batch_measure(torch, nsim=256, steps=20):
    """256 independent periodic drops of uneven size (64..512) stepped by one
    launch per step, after the autotuner picked the tile shape; against the same
    lattices stepped one launch per lattice."""
    from paper_2005_04642_amd import lbm, workloads as Wk
    lats = Wk.config_batch(nsim=nsim, seed=1)
    sites = sum(nx * ny for nx, ny, _, _ in lats)
    b = lbm.Batch(lats, storage="f32", device="cuda:0")
    b.step(3)
    t0 = time.time()
    chosen = b.autotune(5)
    tune_s = time.time() - t0
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    b.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1) / steps
    finite = all(all(v == v for v in b.masses(k)) for k in range(nsim))
    info = b.plan_info()
    b.close()
    sims = [lbm.Simulation(nx, ny, prm, rn, storage="f32", device="cuda:0") for nx, ny, prm, rn in lats]
    for s_ in sims:
        s_.step(1)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(5):
        for s_ in sims:
            s_.step(1)
    e1.record()
    torch.cuda.synchronize()
    ms_s = e0.elapsed_time(e1) / 5
    for s_ in sims:
        s_.close()
    return {"workload": "%d periodic drops, side ~U{64,128,256,512}, Lambda ~U{1,10,100}, sigma 10^U[-3,-1], "
                        "elliptic, FP32, %d sites" % (nsim, sites),
            "ms_per_step": round(ms_b, 4), "MLUPS": round(sites / ms_b / 1e3, 1),
            "ms_per_step_one_launch_per_lattice": round(ms_s, 4),
            "MLUPS_one_launch_per_lattice": round(sites / ms_s / 1e3, 1),
            "autotune": {"chosen_ntx": chosen[0], "chosen_chunk_cap": chosen[1], "seconds": round(tune_s, 3),
                         "work_items": info["items"], "bins": info["bins"]},
            "finite": finite}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--stencil", default="3333")
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"],
                    help="population storage: FP32, or the 16-bit offset formats (FP32 arithmetic)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-copy-roof", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-shard", action="store_true")
    ap.add_argument("--no-storage16", action="store_true")
    ap.add_argument("--no-solid", action="store_true")
    ap.add_argument("--no-rollout", action="store_true",
                    help="with the adjoint legs, skip the two 2000-step rollouts (for counter runs)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="first run one plain 1 GiB device copy (reference dispatch for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (the lattice would be "
              "split into slabs with a halo exchange per step, not implemented). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2005_04642_amd import lbm, workloads as Wk

    if args.copy_calib:
        a = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)          # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del a, b
    n = args.size
    stencil = tuple(int(c) for c in args.stencil)
    cfg = Wk.config_emulsion(nx=n, ny=n)
    params = dict(cfg["params"], stencil=stencil)
    rn = cfg["rhoN0"] if cfg["rhoN0"] is not None else Wk.emulsion(n, n, 50, 20.0, 80.0, 6.0, 0)
    sim = lbm.Simulation(n, n, params, rn, storage=args.storage, device="cuda:0")
    print("bench: emulsion %dx%d %s stencil %s, warmup %d, steps %d" % (n, n, args.storage, args.stencil,
                                                                        args.warmup, args.steps),
          file=sys.stderr, flush=True)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.time()
    ev0.record(stream)
    sim.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.time() - t0
    ms_event = ev0.elapsed_time(ev1)
    m = sim.masses()   # finite-state check (raises on NaN)
    sites = n * n
    ms_per_step = ms_event / args.steps
    mlups = sites / (ms_per_step * 1e-3) / 1e6
    bytes_launch = BYTES_PER_LU[args.storage] * sites
    achieved = bytes_launch / (ms_per_step * 1e-3) / 1e9
    traffic = measured_traffic(args.storage)
    out = {
        "metric": "MLUPS, D2Q9 chromodynamic MRT step (4096^2 emulsion)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "emulsion %dx%d periodic, 50 drops r~U[20,80], Lambda=10, sigma=0.005, "
                               "beta=0.67, nu=1/6, stencil radii %s, %s storage"
                               % (n, n, args.stencil, STORAGE_NAME[args.storage]),
                   "nx": n, "ny": n, "stencil": list(stencil), "storage": args.storage},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic},
        "wall_s": round(wall, 3),
        "masses": [m[0], m[1]],
    }
    sim.close()
    if not args.no_copy_roof:
        out["copy_roof"] = copy_roof(n, params, rn, torch, args.storage)
        out["roofline"]["frac_of_copy"] = round(achieved / out["copy_roof"]["GB_s"], 4)
    if not args.no_storage16 and args.storage == "f32":
        out["storage16"] = storage16_measure(n, params, rn, torch)
    if not args.no_solid and args.storage == "f32":
        out["solid_mask"] = solid_measure(n, params, rn, torch, ms_per_step)
    if not args.no_adjoint:
        out["adjoint"] = dict({"workload": "same lattice and state, one adjoint step vs one forward step, FP32"},
                              **adjoint_measure(n, params, rn, torch))
        rn_d, _, f_d, p_d = Wk.drop_to_ellipse(512)
        out["adjoint_512"] = dict({"workload": "512^2 drop of the rollout below (with its force field), one adjoint "
                                               "step vs one forward step, FP32"},
                                  **adjoint_measure(512, p_d, rn_d, torch, steps=200,
                                                    force=torch.tensor(f_d, dtype=torch.float32, device="cuda:0")))
        if not args.no_rollout:
            out["adjoint_rollout"] = adjoint_rollout(torch)
            out["adjoint_rollout_every_state"] = adjoint_rollout(torch, checkpoint=1)
    if not args.no_shard and args.storage == "f32":
        out["shard"] = shard_measure(n, params, rn, torch)
    if not args.no_batch:
        out["batch"] = batch_measure(torch)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark: D2Q9 chromodynamic MRT step on the 4096x4096 emulsion (FP32).

python bench.py [--gpus 1] [--steps K] [--warmup W] [--stencil 3333]
                [--storage f32|f16|bf16] [--no-cpu]

Prints one JSON line: MLUPS of the whole step (all stages: gather, fields,
stencils, force, collision, recolour, store) with the populations resident in
HBM, the roofline of the step kernel (HBM bound: algorithmic bytes per lattice
update = read + write of one site's population words: 144 B for FP32 storage,
80 B for the 16-bit offset formats) and the CPU oracle timed on a bounded
sample of the same workload.
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
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2005_04642_amd", "csrc", f)
                  for f in ("chromo_kernels.hpp", "chromo_launch.hpp", "chromo_host.hpp", "chromo_api.hip")]


STORAGE_NAME = {"f32": "FP32", "f16": "FP16-offset (16-bit words, FP32 arithmetic)",
                "bf16": "BF16-offset (16-bit words, FP32 arithmetic)"}


def traffic_file(storage):
    return os.path.join(ROOT, "profiles", "traffic_step_emulsion4096_%s.json" % storage)


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
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


def cpu_baseline(seconds_target=15.0):
    """The oracle (torch-CPU float64, untuned) on a 256x256 crop of the emulsion
    workload: Lambda = 10, sigma = 0.005, drops with the emulsion's radius law."""
    import torch
    from oracle import chromo as O
    from paper_2005_04642_amd import workloads as Wk
    threads = os.cpu_count() or 1
    torch.set_num_threads(threads)
    n = 256
    cfg = Wk.config_emulsion(nx=n, ny=n)
    rn = Wk.emulsion(n, n, ndrops=3, rmin=20.0, rmax=40.0, gap=6.0, seed=0)
    o = O.Oracle(O.Params(nx=n, ny=n, **cfg["params"])).init(rn)
    o.step(1)                      # warm-up
    t0 = time.time()
    steps = 0
    while time.time() - t0 < seconds_target:
        o.step(1)
        steps += 1
    dt = time.time() - t0
    return {"value": round(n * n * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "%d steps of a %dx%d crop of the emulsion workload (3 drops, Lambda=10, sigma=0.005), "
                      "torch-CPU float64, %.1f s" % (steps, n, n, dt)}


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
    ap.add_argument("--copy-calib", action="store_true",
                    help="first run one plain 1 GiB device copy (reference dispatch for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (the lattice would be "
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
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

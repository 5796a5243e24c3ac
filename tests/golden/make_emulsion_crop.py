"""Writes emulsion_crop512_1000.npz: the oracle's fields after 1000 steps of the
512x512 three-drop crop of the emulsion workload (Lambda = 10, sigma = 0.005,
beta = 0.67, nu = 1/6, stencil radii 3333), at 2048 seeded random sites and
2048 seeded interface sites (|rho^N| < 0.9 at the end), for the oracle in
float64 and in float32 arithmetic, and for the float64 oracle with its state
rounded to float32 after every step (the error FP32 storage alone leaves).  Calls only oracle/ and the seeded input
generators; nothing here comes from the GPU path.

usage: python tests/golden/make_emulsion_crop.py   (about 8 minutes on 8 cores)"""
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import chromo as O  # noqa: E402
from paper_2005_04642_amd import workloads as Wk  # noqa: E402

N, STEPS, NSITE = 512, 1000, 2048
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "emulsion_crop512_1000.npz")


def run(dtype, round_state=False):
    rn = Wk.emulsion_crop(N, 3, 0)
    p = Wk.config_emulsion(nx=N, ny=N)["params"]
    o = O.Oracle(O.Params(nx=N, ny=N, **p), dtype=dtype).init(rn)
    if not round_state:
        o.step(STEPS)
    else:
        o.R, o.B = o.R.float().double(), o.B.float().double()
        for _ in range(STEPS):
            o.step(1)
            o.R, o.B = o.R.float().double(), o.B.float().double()
    return {k: v.double().numpy() for k, v in o.fields().items()}


def main():
    torch.set_num_threads(os.cpu_count() or 1)
    f64 = run(torch.float64)
    f32 = run(torch.float32)
    s32 = run(torch.float64, round_state=True)
    rng = np.random.default_rng(20050464)
    ys = rng.integers(0, N, NSITE)
    xs = rng.integers(0, N, NSITE)
    iy, ix = np.nonzero(np.abs(f64["rhoN"]) < 0.9)
    k = rng.choice(len(iy), NSITE, replace=False)
    ys = np.concatenate([ys, iy[k]]).astype(np.int32)
    xs = np.concatenate([xs, ix[k]]).astype(np.int32)
    out = {"ys": ys, "xs": xs, "umax64": np.float64(np.max(np.hypot(f64["ux"], f64["uy"]))),
           "steps": np.int32(STEPS), "n": np.int32(N)}
    for key in ("rho", "ux", "uy", "rhoN"):
        out[key + "64"] = f64[key][ys, xs].astype(np.float64)
        out[key + "32"] = f32[key][ys, xs].astype(np.float32)
        out[key + "_s32"] = s32[key][ys, xs].astype(np.float64)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT, "umax64 %.4e" % out["umax64"])


if __name__ == "__main__":
    main()

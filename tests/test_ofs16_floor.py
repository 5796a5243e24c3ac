"""Rounding floor of the 16-bit offset formats: the FP64 oracle with its state
passed through the format's words (tests/ofs16.py) after every step, against
the plain FP64 oracle, on the 64x64 static drop after 1000 steps and on the
layered channel (walls, body force) after 400 steps.  The GPU tolerances of
the 16-bit formats are set at about twice these floors."""
import numpy as np
import pytest
import torch

import ofs16
from oracle import chromo as O
from paper_2005_04642_amd import workloads as Wk

pytestmark = pytest.mark.slow

# GPU tolerances of the 16-bit formats (static drop, 1000 steps): relative rho,
# u relative to max |u| (the micro-current), rho^N absolute, masses relative.
OFS16_TOL = {
    "f16": dict(rho=2e-4, u=0.1, rhoN=2e-4, mass=2e-5),
    "bf16": dict(rho=1e-3, u=0.3, rhoN=1e-3, mass=1e-4),
}


# layered channel: relative rho and u relative to max |u| (the driven flow)
CHANNEL_TOL = {
    "f16": dict(rho=1e-3, u=1e-2),
    "bf16": dict(rho=2e-3, u=0.1),
}


def channel_case():
    """48x66 channel between walls, Lambda = 10, viscosity ratio 10, body
    force 1e-5 along x, two layers with a tanh interface; 400 steps."""
    nx, ny, steps = 48, 66, 400
    params = Wk.base_params(Lambda=10.0, sigma=0.01)
    params.update(walls=True, nu_R=1.0 / 6.0, nu_B=10.0 / 6.0, gx=1e-5)
    yy = (np.arange(ny) - 0.5)[:, None] * np.ones((1, nx))
    rn = np.tanh(0.6 * (ny / 2.0 - yy))
    return nx, ny, steps, params, rn


def round_through_format(o, params, fmt):
    # the oracle holds fluid rows only; the words are per site, so no layout
    # change is needed to round them
    R, B = ofs16.decode(ofs16.encode(o.R.numpy(), o.B.numpy(), params, fmt), params, fmt)
    o.R = torch.from_numpy(R.astype(np.float64))
    o.B = torch.from_numpy(B.astype(np.float64))


def errors(f, fo, m, mo):
    e_rho = float(np.max(np.abs(f["rho"] - fo["rho"]) / fo["rho"]))
    e_u = float(np.max(np.hypot(f["ux"] - fo["ux"], f["uy"] - fo["uy"])) / np.max(np.hypot(fo["ux"], fo["uy"])))
    e_rn = float(np.max(np.abs(f["rhoN"] - fo["rhoN"])))
    e_m = max(abs(m[0] - mo[0]) / mo[0], abs(m[1] - mo[1]) / mo[1])
    return dict(rho=e_rho, u=e_u, rhoN=e_rn, mass=e_m)


def test_ofs16_rounding_floor_of_static_drop():
    cfg = Wk.config_static_drop()
    params = cfg["params"]
    p = O.Params(nx=64, ny=64, **params)
    exact = O.Oracle(p).init(cfg["rhoN0"])
    rounded = {fmt: O.Oracle(p).init(cfg["rhoN0"]) for fmt in OFS16_TOL}
    for fmt, o in rounded.items():
        round_through_format(o, params, fmt)
    for _ in range(1000):
        exact.step(1)
        for fmt, o in rounded.items():
            o.step(1)
            round_through_format(o, params, fmt)
    fe = {k: v.numpy() for k, v in exact.fields().items()}
    for fmt, o in rounded.items():
        e = errors({k: v.numpy() for k, v in o.fields().items()}, fe, o.masses(), exact.masses())
        print("%s storage floor: " % fmt + " ".join("e_%s %.3e" % kv for kv in e.items()))
        for k, tol in OFS16_TOL[fmt].items():
            assert e[k] < tol / 2, (fmt, k, e[k])


def test_ofs16_rounding_floor_of_layered_channel():
    nx, ny, steps, params, rn = channel_case()
    p = O.Params(nx=nx, ny=ny, **params)
    exact = O.Oracle(p).init(rn)
    rounded = {fmt: O.Oracle(p).init(rn) for fmt in CHANNEL_TOL}
    for fmt, o in rounded.items():
        round_through_format(o, params, fmt)
    for _ in range(steps):
        exact.step(1)
        for fmt, o in rounded.items():
            o.step(1)
            round_through_format(o, params, fmt)
    fe = {k: v.numpy()[1:-1] for k, v in exact.fields().items()}
    for fmt, o in rounded.items():
        f = {k: v.numpy()[1:-1] for k, v in o.fields().items()}
        e = errors(f, fe, o.masses(), exact.masses())
        print("%s channel floor: e_rho %.3e e_u %.3e" % (fmt, e["rho"], e["u"]))
        for k, tol in CHANNEL_TOL[fmt].items():
            assert e[k] < tol / 2, (fmt, k, e[k])

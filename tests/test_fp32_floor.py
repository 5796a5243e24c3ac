"""Derivation of the FP32 tolerance on u used by the GPU parity tests: the
oracle in FP64 arithmetic with its state rounded to FP32 after every step
(storage rounding only) already differs from the FP64 oracle by more than
1e-5 of the static drop's micro-current after 1000 steps, while keeping rho
within 1e-6."""
import numpy as np
import pytest
import torch

from oracle import chromo as O
from paper_2005_04642_amd import workloads as Wk

pytestmark = pytest.mark.slow


def test_fp32_storage_floor_of_static_drop():
    cfg = Wk.config_static_drop()
    p = O.Params(nx=64, ny=64, **cfg["params"])
    exact = O.Oracle(p).init(cfg["rhoN0"])
    rounded = O.Oracle(p).init(cfg["rhoN0"])
    for _ in range(1000):
        exact.step(1)
        rounded.step(1)
        rounded.R = rounded.R.float().double()
        rounded.B = rounded.B.float().double()
    fe, fr = exact.fields(), rounded.fields()
    umax = float(torch.hypot(fe["ux"], fe["uy"]).max())
    e_u = float(torch.hypot(fr["ux"] - fe["ux"], fr["uy"] - fe["uy"]).max()) / umax
    e_rho = float(((fr["rho"] - fe["rho"]) / fe["rho"]).abs().max())
    print("fp32 storage floor: e_u %.3e (max|u| %.3e), e_rho %.3e" % (e_u, umax, e_rho))
    assert 1e-5 < e_u < 1e-3
    assert e_rho < 1e-6

"""Differentiable rollouts of the chromodynamic step on the GPU.

``rollout(rhoN0, sigma, force, params, nsteps, checkpoint=100)`` runs
``nsteps`` steps from the rest state of ``rhoN0`` and returns the colour index
rho^N of the final state.  It is a ``torch.autograd.Function``: the backward
pass runs the library's hand-written adjoint (``lbm_adjoint_step``) step by
step in reverse, recomputing the states of each checkpoint segment forward
from the state saved at its start, and returns dL/drho^N_0, dL/dsigma and
dL/dG_ext (the per-site force density).  Every step, forward or adjoint, runs
in the HIP library; torch only holds buffers.

F64 or F32 storage, periodic or walled lattices.  dL/dsigma is summed in FP64 on the
device.
"""
import torch

from . import lbm


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rhoN0, sigma, force, params, nsteps, checkpoint, storage, device):
        p = dict(params)
        p["sigma"] = float(sigma)
        ny, nx = rhoN0.shape
        sim = lbm.Simulation(nx, ny, p, rhoN0.detach(), storage=storage, device=device,
                             force=None if force is None else force.detach())
        ckpts = {}
        for t in range(0, nsteps, checkpoint):
            ckpts[t] = sim.live_pops().clone()
            sim.step(min(checkpoint, nsteps - t))
        out = sim.fields()["rhoN"]
        ctx.sim = sim
        ctx.ckpts = ckpts
        ctx.nsteps = nsteps
        ctx.checkpoint = checkpoint
        ctx.final = sim.live_pops().clone()
        ctx.has_force = force is not None
        ctx.sigma_dtype = sigma.dtype
        ctx.sigma_device = sigma.device
        return out

    @staticmethod
    def backward(ctx, grad_rhoN):
        sim = ctx.sim
        T = sim.dtype
        lam = sim.pops_like()
        lam_prev = sim.pops_like()
        sim.rhoN_adjoint(ctx.final, grad_rhoN.to(T), lam)
        dsigma = torch.zeros(1, dtype=torch.float64, device=sim.device)
        dforce = torch.zeros((2, sim.ny, sim.nx), dtype=T, device=sim.device)
        starts = sorted(ctx.ckpts)
        for k in reversed(range(len(starts))):
            t0 = starts[k]
            t1 = starts[k + 1] if k + 1 < len(starts) else ctx.nsteps
            # states t0 .. t1-1 of this segment, recomputed from its checkpoint,
            # each step written straight into a buffer of its own
            states = [ctx.ckpts[t0]]
            for _ in range(t0 + 1, t1):
                nxt = sim.pops_like()
                sim.set_pops(states[-1], nxt)
                sim.step(1)
                states.append(nxt)
            for t in reversed(range(t0, t1)):
                sim.adjoint_step(states[t - t0], lam, lam_prev, dsigma, dforce)
                lam, lam_prev = lam_prev, lam
        drhoN0 = torch.zeros((sim.ny, sim.nx), dtype=T, device=sim.device)
        sim.init_adjoint(lam, drhoN0)
        sim.close()
        ctx.sim = None
        ctx.ckpts = None
        dsig = dsigma.to(device=ctx.sigma_device, dtype=ctx.sigma_dtype).reshape(())
        return (drhoN0, dsig, dforce if ctx.has_force else None,
                None, None, None, None, None)


def rollout(rhoN0, sigma, force, params, nsteps, checkpoint=100, storage="f32", device="cuda:0"):
    """rho^N after ``nsteps`` steps from the rest state of ``rhoN0`` ([ny, nx]);
    differentiable with respect to rhoN0, sigma (0-dim tensor) and force
    ([2, ny, nx] tensor or None)."""
    if not torch.is_tensor(sigma):
        sigma = torch.tensor(float(sigma), dtype=torch.float64)
    return _Rollout.apply(rhoN0, sigma, force, params, int(nsteps), int(checkpoint), storage, device)

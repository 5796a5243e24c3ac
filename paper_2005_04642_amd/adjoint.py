"""Differentiable rollouts of the chromodynamic step on the GPU.

``rollout(rhoN0, sigma, force, params, nsteps, checkpoint=100)`` runs
``nsteps`` steps from the rest state of ``rhoN0`` and returns the colour index
rho^N of the final state.  It is a ``torch.autograd.Function``: the backward
pass runs the library's hand-written adjoint (``lbm_adjoint_step``) step by
step in reverse, recomputing the states of each checkpoint segment forward
from the state saved at its start, and returns dL/drho^N_0, dL/dsigma and
dL/dG_ext (the per-site force density).  Every step, forward or adjoint, runs
in the HIP library; torch only holds buffers.

F64 or F32 storage; periodic, walled or masked lattices.  dL/dsigma is summed in FP64 on the
device.
"""
import torch

from . import lbm


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rhoN0, sigma, force, params, nsteps, checkpoint, storage, device):
        p = dict(params)
        p["sigma"] = float(sigma)
        solid = p.pop("solid", None)
        ny, nx = rhoN0.shape
        sim = lbm.Simulation(nx, ny, p, rhoN0.detach(), storage=storage, device=device,
                             force=None if force is None else force.detach(), solid=solid)
        # Every checkpointed state (and the final one) gets a buffer of its own,
        # written directly by the step that produces it (lbm_set_pops); the steps
        # in between alternate between two scratch buffers.  No state is copied
        # after the first, so a checkpoint every step costs no extra traffic.
        # All of them come from one allocation.
        nseg = len(range(0, nsteps, checkpoint))
        block = torch.empty((nseg + 3, ny, 2, 9, nx), dtype=sim.dtype, device=sim.device)
        bufs = [block[i].permute(1, 2, 0, 3) for i in range(nseg + 3)]   # pops_like() views
        cur = bufs[0]
        cur.copy_(sim.live_pops())
        scratch = (bufs[1], bufs[2])
        # (straight C calls with the stream looked up once: with a checkpoint
        # every step the Python wrappers would cost more than the step itself)
        h, stream = sim.h, sim.stream()

        def steps_into(src, dst, n):
            lbm.lbm_set_pops(h, src.data_ptr(), dst.data_ptr())
            lbm.lbm_step(h, n, None, stream)

        ckpts = {}
        for j, t in enumerate(range(0, nsteps, checkpoint)):
            ckpts[t] = cur
            k = min(checkpoint, nsteps - t)
            dst = bufs[3 + j]
            if k >= 2:
                steps_into(cur, scratch[0], 1)
                steps_into(scratch[0], scratch[1], k - 2)
                cur = scratch[(k - 2) % 2]   # live after the k - 1 steps so far
            steps_into(cur, dst, 1)
            cur = dst
        sim.set_pops(cur, scratch[0])        # the Simulation's own views follow the handle again
        out = sim.fields()["rhoN"]
        ctx.sim = sim
        ctx.ckpts = ckpts
        ctx.nsteps = nsteps
        ctx.checkpoint = checkpoint
        ctx.final = cur
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
    ([2, ny, nx] tensor or None).

    Device memory: ceil(nsteps / checkpoint) + 3 population states are held
    from the forward pass to the end of the backward one (checkpoint = 1 keeps
    every state and recomputes nothing), plus ``checkpoint`` states during the
    backward recompute of one segment.  ``params`` may hold ``solid``, a mask of
    solid sites ([ny, nx]; F64/F32 storage, stencil profiles 3333, 3131 and 1111)."""
    if not torch.is_tensor(sigma):
        sigma = torch.tensor(float(sigma), dtype=torch.float64)
    return _Rollout.apply(rhoN0, sigma, force, params, int(nsteps), int(checkpoint), storage, device)

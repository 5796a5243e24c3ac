"""Differentiable rollouts of the chromodynamic step on the GPU.

``rollout(rhoN0, sigma, force, params, nsteps, checkpoint=100)`` runs
``nsteps`` steps from the rest state of ``rhoN0`` and returns the colour index
rho^N of the final state.  It is a ``torch.autograd.Function``: the backward
pass runs the library's hand-written adjoint (``lbm_adjoint_steps``, one
call per segment) step by step in reverse, recomputing the states of each checkpoint segment forward
from the state saved at its start (the next segment's recompute overlaps the
current segment's adjoint steps on a second stream), and returns dL/drho^N_0, dL/dsigma and
dL/dG_ext (the per-site force density).  Every step, forward or adjoint, runs
in the HIP library; torch only holds buffers.

F64 or F32 storage; periodic, walled or masked lattices.  dL/dsigma is summed in FP64 on the
device.
"""
import torch

from . import lbm


# Backward passes of lattices up to this many sites confine the recompute to
# the first RECOMPUTE_CUS CUs and the adjoint steps to the others (512^2 FP32
# drop: a forward step takes 23 us on 256 CUs and 40 us on 64, the adjoint step
# 51 us on 256 and 54 us on 192).
PARTITION_MAX_SITES = 1 << 20
RECOMPUTE_CUS = 64

_partitions = {}


def _partition(device, first, count):
    """A stream confined to CUs [first, first + count) of `device`, created
    once per process and kept (torch.cuda.ExternalStream over
    lbm_partition_stream)."""
    key = (torch.device(device).index or 0, first, count)
    if key not in _partitions:
        with torch.cuda.device(device):
            ptr = lbm.lbm_partition_stream(first, count)
        _partitions[key] = torch.cuda.ExternalStream(ptr, device=device)
    return _partitions[key]


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rhoN0, sigma, force, params, nsteps, checkpoint, storage, device, overlap, recompute_cus):
        p = dict(params)
        p["sigma"] = float(sigma)
        solid = p.pop("solid", None)
        ny, nx = rhoN0.shape
        sim = lbm.Simulation(nx, ny, p, rhoN0.detach(), storage=storage, device=device,
                             force=None if force is None else force.detach(), solid=solid)
        # Every checkpointed state (and the final one) gets a buffer of its own,
        # written directly by the step that produces it; the steps in between
        # alternate between two scratch buffers.  No state is copied after the
        # first, so a checkpoint every step costs no extra traffic.  All of
        # them come from one allocation, and the whole trajectory is one call
        # (lbm_step_into: no host call per step).
        nseg = len(range(0, nsteps, checkpoint))
        block = torch.empty((nseg + 3, ny, 2, 9, nx), dtype=sim.dtype, device=sim.device)
        bufs = [block[i].permute(1, 2, 0, 3) for i in range(nseg + 3)]   # pops_like() views
        cur = bufs[0]
        cur.copy_(sim.live_pops())
        scratch = (bufs[1], bufs[2])
        h, stream = sim.h, sim.stream()
        ckpts = {}
        ptrs = []
        for j, t in enumerate(range(0, nsteps, checkpoint)):
            ckpts[t] = cur
            k = min(checkpoint, nsteps - t)
            ptrs += [scratch[i % 2].data_ptr() for i in range(k - 1)]
            cur = bufs[3 + j]
            ptrs.append(cur.data_ptr())
        lbm.lbm_step_into(h, bufs[0].data_ptr(), ptrs, stream)
        sim.set_pops(cur, scratch[0])        # the Simulation's own views follow the handle again
        out = sim.fields()["rhoN"]
        ctx.sim = sim
        ctx.ckpts = ckpts
        ctx.nsteps = nsteps
        ctx.checkpoint = checkpoint
        ctx.overlap = overlap
        ctx.recompute_cus = recompute_cus
        ctx.final = cur
        ctx.has_force = force is not None
        ctx.sigma_dtype = sigma.dtype
        ctx.sigma_device = sigma.device
        return out

    @staticmethod
    def backward(ctx, grad_rhoN):
        sim = ctx.sim
        torch_ = sim.torch
        T = sim.dtype
        lam = sim.pops_like()
        lam_prev = sim.pops_like()
        sim.rhoN_adjoint(ctx.final, grad_rhoN.to(T), lam)
        dsigma = torch.zeros(1, dtype=torch.float64, device=sim.device)
        dforce = torch.zeros((2, sim.ny, sim.nx), dtype=T, device=sim.device)
        starts = sorted(ctx.ckpts)
        ends = starts[1:] + [ctx.nsteps]
        nseg = len(starts)
        # States after a segment's checkpoint are recomputed into a set of
        # buffers of their own.  With two sets, segment k - 1 is recomputed on
        # a second stream while the adjoint steps of segment k run; each set is
        # reused only after the adjoint steps that read it have finished
        # (events).  On small lattices the two streams are confined to disjoint
        # CUs (lbm_partition_stream, tiles planned for each share with
        # lbm_set_cu_budget): there a step's march keeps each CU busy for long
        # with one workgroup, and unconfined streams queue one kernel's
        # workgroups behind the other's.  Same kernels in the same order on
        # each stream: the gradients depend on none of this.
        longest = max(e - s for s, e in zip(starts, ends))
        per = max(longest - 1, 1)
        state_bytes = sim.ny * sim.nx * 18 * (8 if T == torch.float64 else 4)
        overlap = ctx.overlap
        if overlap is None:
            free, _ = torch_.cuda.mem_get_info(sim.device)
            overlap = 2 * per * state_bytes <= free // 2
        nsets = 2 if overlap and nseg >= 2 and longest >= 2 else 1   # (checkpoint 1: nothing to recompute)
        rcus = ctx.recompute_cus
        ncu = torch_.cuda.get_device_properties(sim.device).multi_processor_count // 8 * 8
        if rcus is None:
            rcus = RECOMPUTE_CUS if sim.nx * sim.ny <= PARTITION_MAX_SITES else 0
        if nsets == 1 or not 0 < rcus < ncu:
            rcus = 0
        block = torch.empty((nsets, per, sim.ny, 2, 9, sim.nx), dtype=T, device=sim.device)
        base = block.data_ptr()
        caller = torch_.cuda.current_stream(sim.device)
        if rcus:
            try:
                side = _partition(sim.device, 0, rcus)
                main = _partition(sim.device, rcus, ncu - rcus)
            except lbm.LbmError:
                if ctx.recompute_cus:       # asked for explicitly: report it
                    raise
                rcus = 0                    # the runtime refused CU masks: unconfined streams
        if rcus:
            lbm.lbm_set_cu_budget(sim.h, rcus, ncu - rcus)
            main.wait_stream(caller)        # the checkpoints and lambda come from the caller's stream
        else:
            main = caller
            side = torch_.cuda.Stream(device=sim.device) if nsets == 2 else main
        h = sim.h
        ws = sim.adjoint_workspace()
        wsp, wsb = ws.data_ptr(), ws.numel()
        dsp, dfp = dsigma.data_ptr(), dforce.data_ptr()
        ms, ss = main.cuda_stream, side.cuda_stream
        step_into, adj_steps = lbm.lbm_step_into, lbm.lbm_adjoint_steps

        def states_of(k):
            # device pointers of the states t0 .. t1-1 of segment k
            n = ends[k] - starts[k]
            b = base + (k % nsets) * per * state_bytes
            return [ctx.ckpts[starts[k]].data_ptr()] + [b + j * state_bytes for j in range(n - 1)]

        def recompute(k, stream):
            st = states_of(k)
            if len(st) > 1:
                step_into(h, st[0], st[1:], stream)

        lptr = (lam.data_ptr(), lam_prev.data_ptr())
        cur = 0                              # lptr[cur] holds dL/d(the state reached so far)
        ev_rec, ev_adj = {}, {}
        if nsets == 2:
            side.wait_stream(caller)
            recompute(nseg - 1, ss)
            ev_rec[nseg - 1] = side.record_event()
        for k in reversed(range(nseg)):
            if nsets == 2:
                if k >= 1:
                    if k + 1 < nseg:
                        side.wait_event(ev_adj[k + 1])   # set (k - 1) % 2 was read by segment k + 1
                    recompute(k - 1, ss)
                    ev_rec[k - 1] = side.record_event()
                main.wait_event(ev_rec[k])
            else:
                recompute(k, ms)
            st = states_of(k)
            adj_steps(h, st, lptr[cur], lptr[1 - cur], wsp, wsb, dsp, dfp, ms)
            cur ^= len(st) & 1
            if nsets == 2:
                ev_adj[k] = main.record_event()
        if rcus:
            caller.wait_stream(main)        # (main waited for every recompute)
            lbm.lbm_set_cu_budget(h, 0, 0)
        L = lam_prev if cur else lam
        drhoN0 = torch.zeros((sim.ny, sim.nx), dtype=T, device=sim.device)
        sim.init_adjoint(L, drhoN0)
        del block
        sim.close()
        ctx.sim = None
        ctx.ckpts = None
        dsig = dsigma.to(device=ctx.sigma_device, dtype=ctx.sigma_dtype).reshape(())
        return (drhoN0, dsig, dforce if ctx.has_force else None,
                None, None, None, None, None, None, None)


def rollout(rhoN0, sigma, force, params, nsteps, checkpoint=100, storage="f32", device="cuda:0", overlap=None,
            recompute_cus=None):
    """rho^N after ``nsteps`` steps from the rest state of ``rhoN0`` ([ny, nx]);
    differentiable with respect to rhoN0, sigma (0-dim tensor) and force
    ([2, ny, nx] tensor or None).

    Device memory: ceil(nsteps / checkpoint) + 3 population states are held
    from the forward pass to the end of the backward one (checkpoint = 1 keeps
    every state and recomputes nothing), plus checkpoint - 1 recomputed states
    per segment in the backward pass (twice that with ``overlap``).  ``params`` may hold ``solid``, a mask of
    solid sites ([ny, nx]; F64/F32 storage, stencil profiles 3333, 3131 and 1111).

    ``overlap``: recompute the next segment's states on a second stream while
    the adjoint steps of the current one run (True), or one after the other
    (False); None chooses True when two segments' states take at most half of
    the free device memory.  ``recompute_cus``: with the overlap, confine the
    recompute to that many CUs (a multiple of 8; multiples of 32 run best) and
    the adjoint steps to the rest; None chooses RECOMPUTE_CUS for lattices of
    at most PARTITION_MAX_SITES sites, 0 leaves both streams on every CU.  The
    gradients are the same either way."""
    if not torch.is_tensor(sigma):
        sigma = torch.tensor(float(sigma), dtype=torch.float64)
    return _Rollout.apply(rhoN0, sigma, force, params, int(nsteps), int(checkpoint), storage, device, overlap,
                          recompute_cus)

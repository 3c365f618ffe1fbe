"""Reverse-mode differentiation of whole runs through the hand-written adjoint.

``final_electric_energy(f0, solver, nsteps, tau, every)`` returns the electric
energy W(f^N) after ``nsteps`` Strang steps from ``f0`` as a differentiable
torch scalar.  Its backward pass runs the library's adjoint: dW/df^N from
``vp_energy_gradient``, then one ``vp_strang_adjoint`` per step, last step
first.  The forward pass keeps a checkpoint of the state every ``every``
steps; the backward pass recomputes the states of one segment at a time from
its checkpoint (memory: nsteps/every + every + 4 copies of f).
"""

import torch


class _FinalElectricEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f0, solver, nsteps, tau, every):
        f = f0.detach().clone()
        tmp = torch.empty_like(f)
        ckpts = [f.clone()]
        done = 0
        while done < nsteps:
            n = min(every, nsteps - done)
            solver.step(f, tmp, n, tau)
            done += n
            if done < nsteps:
                ckpts.append(f.clone())
        W = torch.empty(1, dtype=torch.float64, device=f.device)
        lam = torch.empty_like(f)
        solver.energy_gradient(f, lam, W)
        ctx.solver, ctx.nsteps, ctx.tau, ctx.every = solver, nsteps, tau, every
        ctx.ckpts, ctx.lam = ckpts, lam
        return W[0]

    @staticmethod
    def backward(ctx, gW):
        solver, tau, every = ctx.solver, ctx.tau, ctx.every
        lam = ctx.lam
        if not torch.equal(gW, torch.ones_like(gW)):
            lam = lam * gW.to(lam.dtype)
        work = solver.adjoint_workspace(lam.device)
        tmp = torch.empty_like(lam)
        starts = list(range(0, ctx.nsteps, every))
        for seg in range(len(starts) - 1, -1, -1):
            n = min(every, ctx.nsteps - starts[seg])
            states = [ctx.ckpts[seg].clone()]
            for _ in range(n - 1):
                nxt = states[-1].clone()
                solver.step(nxt, tmp, 1, tau)
                states.append(nxt)
            for m in range(n - 1, -1, -1):
                solver.adjoint_step(states[m], lam, tau, work)
            del states
        ctx.ckpts = ctx.lam = None
        return lam, None, None, None, None


def final_electric_energy(f0, solver, nsteps, tau, every=10):
    """W(f^N) as a differentiable scalar (float64); gradients flow to f0."""
    return _FinalElectricEnergy.apply(f0, solver, int(nsteps), float(tau), int(every))

"""Reverse-mode differentiation of whole runs through the hand-written adjoint.

``final_electric_energy(f0, solver, nsteps, tau, every)`` returns the electric
energy W(f^N) after ``nsteps`` Strang steps from ``f0`` as a differentiable
torch scalar.  Its backward pass runs the library's adjoint: dW/df^N from
``vp_energy_gradient``, then one ``vp_strang_adjoint`` per step, last step
first.  The forward pass keeps ``f0`` and a checkpoint of the state every
``every`` steps after it.  The backward pass rebuilds the states of one
segment at a time from its checkpoint, either keeping all of them
(``store_segment=True``: ``every - 1`` steps recomputed per segment, memory
nsteps/every + every + 3 copies of f) or recomputing each one from the
checkpoint when it is needed (``store_segment=False``: every*(every-1)/2
steps per segment, memory nsteps/every + 4 copies of f).  During the
recomputation the first half of the adjoint workspace serves as the second
buffer of the forward steps.
"""

import torch


def _as_state(buf, like):
    """View the first bytes of a uint8 workspace as a state-shaped tensor."""
    nbytes = like.numel() * like.element_size()
    return buf[:nbytes].view(like.dtype).view(like.shape)


class _FinalElectricEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f0, solver, nsteps, tau, every, store_segment):
        f = f0.detach().clone()
        tmp = torch.empty_like(f)
        ckpts = [None]          # segment 0 starts from f0 itself
        done = 0
        while done < nsteps:
            n = min(every, nsteps - done)
            solver.step(f, tmp, n, tau)
            done += n
            if done < nsteps:
                ckpts.append(f.clone())
        del tmp
        W = torch.empty(1, dtype=torch.float64, device=f.device)
        lam = torch.empty_like(f)
        solver.energy_gradient(f, lam, W)
        del f
        ctx.save_for_backward(f0)
        ctx.solver, ctx.nsteps, ctx.tau, ctx.every = solver, nsteps, tau, every
        ctx.store_segment = store_segment
        ctx.ckpts, ctx.lam = ckpts, lam
        return W[0]

    @staticmethod
    def backward(ctx, gW):
        (f0,) = ctx.saved_tensors
        solver, tau, every = ctx.solver, ctx.tau, ctx.every
        lam = ctx.lam
        ctx.lam = None
        if not torch.equal(gW, torch.ones_like(gW)):
            lam.mul_(gW.to(lam.dtype))
        work = solver.adjoint_workspace(lam.device)
        tmp = _as_state(work, lam)
        starts = list(range(0, ctx.nsteps, every))
        for seg in range(len(starts) - 1, -1, -1):
            n = min(every, ctx.nsteps - starts[seg])
            ck = f0.detach() if seg == 0 else ctx.ckpts[seg]
            if ctx.store_segment:
                states = [ck]
                for _ in range(n - 1):
                    nxt = states[-1].clone()
                    solver.step(nxt, tmp, 1, tau)
                    states.append(nxt)
                for m in range(n - 1, -1, -1):
                    solver.adjoint_step(states[m], lam, tau, work)
                    states.pop()
            else:
                cur = torch.empty_like(lam)
                for m in range(n - 1, -1, -1):
                    if m == 0:
                        solver.adjoint_step(ck, lam, tau, work)
                    else:
                        cur.copy_(ck)
                        solver.step(cur, tmp, m, tau)
                        solver.adjoint_step(cur, lam, tau, work)
                del cur
            if seg > 0:
                ctx.ckpts[seg] = None
        ctx.ckpts = None
        return lam, None, None, None, None, None


def final_electric_energy(f0, solver, nsteps, tau, every=10, store_segment=True):
    """W(f^N) as a differentiable scalar (float64); gradients flow to f0."""
    return _FinalElectricEnergy.apply(f0, solver, int(nsteps), float(tau), int(every),
                                      bool(store_segment))

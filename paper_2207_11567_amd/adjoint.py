"""Differentiation of a rollout of the hybrid step with the hand-written adjoint kernels:
``HybridRollout`` is a torch.autograd.Function mapping the initial velocity (and passive
temperature) to J = sum rho|u|^2/2 + sum (T - mean T)^2 after n steps.  The forward pass
keeps a checkpoint of the state every ``seg`` steps; the backward pass recomputes one
segment at a time from its checkpoint, keeping that segment's states, and runs the
adjoint steps through it in reverse."""
import torch


class HybridRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, T0, solver, P_h0, nsteps, seg):
        nsteps, seg = int(nsteps), int(seg)
        solver.init_fields(P_h0, u0, T0 if solver.NS else None)
        ckpts = []
        done = 0
        while done < nsteps:
            pops, scal, step = solver.get_state()
            ckpts.append((pops, scal, step))
            k = min(seg, nsteps - done)
            solver.step(k)
            done += k
        final = solver.get_state()
        J, _, _ = solver.objective(final, with_grad=False)
        ctx.solver, ctx.ckpts, ctx.final, ctx.nsteps, ctx.seg = solver, ckpts, final, nsteps, seg
        ctx.save_for_backward(u0)
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        (u0,) = ctx.saved_tensors
        s = ctx.solver
        _, lp, ls = s.objective(ctx.final, with_grad=True)
        g = float(gJ)
        lp.mul_(g)
        ls.mul_(g)
        _, _, work = s.adjoint_buffers()
        op, osc = torch.empty_like(lp), torch.empty_like(ls)
        for c, (pops, scal, step) in reversed(list(enumerate(ctx.ckpts))):
            k = min(ctx.seg, ctx.nsteps - c * ctx.seg)
            # recompute the segment's states straight into its buffer
            states = [(pops, scal)]
            for j in range(k - 1):
                nxt = (torch.empty_like(pops), torch.empty_like(scal))
                s.step_from(states[-1], nxt, step + j)
                states.append(nxt)
            for st in reversed(states):
                s.adjoint_step(st, lp, ls, work, op, osc)
                lp, op = op, lp
                ls, osc = osc, ls
            del states
        gu, gT = s.init_adjoint(lp, ls, u0)
        return gu, (gT[0] if s.NS else None), None, None, None, None


def rollout_objective(solver, u0, T0, P_h0, nsteps, seg=100):
    return HybridRollout.apply(u0, T0, solver, P_h0, nsteps, seg)

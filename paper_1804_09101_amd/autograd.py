"""torch.autograd wrappers of the evolution and of the constraint norm.

GHEvolve runs n SSP-RK3 steps with the HIP library and, in backward, walks the
steps in reverse.  It keeps a copy of the state every `checkpoint_every` steps
during the forward pass; backward re-runs each segment forward from its
checkpoint with gh_step_stages (storing every step's start state and its two
RK stage states) and then applies gh_step_vjp_stages in reverse order, so each
step costs one forward step plus three RHS transposes.  With save_derivatives
the segment re-run also keeps the spatial derivatives of the three stage
states (150 P doubles each), which the transposes then reuse instead of
recomputing them (about a sixth of the backward time).  Memory: n/k
checkpoints plus 3k segment states of 50 P doubles each, and with
save_derivatives 3k more sets of 150 P doubles.

GHConstraintNorm returns the per-instance constraint norm of a state; its
backward is gh_constraints_vjp.

The damping parameters enter as a CPU float64 tensor [n_inst, 3]; they are
pushed to the library with gh_set_params before the forward and backward
passes, and their gradient is accumulated on the device by the library.
Every computation runs in the library; this module only orders the calls.
"""

import numpy as np
import torch


def _push_params(solver, gamma, dt):
    solver.set_params(gamma.detach().cpu().numpy().astype(np.float64), dt)


class GHEvolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, gamma, solver, dt, n_steps, checkpoint_every, save_derivatives=None):
        _push_params(solver, gamma, dt)
        k = max(1, int(checkpoint_every))
        u = u0.detach().clone().contiguous()
        ckpts = []
        for s in range(n_steps):
            if s % k == 0:
                ckpts.append(u.clone())
            solver.step(u, 1)
        ctx.solver, ctx.dt, ctx.n_steps, ctx.k = solver, dt, n_steps, k
        if save_derivatives is None:
            need = 3 * k * 150 * solver.P * 8
            free, _ = torch.cuda.mem_get_info(u.device)
            save_derivatives = need < 0.5 * free
        ctx.save_derivatives = bool(save_derivatives)
        ctx.gamma = gamma.detach().clone()
        ctx.ckpts = ckpts
        return u

    @staticmethod
    def backward(ctx, grad_u):
        solver, n, k = ctx.solver, ctx.n_steps, ctx.k
        _push_params(solver, ctx.gamma, ctx.dt)
        lam = grad_u.detach().contiguous().clone()
        g = torch.zeros(solver.n_inst * 3, dtype=torch.float64, device=lam.device)
        for seg in reversed(range(len(ctx.ckpts))):
            s0 = seg * k
            s1 = min(n, s0 + k)
            # re-run the segment, keeping every step's start state and its two stage states
            states, stages = [ctx.ckpts[seg].clone()], []
            for j in range(s1 - s0):
                nxt = states[-1].clone()
                u1, u2 = torch.empty_like(nxt), torch.empty_like(nxt)
                d = (torch.empty(450 * solver.P, dtype=torch.float64, device=nxt.device)
                     if ctx.save_derivatives else None)
                solver.step_stages(nxt, u1, u2, derivs=d)
                stages.append((u1, u2, d))
                if j < s1 - s0 - 1:
                    states.append(nxt)
            for j in reversed(range(s1 - s0)):
                u1, u2, d = stages[j]
                solver.step_vjp_stages(states[j], u1, u2, lam, g_gamma=g, out=lam, derivs=d)
                stages[j] = None
            del states, stages
        return lam, g.view(solver.n_inst, 3).cpu(), None, None, None, None, None


class GHConstraintNorm(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, solver):
        _, norm = solver.constraints(u.detach().contiguous(), want_C=False)
        ctx.solver = solver
        ctx.save_for_backward(u)
        return norm

    @staticmethod
    def backward(ctx, grad_norm):
        (u,) = ctx.saved_tensors
        lam = ctx.solver.constraints_vjp(u.detach().contiguous(), grad_norm.detach().contiguous())
        return lam, None


def evolve(u0, gamma, solver, dt, n_steps, checkpoint_every=20, save_derivatives=None):
    """save_derivatives: keep the stage derivatives of a segment for its
    reverse sweep (None: when they take under half of the free device memory)."""
    return GHEvolve.apply(u0, gamma, solver, dt, n_steps, checkpoint_every, save_derivatives)


def constraint_norm(u, solver):
    return GHConstraintNorm.apply(u, solver)

"""torch.autograd wrappers of the evolution and of the constraint norm.

GHEvolve runs n SSP-RK3 steps with the HIP library and, in backward, walks the
steps in reverse with checkpointed recomputation, in one or two levels:

* one level (checkpoint_every = k): a copy of the state every k steps in the
  forward pass; backward re-runs each segment from its checkpoint with
  gh_step_stages (storing every step's start state and its two RK stage
  states) and applies gh_step_vjp_stages in reverse order.  Each step costs
  one forward step plus three RHS transposes.  Live states: ceil(n/k)
  checkpoints plus 3k segment states (plus the cotangent and one work state).
* two levels (checkpoint_every = k1, inner_every = k2 < k1): the same k1
  checkpoints; backward first re-runs a k1-segment with plain steps keeping a
  state every k2 steps, then treats each k2-subsegment as above.  One more
  forward step per step, and ceil(n/k1) + ceil(k1/k2) + 3 k2 live states.
  This is what fits a long evolution of a large batch into device memory
  (the 2000-step gradient of four 20-shell holes: 58 states of 2.16 GB
  instead of 158 for the best one-level choice).

plan_checkpoints picks the cheapest schedule that fits a memory budget.
With save_derivatives a segment re-run also keeps the spatial derivatives of
the three stage states (150 P doubles each, i.e. 9 states per step), which the
transposes then reuse instead of recomputing them (about a sixth of the
backward time); by default only when they fit in half the free memory.

GHConstraintNorm returns the per-instance constraint norm of a state; its
backward is gh_constraints_vjp.

The damping parameters enter as a CPU float64 tensor [n_inst, 3]; they are
pushed to the library with gh_set_params before the forward and backward
passes, and their gradient is accumulated on the device by the library.
Every computation runs in the library; this module only orders the calls.
"""

import math

import numpy as np
import torch


def _push_params(solver, gamma, dt):
    solver.set_params(gamma.detach().cpu().numpy().astype(np.float64), dt)


def live_states(n_steps, k1, k2=None):
    """Peak number of live [50 P] states of the backward pass of a schedule:
    checkpoints, inner checkpoints, segment states, the incoming and the
    running cotangent and one work state (derivatives not counted)."""
    k1 = max(1, min(int(k1), n_steps))
    outer = math.ceil(n_steps / k1)
    if k2 is None or k2 >= k1:
        return outer + 3 * k1 + 3
    k2 = max(1, int(k2))
    return outer + math.ceil(k1 / k2) + 3 * k2 + 3


def plan_checkpoints(n_steps, state_bytes, budget_bytes):
    """(k1, k2) of the cheapest schedule whose live states fit the budget:
    one level (k2 None: one recomputed forward step per step) when some k
    fits, else two levels (two recomputed forward steps per step) with the
    fewest live states.  Raises ValueError if nothing fits."""
    if n_steps <= 0:
        return 1, None
    cap = budget_bytes // max(1, int(state_bytes))
    best = None
    for k in range(1, n_steps + 1):
        m = live_states(n_steps, k)
        if m <= cap and (best is None or m < best[0]):
            best = (m, k)
    if best is not None:
        return best[1], None
    best = None
    for k1 in range(2, n_steps + 1):
        k2 = max(1, int(round(math.sqrt(k1 / 3.0))))
        for kk in (k2 - 1, k2, k2 + 1):
            if 1 <= kk < k1:
                m = live_states(n_steps, k1, kk)
                if best is None or m < best[0]:
                    best = (m, k1, kk)
    if best is None or best[0] > cap:
        raise ValueError(f"no checkpoint schedule of {n_steps} steps fits {budget_bytes} bytes "
                         f"({cap} states of {state_bytes} bytes)")
    return best[1], best[2]


class GHEvolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, gamma, solver, dt, n_steps, checkpoint_every, save_derivatives=None, inner_every=None):
        _push_params(solver, gamma, dt)
        k = max(1, int(checkpoint_every))
        u = u0.detach().clone().contiguous()
        ckpts = []
        for s in range(n_steps):
            if s % k == 0:
                ckpts.append(u.clone())
            solver.step(u, 1)
        k2 = None if inner_every is None or int(inner_every) >= k else max(1, int(inner_every))
        ctx.solver, ctx.dt, ctx.n_steps, ctx.k, ctx.k2 = solver, dt, n_steps, k, k2
        seg = k if k2 is None else k2
        if save_derivatives is None:
            need = 3 * seg * 150 * solver.P * 8
            free, _ = torch.cuda.mem_get_info(u.device)
            save_derivatives = need < 0.5 * free
        ctx.save_derivatives = bool(save_derivatives)
        ctx.gamma = gamma.detach().clone()
        ctx.ckpts = ckpts
        return u

    @staticmethod
    def _reverse_segment(ctx, start, n, lam, g):
        """Reverse sweep over the n steps from state `start` (not modified)."""
        solver = ctx.solver
        states, stages = [start], []
        for j in range(n):
            nxt = states[-1].clone()
            u1, u2 = torch.empty_like(nxt), torch.empty_like(nxt)
            d = (torch.empty(450 * solver.P, dtype=torch.float64, device=nxt.device)
                 if ctx.save_derivatives else None)
            solver.step_stages(nxt, u1, u2, derivs=d)
            stages.append((u1, u2, d))
            if j < n - 1:
                states.append(nxt)
            del nxt
        for j in reversed(range(n)):
            u1, u2, d = stages[j]
            solver.step_vjp_stages(states[j], u1, u2, lam, g_gamma=g, out=lam, derivs=d)
            stages[j] = None
            states[j] = None
            del u1, u2, d

    @staticmethod
    def backward(ctx, grad_u):
        solver, n, k, k2 = ctx.solver, ctx.n_steps, ctx.k, ctx.k2
        _push_params(solver, ctx.gamma, ctx.dt)
        lam = grad_u.detach().contiguous().clone()
        g = torch.zeros(solver.n_inst * 3, dtype=torch.float64, device=lam.device)
        for seg in reversed(range(len(ctx.ckpts))):
            s0 = seg * k
            s1 = min(n, s0 + k)
            if k2 is None:
                GHEvolve._reverse_segment(ctx, ctx.ckpts[seg], s1 - s0, lam, g)
            else:
                # inner checkpoints every k2 steps of this segment
                inner = [ctx.ckpts[seg]]
                u = ctx.ckpts[seg].clone()
                for j in range(s1 - s0 - 1):
                    solver.step(u, 1)
                    if (j + 1) % k2 == 0:
                        inner.append(u.clone())
                del u
                for i in reversed(range(len(inner))):
                    a = s0 + i * k2
                    b = min(s1, a + k2)
                    GHEvolve._reverse_segment(ctx, inner[i], b - a, lam, g)
                    inner[i] = None
            ctx.ckpts[seg] = None
        return lam, g.view(solver.n_inst, 3).cpu(), None, None, None, None, None, None


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


def evolve(u0, gamma, solver, dt, n_steps, checkpoint_every=20, save_derivatives=None, inner_every=None):
    """n_steps RK3 steps with a checkpointed reverse pass.  checkpoint_every:
    outer checkpoint spacing; inner_every (smaller): two-level schedule.
    save_derivatives: keep the stage derivatives of a segment for its reverse
    sweep (None: when they take under half of the free device memory)."""
    return GHEvolve.apply(u0, gamma, solver, dt, n_steps, checkpoint_every, save_derivatives, inner_every)


def evolve_in_budget(u0, gamma, solver, dt, n_steps, budget_bytes=None, save_derivatives=None):
    """evolve with the schedule plan_checkpoints picks for the budget (default:
    80% of the free device memory)."""
    if budget_bytes is None:
        free, _ = torch.cuda.mem_get_info(u0.device)
        budget_bytes = int(0.8 * free)
    k1, k2 = plan_checkpoints(n_steps, u0.numel() * u0.element_size(), budget_bytes)
    return evolve(u0, gamma, solver, dt, n_steps, k1, save_derivatives, k2)


def constraint_norm(u, solver):
    return GHConstraintNorm.apply(u, solver)

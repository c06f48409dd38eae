"""The checkpoint schedules of the reverse pass (paper_1804_09101_amd/autograd.py),
on the CPU with a stand-in solver.

The stand-in steps a linear system u' = M u with SSP-RK3 exactly as the library
orders its calls (step, step_stages, step_vjp_stages), so the gradient of a
linear loss after n steps is known in closed form: lam_0 = R(h M)^T^n lam_n,
with R the RK3 amplification polynomial.  Checked here:
  * one- and two-level schedules give that gradient (to rounding), for
    segment lengths that do and do not divide the step count;
  * the live [50 P] states counted during the backward pass never exceed the
    memory model the planner uses (live_states), and reach it to within a few;
  * the planner's choice for the 2000-step gradient of the 4-instance
    20-shell batch fits 288 GB of HBM, where the best one-level schedule
    does not.
"""

import gc
import math

import numpy as np
import pytest
import torch

from paper_1804_09101_amd import autograd as gha


class _LinearSolver:
    """Stand-in for ghmi.GHSolver: u' = M u, SSP-RK3 with step h."""

    def __init__(self, P, h, seed=0):
        self.P = P
        self.n_inst = 1
        n = 50 * P
        rng = np.random.default_rng(seed)
        self.M = torch.from_numpy(rng.standard_normal((n, n)) / math.sqrt(n))
        self.h = h
        self.peak = 0
        self.counting = False

    def _count(self):
        if not self.counting:
            return
        live = sum(1 for o in gc.get_objects() if torch.is_tensor(o) and o.numel() == 50 * self.P)
        self.peak = max(self.peak, live)

    def set_params(self, gamma, dt):
        pass

    def _f(self, v):
        return self.M @ v

    def step(self, u, n=1):
        for _ in range(n):
            u1 = u + self.h * self._f(u)
            u2 = 0.75 * u + 0.25 * (u1 + self.h * self._f(u1))
            u.copy_(u / 3.0 + 2.0 / 3.0 * (u2 + self.h * self._f(u2)))
        self._count()

    def step_stages(self, u, u1, u2, derivs=None):
        u1.copy_(u + self.h * self._f(u))
        u2.copy_(0.75 * u + 0.25 * (u1 + self.h * self._f(u1)))
        u.copy_(u / 3.0 + 2.0 / 3.0 * (u2 + self.h * self._f(u2)))
        self._count()

    def step_vjp_stages(self, u_n, u1, u2, lam, g_gamma=None, out=None, derivs=None):
        A = self.h * self.M.T
        x = lam.clone()
        r = x + A @ x + A @ (A @ x) / 2.0 + A @ (A @ (A @ x)) / 6.0
        out.copy_(r)
        self._count()


def _exact_gradient(s, lam_n, n):
    A = s.h * s.M.T
    lam = lam_n.clone()
    for _ in range(n):
        lam = lam + A @ lam + A @ (A @ lam) / 2.0 + A @ (A @ (A @ lam)) / 6.0
    return lam


@pytest.mark.parametrize("n,k1,k2", [(12, 12, None), (12, 5, None), (23, 7, 3), (30, 10, 2), (17, 17, 4)])
def test_schedules_give_the_exact_gradient(n, k1, k2):
    s = _LinearSolver(P=2, h=0.05)
    rng = np.random.default_rng(1)
    u0 = torch.from_numpy(rng.standard_normal(100)).requires_grad_(True)
    w = torch.from_numpy(rng.standard_normal(100))
    gamma = torch.zeros(1, 3, dtype=torch.float64)
    un = gha.evolve(u0, gamma, s, np.array([0.05]), n, checkpoint_every=k1, save_derivatives=False,
                    inner_every=k2)
    (un * w).sum().backward()
    want = _exact_gradient(s, w, n)
    assert torch.max(torch.abs(u0.grad - want)) < 1e-12 * torch.max(torch.abs(want))


@pytest.mark.parametrize("n,k1,k2", [(40, 8, None), (60, 20, 3), (45, 15, 4)])
def test_live_states_stay_within_the_model(n, k1, k2):
    gc.collect()
    s = _LinearSolver(P=3, h=0.02)
    u0 = torch.ones(150, dtype=torch.float64).requires_grad_(True)
    gamma = torch.zeros(1, 3, dtype=torch.float64)
    s.counting = True
    s._count()
    base = s.peak
    s.counting = False
    un = gha.evolve(u0, gamma, s, np.array([0.02]), n, checkpoint_every=k1, save_derivatives=False,
                    inner_every=k2)
    s.peak = 0
    s.counting = True
    loss = un.sum()
    del un                      # the loss keeps only the shape of the final state
    loss.backward()
    model = gha.live_states(n, k1, k2)
    used = s.peak - base
    print(f"n {n}, k1 {k1}, k2 {k2}: {used} live states above the baseline, model {model}")
    assert used <= model and used >= model - 4


def test_plan_fits_the_large_batch_gradient_in_hbm():
    """Four 20-shell holes: 5 406 720 points, one state 50 P doubles = 2.16 GB."""
    state = 50 * 5406720 * 8
    hbm = 288 * 10 ** 9
    budget = int(0.9 * hbm)
    n = 2000
    best_one_level = min(gha.live_states(n, k) for k in range(1, n + 1))
    assert best_one_level * state > hbm                  # one level does not fit
    k1, k2 = gha.plan_checkpoints(n, state, budget)
    assert k2 is not None and k2 < k1
    assert gha.live_states(n, k1, k2) * state <= budget
    print(f"plan k1 = {k1}, k2 = {k2}: {gha.live_states(n, k1, k2)} states, "
          f"{gha.live_states(n, k1, k2) * state / 1e9:.0f} GB (one level at best {best_one_level} states)")
    # a small run still uses one level
    assert gha.plan_checkpoints(200, 50 * 86016 * 8, budget)[1] is None
    with pytest.raises(ValueError):
        gha.plan_checkpoints(n, state, 10 * state)

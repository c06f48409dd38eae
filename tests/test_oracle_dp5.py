"""Pins of the oracle's Dormand-Prince 5(4) stepper.

* The tableau, in exact rationals, satisfies the row-sum conditions, all 17
  order conditions up to order five for the advanced weights and the 8 up to
  order four for the embedded ones, and fails an order-five condition with
  the embedded ones (so the error estimate is a true fifth-order term).
* On an ODE with a closed-form solution the global error falls as h^5 and the
  error estimate of one step as h^5.
* The step controller's limits (Numerical Recipes' safe/minscale/maxscale).
* On the domain: a small step on Kerr-Schild data is accepted, grows the step
  and agrees with the SSP-RK3 step; an overlong step on a perturbed state is
  rejected and the state kept; each instance is decided on its own values.
"""

from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import domain, dp5
from paper_1804_09101_amd import configs, inputs

C, A, B, BH = dp5.C, dp5.A, dp5.B, dp5.BHAT


def _a(i, j):
    return A[i][j] if j < len(A[i]) else Fr(0)


def _sum_b(w, f):
    return sum(w[i] * f(i) for i in range(7))


def _ac(i, p=1):
    return sum(_a(i, j) * C[j] ** p for j in range(7))


def _aac(i):
    return sum(_a(i, j) * _ac(j) for j in range(7))


def _conditions(w):
    """The rooted-tree order conditions up to order 5 as (value, required)."""
    return [
        (_sum_b(w, lambda i: 1), Fr(1)),
        (_sum_b(w, lambda i: C[i]), Fr(1, 2)),
        (_sum_b(w, lambda i: C[i] ** 2), Fr(1, 3)),
        (_sum_b(w, lambda i: _ac(i)), Fr(1, 6)),
        (_sum_b(w, lambda i: C[i] ** 3), Fr(1, 4)),
        (_sum_b(w, lambda i: C[i] * _ac(i)), Fr(1, 8)),
        (_sum_b(w, lambda i: _ac(i, 2)), Fr(1, 12)),
        (_sum_b(w, lambda i: _aac(i)), Fr(1, 24)),
        (_sum_b(w, lambda i: C[i] ** 4), Fr(1, 5)),
        (_sum_b(w, lambda i: C[i] ** 2 * _ac(i)), Fr(1, 10)),
        (_sum_b(w, lambda i: C[i] * _ac(i, 2)), Fr(1, 15)),
        (_sum_b(w, lambda i: C[i] * _aac(i)), Fr(1, 30)),
        (_sum_b(w, lambda i: _ac(i) ** 2), Fr(1, 20)),
        (_sum_b(w, lambda i: _ac(i, 3)), Fr(1, 20)),
        (_sum_b(w, lambda i: sum(_a(i, j) * C[j] * _ac(j) for j in range(7))), Fr(1, 40)),
        (_sum_b(w, lambda i: sum(_a(i, j) * _ac(j, 2) for j in range(7))), Fr(1, 60)),
        (_sum_b(w, lambda i: sum(_a(i, j) * _aac(j) for j in range(7))), Fr(1, 120)),
    ]


def test_row_sums_equal_nodes():
    for i in range(1, 7):
        assert sum(A[i]) == C[i]


def test_fifth_order_weights_satisfy_all_conditions_to_order_five():
    assert all(v == r for v, r in _conditions(B))
    assert B[6] == 0 and B[:6] == A[6]      # first-same-as-last


def test_embedded_weights_are_fourth_order_only():
    conds = _conditions(BH)
    assert all(v == r for v, r in conds[:8])
    assert any(v != r for v, r in conds[8:])


def _ode(u, t):
    # u' = cos t + (sin t + 2)^2 - u^2, whose solution through u(0) = 2 is
    # u = sin t + 2 (nonlinear in u, so every stage matters)
    return np.cos(t) + (np.sin(t) + 2.0) ** 2 - u * u


def _integrate(h, T):
    # state (u, t) so the stepper sees an autonomous system
    y = np.array([2.0, 0.0])
    f = lambda v: np.array([_ode(v[0], v[1]), 1.0])
    n = int(round(T / h))
    for _ in range(n):
        y, _ = dp5.stages(y, h, f)
    return y[0] - (np.sin(T) + 2.0)


def test_global_error_is_fifth_order():
    e1, e2 = abs(_integrate(0.1, 2.0)), abs(_integrate(0.05, 2.0))
    rate = np.log2(e1 / e2)
    assert 4.7 < rate < 5.5


def test_error_estimate_is_fifth_order_in_h():
    f = lambda v: np.array([_ode(v[0], v[1]), 1.0])
    y = np.array([2.3, 0.4])
    es = []
    for h in (0.08, 0.04):
        _, k = dp5.stages(y, h, f)
        es.append(abs(dp5.error_vector(k, h)[0]))
    assert 4.5 < np.log2(es[0] / es[1]) < 5.5


def test_controller_limits():
    assert dp5.control(0.0, False) == (True, dp5.MAXSCALE)
    assert dp5.control(1e-12, False) == (True, dp5.MAXSCALE)
    acc, s = dp5.control(1.0, False)
    assert acc and s == pytest.approx(0.9)
    assert dp5.control(1e-3, True) == (True, 1.0)
    acc, s = dp5.control(1.0 + 1e-12, False)
    assert not acc and s == pytest.approx(0.9, rel=1e-9)
    assert dp5.control(1e9, False) == (False, dp5.MINSCALE)


def _pair():
    shells = [(0, 7, 5, 1.8, 3.0), (0, 7, 5, 3.0, 4.5), (1, 7, 3, 1.9, 3.2)]
    holes = [(1.0, 0.0, (0, 0, 1)), (1.0, 0.5, (0, 0, 1))]
    wl = configs.Workload("dp5", shells, holes, [(1.0, -1.0, 1.0)] * 2, [0.01, 0.01], None, 1, None)
    d = domain.Domain([domain.Shell(*s) for s in shells])
    u0, ubg, H, dH = wl.initial_data(d.xyz(), d.offsets)
    return wl, d, u0, ubg, H, dH


def test_smooth_state_is_accepted_and_agrees_with_rk3():
    """On the (coarsely resolved) Kerr-Schild data a small step is accepted,
    the step grows, and the fifth-order step agrees with the independent
    SSP-RK3 step of the same dt far below the size of the step."""
    wl, d, u0, ubg, H, dH = _pair()
    un, acc, dtn, err = d.dp5_attempt(u0, H, dH, ubg, wl.gamma, wl.dt, 1e-8, 1e-8, [False, False])
    assert acc.all() and np.all(err < 1e-2)
    assert np.all(dtn > wl.dt)
    rk3 = d.rk3_step(u0, H, dH, ubg, wl.gamma, wl.dt)
    change = np.max(np.abs(un - u0))
    assert change > 0 and np.max(np.abs(un - rk3)) < 1e-4 * change


def test_overlong_step_is_rejected_per_instance_and_state_kept():
    wl, d, u0, ubg, H, dH = _pair()
    pert = d.to_layout(inputs.smooth_random_field(d.xyz(), 1e-2, 3, 3, 2.0))
    owner = d.instance_of_value()
    u = u0 + np.where(owner == 0, pert, 0.0)
    dt = np.array([0.2, 0.01])
    un, acc, dtn, err = d.dp5_attempt(u, H, dH, ubg, wl.gamma, dt, 1e-10, 1e-10, [False, False])
    assert not acc[0] and acc[1]
    assert np.array_equal(un[owner == 0], u[owner == 0])
    assert dtn[0] < dt[0] and dtn[0] >= dp5.MINSCALE * dt[0]

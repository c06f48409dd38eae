"""Counting scalars do not change the oracle's pointwise results, and the
counts are stable figures for the pointwise kernel's arithmetic."""

import numpy as np

from oracle import flopcount, gh


def _point(seed=0):
    rng = np.random.default_rng(seed)
    u = 0.1 * rng.standard_normal((50, 1))
    eta = np.diag([-1.0, 1.0, 1.0, 1.0])
    for n, (a, b) in enumerate(gh.PAIRS):
        u[n] += eta[a, b]
    return u, 0.1 * rng.standard_normal((3, 50, 1)), rng.standard_normal((4, 1)), rng.standard_normal((4, 4, 1))


def test_counted_rhs_equals_float_rhs():
    u, du, H, dH = _point()
    gam = (0.7, -0.4, 1.3)
    ref = gh.rhs_pointwise(u, du, H, dH, *gam)
    for optimal in (False, True):
        n, out = flopcount.pointwise_rhs_flops(u, du, H, dH, gam, optimal=optimal)
        assert np.max(np.abs(out - ref)) <= 1e-14 * np.max(np.abs(ref))
        assert n > 1000
    n_as_written, _ = flopcount.pointwise_rhs_flops(u, du, H, dH, gam, optimal=False)
    n_opt, _ = flopcount.pointwise_rhs_flops(u, du, H, dH, gam, optimal=True)
    assert n_opt < n_as_written
    # the count is per point: two points cost twice one
    u2, du2, H2, dH2 = (np.concatenate([a, b], axis=-1) for a, b in zip(_point(0), _point(1)))
    n2, _ = flopcount.pointwise_rhs_flops(u2, du2, H2, dH2, gam, optimal=True)
    assert n2 == 2 * n_opt


def test_counted_constraints_equal_float_constraints():
    u, du, H, _ = _point(2)
    ref = gh.constraints_pointwise(u, du, H)
    n, out = flopcount.constraint_flops(u, du, H)
    assert np.max(np.abs(out - ref)) <= 1e-14 * np.max(np.abs(ref))
    assert n > 0

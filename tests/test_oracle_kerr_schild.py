"""Pins of the oracle's own Kerr-Schild generator (oracle/kerr_schild.py), and
of the seeded input generator against it.

The paper's test problem is an isolated Kerr-Schild hole (port overview, eq.
dimensionlessspin) but the paper prints no formulas, so the generator is pinned
by closed forms and invariants that a wrong sign, a dropped factor or a
transposed index would break:
  * hyper-dual arithmetic: exact first and mixed second derivatives of a
    closed-form function;
  * Schwarzschild (chi = 0): metric, lapse, shift, Pi, Phi, the gauge source
    H_a = -(2M/r^2)(1, x_i/r) and its gradient in closed form;
  * Kerr: det psi = -1 (a Kerr-Schild property) and the metric on the spin
    axis in closed form;
  * a boosted hole moves rigidly: d_t q = -v^i d_i q for every field and for H;
  * the seeded input generator (torch.func autodiff, another rotation) equals
    this one to rounding, which pins the inputs both the GPU path and the
    oracle's other tests use.
"""

import math

import numpy as np
import pytest

from oracle import grid
from oracle import kerr_schild as ks
from paper_1804_09101_amd import inputs


def _points(n=5, L=4, r_in=1.9, r_out=6.0):
    return grid.ShellGrid(n, L, r_in, r_out).xyz()


def test_hyperdual_derivatives_closed_form():
    x0, y0 = 1.3, 0.7
    X = ks.HyperDual(np.array([x0]), 1.0, 0.0, 0.0)
    Y = ks.HyperDual(np.array([y0]), 0.0, 1.0, 0.0)
    f = (X * Y).sqrt() / (X + Y) - 3.0 * X * X * Y
    # f = sqrt(xy)/(x+y) - 3x^2 y
    s = math.sqrt(x0 * y0)
    fx = 0.5 * y0 / s / (x0 + y0) - s / (x0 + y0) ** 2 - 6 * x0 * y0
    fy = 0.5 * x0 / s / (x0 + y0) - s / (x0 + y0) ** 2 - 3 * x0 * x0
    # d/dy of fx
    fxy = (0.5 / s - 0.25 * y0 * x0 / s ** 3) / (x0 + y0) - 0.5 * y0 / s / (x0 + y0) ** 2 \
        - 0.5 * x0 / s / (x0 + y0) ** 2 + 2 * s / (x0 + y0) ** 3 - 6 * x0
    assert abs(f.a[0] - (s / (x0 + y0) - 3 * x0 * x0 * y0)) < 1e-15
    assert abs(f.b1[0] - fx) < 1e-14
    assert abs(f.b2[0] - fy) < 1e-14
    assert abs(f.b12[0] - fxy) < 1e-14


def test_schwarzschild_closed_form():
    M = 1.3
    xyz = _points(4, 3, 2.2, 7.0)
    ex = ks.exact_fields(xyz, M=M, chi=0.0)
    x = xyz
    r = np.sqrt(np.sum(x * x, axis=0))
    n = x / r
    Hs = M / r
    # psi_ab = eta + 2 (M/r) l_a l_b, l = (1, n)
    l = np.concatenate([np.ones((1,) + r.shape), n])
    psi = np.zeros((4, 4) + r.shape)
    for a in range(4):
        for b in range(4):
            psi[a, b] = (-1.0 if a == b == 0 else (1.0 if a == b else 0.0)) + 2 * Hs * l[a] * l[b]
    for m, (a, b) in enumerate(ks.PAIRS):
        assert np.max(np.abs(ex["u"][m] - psi[a, b])) < 1e-15
    # Phi_kab = d_k (2M/r l_a l_b): d_k(M/r) = -M n_k/r^2, d_k n_i = (delta_ki - n_k n_i)/r
    for k in range(3):
        for m, (a, b) in enumerate(ks.PAIRS):
            dl = np.zeros((4,) + r.shape)
            for i in range(3):
                dl[i + 1] = ((1.0 if i == k else 0.0) - n[k] * n[i]) / r
            want = 2 * (-M * n[k] / r ** 2) * l[a] * l[b] + 2 * Hs * (dl[a] * l[b] + l[a] * dl[b])
            assert np.max(np.abs(ex["u"][20 + 10 * k + m] - want)) < 1e-14
    # stationary: Pi_ab = N^k Phi_kab / N with N = (1+2M/r)^-1/2, N^k = 2H n^k/(1+2H)
    N = 1.0 / np.sqrt(1 + 2 * Hs)
    shift = 2 * Hs * n / (1 + 2 * Hs)
    for m in range(10):
        want = sum(shift[k] * ex["u"][20 + 10 * k + m] for k in range(3)) / N
        assert np.max(np.abs(ex["u"][10 + m] - want)) < 1e-14
    # gauge source H_a = -(2M/r^2)(1, n_i); d_k H_0 = 4M n_k/r^3;
    # d_k H_i = -2M (delta_ki - 3 n_k n_i)/r^3
    H = ex["H"]
    assert np.max(np.abs(H[0] + 2 * M / r ** 2)) < 1e-14
    for i in range(3):
        assert np.max(np.abs(H[i + 1] + 2 * M * n[i] / r ** 2)) < 1e-14
    dH = ex["dH"].reshape(4, 4, -1)
    assert np.max(np.abs(dH[0])) == 0.0
    for k in range(3):
        assert np.max(np.abs(dH[k + 1, 0] - 4 * M * n[k] / r ** 3)) < 1e-14
        for i in range(3):
            want = -2 * M * ((1.0 if i == k else 0.0) - 3 * n[k] * n[i]) / r ** 3
            assert np.max(np.abs(dH[k + 1, i + 1] - want)) < 1e-14
    assert np.max(np.abs(ex["dtu"])) == 0.0


@pytest.mark.parametrize("chi,axis", [(0.7, (0.2, 0.3, 0.4)), (0.95, (0.0, 0.0, 1.0)), (0.5, (-1.0, 0.2, 0.0))])
def test_kerr_determinant(chi, axis):
    """Kerr-Schild metrics have det psi = -1, since l_a is null for eta."""
    xyz = _points(4, 3, 1.7, 5.0)
    gfun = ks.metric(1.0, chi, axis)
    X = [ks.HyperDual(np.zeros(xyz.shape[1]))] + [ks.HyperDual(xyz[i]) for i in range(3)]
    G = gfun(X)
    g = np.stack([np.stack([G[a][b].a for b in range(4)]) for a in range(4)])
    det = np.linalg.det(np.moveaxis(g, -1, 0))
    assert np.max(np.abs(det + 1.0)) < 1e-13
    assert np.max(np.abs(g - np.swapaxes(g, 0, 1))) < 1e-15


def test_kerr_on_spin_axis_closed_form():
    """On the spin axis (x = y = 0) r = |z|, H = M z/(z^2 + a^2) and
    l = (1, 0, 0, 1), so psi_00 = -1 + 2H, psi_03 = 2H, psi_33 = 1 + 2H."""
    M, chi = 1.0, 0.6
    a = chi * M
    z = np.array([1.2, 2.0, 3.5])
    xyz = np.stack([np.zeros(3), np.zeros(3), z])
    ex = ks.exact_fields(xyz, M=M, chi=chi)
    H = M * z * z ** 2 / (z ** 4 + a * a * z * z)
    assert np.max(np.abs(ex["u"][0] - (-1 + 2 * H))) < 1e-15
    # l_z = z/r = 1 on the axis: psi_33 = 1 + 2H, psi_03 = 2H
    assert np.max(np.abs(ex["u"][9] - (1 + 2 * H))) < 1e-15
    assert np.max(np.abs(ex["u"][3] - 2 * H)) < 1e-15


def test_boosted_hole_moves_rigidly():
    v = np.array([0.25, -0.1, 0.15])
    xyz = _points(4, 3, 2.6, 7.0)
    ex = ks.exact_fields(xyz, M=1.0, chi=0.4, axis=(0.1, 0.5, 0.3), boost=v)
    assert np.max(np.abs(ex["dtu"])) > 1e-2
    adv = sum(v[i] * ex["du"][i] for i in range(3))
    assert np.max(np.abs(ex["dtu"] + adv)) < 1e-14
    dH = ex["dH"].reshape(4, 4, -1)
    assert np.max(np.abs(dH[0] + sum(v[i] * dH[i + 1] for i in range(3)))) < 1e-14


@pytest.mark.parametrize("M,chi,axis,boost", [
    (1.0, 0.7, (0.2, 0.3, 0.4), None),
    (0.6, 0.9, (0.0, 0.0, -1.0), None),
    (1.0, 0.4, (0.1, 0.5, 0.3), (0.25, -0.1, 0.15)),
])
def test_input_generator_matches_oracle_generator(M, chi, axis, boost):
    xyz = _points(5, 4, 1.9 * M, 6.0 * M)
    gf = inputs.kerr_schild_metric(M, chi, axis, boost=boost)
    want = inputs.exact_spacetime(xyz, gf, with_derivs=True)
    got = ks.exact_fields(xyz, M=M, chi=chi, axis=axis, boost=boost)
    for k in ("u", "du", "dtu", "H", "dH"):
        scale = max(1.0, float(np.max(np.abs(want[k]))))
        assert np.max(np.abs(got[k] - want[k])) < 2e-14 * scale, k

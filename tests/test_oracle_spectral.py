"""Pins of the oracle's grid and spectral transforms against closed forms.

Each test compares the oracle with something other than itself: exact integrals
and derivatives of polynomials, explicit low-degree spherical harmonics, and
the chain rule applied to Cartesian polynomials.
"""

import math

import numpy as np
import pytest

from oracle import grid, spectral, domain


@pytest.mark.parametrize("n", [5, 8, 11, 21])
def test_clenshaw_curtis_integrates_polynomials(n):
    xi = grid.cgl_nodes(n)
    w = grid.clenshaw_curtis_weights(n)
    for k in range(n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(w @ xi ** k - exact) < 1e-14 * max(1.0, n)


@pytest.mark.parametrize("n", [5, 9, 16, 33])
def test_radial_derivative_exact_on_polynomials(n):
    rng = np.random.default_rng(n)
    c = rng.standard_normal(n)                      # degree n-1 in xi
    xi = grid.cgl_nodes(n)
    p = np.polynomial.Polynomial(c)
    got = spectral.d_dxi(p(xi))
    want = p.deriv()(xi)
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want)) * n


def test_chebyshev_recurrence_matches_closed_form():
    # T_k'(xi) = k sin(k t)/sin(t) with xi = cos t; T_k'(+-1) = (+-1)^(k+1) k^2
    n = 13
    xi = grid.cgl_nodes(n)
    t = np.arccos(xi)
    for k in range(n):
        got = spectral.d_dxi(np.cos(k * t))
        want = np.empty(n)
        want[1:-1] = k * np.sin(k * t[1:-1]) / np.sin(t[1:-1])
        want[0] = (-1.0) ** (k + 1) * k * k
        want[-1] = k * k
        assert np.max(np.abs(got - want)) < 1e-12 * max(1, k * k)


def test_ylm_low_degree_closed_forms():
    L = 4
    Y, dT, dP = spectral.ylm_tables(L)
    x, _ = grid.gauss_legendre(L)
    th = np.arccos(x)[:, None]
    ph = grid.phi_nodes(L)[None, :]
    s, c = np.sin(th), np.cos(th)
    k0 = 1.0 / math.sqrt(4 * math.pi)
    k1 = math.sqrt(3.0 / (4 * math.pi))
    k2 = math.sqrt(15.0 / (4 * math.pi))
    want = {
        (0, 0): k0 + 0 * th * ph,
        (1, 0): k1 * c + 0 * ph,
        (1, 1): k1 * s * np.cos(ph),
        (1, -1): k1 * s * np.sin(ph),
        (2, 0): math.sqrt(5.0 / (16 * math.pi)) * (3 * c * c - 1) + 0 * ph,
        (2, 1): k2 * s * c * np.cos(ph),
        (2, -1): k2 * s * c * np.sin(ph),
        (2, 2): 0.5 * k2 * s * s * np.cos(2 * ph),
        (2, -2): 0.5 * k2 * s * s * np.sin(2 * ph),
    }
    for (l, m), w in want.items():
        i = spectral.lm_index(l, m)
        assert np.max(np.abs(Y[i] - w)) < 1e-14
    # d/dtheta and d/dphi of Y_11 = k1 sin(th) cos(ph)
    i = spectral.lm_index(1, 1)
    assert np.max(np.abs(dT[i] - k1 * c * np.cos(ph))) < 1e-14
    assert np.max(np.abs(dP[i] + k1 * s * np.sin(ph))) < 1e-14


@pytest.mark.parametrize("L", [3, 7, 15])
def test_ylm_orthonormal_under_quadrature(L):
    sph = spectral.Sphere(L)
    G = np.einsum("aik,bik->ab", sph.Y * sph.W, sph.Y)
    assert np.max(np.abs(G - np.eye(G.shape[0]))) < 1e-13


def _monomials(deg):
    return [(i, j, k) for i in range(deg + 1) for j in range(deg + 1 - i)
            for k in range(deg + 1 - i - j)]


def _poly_and_grad(coef, monos, x, y, z):
    p = sum(c * x ** i * y ** j * z ** k for c, (i, j, k) in zip(coef, monos))
    gx = sum(c * i * x ** max(i - 1, 0) * y ** j * z ** k for c, (i, j, k) in zip(coef, monos) if i)
    gy = sum(c * j * x ** i * y ** max(j - 1, 0) * z ** k for c, (i, j, k) in zip(coef, monos) if j)
    gz = sum(c * k * x ** i * y ** j * z ** max(k - 1, 0) for c, (i, j, k) in zip(coef, monos) if k)
    return p, gx, gy, gz


@pytest.mark.parametrize("L", [3, 6, 11])
def test_angular_derivatives_exact_on_band_limited(L):
    """f = polynomial of degree <= L in the unit vector n is band-limited to l <= L."""
    rng = np.random.default_rng(L)
    monos = _monomials(L)
    coef = rng.standard_normal(len(monos))
    x, _ = grid.gauss_legendre(L)
    th = np.arccos(x)[:, None] + 0 * grid.phi_nodes(L)[None, :]
    ph = grid.phi_nodes(L)[None, :] + 0 * th
    nx, ny, nz = np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)
    f, gx, gy, gz = _poly_and_grad(coef, monos, nx, ny, nz)
    # chain rule: d_theta n = (c_th c_ph, c_th s_ph, -s_th), d_phi n = (-s_th s_ph, s_th c_ph, 0)
    want_t = gx * np.cos(th) * np.cos(ph) + gy * np.cos(th) * np.sin(ph) - gz * np.sin(th)
    want_p = -gx * np.sin(th) * np.sin(ph) + gy * np.sin(th) * np.cos(ph)
    sph = spectral.Sphere(L)
    scale = np.max(np.abs(f)) * (L + 1)
    assert np.max(np.abs(sph.d_dtheta(f) - want_t)) < 1e-12 * scale
    assert np.max(np.abs(sph.d_dphi(f) - want_p)) < 1e-12 * scale


@pytest.mark.parametrize("n_r,L,deg", [(5, 4, 4), (9, 7, 6), (11, 5, 5)])
def test_cartesian_gradient_exact_on_3d_polynomials(n_r, L, deg):
    """A Cartesian polynomial of degree <= min(N_r-1, L) is resolved exactly."""
    d = domain.Domain([domain.Shell(0, n_r, L, 1.3, 2.9)])
    g = d.grids[0]
    rng = np.random.default_rng(deg)
    monos = _monomials(deg)
    coef = rng.standard_normal(len(monos))
    p, gx, gy, gz = _poly_and_grad(coef, monos, g.X, g.Y, g.Z)
    got = d.cartesian_derivs(0, p[None])[:, 0]
    scale = max(np.max(np.abs(gx)), np.max(np.abs(gy)), np.max(np.abs(gz)))
    for k, w in enumerate([gx, gy, gz]):
        assert np.max(np.abs(got[k] - w)) < 1e-11 * scale


@pytest.mark.parametrize("L", [6, 15])
def test_projection_and_filter_factors(L):
    sph = spectral.Sphere(L)
    rng = np.random.default_rng(1)
    u = rng.standard_normal((sph.nth, sph.nph))
    proj = sph.synthesis(sph.analysis(u))
    # SpecToPhys after PhysToSpec is a projection (idempotent), not the identity
    assert np.max(np.abs(sph.synthesis(sph.analysis(proj)) - proj)) < 1e-13
    assert np.max(np.abs(proj - u)) > 1e-2
    sig = spectral.exp_filter_sigma(L, 2.0 / 3.0, 36.0, 8.0)
    # identity on band-limited data with l <= 2L/3
    c = rng.standard_normal((L + 1) ** 2) * (sph.l <= 2 * L / 3)
    low = sph.synthesis(c)
    assert np.max(np.abs(sph.filter(low, sig) - low)) < 1e-13
    # a single top-degree harmonic is multiplied by sigma_L = exp(-36)
    top = sph.Y[spectral.lm_index(L, -L + 1)]
    assert np.max(np.abs(sph.filter(top, sig) - math.exp(-36.0) * top)) < 1e-14
    assert abs(sig[L] - math.exp(-36.0)) < 1e-30
    lmid = int(np.ceil(2 * L / 3 + 1e-9))
    q = (lmid / L - 2.0 / 3.0) * 3.0
    assert abs(sig[lmid] - math.exp(-36.0 * q ** 8)) < 1e-15


def test_volume_weights_give_shell_volume():
    for (n_r, L, a, b) in [(5, 3, 1.0, 2.0), (11, 7, 1.8, 5.0)]:
        g = grid.ShellGrid(n_r, L, a, b)
        vol = np.sum(g.volume_weights())
        assert abs(vol - 4.0 * math.pi / 3.0 * (b ** 3 - a ** 3)) < 1e-12 * vol


@pytest.mark.parametrize("L", [0, 1, 4, 15, 31, 63])
def test_gauss_legendre_rule_is_exact_to_degree_2L_plus_1(L):
    """Closed forms: int_{-1}^{1} x^k dx = 2/(k+1) (k even), 0 (k odd), and the
    nodes are the roots of P_{L+1}, which numpy's leggauss also returns."""
    x, w = grid.gauss_legendre(L)
    assert np.all(np.diff(x) > 0)
    for k in range(2 * L + 2):
        want = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.sum(w * x ** k) - want) < 4e-16 * (L + 1)
    xn, wn = np.polynomial.legendre.leggauss(L + 1)
    assert np.max(np.abs(x - xn)) < 1e-14 and np.max(np.abs(w - wn)) < 1e-13


@pytest.mark.parametrize("L", [15, 31])
def test_angular_derivatives_of_a_constant_vanish_to_rounding(L):
    """d/dtheta and d/dphi of a constant are zero; the transforms must give
    zero to a few ulps of the derivative tables (not the 1e-12 that a
    1e-15 quadrature-weight error or cos(m phi) of a rounded product give)."""
    sph = spectral.Sphere(L)
    one = np.ones((sph.nth, sph.nph))
    assert np.max(np.abs(sph.d_dtheta(one))) < 2e-13
    assert np.max(np.abs(sph.d_dphi(one))) < 2e-13

"""Pins of the oracle's pointwise GH algebra.

The paper does not print the GH equations, so the oracle's transcription is
pinned by properties that a dropped term, a wrong sign or a swapped index would
break:
  P1  exact vacuum solutions: with exact derivatives, the RHS of a rotated
      spinning Kerr-Schild hole vanishes, and the RHS of a boosted hole equals
      its analytic time derivative, for any damping parameters;
  P2  gamma2 damps the three-index constraint: d_t C_iab = -gamma2 C_iab on flat
      space (linear order, via complex-step linearisation);
  P3  the principal symbol has the published characteristic fields as left
      eigenvectors with the published speeds;
  gamma0: a homogeneous constraint violation on flat space decays
      (d_t C_0 = -2 gamma0 C_0, d_t C_i = -gamma0 C_i at linear order);
  the gauge constraint written two ways agrees and vanishes on Kerr-Schild;
  the characteristic projection used at boundaries (char_fields) is, row by
  row, a left eigenvector of that principal symbol with the published speed
  (so its gamma2 term is fixed by the RHS, not only by its own inverse).
The exact spacetimes come from the oracle's own generator
(oracle/kerr_schild.py), not from the seeded input generator.
"""

import math

import numpy as np
import pytest

from oracle import gh, grid
from oracle import kerr_schild as ks

GAMMAS = [(1.0, -1.0, 1.0), (0.3, 0.7, -0.2), (2.5, 0.0, 0.4)]


def _points(n=5, L=4, r_in=1.9, r_out=6.0):
    return grid.ShellGrid(n, L, r_in, r_out).xyz()


@pytest.fixture(scope="module")
def kerr():
    xyz = _points()
    return ks.exact_fields(xyz, M=1.0, chi=0.7, axis=(0.2, 0.3, 0.4))


@pytest.mark.parametrize("gam", GAMMAS)
def test_p1_kerr_schild_rhs_vanishes(kerr, gam):
    ex = kerr
    r = gh.rhs_pointwise(ex["u"], ex["du"], ex["H"], ex["dH"].reshape(4, 4, -1), *gam)
    scale = np.max(np.abs(ex["du"]))
    assert np.max(np.abs(r)) < 1e-13 * max(1.0, scale)


@pytest.mark.parametrize("gam", GAMMAS)
def test_p1_boosted_hole_rhs_is_time_derivative(gam):
    xyz = _points(5, 4, 2.6, 7.0)
    ex = ks.exact_fields(xyz, M=1.0, chi=0.4, axis=(0.1, 0.5, 0.3), boost=(0.25, -0.1, 0.15))
    assert np.max(np.abs(ex["dtu"])) > 1e-2           # genuinely time dependent
    assert np.max(np.abs(ex["dH"].reshape(4, 4, -1)[0])) > 1e-3   # d_t H_a != 0
    r = gh.rhs_pointwise(ex["u"], ex["du"], ex["H"], ex["dH"].reshape(4, 4, -1), *gam)
    assert np.max(np.abs(r - ex["dtu"])) < 1e-13 * max(1.0, np.max(np.abs(ex["du"])))


def test_gauge_constraint_two_forms(kerr):
    ex = kerr
    rng = np.random.default_rng(0)
    u = ex["u"] + 1e-2 * rng.standard_normal(ex["u"].shape)
    psi, Pi, Phi = gh.unpack_fields(u)
    geo = gh.Geometry(psi)
    c1 = gh.gauge_constraint(geo, Pi, Phi, ex["H"])
    c2 = gh.gauge_constraint_from_gamma(geo, Pi, Phi, ex["H"])
    assert np.max(np.abs(c1)) > 1e-3
    assert np.max(np.abs(c1 - c2)) < 1e-14
    psi, Pi, Phi = gh.unpack_fields(ex["u"])
    c0 = gh.gauge_constraint(gh.Geometry(psi), Pi, Phi, ex["H"])
    assert np.max(np.abs(c0)) < 1e-14
    C = gh.constraints_pointwise(ex["u"], ex["du"], ex["H"])
    assert C.shape[0] == 64 and np.max(np.abs(C)) < 1e-13


def _flat(npts):
    u = np.zeros((50, npts), dtype=complex)
    for n, (a, b) in enumerate(gh.PAIRS):
        if a == b:
            u[n] = -1.0 if a == 0 else 1.0
    return u


@pytest.mark.parametrize("g2", [1.0, 0.35])
def test_p2_gamma2_damps_three_index_constraint(g2):
    rng = np.random.default_rng(2)
    npts, h = 6, 1e-30
    u = _flat(npts)
    f = rng.standard_normal((30, npts))
    u[20:50] += 1j * h * f                     # Phi = eps f, psi flat, Pi = 0
    du = np.zeros((3, 50, npts), dtype=complex)
    du[:, 20:50] = 1j * h * rng.standard_normal((3, 30, npts))   # arbitrary d_k Phi
    H = np.zeros((4, npts), dtype=complex)
    dH = np.zeros((4, 4, npts), dtype=complex)
    r = gh.rhs_pointwise(u, du, H, dH, 0.8, 0.6, g2)
    lin = r.imag / h
    # d_t psi vanishes at linear order everywhere, so d_t C_iab = -d_t Phi_iab
    assert np.max(np.abs(lin[0:10])) < 1e-14
    C = -f                                     # C_iab = d_i psi - Phi = -eps f
    dtC = -lin[20:50]
    assert np.max(np.abs(dtC + g2 * C)) < 1e-13


@pytest.mark.parametrize("g0", [1.0, 0.4])
def test_gamma0_damps_homogeneous_gauge_constraint(g0):
    rng = np.random.default_rng(5)
    npts, h = 4, 1e-30
    u = _flat(npts)
    p = rng.standard_normal((10, npts))
    u[10:20] += 1j * h * p                    # Pi = eps p, constant in space
    du = np.zeros((3, 50, npts), dtype=complex)
    H = np.zeros((4, npts), dtype=complex)
    dH = np.zeros((4, 4, npts), dtype=complex)
    r = gh.rhs_pointwise(u, du, H, dH, g0, -0.3, 0.9)
    dPi = gh.sym_unpack(r[10:20].imag / h)
    P = gh.sym_unpack(p)
    # flat space, t^a = (1,0,0,0): C_0 = (Pi_00 + sum_i Pi_ii)/2, C_i = Pi_0i
    def C_of(X):
        return np.stack([0.5 * (X[0, 0] + X[1, 1] + X[2, 2] + X[3, 3]), X[0, 1], X[0, 2], X[0, 3]])
    C = C_of(P)
    dC = C_of(dPi)
    assert np.max(np.abs(dC[0] + 2.0 * g0 * C[0])) < 1e-13
    assert np.max(np.abs(dC[1:] + g0 * C[1:])) < 1e-13


def _principal_matrix(u, s_lo, gam):
    """A(s) with rhs(u, d_k u = s_k v) - rhs(u, 0) = A v (the RHS is affine in du)."""
    npts = u.shape[1]
    H = np.zeros((4, npts))
    dH = np.zeros((4, 4, npts))
    base = gh.rhs_pointwise(u, np.zeros((3, 50, npts)), H, dH, *gam)
    A = np.zeros((npts, 50, 50))
    for f in range(50):
        v = np.zeros((50, npts))
        v[f] = 1.0
        du = s_lo[:, None, :] * v[None]
        A[:, :, f] = (gh.rhs_pointwise(u, du, H, dH, *gam) - base).T
    return A


@pytest.mark.parametrize("gam", GAMMAS)
def test_p3_principal_symbol_characteristic_structure(kerr, gam):
    g0, g1, g2 = gam
    u = kerr["u"][:, :7] + 1e-2 * np.random.default_rng(3).standard_normal((50, 7))
    psi, Pi, Phi = gh.unpack_fields(u)
    geo = gh.Geometry(psi)
    n = np.random.default_rng(4).standard_normal((3, 7))
    s_lo, s_up = gh.unit_normal(geo, n)
    A = _principal_matrix(u, s_lo, gam)
    v_psi, v_0, v_p, v_m = gh.char_speeds(geo, s_lo, g1)
    for p in range(7):
        rows, speeds = [], []
        for m in range(10):
            e = np.zeros(50)
            e[m] = 1.0
            rows.append(e)
            speeds.append(v_psi[p])
            for sign, vs in ((1.0, v_p[p]), (-1.0, v_m[p])):
                e = np.zeros(50)
                e[10 + m] = 1.0
                for k in range(3):
                    e[20 + 10 * k + m] = sign * s_up[k, p]
                e[m] = -g2
                rows.append(e)
                speeds.append(vs)
            for i in range(3):
                e = np.zeros(50)
                e[20 + 10 * i + m] = 1.0
                for k in range(3):
                    e[20 + 10 * k + m] -= s_lo[i, p] * s_up[k, p]
                rows.append(e)
                speeds.append(v_0[p])
        for e, v in zip(rows, speeds):
            # d_t (e.u) = -v d_s (e.u) in the principal part
            assert np.max(np.abs(e @ A[p] + v * e)) < 1e-12


@pytest.mark.parametrize("gam", GAMMAS)
def test_char_fields_are_left_eigenvectors_of_principal_symbol(kerr, gam):
    """Every row of the projection char_fields (the map the boundary treatment
    uses) is a left eigenvector of the RHS's principal symbol A(s) with the
    speed char_speeds gives it: e A = -v e.  The rows are read off by applying
    char_fields to the 50 unit vectors; a sign or a missing gamma2 term in any
    projection breaks the relation for that row."""
    g0, g1, g2 = gam
    npt = 5
    u = kerr["u"][:, 3:3 + npt] + 1e-2 * np.random.default_rng(8).standard_normal((50, npt))
    psi, _, _ = gh.unpack_fields(u)
    geo = gh.Geometry(psi)
    s_lo, s_up = gh.unit_normal(geo, np.random.default_rng(9).standard_normal((3, npt)))
    A = _principal_matrix(u, s_lo, gam)
    v_psi, v_0, v_p, v_m = gh.char_speeds(geo, s_lo, g1)
    eye = np.eye(50)
    for p in range(npt):
        sl = np.repeat(s_lo[:, p:p + 1], 50, axis=1)
        su = np.repeat(s_up[:, p:p + 1], 50, axis=1)
        upsi, u0, up, um = gh.char_fields(eye, sl, su, g2)      # [.., 50]: rows of the map
        groups = [(upsi, v_psi[p]), (up, v_p[p]), (um, v_m[p])] + [(u0[i], v_0[p]) for i in range(3)]
        for rows, v in groups:
            assert np.linalg.matrix_rank(rows, tol=1e-10) >= 3       # not vacuous
            for e in rows:
                assert np.max(np.abs(e @ A[p] + v * e)) < 1e-12
        # the rows span the whole field space (the boundary map can be inverted)
        R = np.concatenate([upsi, u0.reshape(30, 50), up, um])
        assert np.linalg.matrix_rank(R, tol=1e-10) == 50
        # and the reconstruction inverts them on every field vector
        v = np.random.default_rng(p).standard_normal((50, 50))
        back = gh.char_reconstruct(*gh.char_fields(v, sl, su, g2), sl, g2)
        assert np.max(np.abs(back - v)) < 1e-13


def test_characteristic_roundtrip(kerr):
    rng = np.random.default_rng(7)
    v = rng.standard_normal((50, 9))
    psi, _, _ = gh.unpack_fields(kerr["u"][:, :9])
    geo = gh.Geometry(psi)
    s_lo, s_up = gh.unit_normal(geo, rng.standard_normal((3, 9)))
    for g2 in (1.0, -0.6):
        back = gh.char_reconstruct(*gh.char_fields(v, s_lo, s_up, g2), s_lo, g2)
        assert np.max(np.abs(back - v)) < 1e-13


def test_excision_speeds_closed_form():
    """Schwarzschild in Kerr-Schild form at r = 1.8 M with s = -r_hat.

    N = (1+2M/r)^(-1/2), N^i = 2M/r/(1+2M/r) r_hat^i, |r_hat|_g = N, so
    s.N = -(2M/r)/(1+2M/r)/N and the speeds are -s.N, -s.N +- N.
    """
    M, r = 1.0, 1.8
    xyz = np.array([[r], [0.0], [0.0]])
    ex = ks.exact_fields(xyz, M=M, chi=0.0)
    psi, _, _ = gh.unpack_fields(ex["u"])
    geo = gh.Geometry(psi)
    s_lo, _ = gh.unit_normal(geo, np.array([[-1.0], [0.0], [0.0]]))
    _, v0, vp, vm = gh.char_speeds(geo, s_lo, -1.0)
    H = M / r
    N = 1.0 / math.sqrt(1 + 2 * H)
    sN = -(2 * H / (1 + 2 * H)) / N
    assert abs(v0[0] - (-sN)) < 1e-14
    assert abs(vp[0] - (-sN + N)) < 1e-14
    assert abs(vm[0] - (-sN - N)) < 1e-14
    assert abs(vp[0] - 1.4530) < 1e-4 and abs(vm[0] - 0.0765) < 1e-4 and abs(v0[0] - 0.7647) < 1e-4

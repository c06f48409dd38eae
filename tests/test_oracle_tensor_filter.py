"""Pins of the oracle's tensor-coupled angular filter (filtering in total
angular momentum), against facts that do not depend on the oracle's code:

* the orbital generators (r x grad)_k equal the differential operators
  applied on the grid, are antisymmetric, obey the rotation algebra
  [A_x, A_y] = -A_z (cyclic) and sum to -l(l+1) in square on degree l;
  the index generators obey [S_x, S_y] = S_z (cross products);
* J^2 on a vector field of degree l >= 1 has the eigenvalues j(j+1),
  j = l-1, l, l+1, each 2j+1 times (addition of angular momenta);
* closed forms: fields built from Y_lm with the radial unit vector n, the
  tangential gradient, r x grad, delta_ij or n_i n_j have j = l and come out
  multiplied by sigma(l); a constant vector has j = 1;
* the Heaviside filter is a projector (F F = F); F commutes with rotating the
  whole tensor field (positions and indices) by an arbitrary rotation; on the
  time-time components it is the scalar degree filter; with sigma = 1 it is
  the identity on band-limited data.
"""

import numpy as np
import pytest

from oracle import grid, spectral
from oracle import tensor_filter as tf

L = 6


def _sphere(L=L):
    return spectral.Sphere(L)


def _nodes(L=L):
    x, _ = grid.gauss_legendre(L)
    th = np.arccos(x)
    ph = grid.phi_nodes(L)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    n = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)])
    return TH, PH, n


def _ylm_at(L, l, m, n):
    """Real orthonormal Y_lm at unit vectors n[3, ...] (independent evaluation)."""
    th = np.arccos(np.clip(n[2], -1, 1))
    ph = np.arctan2(n[1], n[0])
    P = spectral.assoc_legendre(L, np.cos(th))
    am = abs(m)
    base = spectral.ylm_norm(l, am) * P[l, am]
    if m == 0:
        return base
    return np.sqrt(2.0) * base * (np.cos(am * ph) if m > 0 else np.sin(am * ph))


def _expcheb(L=L):
    # strong, strictly decreasing in j so that every j has its own factor
    return tf.sigma_function("expcheb", L, (0.0, 3.0, 2.0))


def _state(**fields):
    sp = _sphere()
    u = np.zeros((50, 1, sp.nth, sp.nph))
    for k, v in fields.items():
        u[int(k[1:]), 0] = v
    return u


def _pair(a, b):
    return tf.PAIRS.index((min(a, b), max(a, b)))


def test_orbital_generators_algebra():
    A = tf.orbital_generators(L)
    for k in range(3):
        assert np.abs(A[k] + A[k].T).max() < 1e-13
    for a, b, c in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        comm = A[a] @ A[b] - A[b] @ A[a]
        assert np.abs(comm + A[c]).max() < 1e-12
    sq = sum(A[k] @ A[k] for k in range(3))
    lm = spectral.l_of_mode(L)
    assert np.abs(sq + np.diag(lm * (lm + 1.0))).max() < 1e-11


def test_orbital_generators_equal_the_differential_operators_on_the_grid():
    """The ladder-formula matrices equal (r x grad)_k applied to every basis
    function on the grid and analysed back (quadrature rounding only)."""
    for Lg in (3, L, 11):
        A = tf.orbital_generators(Lg)
        G = tf.orbital_generators_on_grid(Lg)
        assert np.abs(A - G).max() < 1e-13 * Lg


def test_index_generators_algebra():
    for dims in ((3,), (4, 4), (3, 4, 4)):
        S = tf.index_generators(dims)
        for a, b, c in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
            assert np.abs(S[a] @ S[b] - S[b] @ S[a] - S[c]).max() == 0.0


def test_vector_spectrum_is_addition_of_angular_momenta():
    for l in range(1, L + 1):
        ev = np.sort(np.linalg.eigvalsh(tf.total_j2(L, l, (3,))))
        want = np.sort(np.concatenate([np.full(2 * j + 1, j * (j + 1.0)) for j in (l - 1, l, l + 1)]))
        assert np.abs(ev - want).max() < 1e-10


def _sig(j):
    return tf._SIGMAS[_expcheb()](j)


@pytest.mark.parametrize("l,m", [(1, 0), (2, 1), (3, -2), (4, 3)])
def test_vector_harmonics_have_j_equal_l(l, m):
    sp = _sphere()
    TH, PH, n = _nodes()
    Y = _ylm_at(L, l, m, n)
    k = spectral.lm_index(l, m)
    dth, dph = sp.dY_dth[k], sp.dY_dph[k]
    e_th = np.stack([np.cos(TH) * np.cos(PH), np.cos(TH) * np.sin(PH), -np.sin(TH)])
    e_ph = np.stack([-np.sin(PH), np.cos(PH), np.zeros_like(PH)])
    grad = e_th * dth + e_ph * dph / np.sin(TH)           # r grad Y
    curl = np.cross(n, grad, axis=0)                       # r x grad Y
    for V in (n * Y, grad, curl):
        u = _state(**{f"f{_pair(0, i + 1)}": V[i] for i in range(3)})
        out = tf.apply(sp, u, _expcheb())
        assert np.abs(out - _sig(l) * u).max() < 1e-12 * np.abs(u).max()


@pytest.mark.parametrize("l,m", [(0, 0), (2, -1), (3, 2)])
def test_rank_two_and_three_fields_have_j_equal_l(l, m):
    sp = _sphere()
    _, _, n = _nodes()
    Y = _ylm_at(L, l, m, n)
    cases = []
    # psi_ij = delta_ij Y and n_i n_j Y
    for T in (np.einsum("ij,...->ij...", np.eye(3), Y), np.einsum("i...,j...->ij...", n, n) * Y):
        cases.append({f"f{_pair(i + 1, j + 1)}": T[i, j] for i in range(3) for j in range(i, 3)})
    # Pi_0i = n_i Y (fields 10..19), Phi_k00 = n_k Y, Phi_kij = n_k n_i n_j Y
    cases.append({f"f{10 + _pair(0, i + 1)}": n[i] * Y for i in range(3)})
    cases.append({f"f{20 + 10 * k}": n[k] * Y for k in range(3)})
    nnn = np.einsum("k...,i...,j...->kij...", n, n, n) * Y
    cases.append({f"f{20 + 10 * k + _pair(i + 1, j + 1)}": nnn[k, i, j]
                  for k in range(3) for i in range(3) for j in range(i, 3)})
    for fields in cases:
        u = _state(**fields)
        out = tf.apply(sp, u, _expcheb())
        assert np.abs(out - _sig(l) * u).max() < 1e-12 * np.abs(u).max(), fields.keys()


def test_constant_vector_has_j_one_and_scalar_part_is_degree_filter():
    sp = _sphere()
    TH, _, _ = _nodes()
    u = _state(**{f"f{_pair(0, 3)}": np.ones_like(TH)})      # psi_0z = 1
    out = tf.apply(sp, u, _expcheb())
    assert np.abs(out - _sig(1) * u).max() < 1e-12
    rng = np.random.default_rng(1)
    c = rng.standard_normal((50, 2, (L + 1) ** 2))
    v = sp.synthesis(c)
    out = tf.apply(sp, v, _expcheb())
    sig_l = np.array([_sig(l) for l in range(L + 1)])
    for f in (0, 10):                                         # psi_00, Pi_00
        assert np.abs(out[f] - sp.filter(v[f], sig_l)).max() < 1e-12


def test_heaviside_is_a_projector_and_unit_sigma_is_identity():
    sp = _sphere()
    rng = np.random.default_rng(2)
    v = sp.synthesis(rng.standard_normal((50, 2, (L + 1) ** 2)))
    h = tf.sigma_function("heaviside", L, (0.5,))
    once = tf.apply(sp, v, h)
    twice = tf.apply(sp, once, h)
    assert np.abs(twice - once).max() < 1e-12 * np.abs(v).max()
    assert np.abs(once - v).max() > 0.1 * np.abs(v).max()
    one = tf.sigma_function("expcheb", L, (10.0, 36.0, 8.0))
    assert np.abs(tf.apply(sp, v, one) - v).max() < 1e-12 * np.abs(v).max()
    for dims in ((4, 4), (3, 4, 4)):
        F = tf.filter_block(L, 3, dims, h)
        assert np.abs(F - F.T).max() < 1e-12


def _rotation(axis, ang):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K


def _rotate_state(c, R, n):
    """(R.u)(n) = R applied to every spatial index of u(R^T n), for band-limited
    u given by its coefficients c[50, N_s]."""
    src = np.einsum("ba,b...->a...", R, n)                  # R^T n
    Ysrc = np.stack([_ylm_at(L, l, m, src) for l in range(L + 1) for m in range(-l, l + 1)])
    vals = np.einsum("fs,s...->f...", c, Ysrc)               # u at R^T n
    R4 = np.eye(4)
    R4[1:, 1:] = R
    out = np.zeros_like(vals)
    full = np.zeros((4, 4) + vals.shape[1:])
    for base in (0, 10):
        for p, (a, b) in enumerate(tf.PAIRS):
            full[a, b] = full[b, a] = vals[base + p]
        rot = np.einsum("ac,bd,cd...->ab...", R4, R4, full)
        for p, (a, b) in enumerate(tf.PAIRS):
            out[base + p] = rot[a, b]
    fullp = np.zeros((3, 4, 4) + vals.shape[1:])
    for k in range(3):
        for p, (a, b) in enumerate(tf.PAIRS):
            fullp[k, a, b] = fullp[k, b, a] = vals[20 + 10 * k + p]
    rot = np.einsum("kq,ac,bd,qcd...->kab...", R, R4, R4, fullp)
    for k in range(3):
        for p, (a, b) in enumerate(tf.PAIRS):
            out[20 + 10 * k + p] = rot[k, a, b]
    return out


def test_filter_commutes_with_rotating_the_tensor_field():
    sp = _sphere()
    _, _, n = _nodes()
    rng = np.random.default_rng(3)
    c = rng.standard_normal((50, (L + 1) ** 2))
    R = _rotation([0.3, -0.5, 0.8], 0.9)
    key = _expcheb()
    v = sp.synthesis(c)[:, None]
    rv = _rotate_state(c, R, n)[:, None]
    left = tf.apply(sp, rv, key)
    fv = tf.apply(sp, v, key)
    right = _rotate_state(sp.analysis(fv[:, 0]), R, n)[:, None]
    assert np.abs(left - right).max() < 1e-11 * np.abs(v).max()
    # the rotation does mix components, so the check is not vacuous
    assert np.abs(rv - v).max() > 0.1 * np.abs(v).max()


def test_domain_applies_the_tensor_filter_per_shell():
    from oracle import domain
    shells = [domain.Shell(0, 3, 4, 1.8, 2.5), domain.Shell(0, 3, 4, 2.5, 3.5), domain.Shell(1, 4, 3, 2.0, 3.0)]
    params = (0.5, 8.0, 4.0)
    d = domain.Domain(shells, filter_params=params, filter_kind=2)
    rng = np.random.default_rng(4)
    u = np.concatenate([d.spheres[s.L].synthesis(rng.standard_normal((50, s.n_r, (s.L + 1) ** 2))).ravel()
                        for s in shells])
    out = d.split(d.apply_filter(u), 50)
    for k, s in enumerate(shells):
        key = tf.sigma_function("expcheb", s.L, params)
        ref = tf.apply(d.spheres[s.L], d.split(u, 50)[k], key)
        assert np.array_equal(out[k], ref)
    assert domain.Domain(shells).filter_kind == 0

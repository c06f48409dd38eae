"""Host-side checks of the C library (no GPU): it loads, exports every symbol of
include/ghmi.h, and its host-built operators equal the oracle's transforms
traced column by column with Kronecker-delta inputs (the paper's tracing
method, eq. Differentiation and the paragraph after it)."""

import os
import re

import numpy as np
import pytest

from oracle import domain, grid, spectral

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ghmi = pytest.importorskip("paper_1804_09101_amd.ghmi")


@pytest.fixture(scope="module")
def lib():
    try:
        return ghmi.load_library()
    except OSError as e:
        pytest.fail(f"libghmi.so not built: {e}")


def test_library_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "ghmi.h")).read()
    declared = set(re.findall(r"^\s*(?:int|const char\*)\s+(gh_\w+)\s*\(", hdr, re.M))
    assert declared == set(ghmi.EXPORTS)
    for name in declared:
        assert hasattr(lib, name)


def _trace(fn, n):
    """Matrix of a linear map by feeding Kronecker deltas (column k = fn(e_k))."""
    cols = []
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        cols.append(fn(e))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("n", [3, 5, 11, 21, 33])
def test_radial_operator_matches_traced_transform(lib, n):
    D = ghmi.host_operator(0, n)
    T = _trace(spectral.d_dxi, n)
    assert np.max(np.abs(D - T)) < 1e-12 * n * n


@pytest.mark.parametrize("L", [1, 3, 5, 7, 15])
def test_angular_operators_match_traced_transforms(lib, L):
    sph = spectral.Sphere(L)
    S = sph.S
    shape = (sph.nth, sph.nph)
    Th = _trace(lambda e: sph.d_dtheta(e.reshape(shape)).ravel(), S)
    Ph = _trace(lambda e: sph.d_dphi(e.reshape(shape)).ravel(), S)
    assert np.max(np.abs(ghmi.host_operator(1, L) - Th)) < 1e-12 * (L + 1)
    assert np.max(np.abs(ghmi.host_operator(2, L) - Ph)) < 1e-12 * (L + 1)
    par = (2.0 / 3.0, 36.0, 8.0)
    sig = spectral.exp_filter_sigma(L, *par)
    Fo = _trace(lambda e: sph.filter(e.reshape(shape), sig).ravel(), S)
    assert np.max(np.abs(ghmi.host_operator(3, L, par) - Fo)) < 1e-13 * (L + 1)


@pytest.mark.parametrize("L", [1, 4, 15, 31])
def test_gemm_operands_are_the_transposed_operators(lib, L):
    """The B operands uploaded for the derivative and filter GEMMs are written
    transposed in place; they must equal the transposes of the operators
    (bitwise: the same sums, only stored elsewhere)."""
    Th, Ph = ghmi.host_operator(1, L), ghmi.host_operator(2, L)
    B = ghmi.host_operator(6, L)
    assert np.array_equal(B, np.hstack([Th.T, Ph.T]))
    par = (2.0 / 3.0, 36.0, 8.0)
    assert np.array_equal(ghmi.host_operator(7, L, par), ghmi.host_operator(3, L, par).T)


@pytest.mark.parametrize("n", [2, 3, 6, 11, 33])
def test_quadrature_matches_oracle(lib, n):
    assert np.max(np.abs(ghmi.host_operator(4, n) - grid.clenshaw_curtis_weights(n))) < 1e-14
    x, w = grid.gauss_legendre(n)
    xw = ghmi.host_operator(5, n)
    assert np.max(np.abs(xw[0] - x)) < 1e-15 and np.max(np.abs(xw[1] - w)) < 1e-14


def test_grid_coords_match_oracle(lib):
    shells = [(0, 7, 5, 1.8, 3.0), (0, 9, 5, 3.0, 6.5), (1, 5, 3, 2.0, 4.0)]
    d = domain.Domain([domain.Shell(*s) for s in shells])
    got = ghmi.grid_coords(shells)
    assert got.shape == (3, d.P)
    assert np.max(np.abs(got - d.xyz())) < 1e-14 * 6.5


def test_host_calls_reject_bad_arguments(lib):
    with pytest.raises(ghmi.GHError):
        ghmi.host_operator(0, 1)
    with pytest.raises(ValueError):
        ghmi.host_operator(9, 3)
    with pytest.raises(ghmi.GHError):
        ghmi.host_operator(1, 64)


def _oracle_coupling(L, kind, params):
    """The oracle's coupling matrix, column by column (unit coefficient vectors)."""
    from oracle import tensor_filter as tf
    key = tf.sigma_function(kind, L, params)
    ns = (L + 1) ** 2
    n = 50 * ns
    M = np.zeros((n, n))
    for col in range(n):
        c = np.zeros((50, ns))
        c[col // ns, col % ns] = 1.0
        M[:, col] = tf.filter_coefficients(c, L, key).ravel()
    return M


def _dense(row_ptr, col, val):
    n = len(row_ptr) - 1
    M = np.zeros((n, n))
    for r in range(n):
        M[r, col[row_ptr[r]:row_ptr[r + 1]]] = val[row_ptr[r]:row_ptr[r + 1]]
    return M


@pytest.mark.parametrize("L,kind,params", [(3, 2, (0.0, 3.0, 2.0)), (5, 2, (2.0 / 3.0, 36.0, 8.0)),
                                           (6, 3, (0.5,))])
def test_tensor_filter_matrix_matches_oracle(lib, L, kind, params):
    """The library's coupling matrix (ladder-operator generators, Newton form
    of sigma(J^2), sparse) equals the oracle's (generators from the grid,
    Lagrange projectors, dense) entry by entry, and so does its transpose."""
    O = _oracle_coupling(L, "expcheb" if kind == 2 else "heaviside", params)
    H = _dense(*ghmi.tensor_filter_matrix(L, kind, params))
    HT = _dense(*ghmi.tensor_filter_matrix(L, kind, params, transpose=True))
    assert np.max(np.abs(H - O)) < 1e-14
    assert np.max(np.abs(HT - O.T)) < 1e-14
    # sparse: at most a few percent of the entries
    assert np.count_nonzero(H) < 0.05 * H.size


def test_tensor_filter_matrix_is_block_diagonal_in_degree_and_tensor(lib):
    L = 7
    row_ptr, col, val = ghmi.tensor_filter_matrix(L, 2, (2.0 / 3.0, 36.0, 8.0))
    ns = (L + 1) ** 2
    deg = np.concatenate([np.full(2 * l + 1, l) for l in range(L + 1)])
    group = np.array([0] * 10 + [1] * 10 + [2] * 30)
    rows = np.repeat(np.arange(len(row_ptr) - 1), np.diff(row_ptr))
    assert np.array_equal(deg[rows % ns], deg[col % ns])
    assert np.array_equal(group[rows // ns], group[col // ns])
    # psi_00 and Pi_00 (time-time components) are the plain degree filter: diagonal
    for f in (0, 10):
        sel = rows // ns == f
        assert np.array_equal(rows[sel], col[sel])


def test_tensor_filter_matrix_rejects_bad_arguments(lib):
    for L, kind, params in ((0, 2, (0.5, 1.0, 2.0)), (64, 2, (0.5, 1.0, 2.0)), (5, 1, (0.5, 1.0, 2.0)),
                            (5, 2, (1.0, 1.0, 2.0)), (5, 2, (0.5, 1.0, 0.0)), (5, 3, (-0.1,))):
        with pytest.raises(ghmi.GHError) as ei:
            ghmi.tensor_filter_matrix(L, kind, params)
        assert ei.value.code == -1

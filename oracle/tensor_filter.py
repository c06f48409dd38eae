"""Tensor-coupled angular filter on I1 x S2 shells -- oracle side.

Test infrastructure only (see package docstring).

The paper (section on spectral filtering on I1 x S2 shells, after the
differentiator benchmarks) filters a tensor field in three steps: every
component is taken to its N_s angular coefficients separately (PhysToSpec, eq.
PhysToSpec), the coefficient array, viewed as an (N_e N_s) x N_r matrix, is
multiplied by one (N_e N_s) x (N_e N_s) matrix that couples the N_e tensor
components (sparse, stored as CSR), and every component is taken back
(SpecToPhys, eq. SpecToPhys).  It profiles two filter functions, Heaviside and
ExpCheb, and says neither what the coupling is nor what the functions'
parameters are.  Readings used here:

* The coupling comes from filtering in total angular momentum.  A tensor field
  on the sphere rotates as a whole: positions and the tensor's spatial indices
  together.  The generator of that rotation about axis k is
      G_k = -(r x grad)_k  (on every component)  +  Sigma_k  (on the indices),
  where Sigma_k acts on each spatial index a as (Sigma_k V)_a = (e_k x V)_a and
  leaves time indices alone.  J^2 = -sum_k G_k^2 has eigenvalues j(j+1) for
  integers j, and the filter is
      F = sum_j sigma(j) P_j,   P_j the projector onto the eigenvalue j(j+1).
  J^2 commutes with the orbital degree l, so F acts within each degree; it
  mixes the components and the orders m of one degree (for a scalar it is the
  plain degree filter sigma(l)).  Fields built from Y_lm and the radial unit
  vector, such as n_i Y_lm, r d_i Y_lm, delta_ij Y_lm or n_i n_j Y_lm, all have
  j = l and are multiplied by sigma(l).
* ExpCheb: sigma(j) = 1 for j/L <= eta_c, else
  exp(-alpha ((j/L - eta_c)/(1 - eta_c))^order), the exponential filter of the
  scalar case in j instead of l.  Heaviside: sigma(j) = 1 for j <= eta_c L,
  else 0.
* The GH state filters as three tensors: psi_ab and Pi_ab (two spacetime
  indices, symmetric) and Phi_iab (a spatial index and a symmetric spacetime
  pair); the stored pair components are expanded to the full index range,
  filtered, and read back.

Here the projectors come from the eigendecomposition of J^2 on dense blocks
(one per degree l and tensor), and the matrices of (r x grad)_k on the real
Y_lm are the angular-momentum ladder matrices carried to the real basis.
"""

import functools
import itertools

import numpy as np

from . import grid as _grid
from . import spectral as _spec

PAIRS = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]
# (first stored field, slot dimensions, number of stored components) of the GH tensors
GH_TENSORS = [(0, (4, 4), 10), (10, (4, 4), 10), (20, (3, 4, 4), 30)]


@functools.lru_cache(maxsize=None)
def orbital_generators(L):
    """Matrices of (r x grad)_k, k = x, y, z, on the real Y_lm coefficients
    (out, in), [3, (L+1)^2, (L+1)^2].

    (r x grad)_k = i L_k with the angular momentum L = -i r x grad, whose
    action on the Condon-Shortley harmonics is the textbook one:
    L_z Y_l^m = m Y_l^m, L_+- Y_l^m = sqrt(l(l+1) - m(m+-1)) Y_l^{m+-1},
    L_x = (L_+ + L_-)/2, L_y = (L_+ - L_-)/(2i).  The real harmonics of this
    package (no Condon-Shortley phase) are Y_l0 = Y_l^0 and, for m > 0,
    sqrt2 Re / Im of (-1)^m Y_l^m; the matrices are carried over by that
    change of basis.  (Applying the differential operators on the grid gives
    the same matrices up to quadrature rounding; a test checks it.)"""
    n = (L + 1) ** 2
    out = np.zeros((3, n, n))
    for l in range(L + 1):
        d = 2 * l + 1
        ms = np.arange(-l, l + 1)
        Lp = np.zeros((d, d))
        for a, m in enumerate(ms[:-1]):
            Lp[a + 1, a] = np.sqrt(l * (l + 1) - m * (m + 1.0))
        Lm = Lp.T
        Lz = np.diag(ms.astype(float))
        Lc = [0.5 * (Lp + Lm), (Lp - Lm) / 2j, Lz]
        # columns: real harmonic (index m + l) in terms of Y_l^m
        C = np.zeros((d, d), dtype=complex)
        C[l, l] = 1.0
        for m in range(1, l + 1):
            ph = (-1.0) ** m
            # sqrt2 Re((-1)^m Y^m) = ((-1)^m Y^m + Y^-m)/sqrt2, since Y^-m = (-1)^m conj(Y^m)
            C[l + m, l + m] = ph / np.sqrt(2.0)
            C[l - m, l + m] = 1.0 / np.sqrt(2.0)
            # sqrt2 Im((-1)^m Y^m) = ((-1)^m Y^m - Y^-m)/(sqrt2 i)
            C[l + m, l - m] = ph / (np.sqrt(2.0) * 1j)
            C[l - m, l - m] = -1.0 / (np.sqrt(2.0) * 1j)
        Cinv = np.linalg.inv(C)
        sl = slice(l * l, (l + 1) * (l + 1))
        for k in range(3):
            M = Cinv @ (1j * Lc[k]) @ C
            out[k, sl, sl] = M.real
    return out


def orbital_generators_on_grid(L):
    """The same matrices from the differential operators applied to every basis
    function on the grid and taken back to coefficients (quadrature):
    (r x grad)_x = -sin(phi) d_theta - cot(theta) cos(phi) d_phi,
    (r x grad)_y =  cos(phi) d_theta - cot(theta) sin(phi) d_phi,
    (r x grad)_z =  d_phi."""
    sp = _spec.Sphere(L)
    x, _ = _grid.gauss_legendre(L)
    th = np.arccos(x)
    ph = _grid.phi_nodes(L)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    cot = np.cos(TH) / np.sin(TH)
    dT, dP = sp.dY_dth, sp.dY_dph
    fields = [-np.sin(PH) * dT - cot * np.cos(PH) * dP,
              np.cos(PH) * dT - cot * np.sin(PH) * dP,
              dP]
    return np.stack([sp.analysis(f).T for f in fields])


def _levi_civita():
    e = np.zeros((3, 3, 3))
    for p in itertools.permutations(range(3)):
        e[p] = np.linalg.det(np.eye(3)[list(p)])
    return e


def index_generators(dims):
    """Sigma_k on a tensor whose index slots have dimension 3 (spatial) or 4
    (spacetime, index 0 = time): sum over slots of e_k x (.) on that slot."""
    eps = _levi_civita()
    n = int(np.prod(dims))
    out = []
    for k in range(3):
        tot = np.zeros((n, n))
        for s, d in enumerate(dims):
            one = np.zeros((d, d))
            sp = eps[:, k, :]                      # (e_k x V)_a = eps_{a k c} V_c
            if d == 3:
                one[:] = sp
            else:
                one[1:, 1:] = sp
            left = int(np.prod(dims[:s]))
            right = int(np.prod(dims[s + 1:]))
            tot += np.kron(np.kron(np.eye(left), one), np.eye(right))
        out.append(tot)
    return out


def total_j2(L, l, dims):
    """J^2 on the block (full tensor component, mode of degree l), component-major."""
    Lk = orbital_generators(L)
    modes = np.where(_spec.l_of_mode(L) == l)[0]
    n = int(np.prod(dims))
    Sig = index_generators(dims)
    J2 = np.zeros((n * len(modes),) * 2)
    for k in range(3):
        G = -np.kron(np.eye(n), Lk[k][np.ix_(modes, modes)]) + np.kron(Sig[k], np.eye(len(modes)))
        J2 -= G @ G
    return J2


def _spin_range(l, dims):
    rank = sum(1 for d in dims if d == 3) + sum(1 for d in dims if d == 4)
    return list(range(max(0, l - rank), l + rank + 1))


@functools.lru_cache(maxsize=None)
def filter_block(L, l, dims, sigma_key):
    """sum_j sigma(j) P_j on the degree-l block.

    The projectors come from the eigendecomposition of the symmetric J^2
    (numpy's eigh): every eigenvalue must be j(j+1) for an integer j, and the
    eigenvectors of j span P_j.  J^2 is block diagonal after a permutation
    (time indices do not rotate, and the real basis splits further), so the
    decomposition is taken on each connected block of its sparsity pattern
    (entries below 1e-12 of the largest are the rounding of exact zeros)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    sigma = _SIGMAS[sigma_key]
    J2 = total_j2(L, l, dims)
    js = _spin_range(l, dims)
    mask = np.abs(J2) > 1e-12 * np.abs(J2).max()
    _, label = connected_components(csr_matrix(mask), directed=False)
    F = np.zeros_like(J2)
    for comp in np.unique(label):
        idx = np.where(label == comp)[0]
        A = J2[np.ix_(idx, idx)]
        lam, V = np.linalg.eigh(0.5 * (A + A.T))
        j = np.rint((np.sqrt(1.0 + 4.0 * np.maximum(lam, 0.0)) - 1.0) / 2.0)
        if np.max(np.abs(lam - j * (j + 1.0))) > 1e-8 * (1.0 + np.max(np.abs(lam))):
            raise ArithmeticError("J^2 has an eigenvalue that is not j(j+1)")
        if not set(j.astype(int)) <= set(js):
            raise ArithmeticError("J^2 has an eigenvalue outside the range of j")
        F[np.ix_(idx, idx)] = (V * np.array([sigma(int(x)) for x in j])) @ V.T
    return F


# ---------------------------------------------------------------------------
# Filter functions (registered so that filter blocks can be cached by key)
# ---------------------------------------------------------------------------
_SIGMAS = {}


def sigma_function(kind, L, params):
    """kind 'expcheb' (eta_c, alpha, order) or 'heaviside' (eta_c,): j -> sigma(j)."""
    key = (kind, L, tuple(float(p) for p in params))
    if key not in _SIGMAS:
        if kind == "expcheb":
            eta_c, alpha, order = key[2]

            def f(j):
                q = j / L if L > 0 else 0.0
                if q <= eta_c:
                    return 1.0
                return float(np.exp(-alpha * ((q - eta_c) / (1.0 - eta_c)) ** order))
        elif kind == "heaviside":
            (eta_c,) = key[2]

            def f(j):
                return 1.0 if j <= eta_c * L else 0.0
        else:
            raise ValueError(kind)
        _SIGMAS[key] = f
    return key


def _expand(dims):
    """Stored (optional first spatial slot) x symmetric pair -> full components."""
    pre = dims[0] if len(dims) == 3 else 1
    nst, nfull = pre * 10, int(np.prod(dims))
    E = np.zeros((nfull, nst))
    R = np.zeros((nst, nfull))
    for i in range(pre):
        for p, (a, b) in enumerate(PAIRS):
            E[(i * 4 + a) * 4 + b, i * 10 + p] = 1.0
            E[(i * 4 + b) * 4 + a, i * 10 + p] = 1.0
            R[i * 10 + p, (i * 4 + a) * 4 + b] = 1.0
    return E, R


def filter_coefficients(c, L, sigma_key):
    """Apply the coupling to a coefficient array c[50, ..., (L+1)^2]."""
    lmode = _spec.l_of_mode(L)
    out = np.zeros_like(c)
    for first, dims, nst in GH_TENSORS:
        E, R = _expand(dims)
        block = c[first:first + nst]                    # [nst, ..., N_s]
        for l in range(L + 1):
            modes = np.where(lmode == l)[0]
            v = block[..., modes]                       # [nst, ..., 2l+1]
            full = np.einsum("fs,s...m->f...m", E, v)   # full components
            F = filter_block(L, l, dims, sigma_key)
            nf, nm = full.shape[0], len(modes)
            F4 = F.reshape(nf, nm, nf, nm)
            filt = np.einsum("amfn,f...n->a...m", F4, full)
            out[first:first + nst][..., modes] = np.einsum("sf,f...m->s...m", R, filt)
    return out


def apply(sphere, u, sigma_key):
    """Filter one shell block u[50, N_r, N_theta, N_phi]: PhysToSpec of every
    component, the component coupling per degree, SpecToPhys."""
    c = sphere.analysis(u)                              # [50, N_r, N_s]
    return sphere.synthesis(filter_coefficients(c, sphere.L, sigma_key))

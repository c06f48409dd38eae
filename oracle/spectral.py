"""Spectral transforms on one shell -- oracle side.

Test infrastructure only (see package docstring).

Follows the paper's description of spectral operations (section "Spectral
Operations: Differentiation and Filtering"): data at collocation points is taken
to spectral coefficients (PhysToSpec, eq. PhysToSpec), the operation acts on the
coefficients (derivative, eq. Deriv; or a filter factor), and the result is taken
back to collocation points (SpecToPhys, eq. SpecToPhys).  On a shell the basis is
T_k(xi) Y_lm(theta, phi) (the series written before eq. DifferentiatorI1S2), with
(L+1)^2 real orthonormal Y_lm on a 2(L+1)^2-point grid, so SpecToPhys after
PhysToSpec is a projection, as the paper notes for SpEC's shells.

Nothing here builds the dense S x S operators the GPU path uses; those are only
ever *traced* from these transforms in the tests (the paper's delta-tracing
method, eq. Differentiation).
"""

import math
import numpy as np

from . import grid as _grid


# ----------------------------------------------------------------------------
# Chebyshev (radial) transforms on CGL points
# ----------------------------------------------------------------------------

def cheb_analysis_matrix(n):
    """PhysToSpec on n CGL points: a_k = sum_j A[k, j] u_j (discrete orthogonality).

    a_k = (2/(n-1)) / c_k * sum_j'' u_j T_k(xi_j), with the end terms of the sum
    halved and c_0 = c_{n-1} = 2, c_k = 1 otherwise.
    """
    T = _grid.cheb_T_at_cgl(n)                # [k, j] = T_k(xi_j)
    half = np.ones(n)
    half[0] = half[-1] = 0.5
    ck = np.ones(n)
    ck[0] = ck[-1] = 2.0
    return (2.0 / (n - 1)) * (T * half[None, :]) / ck[:, None]


def cheb_deriv_coeffs(a):
    """Coefficients of d/dxi of sum_k a_k T_k, by the standard recurrence.

    c_{k-1} b_{k-1} = b_{k+1} + 2 k a_k for k = n-1 .. 1, b_n = b_{n+1} = 0,
    c_0 = 2, c_k = 1 (k>0).  Acts along axis 0.
    """
    n = a.shape[0]
    b = np.zeros_like(a)
    bkp1 = np.zeros_like(a[0])      # b_{k+1}
    bk = np.zeros_like(a[0])        # b_k
    for k in range(n - 1, 0, -1):
        bkm1 = bkp1 + 2.0 * k * a[k]
        b[k - 1] = bkm1
        bkp1, bk = bk, bkm1
    b[0] = 0.5 * b[0]
    return b


def d_dxi(u):
    """d/dxi along axis 0 of CGL samples: PhysToSpec, recurrence, SpecToPhys."""
    n = u.shape[0]
    A = cheb_analysis_matrix(n)
    T = _grid.cheb_T_at_cgl(n)                # SpecToPhys: u_j = sum_k T[k, j] a_k
    a = np.tensordot(A, u, axes=(1, 0))
    b = cheb_deriv_coeffs(a)
    return np.tensordot(T.T, b, axes=(1, 0))


# ----------------------------------------------------------------------------
# Real orthonormal spherical harmonics on the Gauss-Legendre x uniform grid
# ----------------------------------------------------------------------------

def lm_index(l, m):
    return l * l + l + m


def assoc_legendre(L, x):
    """Unnormalised P_l^m(x), 0 <= m <= l <= L, no Condon-Shortley phase.

    P_m^m = (2m-1)!! (1-x^2)^{m/2};  P_{m+1}^m = x (2m+1) P_m^m;
    (l-m) P_l^m = x (2l-1) P_{l-1}^m - (l+m-1) P_{l-2}^m.
    Returns array [L+1 (l), L+1 (m), len(x)] (zero for m > l).
    """
    x = np.asarray(x, dtype=float)
    s = np.sqrt(1.0 - x * x)
    P = np.zeros((L + 1, L + 1) + x.shape)
    for m in range(L + 1):
        dfact = 1.0
        for j in range(1, 2 * m, 2):
            dfact *= j
        P[m, m] = dfact * s ** m
        if m + 1 <= L:
            P[m + 1, m] = x * (2 * m + 1) * P[m, m]
        for l in range(m + 2, L + 1):
            P[l, m] = (x * (2 * l - 1) * P[l - 1, m] - (l + m - 1) * P[l - 2, m]) / (l - m)
    return P


def ylm_norm(l, m):
    """N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), from exact integer factorials."""
    return math.sqrt((2 * l + 1) / (4.0 * math.pi)
                     * (math.factorial(l - m) / math.factorial(l + m)))


def ylm_tables(L):
    """Y_lm, dY_lm/dtheta, dY_lm/dphi at the shell's angular nodes.

    Real basis: Y_l0 = N P_l, Y_lm = sqrt2 N P_l^m cos(m phi) (m>0),
    Y_l,-m = sqrt2 N P_l^m sin(m phi) (m>0).  dP_l^m/dtheta is taken from
    (x^2-1) dP_l^m/dx = l x P_l^m - (l+m) P_{l-1}^m with d/dtheta = -sin(theta) d/dx.
    Returns three arrays [(L+1)^2, N_theta, N_phi].
    """
    x, _ = _grid.gauss_legendre(L)
    phi = _grid.phi_nodes(L)
    s = np.sqrt(1.0 - x * x)
    P = assoc_legendre(L, x)
    nm = (L + 1) ** 2
    Y = np.zeros((nm, len(x), len(phi)))
    dT = np.zeros_like(Y)
    dP = np.zeros_like(Y)
    for l in range(L + 1):
        for m in range(0, l + 1):
            Plm = P[l, m]
            Plm1 = P[l - 1, m] if l - 1 >= m else np.zeros_like(x)
            dPlm = (l * x * Plm - (l + m) * Plm1) / s       # dP_l^m / dtheta
            nrm = ylm_norm(l, m)
            if m == 0:
                Y[lm_index(l, 0)] = (nrm * Plm)[:, None] * np.ones_like(phi)[None, :]
                dT[lm_index(l, 0)] = (nrm * dPlm)[:, None] * np.ones_like(phi)[None, :]
                dP[lm_index(l, 0)] = 0.0
            else:
                c, sn = _grid.azimuthal_factors(L, m)
                f = math.sqrt(2.0) * nrm
                Y[lm_index(l, m)] = f * np.outer(Plm, c)
                Y[lm_index(l, -m)] = f * np.outer(Plm, sn)
                dT[lm_index(l, m)] = f * np.outer(dPlm, c)
                dT[lm_index(l, -m)] = f * np.outer(dPlm, sn)
                dP[lm_index(l, m)] = -m * f * np.outer(Plm, sn)
                dP[lm_index(l, -m)] = m * f * np.outer(Plm, c)
    return Y, dT, dP


def l_of_mode(L):
    """Degree l of each mode index, shape [(L+1)^2]."""
    return np.concatenate([np.full(2 * l + 1, l) for l in range(L + 1)])


def quad_weights_sphere(L):
    """Angular quadrature weights [N_theta, N_phi]: w_GL(theta) * 2 pi / N_phi."""
    _, w = _grid.gauss_legendre(L)
    nphi = 2 * (L + 1)
    return np.outer(w, np.full(nphi, 2.0 * math.pi / nphi))


class Sphere:
    """Transforms for one L: PhysToSpec (quadrature analysis) and SpecToPhys."""

    def __init__(self, L):
        self.L = L
        self.Y, self.dY_dth, self.dY_dph = ylm_tables(L)
        self.W = quad_weights_sphere(L)
        self.nth, self.nph = self.W.shape
        self.S = self.nth * self.nph
        self.l = l_of_mode(L)

    def analysis(self, u):
        """u[..., N_theta, N_phi] -> coefficients [..., (L+1)^2]."""
        return np.einsum("...ik,mik->...m", u * self.W, self.Y)

    def synthesis(self, c, table=None):
        t = self.Y if table is None else table
        return np.einsum("...m,mik->...ik", c, t)

    def d_dtheta(self, u):
        return self.synthesis(self.analysis(u), self.dY_dth)

    def d_dphi(self, u):
        return self.synthesis(self.analysis(u), self.dY_dph)

    def filter(self, u, sigma_l):
        """Multiply each degree-l coefficient by sigma_l[l] and go back."""
        c = self.analysis(u) * sigma_l[self.l]
        return self.synthesis(c)


def exp_filter_sigma(L, eta_c, alpha, order):
    """Angular exponential filter factors sigma_l, l = 0..L.

    sigma_l = 1 for l/L <= eta_c, else exp(-alpha ((l/L - eta_c)/(1 - eta_c))^order).
    (The paper names Heaviside and exponential filters on S2 but gives no
    parameters; the defaults of the evolutions here are eta_c = 2/3, alpha = 36,
    order = 8, i.e. the top third of the degrees is damped.)
    """
    l = np.arange(L + 1, dtype=float)
    if L == 0:
        return np.ones(1)
    q = l / L
    out = np.ones(L + 1)
    hi = q > eta_c
    out[hi] = np.exp(-alpha * ((q[hi] - eta_c) / (1.0 - eta_c)) ** order)
    return out

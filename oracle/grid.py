"""Collocation grid of one spherical shell (topology I1 x S2) -- oracle side.

Test infrastructure only (see package docstring).

The paper's shell differentiator (section "Spectral Operations: Differentiation
and Filtering", eq. DifferentiatorI1S2) works on data u(r_k, theta_l, phi_m) with
a Chebyshev basis in a rescaled radius and Y_lm on the sphere; it does not name
the collocation points.  Readings used here:

* radius: Chebyshev-Gauss-Lobatto points xi_j = -cos(pi j/(N_r-1)), mapped
  affinely r = (r_in+r_out)/2 + xi (r_out-r_in)/2, so neighbouring shells share
  the interface radius;
* polar angle: theta_i = arccos(x_i), x_i the N_theta = L+1 Gauss-Legendre
  nodes in increasing x;
* azimuth: phi_k = 2 pi k / N_phi with N_phi = 2(L+1)  (the paper's grids use
  N_phi = 2 N_theta).
"""

import functools
import math

import mpmath
import numpy as np


def cgl_nodes(n):
    """Chebyshev-Gauss-Lobatto nodes on [-1, 1], increasing (xi_0 = -1)."""
    if n < 2:
        raise ValueError("need at least 2 radial points")
    j = np.arange(n)
    return -np.cos(np.pi * j / (n - 1))


def _legendre_and_derivative(n, x):
    """P_n(x) and P_n'(x) by the three-term recurrence (x an mpmath number)."""
    p0, p1 = mpmath.mpf(1), x
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    if n == 0:
        return mpmath.mpf(1), mpmath.mpf(0)
    return p1, n * (x * p1 - p0) / (x * x - 1)


@functools.lru_cache(maxsize=None)
def _gauss_legendre_mp(n, dps=40):
    with mpmath.workdps(dps):
        xs, ws = [], []
        for i in range(n):
            x = mpmath.cos(mpmath.pi * (i + mpmath.mpf(3) / 4) / (n + mpmath.mpf(1) / 2))
            for _ in range(200):
                p, dp = _legendre_and_derivative(n, x)
                dx = p / dp
                x -= dx
                if abs(dx) < mpmath.mpf(10) ** (5 - dps):
                    break
            _, dp = _legendre_and_derivative(n, x)
            xs.append(x)
            ws.append(2 / ((1 - x * x) * dp * dp))
        order = sorted(range(n), key=lambda i: xs[i])
        return (tuple(float(xs[i]) for i in order), tuple(float(ws[i]) for i in order))


def gauss_legendre(L):
    """Gauss-Legendre nodes x_i (increasing) and weights for N_theta = L+1.

    The roots of P_{L+1} are found by Newton's method in 40-digit arithmetic
    and the weights are 2 / ((1 - x^2) P'_{L+1}(x)^2), both rounded once to
    double.  (numpy's leggauss weights carry errors near 1e-15, which the
    Y_lm analysis turns into 1e-14 errors in the coefficients at L = 31.)
    """
    x, w = _gauss_legendre_mp(L + 1)
    return np.array(x), np.array(w)


def phi_nodes(L):
    nphi = 2 * (L + 1)
    return 2.0 * np.pi * np.arange(nphi) / nphi


def azimuthal_factors(L, m):
    """cos(m phi_k), sin(m phi_k) at the N_phi = 2(L+1) uniform nodes.

    Evaluated at the exactly reduced angle 2 pi ((m k) mod N_phi) / N_phi, so
    the error does not grow with m k as it does for cos(m * phi_k) with a
    rounded product (about 2e-14 at m k ~ 2000).
    """
    nphi = 2 * (L + 1)
    ang = 2.0 * np.pi * ((m * np.arange(nphi)) % nphi) / nphi
    return np.cos(ang), np.sin(ang)


def cheb_T(n, xi):
    """T_k(xi) for k < n, as an array [k, len(xi)] (definition T_k = cos(k acos xi))."""
    xi = np.asarray(xi, dtype=float)
    ang = np.arccos(np.clip(xi, -1.0, 1.0))
    return np.cos(np.outer(np.arange(n), ang))


def cheb_T_at_cgl(n):
    """T_k(xi_j) at the n CGL nodes, [k, j], from the exact node angle.

    xi_j = cos(pi (N - j)/N) with N = n - 1, so T_k(xi_j) = cos(pi m / N) with
    m = k (N - j) mod 2N.  Same values as cheb_T(n, cgl_nodes(n)) but without the
    rounding of arccos of a rounded node, which the derivative recurrence
    would amplify by ~N^2.
    """
    N = n - 1
    k = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    m = (k * (N - j)) % (2 * N)
    return np.cos(np.pi * m / N)


def clenshaw_curtis_weights(n):
    """Quadrature weights on the CGL nodes: integrate the Chebyshev interpolant.

    w_j = sum_k (int_{-1}^{1} T_k) * A[k, j], where A is the CGL analysis map
    (PhysToSpec) and int T_k = 2/(1-k^2) for even k, 0 for odd k.
    """
    from .spectral import cheb_analysis_matrix
    A = cheb_analysis_matrix(n)
    k = np.arange(n)
    intT = np.zeros(n)
    even = k % 2 == 0
    intT[even] = 2.0 / (1.0 - k[even].astype(float) ** 2)
    return intT @ A


class ShellGrid:
    """Coordinates of the N_r x N_theta x N_phi collocation points of one shell."""

    def __init__(self, n_r, L, r_in, r_out):
        if not (r_out > r_in > 0):
            raise ValueError("need 0 < r_in < r_out")
        self.n_r, self.L = int(n_r), int(L)
        self.r_in, self.r_out = float(r_in), float(r_out)
        self.n_th = self.L + 1
        self.n_ph = 2 * (self.L + 1)
        self.S = self.n_th * self.n_ph
        self.xi = cgl_nodes(self.n_r)
        self.r = 0.5 * (self.r_in + self.r_out) + 0.5 * (self.r_out - self.r_in) * self.xi
        self.x_gl, self.w_gl = gauss_legendre(self.L)
        self.theta = np.arccos(self.x_gl)
        self.phi = phi_nodes(self.L)
        R, TH, PH = np.meshgrid(self.r, self.theta, self.phi, indexing="ij")
        self.R, self.TH, self.PH = R, TH, PH
        self.X = R * np.sin(TH) * np.cos(PH)
        self.Y = R * np.sin(TH) * np.sin(PH)
        self.Z = R * np.cos(TH)

    @property
    def npts(self):
        return self.n_r * self.S

    def xyz(self):
        """Cartesian coordinates, shape [3, N_r*S] in [r][theta][phi] order."""
        return np.stack([self.X.ravel(), self.Y.ravel(), self.Z.ravel()])

    def volume_weights(self):
        """Weights w_p of the volume quadrature on this shell, shape [N_r, S].

        Clenshaw-Curtis in xi times the radial Jacobian (r_out-r_in)/2 times
        r^2, times Gauss-Legendre in cos(theta) times 2 pi / N_phi in phi.
        """
        wr = clenshaw_curtis_weights(self.n_r) * 0.5 * (self.r_out - self.r_in) * self.r ** 2
        wa = np.repeat(self.w_gl, self.n_ph) * (2.0 * math.pi / self.n_ph)
        return np.outer(wr, wa)

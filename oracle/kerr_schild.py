"""Exact Kerr-Schild spacetimes with exact derivatives -- oracle side.

Test infrastructure only (see package docstring).

The paper's test problem is an isolated Kerr black hole in Kerr-Schild
coordinates (port overview; mass m and dimensionless spin, eq.
dimensionlessspin).  The paper does not write the metric; the standard form is
  psi_ab = eta_ab + 2 H l_a l_b,   eta = diag(-1, 1, 1, 1),   a = chi M,
  r^2 = (rho^2 - a^2)/2 + sqrt((rho^2 - a^2)^2/4 + a^2 z^2),
  H = M r^3 / (r^4 + a^2 z^2),
  l_a = (1, (r x + a y)/(r^2 + a^2), (r y - a x)/(r^2 + a^2), z/r)
for the spin along z.  Another spin axis is reached by rotating the spatial
frame; a moving hole by a Lorentz boost of the coordinates.

This module is the oracle's own generator, independent of the seeded input
generator that feeds the GPU path: derivatives are exact by hyper-dual numbers
(two nilpotent units e1, e2 with e1 e2 != 0, so one evaluation carries a value,
two first derivatives and the mixed second derivative), the frame for a tilted
spin is built from cross products (a different rotation from the input
generator's, equal up to a turn about the axis, which Kerr does not see), and
everything is plain NumPy.

Quantities returned at Cartesian points X = (t, x, y, z):
  u [50]   first-order fields psi_ab, Pi_ab = -(d_t psi_ab - N^i Phi_iab)/N,
           Phi_iab = d_i psi_ab (symmetric pairs 00,01,02,03,11,12,13,22,23,33);
  du [3,50] exact spatial derivatives d_k u;  dtu [50] exact d_t u;
  H [4]    gauge source H_a = -psi^bc Gamma_abc of the exact metric;
  dH [16]  d_a H_b, row a*4 + b (a = 0 is the time derivative).
"""

import math

import numpy as np

PAIRS = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]


class HyperDual:
    """a + b1 e1 + b2 e2 + b12 e1 e2 with e1^2 = e2^2 = 0 (arrays of points)."""

    __slots__ = ("a", "b1", "b2", "b12")

    def __init__(self, a, b1=0.0, b2=0.0, b12=0.0):
        self.a, self.b1, self.b2, self.b12 = a, b1, b2, b12

    @staticmethod
    def lift(x):
        return x if isinstance(x, HyperDual) else HyperDual(x)

    def __add__(self, o):
        o = HyperDual.lift(o)
        return HyperDual(self.a + o.a, self.b1 + o.b1, self.b2 + o.b2, self.b12 + o.b12)

    __radd__ = __add__

    def __neg__(self):
        return HyperDual(-self.a, -self.b1, -self.b2, -self.b12)

    def __sub__(self, o):
        return self + (-HyperDual.lift(o))

    def __rsub__(self, o):
        return HyperDual.lift(o) - self

    def __mul__(self, o):
        o = HyperDual.lift(o)
        return HyperDual(self.a * o.a, self.a * o.b1 + self.b1 * o.a, self.a * o.b2 + self.b2 * o.a,
                         self.a * o.b12 + self.b1 * o.b2 + self.b2 * o.b1 + self.b12 * o.a)

    __rmul__ = __mul__

    def _apply(self, f0, f1, f2):
        """f(x) for f with value f0, first derivative f1, second f2 at x = self.a."""
        return HyperDual(f0, f1 * self.b1, f1 * self.b2, f1 * self.b12 + f2 * self.b1 * self.b2)

    def recip(self):
        inv = 1.0 / self.a
        return self._apply(inv, -inv * inv, 2.0 * inv * inv * inv)

    def __truediv__(self, o):
        return self * HyperDual.lift(o).recip()

    def __rtruediv__(self, o):
        return HyperDual.lift(o) * self.recip()

    def sqrt(self):
        s = np.sqrt(self.a)
        return self._apply(s, 0.5 / s, -0.25 / (s * self.a))


def spin_frame(axis):
    """Proper orthonormal frame R (columns e1, e2, n) with n = axis/|axis|."""
    n = np.asarray(axis, dtype=float)
    n = n / math.sqrt(float(n @ n))
    # the coordinate axis least aligned with n gives a well-conditioned cross product
    k = int(np.argmin(np.abs(n)))
    c = np.zeros(3)
    c[k] = 1.0
    e1 = np.cross(c, n)
    e1 /= math.sqrt(float(e1 @ e1))
    e2 = np.cross(n, e1)
    return np.stack([e1, e2, n], axis=1)


def boost_matrix(v):
    """Lorentz boost Lambda^a_b to the frame moving with velocity v (c = 1)."""
    v = np.asarray(v, dtype=float)
    v2 = float(v @ v)
    B = np.eye(4)
    if v2 == 0.0:
        return B
    gam = 1.0 / math.sqrt(1.0 - v2)
    B[0, 0] = gam
    for i in range(3):
        B[0, i + 1] = B[i + 1, 0] = -gam * v[i]
        for j in range(3):
            B[i + 1, j + 1] = (1.0 if i == j else 0.0) + (gam - 1.0) * v[i] * v[j] / v2
    return B


def _linear(Mx, X):
    """Y^a = M^a_b X^b for a 4x4 float matrix and a list of 4 hyper-duals."""
    return [sum((Mx[a, b] * X[b] for b in range(4)), HyperDual(0.0)) for a in range(4)]


def _metric_spin_z(M, a, X):
    """Kerr-Schild metric components [4][4] (hyper-dual) for spin along z."""
    x, y, z = X[1], X[2], X[3]
    q = 0.5 * (x * x + y * y + z * z - a * a)
    r2 = q + (q * q + a * a * z * z).sqrt()
    r = r2.sqrt()
    Hs = M * r * r2 / (r2 * r2 + a * a * z * z)
    den = r2 + a * a
    l = [HyperDual(1.0), (r * x + a * y) / den, (r * y - a * x) / den, z / r]
    g = [[None] * 4 for _ in range(4)]
    for i in range(4):
        for j in range(4):
            eta = (-1.0 if i == 0 else 1.0) if i == j else 0.0
            g[i][j] = eta + 2.0 * Hs * l[i] * l[j]
    return g


def metric(M, chi, axis=(0.0, 0.0, 1.0), boost=None):
    """g(X) -> [4][4] hyper-duals for a (rotated, optionally boosted) Kerr-Schild hole."""
    a = float(chi) * float(M)
    Lam = np.eye(4)
    Lam[1:, 1:] = spin_frame(axis)
    B = None if boost is None else boost_matrix(boost)

    def g_rot(X):
        # tensor transform: g'_ab(X) = Lam_ac Lam_bd g_cd(Lam^T X)
        g0 = _metric_spin_z(M, a, _linear(Lam.T, X))
        return [[sum((Lam[p, c] * Lam[q, d] * g0[c][d] for c in range(4) for d in range(4)),
                     HyperDual(0.0)) for q in range(4)] for p in range(4)]

    if B is None:
        return g_rot

    def g_boost(X):
        # coordinates X' = B X: g_ab(X) = B_ca B_db g'_cd(B X)
        g0 = g_rot(_linear(B, X))
        return [[sum((B[c, p] * B[d, q] * g0[c][d] for c in range(4) for d in range(4)),
                     HyperDual(0.0)) for q in range(4)] for p in range(4)]

    return g_boost


# -- outer derivative by first-order dual numbers on matrices -----------------

def _dinv(A, dA):
    """Inverse of A + e dA for stacks of matrices [..., n, n]: A^-1 - e A^-1 dA A^-1."""
    Ai = np.linalg.inv(A)
    return Ai, -Ai @ dA @ Ai


def _fields_and_gauge(g, dg, gk, dgk):
    """From g_ab [P,4,4], d_c g_ab [P,4(c),4,4] and their derivatives along one
    direction (gk, dgk), the first-order fields u [P,50], the gauge source
    H [P,4] and their derivatives along that direction."""
    ginv3, ginv3_k = _dinv(g[:, 1:, 1:], gk[:, 1:, 1:])
    b, bk = g[:, 0, 1:], gk[:, 0, 1:]                      # psi_0i
    shift = np.einsum("pij,pj->pi", ginv3, b)
    shift_k = np.einsum("pij,pj->pi", ginv3_k, b) + np.einsum("pij,pj->pi", ginv3, bk)
    lap2 = np.einsum("pi,pi->p", shift, b) - g[:, 0, 0]
    lap2_k = np.einsum("pi,pi->p", shift_k, b) + np.einsum("pi,pi->p", shift, bk) - gk[:, 0, 0]
    lapse = np.sqrt(lap2)
    lapse_k = 0.5 * lap2_k / lapse
    Phi, Phi_k = dg[:, 1:], dgk[:, 1:]                     # [P,i,a,b]
    num = dg[:, 0] - np.einsum("pi,piab->pab", shift, Phi)
    num_k = (dgk[:, 0] - np.einsum("pi,piab->pab", shift_k, Phi)
             - np.einsum("pi,piab->pab", shift, Phi_k))
    Pi = -num / lapse[:, None, None]
    Pi_k = -num_k / lapse[:, None, None] + num * (lapse_k / lap2)[:, None, None]

    def pack(psi, Pi_, Phi_):
        comps = [psi[:, a, b] for (a, b) in PAIRS] + [Pi_[:, a, b] for (a, b) in PAIRS]
        for i in range(3):
            comps += [Phi_[:, i, a, b] for (a, b) in PAIRS]
        return np.stack(comps, axis=1)

    u = pack(g, Pi, Phi)
    u_k = pack(gk, Pi_k, Phi_k)
    # Gamma_abc = 1/2 (d_b g_ac + d_c g_ab - d_a g_bc); dg index order [c(deriv), a, b]
    def gam(d):
        return 0.5 * (np.einsum("pbac->pabc", d) + np.einsum("pcab->pabc", d)
                      - np.einsum("pabc->pabc", d))
    G, G_k = gam(dg), gam(dgk)
    ginv4, ginv4_k = _dinv(g, gk)
    H = -np.einsum("pbc,pabc->pa", ginv4, G)
    H_k = -np.einsum("pbc,pabc->pa", ginv4_k, G) - np.einsum("pbc,pabc->pa", ginv4, G_k)
    return u, u_k, H, H_k


def exact_fields(xyz, M=1.0, chi=0.0, axis=(0.0, 0.0, 1.0), boost=None, t=0.0):
    """Fields, exact derivatives and gauge source of a Kerr-Schild hole at xyz [3, P].

    Returns a dict of float64 arrays: u [50,P], du [3,50,P], dtu [50,P],
    H [4,P], dH [16,P] (row a*4+b = d_a H_b).
    """
    xyz = np.asarray(xyz, dtype=float)
    P = xyz.shape[1]
    gfun = metric(M, chi, axis, boost)
    coords = [np.full(P, float(t)), xyz[0], xyz[1], xyz[2]]
    u = du = H = None
    du = np.zeros((4, 50, P))
    dH = np.zeros((4, 4, P))
    for k in range(4):                   # outer derivative direction (0 = time)
        g = np.zeros((P, 4, 4))
        gk = np.zeros((P, 4, 4))
        dg = np.zeros((P, 4, 4, 4))
        dgk = np.zeros((P, 4, 4, 4))
        for c in range(4):               # inner derivative direction
            X = [HyperDual(coords[m], 1.0 if m == k else 0.0, 1.0 if m == c else 0.0, 0.0)
                 for m in range(4)]
            G = gfun(X)
            for p in range(4):
                for q in range(4):
                    e = G[p][q]
                    g[:, p, q] = e.a
                    gk[:, p, q] = e.b1
                    dg[:, c, p, q] = e.b2
                    dgk[:, c, p, q] = e.b12
        uu, uk, HH, Hk = _fields_and_gauge(g, dg, gk, dgk)
        u, H = uu.T, HH.T
        du[k] = uk.T
        dH[k] = Hk.T
    return {"u": np.ascontiguousarray(u), "du": np.ascontiguousarray(du[1:]),
            "dtu": np.ascontiguousarray(du[0]), "H": np.ascontiguousarray(H),
            "dH": np.ascontiguousarray(dH.reshape(16, P))}

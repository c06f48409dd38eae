"""Seeded synthetic inputs: exact Kerr-Schild black holes and perturbations.

This module is the one source of inputs for both the GPU path and the CPU
oracle.  It evaluates an *exact* spacetime and its chosen gauge source at given
Cartesian points; it contains none of the evolution method's arithmetic (no
collocation grid, no spectral derivative, no GH right-hand side, no boundary
treatment, no time step).  Derivatives of the exact metric are taken by
forward-mode automatic differentiation (torch.func on the CPU, float64).

The paper's test problem is an isolated Kerr-Schild black hole of mass m and
dimensionless spin vector chi (port overview, eq. dimensionlessspin).  The
formulas are the standard Kerr-Schild form (not written in the paper):
  psi_ab = eta_ab + 2 H l_a l_b,  eta = diag(-1, 1, 1, 1),  a = |chi| M,
  r^2 = (rho^2 - a^2)/2 + sqrt((rho^2 - a^2)^2/4 + a^2 z^2),
  H = M r^3 / (r^4 + a^2 z^2),
  l_a = (1, (r x + a y)/(r^2 + a^2), (r y - a x)/(r^2 + a^2), z / r)
for spin along z; other spin axes are obtained by a spatial rotation.

First-order variables: Phi_iab = d_i psi_ab and Pi_ab = -(d_t psi_ab - N^i Phi_iab)/N.
Gauge source (frozen in time): H_a = -psi^bc Gamma_abc of the exact metric, so the
exact solution has zero gauge constraint and is a solution of the evolution
system; d_a H_b is returned with its time row.
"""

import math
import numpy as np
import torch
from torch.func import jacfwd, vmap

PAIRS = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]
_ETA = torch.diag(torch.tensor([-1.0, 1.0, 1.0, 1.0], dtype=torch.float64))


def rotation_to(axis):
    """Proper rotation R (3x3) with R e_z = axis / |axis| (Rodrigues)."""
    n = np.asarray(axis, dtype=float)
    n = n / np.linalg.norm(n)
    z = np.array([0.0, 0.0, 1.0])
    v = np.cross(z, n)
    s = np.linalg.norm(v)
    c = float(np.dot(z, n))
    if s < 1e-15:
        return np.eye(3) if c > 0 else np.diag([1.0, -1.0, -1.0])
    K = np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]]) / s
    return np.eye(3) + s * K + (1 - c) * (K @ K)


def lorentz_boost(vel):
    """Boost matrix B (4x4, symmetric) taking coordinates to the frame moving with vel."""
    v = np.asarray(vel, dtype=float)
    b2 = float(v @ v)
    B = np.eye(4)
    if b2 == 0.0:
        return B
    g = 1.0 / math.sqrt(1.0 - b2)
    B[0, 0] = g
    B[0, 1:] = B[1:, 0] = -g * v
    B[1:, 1:] += (g - 1.0) * np.outer(v, v) / b2
    return B


def kerr_schild_metric(M, chi, axis=(0.0, 0.0, 1.0), boost=None, device="cpu"):
    """Return g(X) -> [4,4] for a Kerr-Schild hole (optionally Lorentz-boosted)."""
    a = float(chi) * float(M)
    Lam = torch.eye(4, dtype=torch.float64)
    Lam[1:, 1:] = torch.tensor(rotation_to(axis), dtype=torch.float64)
    Lam = Lam.to(device)
    eta = _ETA.to(device)
    B = None if boost is None else torch.tensor(lorentz_boost(boost), dtype=torch.float64).to(device)

    def g_spin_z(X):
        x, y, z = X[1], X[2], X[3]
        q = 0.5 * (x * x + y * y + z * z - a * a)
        r2 = q + torch.sqrt(q * q + a * a * z * z)
        r = torch.sqrt(r2)
        Hs = M * r * r2 / (r2 * r2 + a * a * z * z)
        l = torch.stack([torch.ones_like(x), (r * x + a * y) / (r2 + a * a),
                         (r * y - a * x) / (r2 + a * a), z / r])
        return eta + 2.0 * Hs * torch.outer(l, l)

    def g_rot(X):
        # psi'_ab(x) = Lam_a^c Lam_b^d psi_cd(Lam^T x)
        return Lam @ g_spin_z(Lam.T @ X) @ Lam.T

    if B is None:
        return g_rot

    def g_boost(X):
        # linear change of coordinates X' = B X: g'_ab = B_ca B_db g_cd(B X)
        return B.T @ g_rot(B @ X) @ B

    return g_boost


def _pack(psi, Pi, Phi):
    comps = [psi[a, b] for (a, b) in PAIRS] + [Pi[a, b] for (a, b) in PAIRS]
    for i in range(3):
        comps += [Phi[i, a, b] for (a, b) in PAIRS]
    return torch.stack(comps)


def _first_order_fields(gfun):
    def u_of_X(X):
        g = gfun(X)
        dg = jacfwd(gfun)(X)                       # dg[a,b,c] = d_c g_ab
        Phi = dg[:, :, 1:].permute(2, 0, 1)        # [i,a,b]
        ginv = torch.linalg.inv(g[1:, 1:])
        shift = ginv @ g[0, 1:]
        lapse = torch.sqrt(shift @ g[0, 1:] - g[0, 0])
        Pi = -(dg[:, :, 0] - torch.einsum("i,iab->ab", shift, Phi)) / lapse
        return _pack(g, Pi, Phi)

    def H_of_X(X):
        g = gfun(X)
        dg = jacfwd(gfun)(X)
        # Gamma_cab = 1/2 (d_a g_cb + d_b g_ca - d_c g_ab), with dg[a,b,c] = d_c g_ab
        Gam = 0.5 * (torch.einsum("cba->cab", dg) + torch.einsum("cab->cab", dg)
                     - torch.einsum("abc->cab", dg))
        ginv4 = torch.linalg.inv(g)
        return -torch.einsum("ab,cab->c", ginv4, Gam)

    return u_of_X, H_of_X


def exact_spacetime(xyz, gfun, t=0.0, with_derivs=False, chunk=65536, device="cpu"):
    """Fields, gauge source and (optionally) exact derivatives at points xyz [3, P].

    device: where torch evaluates the exact solution ("cpu" or a CUDA device);
    the results are returned on the host either way.
    Returns dict with numpy float64 arrays:
      u [50, P], H [4, P], dH [16, P] (row a*4+b = d_a H_b);
      with_derivs: du [3, 50, P] (spatial), dtu [50, P] (time derivative).
    """
    xyz = np.asarray(xyz, dtype=float)
    P = xyz.shape[1]
    u_of_X, H_of_X = _first_order_fields(gfun)
    f_u = vmap(u_of_X)
    f_H = vmap(H_of_X)
    f_du = vmap(jacfwd(u_of_X))
    f_dH = vmap(jacfwd(H_of_X))
    outs = {"u": [], "H": [], "dH": []}
    if with_derivs:
        outs["du"], outs["dtu"] = [], []
    for s in range(0, P, chunk):
        e = min(P, s + chunk)
        X = torch.empty((e - s, 4), dtype=torch.float64)
        X[:, 0] = t
        X[:, 1:] = torch.from_numpy(xyz[:, s:e].T.copy())
        X = X.to(device)
        outs["u"].append(f_u(X).T.cpu().numpy())
        outs["H"].append(f_H(X).T.cpu().numpy())
        dH = f_dH(X)                                  # [P, b, a] = d_a H_b
        outs["dH"].append(dH.permute(2, 1, 0).reshape(16, e - s).cpu().numpy())
        if with_derivs:
            du = f_du(X)                              # [P, 50, 4]
            outs["du"].append(du[:, :, 1:].permute(2, 1, 0).cpu().numpy())
            outs["dtu"].append(du[:, :, 0].T.cpu().numpy())
    res = {k: np.ascontiguousarray(np.concatenate(v, axis=-1)) for k, v in outs.items()}
    return res


def kerr_schild(xyz, M=1.0, chi=0.0, axis=(0.0, 0.0, 1.0), with_derivs=False, device="cpu"):
    """Stationary Kerr-Schild hole at the origin (see module docstring)."""
    return exact_spacetime(xyz, kerr_schild_metric(M, chi, axis, device=device), with_derivs=with_derivs,
                           device=device)


def random_polarisation(seed):
    """Seeded random symmetric 4x4 with unit Frobenius norm."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((4, 4))
    e = 0.5 * (A + A.T)
    return e / np.linalg.norm(e)


def gaussian_pulse_Pi(xyz, amp, r0, width, seed):
    """delta Pi_ab = amp e_ab exp(-((r - r0)/width)^2), other fields zero; [50, P]."""
    xyz = np.asarray(xyz, dtype=float)
    r = np.sqrt(np.sum(xyz * xyz, axis=0))
    e = random_polarisation(seed)
    prof = amp * np.exp(-((r - r0) / width) ** 2)
    du = np.zeros((50, xyz.shape[1]))
    for n, (a, b) in enumerate(PAIRS):
        du[10 + n] = e[a, b] * prof
    return du


def smooth_random_field(xyz, amp, seed, degree, kappa_max, ncomp=50, chunk=65536):
    """Seeded smooth random perturbation of every component, [ncomp, P].

    Each component is amp * p(n) * cos(kappa ln r + phase), with p a random
    polynomial of total degree <= `degree` in the unit radial vector n (so it
    is band-limited on every sphere) with N(0,1)/sqrt(#monomials) coefficients
    and kappa uniform in [0, kappa_max].  Draw order per component: the
    coefficients, then kappa, then the phase.
    """
    xyz = np.asarray(xyz, dtype=float)
    rng = np.random.default_rng(seed)
    monos = [(i, j, k) for i in range(degree + 1) for j in range(degree + 1 - i)
             for k in range(degree + 1 - i - j)]
    coef = np.zeros((ncomp, len(monos)))
    kap = np.zeros(ncomp)
    ph = np.zeros(ncomp)
    for c in range(ncomp):
        coef[c] = rng.standard_normal(len(monos)) / math.sqrt(len(monos))
        kap[c] = rng.uniform(0.0, kappa_max)
        ph[c] = rng.uniform(0.0, 2 * math.pi)
    P = xyz.shape[1]
    out = np.zeros((ncomp, P))
    for s0 in range(0, P, chunk):
        e = min(P, s0 + chunk)
        x = xyz[:, s0:e]
        r = np.sqrt(np.sum(x * x, axis=0))
        n = x / r
        pw = [[np.ones_like(r)] for _ in range(3)]
        for a in range(3):
            for _ in range(degree):
                pw[a].append(pw[a][-1] * n[a])
        table = np.stack([pw[0][i] * pw[1][j] * pw[2][k] for (i, j, k) in monos])   # [monos, pts]
        out[:, s0:e] = amp * (coef @ table) * np.cos(np.outer(kap, np.log(r)) + ph[:, None])
    return out

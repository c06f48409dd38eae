"""Pointwise algebra of the first-order generalized-harmonic system -- oracle side.

Test infrastructure only (see package docstring).

The paper names this module ("GHEqns", port overview; "GHEqns" kernels in the
DataMesh/ApplyBCs/GHEqns section) but never writes the equations.  They are
restated here from the published first-order GH system of Lindblom, Scheel,
Kidder, Owen & Rinne (2006): evolution equations (their eqs. 35-37), the gauge
constraint (their eq. 40) and the characteristic fields (their eqs. 32-34).

Fields per point (50): psi_ab (10), Pi_ab (10), Phi_iab (30), symmetric pairs
ordered 00,01,02,03,11,12,13,22,23,33 and Phi ordered x, y, z.
Notation: spatial metric g_ij = psi_ij, inverse g^ij; shift N^i = g^ij psi_0j;
lapse N = sqrt(N^i psi_0i - psi_00); normal t^a = (1/N, -N^i/N),
t_a = (-N, 0, 0, 0); psi^ab = g^ab - t^a t^b.

All arrays carry the point index(es) last ("..."), and every function works
for float64 and complex128.
"""

import numpy as np

PAIRS = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]
NF = 50


def sym_unpack(v):
    """[10, ...] symmetric-pair components -> [4, 4, ...] symmetric tensor."""
    out = np.zeros((4, 4) + v.shape[1:], dtype=v.dtype)
    for n, (a, b) in enumerate(PAIRS):
        out[a, b] = v[n]
        out[b, a] = v[n]
    return out


def sym_pack(t):
    """[4, 4, ...] -> [10, ...] (upper triangle in pair order)."""
    return np.stack([t[a, b] for (a, b) in PAIRS])


def unpack_fields(u):
    """u[50, ...] -> psi[4,4,...], Pi[4,4,...], Phi[3,4,4,...]."""
    psi = sym_unpack(u[0:10])
    Pi = sym_unpack(u[10:20])
    Phi = np.stack([sym_unpack(u[20 + 10 * i: 30 + 10 * i]) for i in range(3)])
    return psi, Pi, Phi


def pack_fields(psi, Pi, Phi):
    return np.concatenate([sym_pack(psi), sym_pack(Pi)] + [sym_pack(Phi[i]) for i in range(3)])


def inv3_sym(g):
    """Inverse of a symmetric 3x3 [3,3,...] by cofactors over the determinant."""
    a, b, c = g[0, 0], g[0, 1], g[0, 2]
    d, e, f = g[1, 1], g[1, 2], g[2, 2]
    A = d * f - e * e
    B = c * e - b * f
    C = b * e - c * d
    D = a * f - c * c
    E = b * c - a * e
    F = a * d - b * b
    det = a * A + b * B + c * C
    inv = np.stack([np.stack([A, B, C]), np.stack([B, D, E]), np.stack([C, E, F])]) / det
    return inv


class Geometry:
    """3+1 quantities derived from psi_ab at each point."""

    def __init__(self, psi):
        self.psi = psi
        self.ginv = inv3_sym(psi[1:, 1:])                            # g^ij
        self.shift = np.einsum("ij...,j...->i...", self.ginv, psi[0, 1:])   # N^i
        self.lapse = np.sqrt(np.einsum("i...,i...->...", self.shift, psi[0, 1:]) - psi[0, 0])
        N = self.lapse
        z = np.zeros_like(N)
        self.t_up = np.stack([1.0 / N] + [-self.shift[i] / N for i in range(3)])
        self.t_lo = np.stack([-N, z, z, z])
        # spatial projector with upper indices, extended to 4d: g^ab (only ij nonzero)
        g4 = np.zeros((4, 4) + N.shape, dtype=psi.dtype)
        g4[1:, 1:] = self.ginv
        self.g4up = g4
        self.psi_inv = g4 - np.einsum("a...,b...->ab...", self.t_up, self.t_up)
        # g^i_a: g^i_0 = N^i, g^i_j = delta^i_j
        gia = np.zeros((3, 4) + N.shape, dtype=psi.dtype)
        gia[:, 0] = self.shift
        for i in range(3):
            gia[i, i + 1] = 1.0
        self.g_i_a = gia


def spacetime_dpsi(geo, Pi, Phi):
    """d_a psi_bc from first-order variables: d_0 psi = -N Pi + N^i Phi_i, d_i psi = Phi_i."""
    d0 = -geo.lapse * Pi + np.einsum("i...,iab...->ab...", geo.shift, Phi)
    return np.concatenate([d0[None], Phi], axis=0)               # [4(a),4,4,...]


def christoffel_first(dpsi4):
    """Gamma_cab = 1/2 (d_a psi_cb + d_b psi_ca - d_c psi_ab), index order [c,a,b]."""
    return 0.5 * (np.einsum("acb...->cab...", dpsi4) + np.einsum("bca...->cab...", dpsi4)
                  - dpsi4)


def gauge_constraint(geo, Pi, Phi, H):
    """C_a = H_a + g^ij Phi_ija + t^b Pi_ba - 1/2 g^i_a psi^bc Phi_ibc - 1/2 t_a psi^bc Pi_bc."""
    gPhi = np.einsum("ij...,ija...->a...", geo.ginv, Phi[:, 1:])
    tPi = np.einsum("b...,ba...->a...", geo.t_up, Pi)
    trPhi = np.einsum("bc...,ibc...->i...", geo.psi_inv, Phi)
    trPi = np.einsum("bc...,bc...->...", geo.psi_inv, Pi)
    return (H + gPhi + tPi - 0.5 * np.einsum("ia...,i...->a...", geo.g_i_a, trPhi)
            - 0.5 * geo.t_lo * trPi)


def gauge_constraint_from_gamma(geo, Pi, Phi, H):
    """C_a = H_a + psi^bc Gamma_abc (the same constraint, written with Christoffels)."""
    G = christoffel_first(spacetime_dpsi(geo, Pi, Phi))
    return H + np.einsum("bc...,abc...->a...", geo.psi_inv, G)


def rhs_pointwise(u, du, H, dH, gamma0, gamma1, gamma2):
    """Time derivatives of the 50 GH fields at each point.

    u[50, ...] fields; du[3, 50, ...] Cartesian spatial derivatives d_k u;
    H[4, ...] gauge source H_a; dH[4, 4, ...] = d_a H_b (row a = 0 is d_t);
    gamma0, gamma1, gamma2: constraint-damping parameters (scalars or arrays).

    Evolution equations (Lindblom et al. 2006, eqs. 35-37):
      d_t psi_ab = (1+g1) N^k d_k psi_ab - N Pi_ab - g1 N^i Phi_iab
      d_t Pi_ab  = N^k d_k Pi_ab - N g^ki d_k Phi_iab + g1 g2 N^k d_k psi_ab
                   + 2N psi^cd (g^ij Phi_ica Phi_jdb - Pi_ca Pi_db - psi^ef Gamma_ace Gamma_bdf)
                   - 2N (d_(a H_b) - Gamma^c_ab H_c)
                   - 1/2 N t^c t^d Pi_cd Pi_ab - N t^c Pi_ci g^ij Phi_jab
                   + N g0 (t_a C_b + t_b C_a - psi_ab t^c C_c) - g1 g2 N^i Phi_iab
      d_t Phi_iab = N^k d_k Phi_iab - N d_i Pi_ab + N g2 d_i psi_ab
                   + 1/2 N t^c t^d Phi_icd Pi_ab + N g^jk t^c Phi_ijc Phi_kab - N g2 Phi_iab
    """
    psi, Pi, Phi = unpack_fields(u)
    dpsi = np.stack([sym_unpack(du[k, 0:10]) for k in range(3)])            # [k,a,b]
    dPi = np.stack([sym_unpack(du[k, 10:20]) for k in range(3)])
    dPhi = np.stack([np.stack([sym_unpack(du[k, 20 + 10 * i:30 + 10 * i]) for i in range(3)])
                     for k in range(3)])                                     # [k,i,a,b]
    geo = Geometry(psi)
    N, Nu, gi, pinv = geo.lapse, geo.shift, geo.ginv, geo.psi_inv
    tu, tl = geo.t_up, geo.t_lo

    G = christoffel_first(spacetime_dpsi(geo, Pi, Phi))                     # Gamma_cab
    Gup = np.einsum("cd...,dab...->cab...", pinv, G)                         # Gamma^c_ab
    C = H + np.einsum("bc...,abc...->a...", pinv, G)                         # C_a

    # d_t psi
    adv_psi = np.einsum("k...,kab...->ab...", Nu, dpsi)
    NPhi = np.einsum("i...,iab...->ab...", Nu, Phi)
    dt_psi = (1.0 + gamma1) * adv_psi - N * Pi - gamma1 * NPhi

    # d_t Pi
    adv_Pi = np.einsum("k...,kab...->ab...", Nu, dPi)
    divPhi = np.einsum("ki...,kiab...->ab...", gi, dPhi)
    quad = (np.einsum("cd...,ij...,ica...,jdb...->ab...", pinv, gi, Phi, Phi)
            - np.einsum("cd...,ca...,db...->ab...", pinv, Pi, Pi)
            - np.einsum("cd...,ef...,ace...,bdf...->ab...", pinv, pinv, G, G))
    dHsym = dH + np.einsum("ab...->ba...", dH)
    GH = np.einsum("cab...,c...->ab...", Gup, H)
    ttPi = np.einsum("c...,d...,cd...->...", tu, tu, Pi)
    tPi_i = np.einsum("c...,ci...->i...", tu, Pi[:, 1:])                   # t^c Pi_ci
    tPi_gPhi = np.einsum("i...,ij...,jab...->ab...", tPi_i, gi, Phi)
    tC = np.einsum("c...,c...->...", tu, C)
    damp0 = (np.einsum("a...,b...->ab...", tl, C) + np.einsum("a...,b...->ab...", C, tl)
             - psi * tC)
    dt_Pi = (adv_Pi - N * divPhi + gamma1 * gamma2 * adv_psi
             + 2.0 * N * quad
             - N * dHsym + 2.0 * N * GH
             - 0.5 * N * ttPi * Pi - N * tPi_gPhi
             + gamma0 * N * damp0 - gamma1 * gamma2 * NPhi)

    # d_t Phi
    adv_Phi = np.einsum("k...,kiab...->iab...", Nu, dPhi)
    ttPhi = np.einsum("c...,d...,icd...->i...", tu, tu, Phi)
    tPhi = np.einsum("c...,ijc...->ij...", tu, Phi[:, 1:])                  # t^c Phi_ijc  [i,j]
    gtPhiPhi = np.einsum("jk...,ij...,kab...->iab...", gi, tPhi, Phi)
    dt_Phi = (adv_Phi - N * dPi + gamma2 * N * dpsi
              + 0.5 * N * np.einsum("i...,ab...->iab...", ttPhi, Pi)
              + N * gtPhiPhi - gamma2 * N * Phi)

    return pack_fields(dt_psi, dt_Pi, dt_Phi)


def constraints_pointwise(u, du, H):
    """The 64 constraint components per point, order [C_a (4), C_iab (30), C_ijab (30)].

    C_a    = H_a + psi^bc Gamma_abc                (gauge constraint)
    C_iab  = d_i psi_ab - Phi_iab                  (i = x,y,z; pairs in PAIRS order)
    C_ijab = d_i Phi_jab - d_j Phi_iab             ((i,j) = (x,y), (x,z), (y,z))
    """
    psi, Pi, Phi = unpack_fields(u)
    geo = Geometry(psi)
    Ca = gauge_constraint(geo, Pi, Phi, H)
    C3 = [du[i, 0:10] - u[20 + 10 * i:30 + 10 * i] for i in range(3)]
    C4 = []
    for (i, j) in [(0, 1), (0, 2), (1, 2)]:
        C4.append(du[i, 20 + 10 * j:30 + 10 * j] - du[j, 20 + 10 * i:30 + 10 * i])
    return np.concatenate([Ca] + C3 + C4)


# ----------------------------------------------------------------------------
# Characteristic decomposition (Lindblom et al. 2006, eqs. 32-34)
# ----------------------------------------------------------------------------

def unit_normal(geo, n_cov):
    """Normalise a spatial covector n_i with g^ij: s_i = n_i / |n|, s^i = g^ij s_j."""
    nrm = np.sqrt(np.einsum("ij...,i...,j...->...", geo.ginv, n_cov, n_cov))
    s_lo = n_cov / nrm
    s_up = np.einsum("ij...,j...->i...", geo.ginv, s_lo)
    return s_lo, s_up


def char_speeds(geo, s_lo, gamma1):
    """Speeds of (u^psi, u^0, u^+, u^-): -(1+g1) s.N, -s.N, -s.N + N, -s.N - N."""
    sN = np.einsum("i...,i...->...", s_lo, geo.shift)
    return (-(1.0 + gamma1) * sN, -sN, -sN + geo.lapse, -sN - geo.lapse)


def char_fields(v, s_lo, s_up, gamma2):
    """Characteristic projections of a 50-component vector v (fields or their d_t).

    u^psi_ab = psi_ab; u^0_iab = Phi_iab - s_i s^k Phi_kab;
    u^(+-)_ab = Pi_ab +- s^k Phi_kab - g2 psi_ab.  Returned in pair form:
    (upsi[10], u0[3,10], up[10], um[10]).
    """
    psi, Pi, Phi = v[0:10], v[10:20], v[20:50].reshape((3, 10) + v.shape[1:])
    sPhi = np.einsum("k...,kn...->n...", s_up, Phi)
    u0 = Phi - np.einsum("i...,n...->in...", s_lo, sPhi)
    up = Pi + sPhi - gamma2 * psi
    um = Pi - sPhi - gamma2 * psi
    return psi, u0, up, um


def char_reconstruct(upsi, u0, up, um, s_lo, gamma2):
    """Inverse map: psi = u^psi, Pi = (u^+ + u^-)/2 + g2 u^psi, Phi_i = u^0_i + s_i (u^+ - u^-)/2."""
    Pi = 0.5 * (up + um) + gamma2 * upsi
    Phi = u0 + 0.5 * np.einsum("i...,n...->in...", s_lo, up - um)
    return np.concatenate([upsi, Pi, Phi.reshape((30,) + Phi.shape[2:])])


# ----------------------------------------------------------------------------
# Constraint-preserving treatment of an outer boundary point
# ----------------------------------------------------------------------------

def outer_constraint_preserving(dtu, u, du, s_lo, s_up, geo, gamma1, gamma2):
    """Boundary treatment of d_t u at outer-boundary points (normal s out of the
    domain), reading the paper's constraint-preserving outer condition
    (Conclusions, ApplyBCs case (ii)) for the constraints of the first-order
    system.

    dtu [50, ...] raw time derivatives; u [50, ...] fields; du [3, 50, ...]
    their Cartesian derivatives; s_lo, s_up the unit normal (unit_normal);
    geo the Geometry of u.  With N.s = s_k N^k:

    * u^psi (speed -(1+g1) N.s) carries the three-index constraint
      C_kab = d_k psi_ab - Phi_kab: d_t psi contains (1+g1) N^k C_kab, whose
      normal part (1+g1)(N.s)(s^k C_kab) is the only piece that needs the
      normal derivative of psi.  Where u^psi is incoming it is removed.
    * u^0 (speed -N.s) carries the four-index constraint
      C_klab = d_k Phi_lab - d_l Phi_kab: the normal advection of Phi_l is
      (N.s)(s^k d_l Phi_k + s^k C_klab), and under the transverse projector
      P_i^l = delta_i^l - s_i s^l only the constraint part needs a normal
      derivative.  Where u^0 is incoming, (N.s) P_i^l s^k C_klab is removed.
    * u^- (speed -N.s - N) is incoming at an outer boundary; the published
      condition for it combines physical (Weyl), gauge and two-index
      constraint parts.  Reading: it is frozen, d_t u^- = 0 (no incoming
      radiation rate).  The same holds for u^+ if it were incoming.
    * outgoing fields are left as they are.

    After the treatment the incoming u^psi and u^0 depend on the fields and
    their tangential derivatives only, and on data that satisfy the
    constraints the treatment changes nothing but the incoming u^-.
    """
    v_psi, v_0, v_p, v_m = char_speeds(geo, s_lo, gamma1)
    upsi, u0, up, um = char_fields(dtu, s_lo, s_up, gamma2)
    sN = np.einsum("i...,i...->...", s_lo, geo.shift)
    # C_kab and s^k C_kab
    C3 = np.stack([du[k, 0:10] - u[20 + 10 * k:30 + 10 * k] for k in range(3)])          # [k, n]
    sC3 = np.einsum("k...,kn...->n...", s_up, C3)
    # C_klab and s^k C_klab  [l, n]
    dPhi = np.stack([du[:, 20 + 10 * l:30 + 10 * l] for l in range(3)], axis=1)         # [k, l, n]
    C4 = dPhi - np.swapaxes(dPhi, 0, 1)
    sC4 = np.einsum("k...,kln...->ln...", s_up, C4)
    # P_i^l sC4_l = sC4_i - s_i (s^l sC4_l)
    proj = sC4 - np.einsum("i...,n...->in...", s_lo, np.einsum("l...,ln...->n...", s_up, sC4))
    upsi = np.where(np.real(v_psi) < 0, upsi - (1.0 + gamma1) * sN * sC3, upsi)
    u0 = np.where(np.real(v_0) < 0, u0 - sN * proj, u0)
    up = np.where(np.real(v_p) < 0, 0.0 * up, up)
    um = np.where(np.real(v_m) < 0, 0.0 * um, um)
    return char_reconstruct(upsi, u0, up, um, s_lo, gamma2)

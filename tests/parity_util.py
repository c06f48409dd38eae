"""Helpers shared by the parity tests."""

import numpy as np

from oracle import spectral


def _traced(fn, n):
    return np.stack([fn(np.eye(n)[k]) for k in range(n)], axis=1)


def rounding_scale(d, j, ublk):
    """Term scale kappa of the Cartesian derivatives of one shell block
    [50, n_r, N_theta, N_phi] of oracle domain d:
    max(|D_r| |u| + |Theta| |u| / r + |Phi| |u| / (r sin theta)), the operators
    traced from the oracle's transforms.  An FP64 evaluation of a derivative
    carries a rounding error of order eps times this (the standard bound for a
    sum of products), whatever the size of the derivative itself."""
    g = d.grids[j]
    sph = d.spheres[g.L]
    S = sph.S
    eye = np.eye(S).reshape(S, sph.nth, sph.nph)
    Th = np.abs(sph.d_dtheta(eye).reshape(S, S))          # [input, output]
    Ph = np.abs(sph.d_dphi(eye).reshape(S, S))
    Dr = np.abs(_traced(spectral.d_dxi, g.n_r)) * (2.0 / (g.r_out - g.r_in))
    U = np.abs(ublk).reshape(50, g.n_r, S)
    k_r = np.einsum("ij,fjs->fis", Dr, U)
    k_t = (U @ Th) / g.R.reshape(1, g.n_r, S)
    k_p = (U @ Ph) / (g.R * np.sin(g.TH)).reshape(1, g.n_r, S)
    return float(np.max(k_r + k_t + k_p))


def _abs_operator_by_shifts(fn, nth, nph):
    """|A| [input, output] of an angular operator A that commutes with shifts
    of the uniform phi grid (d/dtheta and d/dphi do: both commute with
    rotations about the axis, and so does the band limit l <= L), from the nth
    columns of the inputs at phi index 0:
    A[(i, k), (i', k')] = A[(i, k - k'), (i', 0)]."""
    E = np.zeros((nth, nth, nph))
    E[np.arange(nth), np.arange(nth), 0] = 1.0
    T = np.abs(fn(E))                                     # [i', i, k] = A[(i, k), (i', 0)]
    ip = np.arange(nth)[:, None, None, None]
    kp = np.arange(nph)[None, :, None, None]
    i = np.arange(nth)[None, None, :, None]
    k = np.arange(nph)[None, None, None, :]
    return T[ip, i, (k - kp) % nph].reshape(nth * nph, nth * nph)


def rounding_scale_by_shifts(d, j, ublk):
    """rounding_scale with the angular operators traced from N_theta inputs
    instead of S (their phi-shift structure), for large L."""
    g = d.grids[j]
    sph = d.spheres[g.L]
    Th = _abs_operator_by_shifts(sph.d_dtheta, sph.nth, sph.nph)
    Ph = _abs_operator_by_shifts(sph.d_dphi, sph.nth, sph.nph)
    Dr = np.abs(_traced(spectral.d_dxi, g.n_r)) * (2.0 / (g.r_out - g.r_in))
    U = np.abs(ublk).reshape(50, g.n_r, sph.S)
    U2 = U.reshape(-1, sph.S)                             # one product over all (field, radius) rows
    k_r = np.einsum("ij,fjs->fis", Dr, U)
    k_t = (U2 @ Th).reshape(U.shape) / g.R.reshape(1, g.n_r, sph.S)
    k_p = (U2 @ Ph).reshape(U.shape) / (g.R * np.sin(g.TH)).reshape(1, g.n_r, sph.S)
    return float(np.max(k_r + k_t + k_p))

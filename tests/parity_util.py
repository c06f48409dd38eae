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

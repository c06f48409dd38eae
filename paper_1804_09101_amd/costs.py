"""Operation counts of the derivative path: the paper's minimum-cost model and
the counts this implementation's kernels are measured against.

The paper's model (section "GPU Benchmarking", eqs. speedup, BWeff, Peff): an operation moving D = w M
bytes (w = 8 for FP64) and doing F floating-point operations has arithmetic
intensity I = F / M; it is memory-bound below I_eq = w P / B.

Dense matrix-multiply differentiator on a shell, I1 x S2 (section "Spectral
Operations: Differentiation and Filtering", the I1 x S2 paragraphs): one radial (N_r x N_r) and two angular
(S x S, S = N_theta N_phi) transforms of each of N_e arrays,
    M = N_e (N_r^2 + 2 S^2 + 6 N_r S),
    F = N_e N_r S (2 N_r + 4 S - 3).
The SingleBH grids use N_r = 9 + 4k, N_theta = 6 + 2k, N_phi = 4k + 12; the BBH
grids N_r = 4 + k, N_theta = 7 + 2k, N_phi = 4k + 14.

DiffJac (section "Jacobian multiplication", eq. DiffJac): a d x d Jacobian
applied per point to the spatial derivative of a tensor with N_e unique
components, M = N_x (2 N_e + d) d, F = N_x N_e (2d - 1) d.

Nothing here takes part in the computation; bench.py reports these figures.
"""

N_FIELDS = 50


def shell_dense_derivative(n_r, S, n_e=N_FIELDS):
    """(M, F) of the paper's dense shell differentiator for one shell."""
    M = n_e * (n_r * n_r + 2 * S * S + 6 * n_r * S)
    F = n_e * n_r * S * (2 * n_r + 4 * S - 3)
    return M, F


def singlebh_grid(k):
    """(N_r, N_theta, N_phi) of the SingleBH resolution k."""
    return 9 + 4 * k, 6 + 2 * k, 4 * k + 12


def bbh_grid(k):
    """(N_r, N_theta, N_phi) of the BBH resolution k."""
    return 4 + k, 7 + 2 * k, 4 * k + 14


def diffjac(n_e, d=3, n_x=1):
    """(M, F) of the DiffJac operation on n_x points."""
    return n_x * (2 * n_e + d) * d, n_x * n_e * (2 * d - 1) * d


def domain_model(shells, n_e=N_FIELDS, w=8):
    """Per-domain totals of the paper's dense model for one derivative pass.

    shells: iterable of (instance, n_r, L, r_in, r_out) with S = 2 (L + 1)^2.
    Returns points, bytes (w M) and flops F summed over shells.
    """
    P = B = F = 0
    for (_, n_r, L, _, _) in shells:
        S = 2 * (L + 1) ** 2
        m, f = shell_dense_derivative(n_r, S, n_e)
        P += n_r * S
        B += w * m
        F += f
    return {"points": P, "bytes": B, "flops": F, "intensity_flop_per_byte": F / B,
            "flops_per_point": F / P, "bytes_per_point": B / P}


def angular_gemm_flops(shells, n_e=N_FIELDS):
    """Flops of one launch of the angular derivative GEMM over the domain.

    Per shell C[n_e n_r x 2S] = U[n_e n_r x S] [Theta^T | Phi^T][S x 2S] costs
    2 n_e n_r (2S) S flops: the angular part of the paper's F above, with
    each multiply-add counted as two operations.
    """
    f = 0
    for (_, n_r, L, _, _) in shells:
        S = 2 * (L + 1) ** 2
        f += 2 * n_e * n_r * 2 * S * S
    return f


def angular_gemm_bytes(shells, n_e=N_FIELDS, w=8):
    """Minimum HBM bytes of one angular derivative GEMM launch: every field
    row read once, each distinct operator [S x 2S] read once, the result
    [n_e n_r x 2S] written once."""
    b = 0
    seen = set()
    for (_, n_r, L, _, _) in shells:
        S = 2 * (L + 1) ** 2
        b += w * n_e * n_r * (S + 2 * S)
        if L not in seen:
            seen.add(L)
            b += w * S * 2 * S
    return b

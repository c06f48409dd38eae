"""The cost model reproduces the figures the paper prints for it.

Pins: the expanded SingleBH and BBH polynomials for M and F (section
"Spectral Operations: Differentiation and Filtering", I1 x S2 paragraphs), the starting intensities 13.7
(SingleBH, k = 0) and 7.2 (BBH, k = 0), and the DiffJac intensities
1.81, 2.17, 2.29, 2.41 for N_e = 4, 10, 16, 40 (section "Jacobian
multiplication"; the first is printed truncated, 20/11 = 1.818)."""

import pytest

from paper_1804_09101_amd import costs


def _singlebh_poly(k):
    M = 128 * k**4 + 1728 * k**3 + 8512 * k**2 + 18216 * k + 14337
    F = 1024 * k**5 + 14848 * k**4 + 85536 * k**3 + 244728 * k**2 + 347760 * k + 196344
    return M, F


def _bbh_poly(k):
    M = 128 * k**4 + 1840 * k**3 + 9937 * k**2 + 23892 * k + 21576
    F = 256 * k**5 + 4624 * k**4 + 33368 * k**3 + 120252 * k**2 + 216426 * k + 155624
    return M, F


@pytest.mark.parametrize("k", range(0, 11))
def test_singlebh_polynomials(k):
    n_r, nt, nph = costs.singlebh_grid(k)
    assert nt * nph == 8 * k * k + 48 * k + 72
    assert costs.shell_dense_derivative(n_r, nt * nph, n_e=1) == _singlebh_poly(k)


@pytest.mark.parametrize("k", range(0, 17))
def test_bbh_polynomials(k):
    n_r, nt, nph = costs.bbh_grid(k)
    assert nt * nph == 8 * k * k + 56 * k + 98
    assert costs.shell_dense_derivative(n_r, nt * nph, n_e=1) == _bbh_poly(k)


def test_starting_intensities():
    for grid, printed in ((costs.singlebh_grid, 13.7), (costs.bbh_grid, 7.2)):
        n_r, nt, nph = grid(0)
        M, F = costs.shell_dense_derivative(n_r, nt * nph)
        assert round(F / M, 1) == printed


def test_diffjac_intensities():
    for n_e, printed in ((4, 1.81), (10, 2.17), (16, 2.29), (40, 2.41)):
        M, F = costs.diffjac(n_e)
        assert F / M == pytest.approx(5 * n_e / (2 * n_e + 3))
        assert abs(F / M - printed) < 0.01
    M, F = costs.diffjac(10**6)
    assert abs(F / M - 2.5) < 1e-5


def test_angular_gemm_is_angular_part_of_model():
    # the angular share of F is N_e N_r S (4S - 2) with the -1 per direction of
    # an (S x S) product; the GEMM count 4 N_e N_r S^2 differs from it by 2 N_e N_r S
    shells = [(0, 21, 15, 1.0, 2.0), (0, 11, 7, 2.0, 3.0)]
    g = costs.angular_gemm_flops(shells)
    ref = sum(4 * 50 * n_r * (2 * (L + 1) ** 2) ** 2 for (_, n_r, L, _, _) in shells)
    assert g == ref
    dm = costs.domain_model(shells)
    assert dm["points"] == 21 * 512 + 11 * 128


def test_angular_gemm_bytes_of_the_8_shell_domain():
    # field matrix 8400 x 512, operator 512 x 1024 (one L), result 8400 x 1024, doubles
    shells = [(0, 21, 15, 1.0 + i, 2.0 + i) for i in range(8)]
    assert costs.angular_gemm_bytes(shells) == 8 * (8400 * 512 + 512 * 1024 + 8400 * 1024)

// Host-side construction of the collocation grid and of the dense spectral
// operators (the paper's traced matrices, section "Spectral Operations",
// eqs. Differentiation and DifferentiatorI1S2).  Pure C++, no HIP.
#pragma once
#include <vector>

namespace ghsetup {

// Chebyshev-Gauss-Lobatto nodes xi_j = -cos(pi j/(n-1)), increasing.
std::vector<double> cgl_nodes(int n);

// CGL first-derivative matrix D[i*n+j] (d/dxi), barycentric closed form
// D_ij = (c_i/c_j) (-1)^(i+j) / (xi_i - xi_j), diagonal = minus the row sum.
std::vector<double> cgl_diff_matrix(int n);

// Clenshaw-Curtis weights on the CGL nodes (Trefethen's closed form).
std::vector<double> clenshaw_curtis(int n);

// Gauss-Legendre nodes (increasing) and weights for L+1 points (Newton on P_{L+1}).
void gauss_legendre(int L, std::vector<double>& x, std::vector<double>& w);

// Normalised P_l^m(x) (including 1/sqrt(4 pi), no Condon-Shortley phase) and
// d/dtheta of it, 0 <= m <= l <= L, at one node: arrays [(L+1)*(L+1)], index l*(L+1)+m.
void legendre_normalised(int L, double x, std::vector<double>& P, std::vector<double>& dP);

// Dense S x S operators on one sphere, row-major (out_j = sum_a M[j*S+a] u_a):
//   which 0: d/dtheta, 1: d/dphi, 2: filter with factors sigma_l (sigma has L+1 entries).
std::vector<double> sphere_operator(int L, int which, const std::vector<double>& sigma);
// The same operator (transposed = false) or its transpose written into out,
// row r at out + r * ld (S rows of S values), without forming it elsewhere.
void sphere_operator_into(int L, int which, const std::vector<double>& sigma, bool transposed, double* out,
                          size_t ld);

// The same operators factorised by azimuthal order m (n = L+1):
//   M u (i, k) = sum_m sum_i' K_m[i][i'] (cos(m phi_k) A_m(i') + sin(m phi_k) B_m(i'))   (which 0, 2)
//   M u (i, k) = sum_m sum_i' K_m[i][i'] (sin(m phi_k) A_m(i') - cos(m phi_k) B_m(i'))   (which 1)
// with A_m(i') = sum_k' cos(m phi_k') u(i', k'), B_m(i') = sum_k' sin(m phi_k') u(i', k').
// sphere_factors returns K as [m][i][i'] (quadrature weight, c_m and -m folded in).
std::vector<double> sphere_factors(int L, int which, const std::vector<double>& sigma);

// Fourier table T[k][m'] (N_phi x 2n): cos(m' phi_k) for m' < n, sin((m'-n) phi_k)
// for m' >= n, at exactly reduced angles.
std::vector<double> fourier_table(int L);

// Filter factors sigma_l = 1 (l/L <= eta_c), else exp(-alpha((l/L-eta_c)/(1-eta_c))^order).
std::vector<double> exp_filter_sigma(int L, double eta_c, double alpha, double order);

// Per angular point (i, k): sin(theta), cos(theta), sin(phi), cos(phi), and the
// angular quadrature weight w_i * 2 pi / N_phi; 5 doubles each, S entries.
std::vector<double> angular_table(int L);

}  // namespace ghsetup

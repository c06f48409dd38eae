// Host-side construction of the tensor-coupled angular filter: the coupling
// matrix on the stored angular coefficients of the 50 GH fields, and the
// real-Y_lm analysis / synthesis matrices the filter is applied between.
// Pure C++, no HIP.
#pragma once
#include <vector>

namespace ghtf {

// Sparse matrix in CSR form; rows and columns e * (L+1)^2 + s with e the
// stored field (0..49) and s = l*l + l + m the real Y_lm (m > 0: cos m phi,
// m < 0: sin |m| phi).
struct Csr {
  int n = 0;
  std::vector<long long> row_ptr;   // n + 1
  std::vector<int> col;
  std::vector<double> val;
};

// Filter factor of total angular momentum j on a sphere of degree L.
//   kind 2 (ExpCheb, params eta_c, alpha, order): 1 for j/L <= eta_c, else
//          exp(-alpha ((j/L - eta_c)/(1 - eta_c))^order);
//   kind 3 (Heaviside, params eta_c): 1 for j <= eta_c L, else 0.
double sigma(int kind, const double* params, int L, int j);

// F = sum_j sigma(j) P_j, P_j the projector onto total angular momentum j of
// psi_ab, Pi_ab (two spacetime indices) and Phi_iab (a spatial index and two
// spacetime indices); transpose: F^T.  Built per degree l on worker threads.
Csr coupling_matrix(int L, int kind, const double* params, bool transpose);

// The transpose of a CSR matrix (columns sorted within each row).
Csr transpose(const Csr& m);

// Real orthonormal Y_lm at the Gauss-Legendre x uniform grid (S = 2(L+1)^2
// points, point index i * N_phi + k):
//   analysis  [ (L+1)^2 ][ S ]: quadrature weight times Y_s at the point;
//   synthesis [ S ][ (L+1)^2 ]: Y_s at the point.
std::vector<double> sphere_analysis(int L);
std::vector<double> sphere_synthesis(int L);

// The same analysis and synthesis factorised by azimuthal order, for Fourier
// coefficients F[i][m'] (m' < n: cos m phi, m' >= n: sin (m' - n) phi; n = L+1):
//   analysis  TA[i][s] = f_m (2 pi / N_phi) w_i P_l^|m|(x_i)   (n x (L+1)^2),
//   synthesis TS[s][i] = f_m P_l^|m|(x_i)                       ((L+1)^2 x n),
// f_0 = 1, f_m = sqrt2, s = l*l + l + m.  Returned as TA followed by TS.
std::vector<double> legendre_tables(int L);

}  // namespace ghtf

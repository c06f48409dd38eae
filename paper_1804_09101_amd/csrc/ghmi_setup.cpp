// Host-side construction of grids and dense spectral operators.
//
// The paper traces each linear spectral operation into an explicit matrix and
// keeps it in a dictionary keyed by what makes it unique (section "Spectral
// Operations", eq. Differentiation; the dictionary paragraph that follows).
// Here the matrices are built directly from closed forms:
//  * radial: the Chebyshev-Gauss-Lobatto differentiation matrix;
//  * angular: Theta = Syn_dtheta * Ana and Phi = Syn_dphi * Ana, with Ana the
//    Gauss-Legendre x trapezoid quadrature onto the (L+1)^2 real orthonormal
//    Y_lm and Syn_d* the derivatives of the Y_lm at the nodes
//    (eq. DifferentiatorI1S2: both angular operators are full S x S matrices);
//  * filter: Syn * diag(sigma_l) * Ana.
// Normalised associated Legendre functions come from the standard normalised
// three-term recurrences (no factorials), their theta-derivative from
// dP_l^m/dtheta = (l x P_l^m - sqrt((2l+1)(l^2-m^2)/(2l-1)) P_{l-1}^m) / sin(theta).
#include "ghmi_setup.h"

#include <algorithm>
#include <cmath>
#include <thread>

namespace ghsetup {

static const double kPi = 3.14159265358979323846;

std::vector<double> cgl_nodes(int n) {
  std::vector<double> xi(n);
  for (int j = 0; j < n; ++j) xi[j] = -std::cos(kPi * j / (n - 1));
  return xi;
}

std::vector<double> cgl_diff_matrix(int n) {
  // Off-diagonal entries use xi_i - xi_j = 2 sin(pi (i+j)/(2N)) sin(pi (i-j)/(2N)), N = n-1,
  // which avoids the cancellation of subtracting clustered end nodes (the
  // trigonometric-identity form of Don & Solomonoff, SIAM J. Sci. Comput. 18, 1997);
  // the diagonal is minus the off-diagonal row sum, so D annihilates constants.
  const int N = n - 1;
  std::vector<double> D(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double ci = (i == 0 || i == N) ? 2.0 : 1.0;
    double rowsum = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double cj = (j == 0 || j == N) ? 2.0 : 1.0;
      double sgn = ((i + j) & 1) ? -1.0 : 1.0;
      double diff = 2.0 * std::sin(kPi * (i + j) / (2.0 * N)) * std::sin(kPi * (i - j) / (2.0 * N));
      double v = (ci / cj) * sgn / diff;
      D[size_t(i) * n + j] = v;
      rowsum += v;
    }
    D[size_t(i) * n + i] = -rowsum;
  }
  return D;
}

std::vector<double> clenshaw_curtis(int n) {
  // N = n-1 intervals, nodes cos(j pi / N); symmetric under j -> N-j, so the
  // increasing ordering of the nodes does not matter.
  int N = n - 1;
  std::vector<double> w(n, 0.0);
  if (N == 0) { w[0] = 2.0; return w; }
  for (int j = 0; j <= N; ++j) {
    double th = kPi * j / N;
    if (j == 0 || j == N) {
      w[j] = (N % 2 == 0) ? 1.0 / (double(N) * N - 1.0) : 1.0 / (double(N) * N);
      continue;
    }
    double v = 1.0;
    if (N % 2 == 0) {
      for (int k = 1; k <= N / 2 - 1; ++k) v -= 2.0 * std::cos(2.0 * k * th) / (4.0 * k * k - 1.0);
      v -= std::cos(N * th) / (double(N) * N - 1.0);
    } else {
      for (int k = 1; k <= (N - 1) / 2; ++k) v -= 2.0 * std::cos(2.0 * k * th) / (4.0 * k * k - 1.0);
    }
    w[j] = 2.0 * v / N;
  }
  return w;
}

void gauss_legendre(int L, std::vector<double>& x, std::vector<double>& w) {
  int n = L + 1;
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double pn = (n == 1) ? z : p1;
      double pm = (n == 1) ? 1.0 : p0;
      dp = n * (z * pn - pm) / (z * z - 1.0);
      double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        // one more update of the derivative at the converged node
        p0 = 1.0; p1 = z;
        for (int k = 2; k <= n; ++k) {
          double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        pn = (n == 1) ? z : p1;
        pm = (n == 1) ? 1.0 : p0;
        dp = n * (z * pn - pm) / (z * z - 1.0);
        break;
      }
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  // sort increasing in x
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return x[a] < x[b]; });
  std::vector<double> xs(n), ws(n);
  for (int i = 0; i < n; ++i) { xs[i] = x[idx[i]]; ws[i] = w[idx[i]]; }
  // enforce exact antisymmetry of the nodes (they come in +- pairs)
  for (int i = 0; i < n / 2; ++i) {
    double a = 0.5 * (xs[n - 1 - i] - xs[i]);
    double b = 0.5 * (ws[n - 1 - i] + ws[i]);
    xs[i] = -a; xs[n - 1 - i] = a;
    ws[i] = b; ws[n - 1 - i] = b;
  }
  if (n % 2 == 1) xs[n / 2] = 0.0;
  x = xs;
  w = ws;
}

// Normalised P_l^m(x) (including 1/sqrt(4 pi), no Condon-Shortley phase) and
// d/dtheta of it, for 0 <= m <= l <= L at one node: arrays [(L+1)*(L+1)], index l*(L+1)+m.
void legendre_normalised(int L, double x, std::vector<double>& P, std::vector<double>& dP) {
  int n = L + 1;
  P.assign(size_t(n) * n, 0.0);
  dP.assign(size_t(n) * n, 0.0);
  double s = std::sqrt(1.0 - x * x);
  double pmm = 1.0 / std::sqrt(4.0 * kPi);
  for (int m = 0; m <= L; ++m) {
    if (m > 0) pmm *= std::sqrt((2.0 * m + 1.0) / (2.0 * m)) * s;
    P[size_t(m) * n + m] = pmm;
    if (m + 1 <= L) P[size_t(m + 1) * n + m] = std::sqrt(2.0 * m + 3.0) * x * pmm;
    for (int l = m + 2; l <= L; ++l) {
      double a = std::sqrt((4.0 * l * l - 1.0) / (double(l) * l - double(m) * m));
      double b = std::sqrt((double(l - 1) * (l - 1) - double(m) * m) / (4.0 * (l - 1) * (l - 1) - 1.0));
      P[size_t(l) * n + m] = a * (x * P[size_t(l - 1) * n + m] - b * P[size_t(l - 2) * n + m]);
    }
  }
  for (int m = 0; m <= L; ++m)
    for (int l = m; l <= L; ++l) {
      double prev = (l - 1 >= m) ? P[size_t(l - 1) * n + m] : 0.0;
      double c = std::sqrt((2.0 * l + 1.0) * (double(l) * l - double(m) * m) / (2.0 * l - 1.0));
      dP[size_t(l) * n + m] = (l * x * P[size_t(l) * n + m] - c * prev) / s;
    }
}

std::vector<double> exp_filter_sigma(int L, double eta_c, double alpha, double order) {
  std::vector<double> sig(L + 1, 1.0);
  if (L == 0) return sig;
  for (int l = 0; l <= L; ++l) {
    double q = double(l) / double(L);
    if (q > eta_c) sig[l] = std::exp(-alpha * std::pow((q - eta_c) / (1.0 - eta_c), order));
  }
  return sig;
}

std::vector<double> sphere_factors(int L, int which, const std::vector<double>& sigma) {
  // M = Syn * Ana with Ana[lm][a] = W_a Y_lm(a).  For a fixed order m the two real
  // harmonics of that order combine into a function of the azimuth difference:
  //   sum_{+-m} Y_lm(j) Y_lm(a) = c_m P_l^m(x_j) P_l^m(x_a) cos(m (phi_j - phi_a)),
  // c_0 = 1, c_m = 2 (normalised P_l^m as in legendre_normalised), so
  //   d/dtheta:  M[j][a] = W_a sum_m c_m Kd_m(i_j, i_a) cos(m dphi)
  //   d/dphi:    M[j][a] = -W_a sum_m c_m m K_m(i_j, i_a) sin(m dphi)
  //   filter:    M[j][a] = W_a sum_m c_m Ks_m(i_j, i_a) cos(m dphi)
  // with theta kernels K_m = sum_l P_l^m P_l^m, Kd_m = sum_l dP_l^m/dtheta P_l^m and
  // Ks_m = sum_l sigma_l P_l^m P_l^m.  Returned: c_m (-m) K_m(i, i') W_i' as [m][i][i'].
  std::vector<double> x, w;
  gauss_legendre(L, x, w);
  const int nth = L + 1, nph = 2 * (L + 1), n = L + 1;
  std::vector<std::vector<double>> P(nth), dP(nth);
  for (int i = 0; i < nth; ++i) legendre_normalised(L, x[i], P[i], dP[i]);
  std::vector<double> K(size_t(n) * nth * nth, 0.0);
  for (int m = 0; m <= L; ++m)
    for (int i = 0; i < nth; ++i)
      for (int ip = 0; ip < nth; ++ip) {
        double acc = 0.0;
        for (int l = m; l <= L; ++l) {
          const double left = (which == 0) ? dP[i][size_t(l) * n + m] : P[i][size_t(l) * n + m];
          const double f = (which == 2) ? sigma[l] : 1.0;
          acc += f * left * P[ip][size_t(l) * n + m];
        }
        K[(size_t(m) * nth + i) * nth + ip] =
            acc * (m == 0 ? 1.0 : 2.0) * (which == 1 ? -double(m) : 1.0) * (w[ip] * 2.0 * kPi / nph);
      }
  return K;
}

std::vector<double> fourier_table(int L) {
  const int n = L + 1, nph = 2 * n;
  std::vector<double> T(size_t(nph) * 2 * n);
  for (int k = 0; k < nph; ++k)
    for (int m = 0; m < n; ++m) {
      const double ang = 2.0 * kPi * double((m * k) % nph) / nph;
      T[size_t(k) * 2 * n + m] = std::cos(ang);
      T[size_t(k) * 2 * n + n + m] = std::sin(ang);
    }
  return T;
}

void sphere_operator_into(int L, int which, const std::vector<double>& sigma, bool transposed, double* out,
                          size_t ld) {
  // assembled from the per-order factors.  An entry depends on the azimuths
  // only through d = k - k' (mod nph), so the order sum is formed once per
  // (theta row, theta column, d), nth^2 nph (L+1) multiply-adds, and the S^2
  // entries are then copies; rows are filled by several host threads.
  const int nth = L + 1, nph = 2 * (L + 1), S = nth * nph, n = L + 1;
  const std::vector<double> K = sphere_factors(L, which, sigma);
  // azimuthal factors for every difference d = k - k' (mod nph)
  std::vector<double> trig(size_t(n) * nph);
  for (int m = 0; m <= L; ++m)
    for (int d = 0; d < nph; ++d) {
      const double ang = 2.0 * kPi * double((m * d) % nph) / nph;
      trig[size_t(m) * nph + d] = (which == 1) ? std::sin(ang) : std::cos(ang);
    }
  // V[ij][ia][d]: the entry of output row (ij, k) and input column (ia, k - d)
  std::vector<double> V(size_t(nth) * nth * nph);
  for (int ij = 0; ij < nth; ++ij)
    for (int ia = 0; ia < nth; ++ia)
      for (int d = 0; d < nph; ++d) {
        double acc = 0.0;
        for (int m = 0; m <= L; ++m) acc += K[(size_t(m) * nth + ij) * nth + ia] * trig[size_t(m) * nph + d];
        V[(size_t(ij) * nth + ia) * nph + d] = acc;
      }
  auto fill = [&](int r0, int r1) {
    for (int r = r0; r < r1; ++r) {
      const int ir = r / nph, kr = r - ir * nph;
      double* row = out + size_t(r) * ld;
      for (int ic = 0; ic < nth; ++ic) {
        if (!transposed) {          // row (ir, kr) = output, column (ic, kc) = input
          const double* v = &V[(size_t(ir) * nth + ic) * nph];
          for (int kc = 0; kc < nph; ++kc) row[ic * nph + kc] = v[(kr - kc + nph) % nph];
        } else {                    // row (ir, kr) = input, column (ic, kc) = output
          const double* v = &V[(size_t(ic) * nth + ir) * nph];
          for (int kc = 0; kc < nph; ++kc) row[ic * nph + kc] = v[(kc - kr + nph) % nph];
        }
      }
    }
  };
  const int nt = S >= 2048 ? std::max(1, std::min(16, int(std::thread::hardware_concurrency()))) : 1;
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t) pool.emplace_back(fill, int(size_t(S) * t / nt), int(size_t(S) * (t + 1) / nt));
  for (auto& th : pool) th.join();
}

std::vector<double> sphere_operator(int L, int which, const std::vector<double>& sigma) {
  const size_t S = size_t(2) * (L + 1) * (L + 1);
  std::vector<double> M(S * S);
  sphere_operator_into(L, which, sigma, false, M.data(), S);
  return M;
}

std::vector<double> angular_table(int L) {
  std::vector<double> x, w;
  gauss_legendre(L, x, w);
  int nth = L + 1, nph = 2 * (L + 1), S = nth * nph;
  std::vector<double> t(size_t(S) * 5);
  for (int i = 0; i < nth; ++i) {
    double st = std::sqrt(1.0 - x[i] * x[i]);
    for (int k = 0; k < nph; ++k) {
      double ph = 2.0 * kPi * k / nph;
      size_t a = size_t(i * nph + k) * 5;
      t[a + 0] = st;
      t[a + 1] = x[i];
      t[a + 2] = std::sin(ph);
      t[a + 3] = std::cos(ph);
      t[a + 4] = w[i] * 2.0 * kPi / nph;
    }
  }
  return t;
}

}  // namespace ghsetup

// Host-side construction of the tensor-coupled angular filter.
//
// The paper filters a tensor field on an I1 x S2 shell in three steps:
// PhysToSpec of every component, one sparse (N_e N_s) x (N_e N_s) matrix that
// couples the tensor components (CSR), SpecToPhys (section on spectral
// filtering on I1 x S2, with the Heaviside and ExpCheb filter functions).  It
// does not say what the coupling is.  Here the filter acts on total angular
// momentum: a tensor field rotates as a whole (positions and spatial indices),
// with generators G_k = -(r x grad)_k + Sigma_k, Sigma_k = e_k x (.) on every
// spatial index; J^2 = -sum_k G_k^2 has eigenvalues j(j+1) and
//   F = sum_j sigma(j) P_j = p(J^2),
// p the polynomial through (j(j+1), sigma(j)) for the j that occur at degree
// l.  J^2 keeps the orbital degree l, so F is built per l.
//
// On one degree l (local mode index mu = m + l):
//  * (r x grad)_k = i L_k with the angular-momentum ladder L_+- = L_x +- i L_y,
//    L_+- Y_l^m = sqrt(l(l+1) - m(m+-1)) Y_l^{m+-1} (Condon-Shortley Y_l^m);
//    the real harmonics are combinations of those, so the real coefficient
//    matrices come from the complex ones by that change of basis;
//  * J^2 = l(l+1) + S^2 + 2 sum_k Sigma_k (x) (r x grad)_k with
//    S^2 = -sum_k Sigma_k^2, a sparse matrix on (component, mode);
//  * p(J^2) in Newton form on the rescaled variable (J^2 - c)/h, applied to
//    the expansion of the stored components (Horner steps of sparse x dense).
#include "ghmi_tensor_filter.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <thread>

#include "ghmi_setup.h"

namespace ghtf {

namespace {

constexpr double kPi = 3.14159265358979323846;
typedef std::complex<double> cplx;

// Coefficient matrices [out][in] of (r x grad)_x, _y, _z on the real
// harmonics of degree l (mode index m + l).
void orbital(int l, std::vector<double> R[3]) {
  const int n = 2 * l + 1;
  // complex harmonics Z_mu = P_l^|mu| e^{i mu phi} (no Condon-Shortley phase):
  // Z_mu = eps_mu Y_l^mu with eps_mu = (-1)^mu for mu >= 0 and 1 for mu < 0
  auto eps = [](int mu) { return (mu >= 0 && (mu & 1)) ? -1.0 : 1.0; };
  auto lad = [l](int mu, int d) { return std::sqrt(double(l) * (l + 1) - double(mu) * (mu + d)); };
  std::vector<cplx> A[3];
  for (int k = 0; k < 3; ++k) A[k].assign(size_t(n) * n, cplx(0, 0));
  const cplx I(0, 1);
  for (int mu = -l; mu <= l; ++mu) {
    const int c = mu + l;
    if (mu + 1 <= l) {           // L_+ Z_mu = (eps_mu / eps_mu+1) a_+ Z_mu+1
      const double v = eps(mu) / eps(mu + 1) * lad(mu, 1);
      A[0][size_t(c + 1) * n + c] += 0.5 * I * v;   // (r x grad)_x = i (L_+ + L_-)/2
      A[1][size_t(c + 1) * n + c] += 0.5 * v;       // (r x grad)_y = (L_+ - L_-)/2
    }
    if (mu - 1 >= -l) {
      const double v = eps(mu) / eps(mu - 1) * lad(mu, -1);
      A[0][size_t(c - 1) * n + c] += 0.5 * I * v;
      A[1][size_t(c - 1) * n + c] -= 0.5 * v;
    }
    A[2][size_t(c) * n + c] = I * double(mu);       // (r x grad)_z = i L_z
  }
  // real harmonics b_s = sum_mu U[s][mu] Z_mu: cos m = (Z_m + Z_-m)/sqrt2,
  // sin m = (Z_m - Z_-m)/(sqrt2 i), m = 0: Z_0; coefficients then transform
  // as c' = conj(U) A U^T
  std::vector<cplx> U(size_t(n) * n, cplx(0, 0));
  const double r2 = 1.0 / std::sqrt(2.0);
  U[size_t(l) * n + l] = 1.0;
  for (int m = 1; m <= l; ++m) {
    U[size_t(l + m) * n + (l + m)] = r2;
    U[size_t(l + m) * n + (l - m)] = r2;
    U[size_t(l - m) * n + (l + m)] = -I * r2;
    U[size_t(l - m) * n + (l - m)] = I * r2;
  }
  for (int k = 0; k < 3; ++k) {
    R[k].assign(size_t(n) * n, 0.0);
    for (int s = 0; s < n; ++s)
      for (int t = 0; t < n; ++t) {
        cplx acc(0, 0);
        for (int a = 0; a < n; ++a) {
          const cplx ua = std::conj(U[size_t(s) * n + a]);
          if (ua == cplx(0, 0)) continue;
          for (int b = 0; b < n; ++b) acc += ua * A[k][size_t(a) * n + b] * U[size_t(t) * n + b];
        }
        R[k][size_t(s) * n + t] = acc.real();
      }
  }
}

// One GH tensor: first stored field, slot dimensions (3 spatial, 4 spacetime).
struct Tensor {
  int first, nst, nslot;
  int dims[3];
};
const Tensor kTensors[2] = {{0, 10, 2, {4, 4, 0}}, {20, 30, 3, {3, 4, 4}}};   // psi (and Pi), Phi
const int kPair[10][2] = {{0, 0}, {0, 1}, {0, 2}, {0, 3}, {1, 1}, {1, 2}, {1, 3}, {2, 2}, {2, 3}, {3, 3}};

int levi(int a, int b, int c) { return (a - b) * (b - c) * (c - a) / 2; }

int nfull(const Tensor& t) {
  int n = 1;
  for (int s = 0; s < t.nslot; ++s) n *= t.dims[s];
  return n;
}

// Sigma_k on the full components of a tensor (dense nf x nf).
std::vector<double> index_generator(const Tensor& t, int k) {
  const int nf = nfull(t);
  std::vector<double> S(size_t(nf) * nf, 0.0);
  for (int row = 0; row < nf; ++row) {
    int idx[3], r = row;
    for (int s = t.nslot - 1; s >= 0; --s) { idx[s] = r % t.dims[s]; r /= t.dims[s]; }
    for (int s = 0; s < t.nslot; ++s) {
      const int off = t.dims[s] == 4 ? 1 : 0;     // spacetime slot: index 0 is time
      const int a = idx[s] - off;
      if (a < 0) continue;
      for (int c = 0; c < 3; ++c) {
        const int e = levi(a, k, c);               // (e_k x V)_a = eps_{a k c} V_c
        if (!e) continue;
        int j[3] = {idx[0], idx[1], idx[2]};
        j[s] = c + off;
        int col = 0;
        for (int q = 0; q < t.nslot; ++q) col = col * t.dims[q] + j[q];
        S[size_t(row) * nf + col] += e;
      }
    }
  }
  return S;
}

// Full component indices of stored component e (local): one or two (pair a != b).
int expand(const Tensor& t, int e, int out[2]) {
  const int pre = e / 10, p = e % 10, a = kPair[p][0], b = kPair[p][1];
  const int base = (t.nslot == 3) ? pre * 16 : 0;
  out[0] = base + a * 4 + b;
  out[1] = base + b * 4 + a;
  return a == b ? 1 : 2;
}

struct Triplet {
  int row, col;
  double v;
};

// Coupling of one tensor at degree l: triplets in global (field, mode) indices.
void degree_block(int L, int l, const Tensor& t, int kind, const double* params, std::vector<Triplet>& out,
                  const std::vector<double> Sig[3], const std::vector<double>& S2) {
  const int nm = 2 * l + 1, nf = nfull(t), dim = nf * nm, ns = (L + 1) * (L + 1);
  std::vector<double> Lr[3];
  orbital(l, Lr);
  // sparse J^2 (rows of (component, mode))
  std::vector<long long> jp(dim + 1, 0);
  std::vector<int> jc;
  std::vector<double> jv;
  std::vector<double> row(dim);
  const double tol = 1e-12 * (double(l) * (l + 1) + 16.0);
  for (int a = 0; a < nf; ++a)
    for (int mu = 0; mu < nm; ++mu) {
      std::fill(row.begin(), row.end(), 0.0);
      row[size_t(a) * nm + mu] += double(l) * (l + 1);
      for (int b = 0; b < nf; ++b) {
        const double s2 = S2[size_t(a) * nf + b];
        if (s2 != 0.0) row[size_t(b) * nm + mu] += s2;
        for (int k = 0; k < 3; ++k) {
          const double sg = Sig[k][size_t(a) * nf + b];
          if (sg == 0.0) continue;
          for (int nu = 0; nu < nm; ++nu) row[size_t(b) * nm + nu] += 2.0 * sg * Lr[k][size_t(mu) * nm + nu];
        }
      }
      for (int q = 0; q < dim; ++q)
        if (std::fabs(row[q]) > tol) { jc.push_back(q); jv.push_back(row[q]); }
      jp[size_t(a) * nm + mu + 1] = (long long)jc.size();
    }
  // interpolation nodes j(j+1), j = max(0, l - rank) .. l + rank, Newton
  // form; evaluated in extended precision (the divided differences of a
  // steep or jumping sigma are large, and double rounding of the Horner steps
  // would reach 1e-13 of F)
  typedef long double ext;
  const int j0 = std::max(0, l - t.nslot), j1 = l + t.nslot, nj = j1 - j0 + 1;
  const ext lo = ext(j0) * (j0 + 1), hi = ext(j1) * (j1 + 1);
  const ext c0 = 0.5L * (lo + hi), h = std::max(0.5L * (hi - lo), 1.0L);
  std::vector<ext> x(nj), dd(nj);
  for (int q = 0; q < nj; ++q) {
    const int j = j0 + q;
    x[q] = (ext(j) * (j + 1) - c0) / h;
    dd[q] = sigma(kind, params, L, j);
  }
  for (int k = 1; k < nj; ++k)
    for (int q = nj - 1; q >= k; --q) dd[q] = (dd[q] - dd[q - 1]) / (x[q] - x[q - k]);
  // Y = p(J^2) E, E the expansion of the stored components (columns (e, nu))
  const int ncol = t.nst * nm;
  std::vector<ext> E(size_t(dim) * ncol, 0.0L);
  for (int e = 0; e < t.nst; ++e) {
    int f[2];
    const int nfe = expand(t, e, f);
    for (int q = 0; q < nfe; ++q)
      for (int nu = 0; nu < nm; ++nu) E[(size_t(f[q]) * nm + nu) * ncol + size_t(e) * nm + nu] = 1.0;
  }
  std::vector<ext> Y(E.size()), Z(E.size());
  for (size_t q = 0; q < Y.size(); ++q) Y[q] = dd[nj - 1] * E[q];
  for (int k = nj - 2; k >= 0; --k) {
    const ext shift = -c0 / h - x[k];
    for (int r = 0; r < dim; ++r) {
      ext* z = &Z[size_t(r) * ncol];
      const ext* yr = &Y[size_t(r) * ncol];
      const ext* er = &E[size_t(r) * ncol];
      for (int q = 0; q < ncol; ++q) z[q] = shift * yr[q] + dd[k] * er[q];
      for (long long p = jp[r]; p < jp[r + 1]; ++p) {
        const ext w = jv[p] / h;
        const ext* yq = &Y[size_t(jc[p]) * ncol];
        for (int q = 0; q < ncol; ++q) z[q] += w * yq[q];
      }
    }
    Y.swap(Z);
  }
  // stored rows: the (a <= b) full component of each stored component
  const int s0 = l * l;
  const int copies = (t.first == 0) ? 2 : 1;      // psi and Pi share the tensor type
  for (int cpy = 0; cpy < copies; ++cpy) {
    const int first = t.first + 10 * cpy;
    for (int e = 0; e < t.nst; ++e) {
      int f[2];
      expand(t, e, f);
      for (int mu = 0; mu < nm; ++mu) {
        const ext* yr = &Y[(size_t(f[0]) * nm + mu) * ncol];
        for (int q = 0; q < ncol; ++q) {
          const double v = double(yr[q]);
          if (std::fabs(v) <= 1e-15) continue;
          const int e2 = q / nm, nu = q % nm;
          out.push_back({(first + e) * ns + s0 + mu, (first + e2) * ns + s0 + nu, v});
        }
      }
    }
  }
}

}  // namespace

double sigma(int kind, const double* params, int L, int j) {
  const double q = L > 0 ? double(j) / L : 0.0;
  if (kind == 3) return (double(j) <= params[0] * L) ? 1.0 : 0.0;
  if (q <= params[0]) return 1.0;
  return std::exp(-params[1] * std::pow((q - params[0]) / (1.0 - params[0]), params[2]));
}

Csr coupling_matrix(int L, int kind, const double* params, bool transpose) {
  const int ns = (L + 1) * (L + 1);
  // tasks (tensor, degree), largest first
  std::vector<std::pair<int, int>> tasks;
  for (int l = L; l >= 0; --l)
    for (int ti = 0; ti < 2; ++ti) tasks.push_back({ti, l});
  std::vector<std::vector<Triplet>> parts(tasks.size());
  std::vector<double> Sig[2][3], S2[2];
  for (int ti = 0; ti < 2; ++ti) {
    const int nf = nfull(kTensors[ti]);
    S2[ti].assign(size_t(nf) * nf, 0.0);
    for (int k = 0; k < 3; ++k) {
      Sig[ti][k] = index_generator(kTensors[ti], k);
      for (int a = 0; a < nf; ++a)
        for (int b = 0; b < nf; ++b) {
          double acc = 0.0;
          for (int q = 0; q < nf; ++q) acc += Sig[ti][k][size_t(a) * nf + q] * Sig[ti][k][size_t(q) * nf + b];
          S2[ti][size_t(a) * nf + b] -= acc;
        }
    }
  }
  std::atomic<size_t> next(0);
  auto worker = [&]() {
    for (size_t q = next++; q < tasks.size(); q = next++) {
      const int ti = tasks[q].first, l = tasks[q].second;
      degree_block(L, l, kTensors[ti], kind, params, parts[q], Sig[ti], S2[ti]);
    }
  };
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const unsigned nt = std::min<unsigned>(hw, unsigned(tasks.size()));
  std::vector<std::thread> pool;
  for (unsigned i = 1; i < nt; ++i) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
  // assemble CSR (rows sorted, columns sorted within a row)
  Csr m;
  m.n = 50 * ns;
  std::vector<Triplet> all;
  for (auto& p : parts) all.insert(all.end(), p.begin(), p.end());
  if (transpose)
    for (auto& t : all) std::swap(t.row, t.col);
  std::sort(all.begin(), all.end(),
            [](const Triplet& a, const Triplet& b) { return a.row != b.row ? a.row < b.row : a.col < b.col; });
  m.row_ptr.assign(m.n + 1, 0);
  m.col.resize(all.size());
  m.val.resize(all.size());
  for (size_t q = 0; q < all.size(); ++q) {
    m.row_ptr[all[q].row + 1]++;
    m.col[q] = all[q].col;
    m.val[q] = all[q].v;
  }
  for (int r = 0; r < m.n; ++r) m.row_ptr[r + 1] += m.row_ptr[r];
  return m;
}

Csr transpose(const Csr& m) {
  Csr t;
  t.n = m.n;
  t.row_ptr.assign(m.n + 1, 0);
  for (size_t q = 0; q < m.col.size(); ++q) t.row_ptr[m.col[q] + 1]++;
  for (int r = 0; r < m.n; ++r) t.row_ptr[r + 1] += t.row_ptr[r];
  t.col.resize(m.col.size());
  t.val.resize(m.val.size());
  std::vector<long long> next(t.row_ptr.begin(), t.row_ptr.end() - 1);
  for (int r = 0; r < m.n; ++r)                    // rows in order: columns of t come out sorted
    for (long long p = m.row_ptr[r]; p < m.row_ptr[r + 1]; ++p) {
      const long long d = next[m.col[p]]++;
      t.col[d] = r;
      t.val[d] = m.val[p];
    }
  return t;
}

namespace {

// Y_s at every grid point, [S][ns].
std::vector<double> ylm_grid(int L, std::vector<double>* weights) {
  std::vector<double> x, w;
  ghsetup::gauss_legendre(L, x, w);
  const int n = L + 1, nph = 2 * n, S = n * nph, ns = n * n;
  std::vector<double> Y(size_t(S) * ns, 0.0), P, dP;
  if (weights) weights->resize(S);
  for (int i = 0; i < n; ++i) {
    ghsetup::legendre_normalised(L, x[i], P, dP);
    for (int k = 0; k < nph; ++k) {
      const int a = i * nph + k;
      if (weights) (*weights)[a] = w[i] * 2.0 * kPi / nph;
      for (int l = 0; l <= L; ++l) {
        Y[size_t(a) * ns + l * l + l] = P[size_t(l) * n + 0];
        for (int m = 1; m <= l; ++m) {
          const double ang = 2.0 * kPi * double((m * k) % nph) / nph;
          const double f = std::sqrt(2.0) * P[size_t(l) * n + m];
          Y[size_t(a) * ns + l * l + l + m] = f * std::cos(ang);
          Y[size_t(a) * ns + l * l + l - m] = f * std::sin(ang);
        }
      }
    }
  }
  return Y;
}

}  // namespace

std::vector<double> sphere_analysis(int L) {
  std::vector<double> w;
  const std::vector<double> Y = ylm_grid(L, &w);
  const int S = 2 * (L + 1) * (L + 1), ns = (L + 1) * (L + 1);
  std::vector<double> A(size_t(ns) * S);
  for (int a = 0; a < S; ++a)
    for (int s = 0; s < ns; ++s) A[size_t(s) * S + a] = w[a] * Y[size_t(a) * ns + s];
  return A;
}

std::vector<double> sphere_synthesis(int L) { return ylm_grid(L, nullptr); }

std::vector<double> legendre_tables(int L) {
  std::vector<double> x, w, P, dP;
  ghsetup::gauss_legendre(L, x, w);
  const int n = L + 1, ns = n * n, nph = 2 * n;
  std::vector<double> T(size_t(2) * ns * n, 0.0);
  for (int i = 0; i < n; ++i) {
    ghsetup::legendre_normalised(L, x[i], P, dP);
    for (int l = 0; l <= L; ++l)
      for (int m = -l; m <= l; ++m) {
        const int s = l * l + l + m, am = m < 0 ? -m : m;
        const double v = (am ? std::sqrt(2.0) : 1.0) * P[size_t(l) * n + am];
        T[size_t(i) * ns + s] = v * w[i] * 2.0 * kPi / nph;
        T[size_t(ns) * n + size_t(s) * n + i] = v;
      }
  }
  return T;
}

}  // namespace ghtf

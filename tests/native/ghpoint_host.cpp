// Host build of the device pointwise reverse pass (paper_1804_09101_amd/csrc/gh_point.h),
// so that CPU tests can check it against the oracle.  Test infrastructure only.
#include "gh_point.h"

extern "C" int ghp_rhs_vjp(int n, const double* u, const double* du, const double* H, const double* dH,
                           const double* g, const double* lam, double* ubar, double* dubar, double* gbar) {
  for (int p = 0; p < n; ++p)
    ghp::rhs_vjp(u + 50 * p, reinterpret_cast<const double(*)[50]>(du + 150 * p), H + 4 * p, dH + 16 * p,
                 g[0], g[1], g[2], lam + 50 * p, ubar + 50 * p, reinterpret_cast<double(*)[50]>(dubar + 150 * p),
                 gbar);
  return 0;
}

extern "C" int ghp_gauge_constraint_vjp(int n, const double* u, const double* H, const double* Cbar, double* ubar) {
  for (int p = 0; p < n; ++p) {
    for (int f = 0; f < 50; ++f) ubar[50 * p + f] = 0.0;
    ghp::gauge_constraint_vjp(u + 50 * p, H + 4 * p, Cbar + 4 * p, ubar + 50 * p);
  }
  return 0;
}

extern "C" int ghp_rhs_vjp_pairs(int n, const double* u, const double* du, const double* H, const double* dH,
                                 const double* g, const double* lam, double* ubar, double* dubar, double* gbar) {
  for (int p = 0; p < n; ++p) {
    const double* d = du + 150 * p;
    double* db = dubar + 150 * p;
    auto load = [&](int m, double* dpsi, double* dPi, double (*dPhi)[3]) {
      for (int k = 0; k < 3; ++k) {
        dpsi[k] = d[50 * k + m];
        dPi[k] = d[50 * k + 10 + m];
        for (int i = 0; i < 3; ++i) dPhi[k][i] = d[50 * k + 20 + 10 * i + m];
      }
    };
    auto store = [&](int m, const double* dpsi_b, const double* dPi_b, const double (*dPhi_b)[3]) {
      for (int k = 0; k < 3; ++k) {
        db[50 * k + m] = dpsi_b[k];
        db[50 * k + 10 + m] = dPi_b[k];
        for (int i = 0; i < 3; ++i) db[50 * k + 20 + 10 * i + m] = dPhi_b[k][i];
      }
    };
    ghp::rhs_vjp_pairs(u + 50 * p, H + 4 * p, dH + 16 * p, g[0], g[1], g[2], lam + 50 * p, load, store,
                       ubar + 50 * p, gbar);
  }
  return 0;
}

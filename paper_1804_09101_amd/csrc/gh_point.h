// Pointwise generalized-harmonic algebra at one collocation point, in a form
// that compiles for the device and the host: the forward RHS and its
// hand-written reverse (vector-Jacobian product).
//
// Equations: the first-order GH system of Lindblom, Scheel, Kidder, Owen &
// Rinne (2006), eqs. 35-37 there (the paper names this "GHEqns" but does not
// print it):
//   d_t psi_ab  = (1+g1) N^k d_k psi_ab - N Pi_ab - g1 N^i Phi_iab
//   d_t Pi_ab   = N^k d_k Pi_ab - N g^ki d_k Phi_iab + g1 g2 N^k d_k psi_ab
//                 + 2N Q_ab - N (d_a H_b + d_b H_a) + 2N Gamma^c_ab H_c
//                 - 1/2 N t^c t^d Pi_cd Pi_ab - N t^c Pi_ci g^ij Phi_jab
//                 + g0 N (t_a C_b + t_b C_a - psi_ab t^c C_c) - g1 g2 N^i Phi_iab
//   d_t Phi_iab = N^k d_k Phi_iab - N d_i Pi_ab + g2 N d_i psi_ab
//                 + 1/2 N t^c t^d Phi_icd Pi_ab + N g^jk t^c Phi_ijc Phi_kab - g2 N Phi_iab
// with Q = psi^cd (g^ij Phi_ica Phi_jdb - Pi_ca Pi_db - psi^ef Gamma_ace Gamma_bdf),
// C_a = H_a + psi^bc Gamma_abc, Gamma_cab = (d_a psi_cb + d_b psi_ca - d_c psi_ab)/2,
// d_0 psi = -N Pi + N^i Phi_i, d_i psi = Phi_i.
//
// Storage: fields in pair form (50 = psi 10, Pi 10, Phi_x 10, Phi_y 10, Phi_z 10,
// pairs 00,01,02,03,11,12,13,22,23,33); derivatives du[k][50] (k = x,y,z);
// H[4]; dH[16] = d_a H_b at a*4+b.  The reverse pass works on full symmetric
// 4x4 tensors: an output pair cotangent is split evenly over (a,b) and (b,a),
// and the adjoint of an input pair is the sum of its two full entries.
#pragma once

#if defined(__HIPCC__)
#define GHP_HD __host__ __device__ inline
#else
#define GHP_HD inline
#endif

#include <math.h>

namespace ghp {

GHP_HD int pair(int a, int b) {
  return a <= b ? (a * 4 - a * (a - 1) / 2 + b - a) : (b * 4 - b * (b - 1) / 2 + a - b);
}

// Forward quantities of one point, full tensors.
struct Fwd {
  double psi[4][4], Pi[4][4], Phi[3][4][4];
  double gi[3][3], beta[3], Nu[3], N, tu[4], P[4][4];
  double d4[4][4][4];          // d_a psi_bc
  double G[4][4][4];           // Gamma_cab, index [c][a][b]
  double C[4], Hup[4], tC;
};

GHP_HD void unpack_sym(const double* v, double (*X)[4]) {
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) X[a][b] = v[pair(a, b)];
}

GHP_HD void forward(const double* u, const double* H, Fwd& F) {
  unpack_sym(u, F.psi);
  unpack_sym(u + 10, F.Pi);
  for (int i = 0; i < 3; ++i) unpack_sym(u + 20 + 10 * i, F.Phi[i]);
  const double g11 = F.psi[1][1], g12 = F.psi[1][2], g13 = F.psi[1][3];
  const double g22 = F.psi[2][2], g23 = F.psi[2][3], g33 = F.psi[3][3];
  const double A = g22 * g33 - g23 * g23, B = g13 * g23 - g12 * g33, Cc = g12 * g23 - g13 * g22;
  const double D = g11 * g33 - g13 * g13, E = g12 * g13 - g11 * g23, Fm = g11 * g22 - g12 * g12;
  const double idet = 1.0 / (g11 * A + g12 * B + g13 * Cc);
  F.gi[0][0] = A * idet; F.gi[0][1] = F.gi[1][0] = B * idet; F.gi[0][2] = F.gi[2][0] = Cc * idet;
  F.gi[1][1] = D * idet; F.gi[1][2] = F.gi[2][1] = E * idet; F.gi[2][2] = Fm * idet;
  for (int i = 0; i < 3; ++i) F.beta[i] = F.psi[0][i + 1];
  double nsq = -F.psi[0][0];
  for (int i = 0; i < 3; ++i) {
    F.Nu[i] = F.gi[i][0] * F.beta[0] + F.gi[i][1] * F.beta[1] + F.gi[i][2] * F.beta[2];
    nsq += F.Nu[i] * F.beta[i];
  }
  F.N = sqrt(nsq);
  F.tu[0] = 1.0 / F.N;
  for (int i = 0; i < 3; ++i) F.tu[i + 1] = -F.Nu[i] / F.N;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      F.P[a][b] = ((a > 0 && b > 0) ? F.gi[a - 1][b - 1] : 0.0) - F.tu[a] * F.tu[b];
  for (int b = 0; b < 4; ++b)
    for (int c = 0; c < 4; ++c) {
      double v = -F.N * F.Pi[b][c];
      for (int i = 0; i < 3; ++i) v += F.Nu[i] * F.Phi[i][b][c];
      F.d4[0][b][c] = v;
      for (int i = 0; i < 3; ++i) F.d4[i + 1][b][c] = F.Phi[i][b][c];
    }
  for (int c = 0; c < 4; ++c)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        F.G[c][a][b] = 0.5 * (F.d4[a][c][b] + F.d4[b][c][a] - F.d4[c][a][b]);
  F.tC = 0.0;
  for (int a = 0; a < 4; ++a) {
    double s = H[a];
    for (int b = 0; b < 4; ++b)
      for (int c = 0; c < 4; ++c) s += F.P[b][c] * F.G[a][b][c];
    F.C[a] = s;
    double h = 0.0;
    for (int c = 0; c < 4; ++c) h += F.P[a][c] * H[c];
    F.Hup[a] = h;
  }
  for (int a = 0; a < 4; ++a) F.tC += F.tu[a] * F.C[a];
}

// 4x4 helpers (full matrices)
GHP_HD void mm(const double (*X)[4], const double (*Y)[4], double (*Z)[4]) {
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      double s = 0.0;
      for (int c = 0; c < 4; ++c) s += X[a][c] * Y[c][b];
      Z[a][b] = s;
    }
}
GHP_HD void mmm(const double (*X)[4], const double (*Y)[4], const double (*W)[4], double (*Z)[4]) {
  double T[4][4];
  mm(X, Y, T);
  mm(T, W, Z);
}

// Shared end of the reverse pass: from the cotangents of C_a, Gamma_cab, psi^ab,
// t^a, N, N^i and g^ij back to psi, Pi, Phi (full tensors, accumulated).
GHP_HD void reverse_tail(const Fwd& F, const double* C_b, double (*G_b)[4][4], double (*P_b)[4],
                         double* tu_b, double& N_b, double* Nu_b, double (*gi_b)[3], double (*psi_b)[4],
                         double (*Pi_b)[4], double (*Phi_b)[4][4]) {
  const double N = F.N;
  // C_a = H_a + P^bc G_abc
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      for (int c = 0; c < 4; ++c) {
        P_b[b][c] += C_b[a] * F.G[a][b][c];
        G_b[a][b][c] += C_b[a] * F.P[b][c];
      }
  // Gamma_cab = (d4_acb + d4_bca - d4_cab)/2
  double d4_b[4][4][4] = {};
  for (int c = 0; c < 4; ++c)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        const double g = 0.5 * G_b[c][a][b];
        d4_b[a][c][b] += g;
        d4_b[b][c][a] += g;
        d4_b[c][a][b] -= g;
      }
  // d4_0 = -N Pi + N^i Phi_i ; d4_(i+1) = Phi_i
  for (int b = 0; b < 4; ++b)
    for (int c = 0; c < 4; ++c) {
      const double g = d4_b[0][b][c];
      N_b += -g * F.Pi[b][c];
      Pi_b[b][c] += -N * g;
      for (int i = 0; i < 3; ++i) {
        Nu_b[i] += g * F.Phi[i][b][c];
        Phi_b[i][b][c] += F.Nu[i] * g + d4_b[i + 1][b][c];
      }
    }
  // P^ab = g^ab - t^a t^b
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      if (a > 0 && b > 0) gi_b[a - 1][b - 1] += P_b[a][b];
      tu_b[a] += -P_b[a][b] * F.tu[b];
      tu_b[b] += -P_b[a][b] * F.tu[a];
    }
  // t^a = (1/N, -N^i/N)
  N_b += -tu_b[0] / (N * N);
  for (int i = 0; i < 3; ++i) {
    N_b += tu_b[i + 1] * F.Nu[i] / (N * N);
    Nu_b[i] += -tu_b[i + 1] / N;
  }
  // N = sqrt(N^i beta_i - psi_00)
  const double nsq_b = N_b / (2.0 * N);
  double beta_b[3];
  for (int i = 0; i < 3; ++i) {
    Nu_b[i] += nsq_b * F.beta[i];
    beta_b[i] = nsq_b * F.Nu[i];
  }
  psi_b[0][0] += -nsq_b;
  // N^i = g^ij beta_j
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      gi_b[i][j] += Nu_b[i] * F.beta[j];
      beta_b[j] += F.gi[i][j] * Nu_b[i];
    }
  for (int i = 0; i < 3; ++i) psi_b[0][i + 1] += beta_b[i];
  // g^ij = inv(g_ij): gbar_ij = -(g^-1 gi_b g^-1)_ij
  {
    double T[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += gi_b[i][k] * F.gi[k][j];
        T[i][j] = s;
      }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += F.gi[i][k] * T[k][j];
        psi_b[i + 1][j + 1] += -s;
      }
  }
}

// Reverse pass.  lam: cotangent of d_t u (50, pair form).  Writes ubar[50],
// dubar[3][50] (cotangents of u and of its Cartesian derivatives) and adds to
// gbar[3] (cotangents of gamma0, gamma1, gamma2).
GHP_HD void rhs_vjp(const double* u, const double (*du)[50], const double* H, const double* dH,
                    double g0, double g1, double g2, const double* lam, double* ubar,
                    double (*dubar)[50], double* gbar) {
  Fwd F;
  forward(u, H, F);
  const double N = F.N;
  double dpsi[3][4][4], dPi[3][4][4], dPhi[3][3][4][4];
  for (int k = 0; k < 3; ++k) {
    unpack_sym(du[k], dpsi[k]);
    unpack_sym(du[k] + 10, dPi[k]);
    for (int i = 0; i < 3; ++i) unpack_sym(du[k] + 20 + 10 * i, dPhi[k][i]);
  }
  // output cotangents, split over the symmetric pair
  double Lpsi[4][4], LPi[4][4], LPhi[3][4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      const double f = (a == b) ? 1.0 : 0.5;
      Lpsi[a][b] = f * lam[pair(a, b)];
      LPi[a][b] = f * lam[10 + pair(a, b)];
      for (int i = 0; i < 3; ++i) LPhi[i][a][b] = f * lam[20 + 10 * i + pair(a, b)];
    }
  // adjoint accumulators (full tensors)
  double psi_b[4][4] = {}, Pi_b[4][4] = {}, Phi_b[3][4][4] = {};
  double dpsi_b[3][4][4] = {}, dPi_b[3][4][4] = {}, dPhi_b[3][3][4][4] = {};
  double Nu_b[3] = {}, N_b = 0.0, gi_b[3][3] = {}, tu_b[4] = {}, P_b[4][4] = {};
  double G_b[4][4][4] = {}, C_b[4] = {}, Hup_b[4] = {}, tC_b = 0.0;
  double gb0 = 0.0, gb1 = 0.0, gb2 = 0.0;

  // secondary forward quantities
  double ttPhi[3], tPhi[3][3], Gt[3][3];
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
    for (int c = 0; c < 4; ++c)
      for (int d = 0; d < 4; ++d) s += F.tu[c] * F.tu[d] * F.Phi[i][c][d];
    ttPhi[i] = s;
    for (int j = 0; j < 3; ++j) {
      double t = 0.0;
      for (int c = 0; c < 4; ++c) t += F.tu[c] * F.Phi[i][j + 1][c];
      tPhi[i][j] = t;
    }
  }
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) {
      double s = 0.0;
      for (int j = 0; j < 3; ++j) s += F.gi[j][k] * tPhi[i][j];
      Gt[i][k] = s;
    }
  double ttPi = 0.0, w[3], v[3];
  for (int c = 0; c < 4; ++c)
    for (int d = 0; d < 4; ++d) ttPi += F.tu[c] * F.tu[d] * F.Pi[c][d];
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
    for (int c = 0; c < 4; ++c) s += F.tu[c] * F.Pi[c][i + 1];
    w[i] = s;
  }
  for (int j = 0; j < 3; ++j) v[j] = w[0] * F.gi[0][j] + w[1] * F.gi[1][j] + w[2] * F.gi[2][j];
  const double tl[4] = {-N, 0.0, 0.0, 0.0};
  double Dm[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) Dm[a][b] = tl[a] * F.C[b] + tl[b] * F.C[a] - F.psi[a][b] * F.tC;
  // Q = sum_j R_j P Phi_j - Pi P Pi - T3, R_j = g^ji Phi_i, T3_ab = <G_a, P G_b P>
  double R[3][4][4];
  for (int j = 0; j < 3; ++j)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        R[j][a][b] = F.gi[j][0] * F.Phi[0][a][b] + F.gi[j][1] * F.Phi[1][a][b] + F.gi[j][2] * F.Phi[2][a][b];
  double PGP[4][4][4];
  for (int b = 0; b < 4; ++b) mmm(F.P, F.G[b], F.P, PGP[b]);
  double Q[4][4];
  {
    double T[4][4];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) Q[a][b] = 0.0;
    for (int j = 0; j < 3; ++j) {
      mmm(R[j], F.P, F.Phi[j], T);
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) Q[a][b] += T[a][b];
    }
    mmm(F.Pi, F.P, F.Pi, T);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        double t3 = 0.0;
        for (int c = 0; c < 4; ++c)
          for (int e = 0; e < 4; ++e) t3 += F.G[a][c][e] * PGP[b][c][e];
        Q[a][b] += -T[a][b] - t3;
      }
  }

  // (A) d_t psi
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      const double L = Lpsi[a][b];
      double adv = 0.0, nphi = 0.0;
      for (int k = 0; k < 3; ++k) {
        dpsi_b[k][a][b] += (1.0 + g1) * F.Nu[k] * L;
        Nu_b[k] += L * ((1.0 + g1) * dpsi[k][a][b] - g1 * F.Phi[k][a][b]);
        Phi_b[k][a][b] += -g1 * F.Nu[k] * L;
        adv += F.Nu[k] * dpsi[k][a][b];
        nphi += F.Nu[k] * F.Phi[k][a][b];
      }
      N_b += -L * F.Pi[a][b];
      Pi_b[a][b] += -N * L;
      gb1 += L * (adv - nphi);
    }

  // (B) d_t Phi_i
  double ttPhi_b[3] = {}, Gt_b[3][3] = {}, tPhi_b[3][3] = {};
  for (int i = 0; i < 3; ++i)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        const double L = LPhi[i][a][b];
        double gtp = 0.0;
        for (int k = 0; k < 3; ++k) {
          dPhi_b[k][i][a][b] += F.Nu[k] * L;
          Nu_b[k] += L * dPhi[k][i][a][b];
          Gt_b[i][k] += N * L * F.Phi[k][a][b];
          Phi_b[k][a][b] += N * Gt[i][k] * L;
          gtp += Gt[i][k] * F.Phi[k][a][b];
        }
        dPi_b[i][a][b] += -N * L;
        dpsi_b[i][a][b] += g2 * N * L;
        N_b += L * (-dPi[i][a][b] + g2 * dpsi[i][a][b] + 0.5 * ttPhi[i] * F.Pi[a][b] + gtp -
                    g2 * F.Phi[i][a][b]);
        gb2 += L * N * (dpsi[i][a][b] - F.Phi[i][a][b]);
        ttPhi_b[i] += 0.5 * N * L * F.Pi[a][b];
        Pi_b[a][b] += 0.5 * N * L * ttPhi[i];
        Phi_b[i][a][b] += -g2 * N * L;
      }
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k)
      for (int j = 0; j < 3; ++j) {
        gi_b[j][k] += Gt_b[i][k] * tPhi[i][j];
        tPhi_b[i][j] += Gt_b[i][k] * F.gi[j][k];
      }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int c = 0; c < 4; ++c) {
        tu_b[c] += tPhi_b[i][j] * F.Phi[i][j + 1][c];
        Phi_b[i][j + 1][c] += tPhi_b[i][j] * F.tu[c];
      }
  for (int i = 0; i < 3; ++i)
    for (int c = 0; c < 4; ++c)
      for (int d = 0; d < 4; ++d) {
        tu_b[c] += 2.0 * ttPhi_b[i] * F.tu[d] * F.Phi[i][c][d];
        Phi_b[i][c][d] += ttPhi_b[i] * F.tu[c] * F.tu[d];
      }

  // (C) d_t Pi
  double Q_b[4][4] = {}, D_b[4][4] = {}, ttPi_b = 0.0, v_b[3] = {};
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      const double L = LPi[a][b];
      double adv = 0.0, nphi = 0.0, div = 0.0, hg = 0.0, vphi = 0.0;
      for (int k = 0; k < 3; ++k) {
        dPi_b[k][a][b] += F.Nu[k] * L;
        Nu_b[k] += L * (dPi[k][a][b] + g1 * g2 * dpsi[k][a][b] - g1 * g2 * F.Phi[k][a][b]);
        dpsi_b[k][a][b] += g1 * g2 * F.Nu[k] * L;
        Phi_b[k][a][b] += -g1 * g2 * F.Nu[k] * L;
        adv += F.Nu[k] * dpsi[k][a][b];
        nphi += F.Nu[k] * F.Phi[k][a][b];
        for (int i = 0; i < 3; ++i) {
          dPhi_b[k][i][a][b] += -N * F.gi[k][i] * L;
          gi_b[k][i] += -N * L * dPhi[k][i][a][b];
          div += F.gi[k][i] * dPhi[k][i][a][b];
        }
        v_b[k] += -N * L * F.Phi[k][a][b];
        Phi_b[k][a][b] += -N * v[k] * L;
        vphi += v[k] * F.Phi[k][a][b];
      }
      for (int d = 0; d < 4; ++d) {
        Hup_b[d] += 2.0 * N * L * F.G[d][a][b];
        G_b[d][a][b] += 2.0 * N * F.Hup[d] * L;
        hg += F.Hup[d] * F.G[d][a][b];
      }
      gb1 += g2 * L * (adv - nphi);
      gb2 += g1 * L * (adv - nphi);
      N_b += L * (-div + 2.0 * Q[a][b] - (dH[a * 4 + b] + dH[b * 4 + a]) + 2.0 * hg -
                  0.5 * ttPi * F.Pi[a][b] - vphi + g0 * Dm[a][b]);
      Q_b[a][b] += 2.0 * N * L;
      ttPi_b += -0.5 * N * L * F.Pi[a][b];
      Pi_b[a][b] += -0.5 * N * ttPi * L;
      D_b[a][b] += g0 * N * L;
      gb0 += N * L * Dm[a][b];
    }
  // D = t_a C_b + t_b C_a - psi_ab tC, t_a = (-N, 0, 0, 0)
  {
    double tl_b[4] = {};
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        const double Db = D_b[a][b];
        tl_b[a] += Db * F.C[b];
        C_b[b] += Db * tl[a];
        tl_b[b] += Db * F.C[a];
        C_b[a] += Db * tl[b];
        psi_b[a][b] += -Db * F.tC;
        tC_b += -Db * F.psi[a][b];
      }
    N_b += -tl_b[0];
  }
  for (int c = 0; c < 4; ++c) {
    tu_b[c] += tC_b * F.C[c];
    C_b[c] += tC_b * F.tu[c];
  }
  for (int d = 0; d < 4; ++d)
    for (int c = 0; c < 4; ++c) P_b[d][c] += Hup_b[d] * H[c];
  for (int c = 0; c < 4; ++c)
    for (int d = 0; d < 4; ++d) {
      tu_b[c] += 2.0 * ttPi_b * F.tu[d] * F.Pi[c][d];
      Pi_b[c][d] += ttPi_b * F.tu[c] * F.tu[d];
    }
  {
    double w_b[3] = {};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        w_b[i] += v_b[j] * F.gi[i][j];
        gi_b[i][j] += v_b[j] * w[i];
      }
    for (int i = 0; i < 3; ++i)
      for (int c = 0; c < 4; ++c) {
        tu_b[c] += w_b[i] * F.Pi[c][i + 1];
        Pi_b[c][i + 1] += w_b[i] * F.tu[c];
      }
  }
  // Q = sum_j R_j P Phi_j - Pi P Pi - T3
  {
    double T1[4][4], T2[4][4], T3[4][4];
    for (int j = 0; j < 3; ++j) {
      double Rb[4][4];
      mmm(Q_b, F.Phi[j], F.P, Rb);          // dQ/dR_j
      mmm(R[j], Q_b, F.Phi[j], T1);         // dQ/dP
      mmm(F.P, R[j], Q_b, T2);              // dQ/dPhi_j
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          P_b[a][b] += T1[a][b];
          Phi_b[j][a][b] += T2[a][b];
        }
      for (int i = 0; i < 3; ++i) {
        double dot = 0.0;
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 4; ++b) {
            Phi_b[i][a][b] += F.gi[j][i] * Rb[a][b];
            dot += Rb[a][b] * F.Phi[i][a][b];
          }
        gi_b[j][i] += dot;
      }
    }
    mmm(Q_b, F.Pi, F.P, T1);
    mmm(F.P, F.Pi, Q_b, T2);
    mmm(F.Pi, Q_b, F.Pi, T3);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        Pi_b[a][b] += -(T1[a][b] + T2[a][b]);
        P_b[a][b] += -T3[a][b];
      }
    // T3 part: cotangent -Q_b (symmetric)
    for (int a = 0; a < 4; ++a) {
      double Y[4][4] = {};
      for (int b = 0; b < 4; ++b)
        for (int c = 0; c < 4; ++c)
          for (int e = 0; e < 4; ++e) {
            G_b[a][c][e] += 2.0 * (-Q_b[a][b]) * PGP[b][c][e];
            Y[c][e] += (-Q_b[a][b]) * F.G[b][c][e];
          }
      double GPY[4][4];
      mmm(F.G[a], F.P, Y, GPY);
      for (int c = 0; c < 4; ++c)
        for (int e = 0; e < 4; ++e) P_b[c][e] += 2.0 * GPY[c][e];
    }
  }
  reverse_tail(F, C_b, G_b, P_b, tu_b, N_b, Nu_b, gi_b, psi_b, Pi_b, Phi_b);
  // fold full-tensor adjoints onto pairs
  for (int a = 0; a < 4; ++a)
    for (int b = a; b < 4; ++b) {
      const int n = pair(a, b);
      const bool off = a != b;
      ubar[n] = psi_b[a][b] + (off ? psi_b[b][a] : 0.0);
      ubar[10 + n] = Pi_b[a][b] + (off ? Pi_b[b][a] : 0.0);
      for (int i = 0; i < 3; ++i) ubar[20 + 10 * i + n] = Phi_b[i][a][b] + (off ? Phi_b[i][b][a] : 0.0);
      for (int k = 0; k < 3; ++k) {
        dubar[k][n] = dpsi_b[k][a][b] + (off ? dpsi_b[k][b][a] : 0.0);
        dubar[k][10 + n] = dPi_b[k][a][b] + (off ? dPi_b[k][b][a] : 0.0);
        for (int i = 0; i < 3; ++i)
          dubar[k][20 + 10 * i + n] = dPhi_b[k][i][a][b] + (off ? dPhi_b[k][i][b][a] : 0.0);
      }
    }
  gbar[0] += gb0;
  gbar[1] += gb1;
  gbar[2] += gb2;
}

// Reverse of the gauge constraint C_a = H_a + psi^bc Gamma_abc: adds the
// cotangent of u (pair form) for the cotangent Cbar[4] of C_a.
GHP_HD void gauge_constraint_vjp(const double* u, const double* H, const double* Cbar, double* ubar) {
  Fwd F;
  forward(u, H, F);
  double psi_b[4][4] = {}, Pi_b[4][4] = {}, Phi_b[3][4][4] = {};
  double Nu_b[3] = {}, N_b = 0.0, gi_b[3][3] = {}, tu_b[4] = {}, P_b[4][4] = {};
  double G_b[4][4][4] = {};
  reverse_tail(F, Cbar, G_b, P_b, tu_b, N_b, Nu_b, gi_b, psi_b, Pi_b, Phi_b);
  for (int a = 0; a < 4; ++a)
    for (int b = a; b < 4; ++b) {
      const int n = pair(a, b);
      const bool off = a != b;
      ubar[n] += psi_b[a][b] + (off ? psi_b[b][a] : 0.0);
      ubar[10 + n] += Pi_b[a][b] + (off ? Pi_b[b][a] : 0.0);
      for (int i = 0; i < 3; ++i) ubar[20 + 10 * i + n] += Phi_b[i][a][b] + (off ? Phi_b[i][b][a] : 0.0);
    }
}


// ---------------------------------------------------------------------------
// Register-lean reverse pass in pair storage.  Same mathematics as rhs_vjp;
// symmetric cotangents are kept as one value per pair ("full entry" values,
// i.e. the cotangent of one of the two equal tensor entries), the spatial
// inverse-metric cotangent as its symmetric part giS = gi_b + gi_b^T and the
// psi^ab cotangent as PS = P_b + P_b^T.  The derivative cotangents are
// produced pair by pair through `load(n, dpsi, dPi, dPhi)` (Cartesian
// derivatives of the five fields of pair n; dPhi[k][i] = d_k Phi_i) and
// `store(n, dpsi_b, dPi_b, dPhi_b)`, so that a kernel can stream them.
// ---------------------------------------------------------------------------
GHP_HD int s3(int i, int j) {
  return i <= j ? (i * 3 - i * (i - 1) / 2 + j - i) : (j * 3 - j * (j - 1) / 2 + i - j);
}
GHP_HD double pmul(int a, int b) { return a == b ? 1.0 : 2.0; }

// The reverse pass in two parts, so that a kernel can run them as two
// register-light passes: rhs_vjp_principal takes the derivative (principal)
// terms, streaming the derivatives and their cotangents pair by pair, and
// returns its partial cotangents of the geometry and of gamma1, gamma2 in
// acc[12] = (N^i_b[3], N_b, giS[6], gamma1_b, gamma2_b), reading the
// cotangent lam of d_t u through lamf(f); rhs_vjp_algebraic
// continues from acc with the algebraic terms and the geometry's reverse.
// rhs_vjp_pairs runs both; the sums are taken in the same order either way.
#define GHP_VJP_ACC 12

template <class LamF, class Load, class Store>
GHP_HD void rhs_vjp_principal(const double* psi, double g1, double g2, LamF lamf, Load load, Store store,
                              double* acc) {
  // geometry
  double gi[6], Nu[3], beta[3], N, tu[4], P[10];
  {
    const double g11 = psi[4], g12 = psi[5], g13 = psi[6], g22 = psi[7], g23 = psi[8], g33 = psi[9];
    const double A = g22 * g33 - g23 * g23, B = g13 * g23 - g12 * g33, Cc = g12 * g23 - g13 * g22;
    const double D = g11 * g33 - g13 * g13, E = g12 * g13 - g11 * g23, F = g11 * g22 - g12 * g12;
    const double idet = 1.0 / (g11 * A + g12 * B + g13 * Cc);
    gi[0] = A * idet; gi[1] = B * idet; gi[2] = Cc * idet; gi[3] = D * idet; gi[4] = E * idet; gi[5] = F * idet;
    beta[0] = psi[1]; beta[1] = psi[2]; beta[2] = psi[3];
    double nsq = -psi[0];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Nu[i] = gi[s3(i, 0)] * beta[0] + gi[s3(i, 1)] * beta[1] + gi[s3(i, 2)] * beta[2];
      nsq += Nu[i] * beta[i];
    }
    N = sqrt(nsq);
    tu[0] = 1.0 / N;
#pragma unroll
    for (int i = 0; i < 3; ++i) tu[i + 1] = -Nu[i] / N;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = a; b < 4; ++b)
        P[pair(a, b)] = ((a > 0 && b > 0) ? gi[s3(a - 1, b - 1)] : 0.0) - tu[a] * tu[b];
  }
  double Nu_b[3] = {0.0, 0.0, 0.0}, N_b = 0.0, giS[6] = {0, 0, 0, 0, 0, 0};
  double gb1 = 0.0, gb2 = 0.0;
  (void)P;
  (void)tu;

  // (1) principal parts, streamed per pair (not unrolled: one pair's
  // derivatives and cotangents live at a time)
#pragma unroll 1
  for (int n = 0; n < 10; ++n) {
    double dpsi[3], dPi[3], dPhi[3][3];
    load(n, dpsi, dPi, dPhi);
    const double lp = lamf(n), lP = lamf(10 + n);
    const double lF[3] = {lamf(20 + n), lamf(30 + n), lamf(40 + n)};
    double dpsi_b[3], dPi_b[3], dPhi_b[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      dpsi_b[k] = (1.0 + g1) * Nu[k] * lp + g1 * g2 * Nu[k] * lP + g2 * N * lF[k];
      dPi_b[k] = Nu[k] * lP - N * lF[k];
#pragma unroll
      for (int i = 0; i < 3; ++i) dPhi_b[k][i] = Nu[k] * lF[i] - N * gi[s3(k, i)] * lP;
    }
    store(n, dpsi_b, dPi_b, dPhi_b);
    double adv = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      adv += Nu[k] * dpsi[k];
      Nu_b[k] += lp * (1.0 + g1) * dpsi[k] + lP * (dPi[k] + g1 * g2 * dpsi[k]);
#pragma unroll
      for (int i = 0; i < 3; ++i) Nu_b[k] += lF[i] * dPhi[k][i];
    }
    double div = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int i = 0; i < 3; ++i) div += gi[s3(k, i)] * dPhi[k][i];
#pragma unroll
    for (int i = 0; i < 3; ++i) N_b += lF[i] * (-dPi[i] + g2 * dpsi[i]);
    N_b += -lP * div;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int i = k; i < 3; ++i)
        giS[s3(k, i)] += -N * lP * (k == i ? 2.0 * dPhi[k][k] : dPhi[k][i] + dPhi[i][k]);
    gb1 += lp * adv + g2 * lP * adv;
    double dps = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) dps += lF[i] * dpsi[i];
    gb2 += N * dps + g1 * lP * adv;
  }

  acc[0] = Nu_b[0]; acc[1] = Nu_b[1]; acc[2] = Nu_b[2]; acc[3] = N_b;
#pragma unroll
  for (int i = 0; i < 6; ++i) acc[4 + i] = giS[i];
  acc[10] = gb1;
  acc[11] = gb2;
}

// u and lam are read through V (a pointer, or any type with v + k and v[i]),
// so a kernel can leave them in memory instead of registers.
template <class V>
GHP_HD void rhs_vjp_algebraic(V u, const double* H, const double* dH, double g0, double g1, double g2, V lam,
                              const double* acc, double* ubar, double* gbar) {
  const V psi = u;
  const V Pi = u + 10;
  const V Phi = u + 20;                  // Phi_i pair n at Phi[10 i + n]
  const V lpsi = lam;
  const V lPi = lam + 10;
  const V lPhi = lam + 20;
  // geometry
  double gi[6], Nu[3], beta[3], N, tu[4], P[10];
  {
    const double g11 = psi[4], g12 = psi[5], g13 = psi[6], g22 = psi[7], g23 = psi[8], g33 = psi[9];
    const double A = g22 * g33 - g23 * g23, B = g13 * g23 - g12 * g33, Cc = g12 * g23 - g13 * g22;
    const double D = g11 * g33 - g13 * g13, E = g12 * g13 - g11 * g23, F = g11 * g22 - g12 * g12;
    const double idet = 1.0 / (g11 * A + g12 * B + g13 * Cc);
    gi[0] = A * idet; gi[1] = B * idet; gi[2] = Cc * idet; gi[3] = D * idet; gi[4] = E * idet; gi[5] = F * idet;
    beta[0] = psi[1]; beta[1] = psi[2]; beta[2] = psi[3];
    double nsq = -psi[0];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Nu[i] = gi[s3(i, 0)] * beta[0] + gi[s3(i, 1)] * beta[1] + gi[s3(i, 2)] * beta[2];
      nsq += Nu[i] * beta[i];
    }
    N = sqrt(nsq);
    tu[0] = 1.0 / N;
#pragma unroll
    for (int i = 0; i < 3; ++i) tu[i + 1] = -Nu[i] / N;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = a; b < 4; ++b)
        P[pair(a, b)] = ((a > 0 && b > 0) ? gi[s3(a - 1, b - 1)] : 0.0) - tu[a] * tu[b];
  }
#pragma unroll
  for (int f = 0; f < 50; ++f) ubar[f] = 0.0;
  double Nu_b[3] = {acc[0], acc[1], acc[2]}, N_b = acc[3];
  double giS[6] = {acc[4], acc[5], acc[6], acc[7], acc[8], acc[9]}, tu_b[4] = {0, 0, 0, 0};
  double PS[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  double gb0 = 0.0, gb1 = acc[10], gb2 = acc[11];

  // (2) algebraic part of d_t psi, and the -g1 g2 N^i Phi_i term of d_t Pi
#pragma unroll
  for (int n = 0; n < 10; ++n) {
    const double NuPhi = Nu[0] * Phi[n] + Nu[1] * Phi[10 + n] + Nu[2] * Phi[20 + n];
    N_b += -lpsi[n] * Pi[n];
    ubar[10 + n] += -N * lpsi[n];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      ubar[20 + 10 * i + n] += -(g1 * lpsi[n] + g1 * g2 * lPi[n]) * Nu[i];
      Nu_b[i] += -(g1 * lpsi[n] + g1 * g2 * lPi[n]) * Phi[10 * i + n];
    }
    gb1 += -(lpsi[n] + g2 * lPi[n]) * NuPhi;
    gb2 += -g1 * lPi[n] * NuPhi;
  }

  // (3) algebraic part of d_t Phi: 1/2 N ttPhi_i Pi + N Gt_ik Phi_k - g2 N Phi_i
  {
    double ttPhi[3], tPhi[3][3], Gt[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int d = c; d < 4; ++d) s += pmul(c, d) * tu[c] * tu[d] * Phi[10 * i + pair(c, d)];
      ttPhi[i] = s;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double t = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) t += tu[c] * Phi[10 * i + pair(j + 1, c)];
        tPhi[i][j] = t;
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        Gt[i][k] = gi[s3(0, k)] * tPhi[i][0] + gi[s3(1, k)] * tPhi[i][1] + gi[s3(2, k)] * tPhi[i][2];
    double ttPhi_b[3] = {0, 0, 0}, Gt_b[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int n = 0; n < 10; ++n) {
        const double l = lPhi[10 * i + n];
        double gtp = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          gtp += Gt[i][k] * Phi[10 * k + n];
          Gt_b[i][k] += N * l * Phi[10 * k + n];
          ubar[20 + 10 * k + n] += N * Gt[i][k] * l;
        }
        N_b += l * (0.5 * ttPhi[i] * Pi[n] + gtp - g2 * Phi[10 * i + n]);
        gb2 += -N * l * Phi[10 * i + n];
        ttPhi_b[i] += 0.5 * N * l * Pi[n];
        ubar[10 + n] += 0.5 * N * l * ttPhi[i];
        ubar[20 + 10 * i + n] += -g2 * N * l;
      }
    double tPhi_b[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        tPhi_b[i][j] = Gt_b[i][0] * gi[s3(j, 0)] + Gt_b[i][1] * gi[s3(j, 1)] + Gt_b[i][2] * gi[s3(j, 2)];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = j; k < 3; ++k) {
        double c = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) c += Gt_b[i][k] * tPhi[i][j] + (k == j ? Gt_b[i][k] * tPhi[i][j] : Gt_b[i][j] * tPhi[i][k]);
        giS[s3(j, k)] += c;
      }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          tu_b[c] += tPhi_b[i][j] * Phi[10 * i + pair(j + 1, c)];
          ubar[20 + 10 * i + pair(j + 1, c)] += tPhi_b[i][j] * tu[c];
        }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double s = 0.0;
#pragma unroll
        for (int d = 0; d < 4; ++d) s += tu[d] * Phi[10 * i + pair(c, d)];
        tu_b[c] += 2.0 * ttPhi_b[i] * s;
#pragma unroll
        for (int d = c; d < 4; ++d) ubar[20 + 10 * i + pair(c, d)] += pmul(c, d) * ttPhi_b[i] * tu[c] * tu[d];
      }
  }

  // (4) the rest of d_t Pi: Christoffels, constraint, Q, damping
  double G[4][10];
  {
    double d0[10];
#pragma unroll
    for (int n = 0; n < 10; ++n) d0[n] = -N * Pi[n] + Nu[0] * Phi[n] + Nu[1] * Phi[10 + n] + Nu[2] * Phi[20 + n];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a; b < 4; ++b) {
          const double x = (a == 0) ? d0[pair(c, b)] : Phi[10 * (a - 1) + pair(c, b)];
          const double y = (b == 0) ? d0[pair(c, a)] : Phi[10 * (b - 1) + pair(c, a)];
          const double z = (c == 0) ? d0[pair(a, b)] : Phi[10 * (c - 1) + pair(a, b)];
          G[c][pair(a, b)] = 0.5 * (x + y - z);
        }
  }
  double C[4], Hup[4], tC = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double s = H[a];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int c = b; c < 4; ++c) s += pmul(b, c) * P[pair(b, c)] * G[a][pair(b, c)];
    C[a] = s;
    Hup[a] = P[pair(a, 0)] * H[0] + P[pair(a, 1)] * H[1] + P[pair(a, 2)] * H[2] + P[pair(a, 3)] * H[3];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) tC += tu[a] * C[a];
  double ttPi = 0.0, w[3], v[3];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int d = c; d < 4; ++d) ttPi += pmul(c, d) * tu[c] * tu[d] * Pi[pair(c, d)];
#pragma unroll
  for (int i = 0; i < 3; ++i) w[i] = tu[0] * Pi[pair(0, i + 1)] + tu[1] * Pi[pair(1, i + 1)] +
                                    tu[2] * Pi[pair(2, i + 1)] + tu[3] * Pi[pair(3, i + 1)];
#pragma unroll
  for (int j = 0; j < 3; ++j) v[j] = w[0] * gi[s3(0, j)] + w[1] * gi[s3(1, j)] + w[2] * gi[s3(2, j)];

  // Q (full symmetric 4x4) for the N cotangent
  double Qm[4][4];
  {
    double Pf[4][4], Pif[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) { Pf[a][b] = P[pair(a, b)]; Pif[a][b] = Pi[pair(a, b)]; }
    double T[4][4], Mx[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) Qm[a][b] = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double Rf[4][4], Ff[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int n = pair(a, b);
          Rf[a][b] = gi[s3(j, 0)] * Phi[n] + gi[s3(j, 1)] * Phi[10 + n] + gi[s3(j, 2)] * Phi[20 + n];
          Ff[a][b] = Phi[10 * j + n];
        }
      mmm(Rf, Pf, Ff, T);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) Qm[a][b] += T[a][b];
    }
    mmm(Pif, Pf, Pif, T);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) Qm[a][b] -= T[a][b];
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      double Gf[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) Gf[a][b] = G[bb][pair(a, b)];
      mmm(Pf, Gf, Pf, Mx);                 // P G_bb P
#pragma unroll
      for (int aa = 0; aa < 4; ++aa) {
        double t3 = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
          for (int e = 0; e < 4; ++e) t3 += G[aa][pair(c, e)] * Mx[c][e];
        Qm[aa][bb] -= t3;
      }
    }
  }
  // scalar-type contributions of d_t Pi
  double Hup_b[4] = {0, 0, 0, 0}, tC_b = 0.0, ttPi_b = 0.0, v_b[3] = {0, 0, 0}, tl_b0 = 0.0;
  double C_b[4] = {0, 0, 0, 0};
  double G_b[4][10];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int n = 0; n < 10; ++n) G_b[c][n] = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a; b < 4; ++b) {
      const int n = pair(a, b);
      const double l = lPi[n];
      const double hg = Hup[0] * G[0][n] + Hup[1] * G[1][n] + Hup[2] * G[2][n] + Hup[3] * G[3][n];
      const double vphi = v[0] * Phi[n] + v[1] * Phi[10 + n] + v[2] * Phi[20 + n];
      const double Dn = -N * ((a == 0 ? C[b] : 0.0) + (b == 0 ? C[a] : 0.0)) - psi[n] * tC;
      N_b += l * (2.0 * Qm[a][b] - (dH[a * 4 + b] + dH[b * 4 + a]) + 2.0 * hg - 0.5 * ttPi * Pi[n] - vphi + g0 * Dn);
      gb0 += N * l * Dn;
      const double half = (a == b) ? 1.0 : 0.5;
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        Hup_b[d] += 2.0 * N * l * G[d][n];
        G_b[d][n] += 2.0 * N * Hup[d] * l * half;
      }
      ttPi_b += -0.5 * N * l * Pi[n];
      ubar[10 + n] += -0.5 * N * ttPi * l;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        v_b[j] += -N * l * Phi[10 * j + n];
        ubar[20 + 10 * j + n] += -N * v[j] * l;
      }
      // damping D = t_a C_b + t_b C_a - psi tC with t_a = (-N, 0, 0, 0)
      const double Db = g0 * N * l * half;     // full-entry cotangent
      if (a == 0) { tl_b0 += 2.0 * Db * C[b] * (b == 0 ? 1.0 : 1.0); C_b[b] += 2.0 * Db * (-N); }
      if (b == 0 && a != 0) { tl_b0 += 2.0 * Db * C[a]; C_b[a] += 2.0 * Db * (-N); }
      ubar[n] += -tC * g0 * N * l;
      tC_b += -g0 * N * l * psi[n];
    }
  N_b += -tl_b0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    tu_b[c] += tC_b * C[c];
    C_b[c] += tC_b * tu[c];
  }
#pragma unroll
  for (int d = 0; d < 4; ++d)
#pragma unroll
    for (int c = d; c < 4; ++c)
      PS[pair(d, c)] += (d == c) ? 2.0 * Hup_b[d] * H[c] : Hup_b[d] * H[c] + Hup_b[c] * H[d];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 4; ++d) s += tu[d] * Pi[pair(c, d)];
    tu_b[c] += 2.0 * ttPi_b * s;
#pragma unroll
    for (int d = c; d < 4; ++d) ubar[10 + pair(c, d)] += pmul(c, d) * ttPi_b * tu[c] * tu[d];
  }
  {
    double w_b[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) w_b[i] = v_b[0] * gi[s3(i, 0)] + v_b[1] * gi[s3(i, 1)] + v_b[2] * gi[s3(i, 2)];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) giS[s3(i, j)] += v_b[j] * w[i] + v_b[i] * w[j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        tu_b[c] += w_b[i] * Pi[pair(c, i + 1)];
        ubar[10 + pair(c, i + 1)] += w_b[i] * tu[c];
      }
  }
  // Q reverse (full matrices), Q_b full-entry = 2 N lPi (1/2 off-diagonal)
  {
    double Qb[4][4], Pf[4][4], Pif[4][4], T1[4][4], T2[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        Qb[a][b] = 2.0 * N * lPi[pair(a, b)] * (a == b ? 1.0 : 0.5);
        Pf[a][b] = P[pair(a, b)];
        Pif[a][b] = Pi[pair(a, b)];
      }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double Rf[4][4], Ff[4][4], Rb[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int n = pair(a, b);
          Rf[a][b] = gi[s3(j, 0)] * Phi[n] + gi[s3(j, 1)] * Phi[10 + n] + gi[s3(j, 2)] * Phi[20 + n];
          Ff[a][b] = Phi[10 * j + n];
        }
      mmm(Qb, Ff, Pf, Rb);       // dQ/dR_j
      mmm(Rf, Qb, Ff, T1);       // dQ/dP
      mmm(Pf, Rf, Qb, T2);       // dQ/dPhi_j
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a; b < 4; ++b) {
          const int n = pair(a, b);
          PS[n] += T1[a][b] + T1[b][a];
          ubar[20 + 10 * j + n] += (a == b) ? T2[a][a] : T2[a][b] + T2[b][a];
          const double rb = (a == b) ? Rb[a][a] : Rb[a][b] + Rb[b][a];
#pragma unroll
          for (int i = 0; i < 3; ++i) ubar[20 + 10 * i + n] += gi[s3(j, i)] * rb;
        }
      // gi_b[j][i] += <Rb, Phi_i>
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        double dot = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) dot += Rb[a][b] * Phi[10 * i + pair(a, b)];
        giS[s3(j, i)] += (i == j) ? 2.0 * dot : dot;
      }
    }
    mmm(Qb, Pif, Pf, T1);        // X = Qb Pi P
    mmm(Pif, Qb, Pif, T2);       // Pi Qb Pi
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = a; b < 4; ++b) {
        const int n = pair(a, b);
        ubar[10 + n] += -((a == b) ? 2.0 * T1[a][a] : 2.0 * (T1[a][b] + T1[b][a]));
        PS[n] += -2.0 * T2[a][b];
      }
    // T3 part, cotangent -Qb
#pragma unroll
    for (int aa = 0; aa < 4; ++aa) {
      double Y[4][4], Ga[4][4], Z[4][4];
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          double y = 0.0;
#pragma unroll
          for (int bb = 0; bb < 4; ++bb) y += -Qb[aa][bb] * G[bb][pair(c, e)];
          Y[c][e] = y;
          Ga[c][e] = G[aa][pair(c, e)];
        }
      double PYP[4][4];
      mmm(Pf, Y, Pf, PYP);       // sum_b T3b[a][b] P G_b P
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int e = c; e < 4; ++e) G_b[aa][pair(c, e)] += 2.0 * PYP[c][e];
      mmm(Ga, Pf, Y, Z);         // G_a P Y_a
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int e = c; e < 4; ++e) PS[pair(c, e)] += 2.0 * (Z[c][e] + Z[e][c]);
    }
  }
  // C_a = H_a + P^bc G_abc
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int n = 0; n < 10; ++n) {
      PS[n] += 2.0 * C_b[a] * G[a][n];
      G_b[a][n] += C_b[a] * P[n];
    }
  // Gamma_cab = (d4_acb + d4_bca - d4_cab)/2: pair cotangents of d_x psi_yz
  {
    double d4b[4][10];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y)
#pragma unroll
        for (int z = y; z < 4; ++z)
          d4b[x][pair(y, z)] = (y == z) ? G_b[y][pair(x, y)] - 0.5 * G_b[x][pair(y, y)]
                                        : G_b[y][pair(x, z)] + G_b[z][pair(x, y)] - G_b[x][pair(y, z)];
#pragma unroll
    for (int n = 0; n < 10; ++n) {
      N_b += -d4b[0][n] * Pi[n];
      ubar[10 + n] += -N * d4b[0][n];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        Nu_b[i] += d4b[0][n] * Phi[10 * i + n];
        ubar[20 + 10 * i + n] += Nu[i] * d4b[0][n] + d4b[i + 1][n];
      }
    }
  }
  // P^ab = g^ab - t^a t^b
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) giS[s3(i, j)] += PS[pair(i + 1, j + 1)];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) s += PS[pair(a, b)] * tu[b];
    tu_b[a] += -s;
  }
  // t^a = (1/N, -N^i/N)
  N_b += -tu_b[0] / (N * N);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    N_b += tu_b[i + 1] * Nu[i] / (N * N);
    Nu_b[i] += -tu_b[i + 1] / N;
  }
  const double nsq_b = N_b / (2.0 * N);
  double beta_b[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Nu_b[i] += nsq_b * beta[i];
    beta_b[i] = nsq_b * Nu[i];
  }
  ubar[0] += -nsq_b;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) giS[s3(i, j)] += Nu_b[i] * beta[j] + Nu_b[j] * beta[i];
#pragma unroll
  for (int j = 0; j < 3; ++j) beta_b[j] += gi[s3(0, j)] * Nu_b[0] + gi[s3(1, j)] * Nu_b[1] + gi[s3(2, j)] * Nu_b[2];
#pragma unroll
  for (int i = 0; i < 3; ++i) ubar[pair(0, i + 1)] += beta_b[i];
  // g^ij = inv(g_ij): psi pair (i+1, j+1) gets -(g^-1 giS g^-1)_ij (1/2 on the diagonal)
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = 0; l < 3; ++l) s += gi[s3(i, k)] * giS[s3(k, l)] * gi[s3(l, j)];
      ubar[pair(i + 1, j + 1)] += -(i == j ? 0.5 : 1.0) * s;
    }
  gbar[0] += gb0;
  gbar[1] += gb1;
  gbar[2] += gb2;}

template <class Load, class Store>
GHP_HD void rhs_vjp_pairs(const double* u, const double* H, const double* dH, double g0, double g1,
                          double g2, const double* lam, Load load, Store store, double* ubar, double* gbar) {
  double acc[GHP_VJP_ACC];
  auto lamf = [&](int f) { return lam[f]; };
  rhs_vjp_principal(u, g1, g2, lamf, load, store, acc);
  rhs_vjp_algebraic(u, H, dH, g0, g1, g2, lam, acc, ubar, gbar);
}

}  // namespace ghp

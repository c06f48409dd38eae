// HIP kernels for gfx950 (MI355X): spectral derivatives, pointwise GH algebra,
// boundary treatment, SSP-RK3 stages, constraints.  All arithmetic is FP64.
#include <hip/hip_runtime.h>
#include <cmath>

#include "ghmi_internal.h"
#include "gh_point.h"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// Symmetric pair index of (a, b), pairs ordered 00,01,02,03,11,12,13,22,23,33.
__host__ __device__ constexpr int SYM(int a, int b) {
  return a <= b ? (a * 4 - a * (a - 1) / 2 + b - a) : (b * 4 - b * (b - 1) / 2 + a - b);
}
// Symmetric 3x3 index of (i, j), i,j in 0..2: 11,12,13,22,23,33.
__host__ __device__ constexpr int SYM3(int i, int j) {
  return i <= j ? (i * 3 - i * (i - 1) / 2 + j - i) : (j * 3 - j * (j - 1) / 2 + i - j);
}

// ---------------------------------------------------------------------------
// Radial derivative: dR[f][r][a] = dscale * sum_r' D[r][r'] u[f][r'][a], one
// thread per point, any n_r (the column form below keeps a column in
// registers and covers n_r <= 64).  TRANS applies D^T; ACC adds into dR.
// ---------------------------------------------------------------------------
template <bool TRANS, bool ACC>
__global__ __launch_bounds__(256) void k_radial(const ShellDev* __restrict__ sh,
                                                const PtBlock* __restrict__ blk,
                                                const double* __restrict__ dtab,
                                                const double* __restrict__ u,
                                                double* __restrict__ dR, int f0) {
  const PtBlock b = blk[blockIdx.x];
  const ShellDev s = sh[b.shell];
  const int P = s.n_r * s.S;
  const int q = b.q0 + threadIdx.x;
  if (q >= P) return;
  const int f = f0 + blockIdx.y;
  const int r = q / s.S, a = q - r * s.S;
  const long long base = 50LL * s.pt_off + (long long)f * P;
  // row r of D (stride 1) or of D^T (column r of D, stride n_r)
  const double* D = dtab + s.d_off + (TRANS ? r : r * s.n_r);
  const int dstride = TRANS ? s.n_r : 1;
  const double* col = u + base + a;
  double acc = 0.0;
  for (int rp = 0; rp < s.n_r; ++rp) acc += D[rp * dstride] * col[(long long)rp * s.S];
  if (ACC) dR[base + q] += s.dscale * acc;
  else dR[base + q] = s.dscale * acc;
}

// Radial derivative, one thread per (field, angular point) column: the n_r
// values of the column are loaded once into registers and all n_r outputs are
// formed from them, so u and dR each cross HBM once.  The CGL matrix entries
// are staged in LDS and read as broadcasts.  TRANS applies D^T instead
// of D; ACC adds into dR instead of overwriting it.
template <int MAXR, bool TRANS, bool ACC>
__global__ __launch_bounds__(256) void k_radial_col(const ShellDev* __restrict__ sh,
                                                    const PtBlock* __restrict__ cblk,
                                                    const double* __restrict__ dtab,
                                                    const double* __restrict__ u,
                                                    double* __restrict__ dR, int f0) {
  const PtBlock b = cblk[blockIdx.x];
  const ShellDev s = sh[b.shell];
  const int n = s.n_r;
  // the n x n matrix is the same for every thread: stage it in LDS once and
  // read it with broadcast loads
  __shared__ double D[MAXR * MAXR];
  for (int i = threadIdx.x; i < MAXR * MAXR; i += blockDim.x) {
    const int r = i / MAXR, rp = i - r * MAXR;
    const int src = TRANS ? rp * n + r : r * n + rp;      // (row r, column rp) of D or D^T
    D[i] = (r < n && rp < n) ? dtab[s.d_off + src] : 0.0;
  }
  __syncthreads();
  const int a = b.q0 + threadIdx.x;
  if (a >= s.S) return;
  const int f = f0 + blockIdx.y;
  const long long base = 50LL * s.pt_off + (long long)f * n * s.S + a;
  double col[MAXR];
  // unconditional loads (index clamped; the padded matrix entries are zero)
#pragma unroll
  for (int r = 0; r < MAXR; ++r) col[r] = u[base + (long long)min(r, n - 1) * s.S];
#pragma unroll
  for (int r = 0; r < MAXR; ++r) {
    if (r < n) {
      double acc = 0.0;
#pragma unroll
      for (int rp = 0; rp < MAXR; ++rp) acc += D[r * MAXR + rp] * col[rp];
      double* o = dR + base + (long long)r * s.S;
      if (ACC) *o += s.dscale * acc;
      else *o = s.dscale * acc;
    }
  }
}

// ---------------------------------------------------------------------------
// Pointwise generalized-harmonic algebra.
// ---------------------------------------------------------------------------

// 3+1 quantities from psi_ab.
struct Geo {
  double gi[6];     // g^ij
  double Nu[3];     // N^i
  double N;         // lapse
  double tu[4];     // t^a
  double pinv[10];  // psi^ab
};

__device__ __forceinline__ void geometry(const double* psi, Geo& G) {
  const double g11 = psi[SYM(1, 1)], g12 = psi[SYM(1, 2)], g13 = psi[SYM(1, 3)];
  const double g22 = psi[SYM(2, 2)], g23 = psi[SYM(2, 3)], g33 = psi[SYM(3, 3)];
  const double A = g22 * g33 - g23 * g23, B = g13 * g23 - g12 * g33, C = g12 * g23 - g13 * g22;
  const double D = g11 * g33 - g13 * g13, E = g12 * g13 - g11 * g23, F = g11 * g22 - g12 * g12;
  const double idet = 1.0 / (g11 * A + g12 * B + g13 * C);
  G.gi[0] = A * idet; G.gi[1] = B * idet; G.gi[2] = C * idet;
  G.gi[3] = D * idet; G.gi[4] = E * idet; G.gi[5] = F * idet;
  const double s1 = psi[SYM(0, 1)], s2 = psi[SYM(0, 2)], s3 = psi[SYM(0, 3)];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    G.Nu[i] = G.gi[SYM3(i, 0)] * s1 + G.gi[SYM3(i, 1)] * s2 + G.gi[SYM3(i, 2)] * s3;
  G.N = sqrt(G.Nu[0] * s1 + G.Nu[1] * s2 + G.Nu[2] * s3 - psi[SYM(0, 0)]);
  const double iN = 1.0 / G.N;
  G.tu[0] = iN;
#pragma unroll
  for (int i = 0; i < 3; ++i) G.tu[i + 1] = -G.Nu[i] * iN;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a; b < 4; ++b) {
      double g4 = (a > 0 && b > 0) ? G.gi[SYM3(a - 1, b - 1)] : 0.0;
      G.pinv[SYM(a, b)] = g4 - G.tu[a] * G.tu[b];
    }
}

// Gamma_cab = 1/2 (d_a psi_cb + d_b psi_ca - d_c psi_ab), with d_0 psi = -N Pi + N^i Phi_i
// and d_i psi = Phi_i; stored Gm[c][SYM(a,b)].
__device__ __forceinline__ void christoffel(const Geo& G, const double* Pi, const double* Phi,
                                            double Gm[4][10]) {
  double d0[10];
#pragma unroll
  for (int n = 0; n < 10; ++n)
    d0[n] = -G.N * Pi[n] + G.Nu[0] * Phi[n] + G.Nu[1] * Phi[10 + n] + G.Nu[2] * Phi[20 + n];
  auto dpsi = [&](int a, int n) -> double { return a == 0 ? d0[n] : Phi[(a - 1) * 10 + n]; };
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = a; b < 4; ++b)
        Gm[c][SYM(a, b)] = 0.5 * (dpsi(a, SYM(c, b)) + dpsi(b, SYM(c, a)) - dpsi(c, SYM(a, b)));
}

// Frobenius product of two symmetric 4x4 matrices in pair storage.
__device__ __forceinline__ double sym_dot(const double* X, const double* Y) {
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a; b < 4; ++b) s += (a == b ? 1.0 : 2.0) * X[SYM(a, b)] * Y[SYM(a, b)];
  return s;
}

// Y = P X P for symmetric X, P (pair storage): raises both indices of X with P = psi^ab.
__device__ __forceinline__ void raise2(const double* P, const double* X, double* Y) {
  double T[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) s += P[SYM(a, c)] * X[SYM(c, d)];
      T[a][d] = s;
    }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a; b < 4; ++b) {
      double s = 0.0;
#pragma unroll
      for (int d = 0; d < 4; ++d) s += T[a][d] * P[SYM(d, b)];
      Y[SYM(a, b)] = s;
    }
}

// out_ab += coef * (X P Y)_ab, symmetrised over pairs (X, Y symmetric, P symmetric).
__device__ __forceinline__ void add_xpy(const double* X, const double* P, const double* Y,
                                        double coef, double* out) {
  double T[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) s += X[SYM(a, c)] * P[SYM(c, d)];
      T[a][d] = s;
    }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a; b < 4; ++b) {
      double s = 0.0;
#pragma unroll
      for (int d = 0; d < 4; ++d) s += T[a][d] * Y[SYM(d, b)];
      out[SYM(a, b)] += coef * s;
    }
}

struct Jac {   // d_x, d_y, d_z in terms of d_r, d_theta, d_phi
  double xr, xt, xp, yr, yt, yp, zr, zt;
};

__device__ __forceinline__ Jac jacobian(const double* ang, double r) {
  const double st = ang[0], ct = ang[1], sp = ang[2], cp = ang[3];
  const double ir = 1.0 / r, irs = 1.0 / (r * st);
  Jac J;
  J.xr = st * cp; J.xt = ct * cp * ir; J.xp = -sp * irs;
  J.yr = st * sp; J.yt = ct * sp * ir; J.yp = cp * irs;
  J.zr = ct; J.zt = -st * ir;
  return J;
}

__device__ __forceinline__ void cart(const Jac& J, double dr, double dt, double dp, double* d) {
  d[0] = J.xr * dr + J.xt * dt + J.xp * dp;
  d[1] = J.yr * dr + J.yt * dt + J.yp * dp;
  d[2] = J.zr * dr + J.zt * dt;
}

// Whether local radial row r of shell s is a face the boundary treatment
// changes: an interface face (the outer face of a shell with an interface
// record, the inner face of a shell that is not an excision shell) or the
// outer face of an instance.
__device__ __forceinline__ bool treated_face(const ShellDev& s, int r) {
  return (r == s.n_r - 1 && (s.outer || s.bc_off >= 0)) || (r == 0 && !s.inner);
}

// STAGE 0: d_t u of every point into rhs (gh_rhs).  STAGE 1, 2: the kernel
// also takes the SSP-RK3 stage out = c0 u0 + c1 (u + dt L), u being the stage
// state it reads anyway (STAGE 1: c0 = 0, no u0).  Points on a face that the
// boundary treatment changes (an interface face, the outer face) still get the
// raw d_t u in rhs, for k_stage_faces; every other point gets only its stage
// value in out.  out may alias u0 (each element is read before it is written,
// by the same thread), not u or rhs.
template <int STAGE>
__global__ __launch_bounds__(256) void k_pointwise_rhs(
    const ShellDev* __restrict__ sh, const PtBlock* __restrict__ blk,
    const double* __restrict__ angtab, const double* __restrict__ radtab,
    const double* __restrict__ u, const double* __restrict__ dR, const double* __restrict__ dA,
    const double* __restrict__ Hin, const double* __restrict__ dHin,
    const double* __restrict__ gamma, double* __restrict__ rhs,
    const double* __restrict__ dtp, double c0, const double* u0, double c1, double* out) {
  const PtBlock b = blk[blockIdx.x];
  const ShellDev s = sh[b.shell];
  const int P = s.n_r * s.S;
  const int q = b.q0 + threadIdx.x;
  if (q >= P) return;
  const int r = q / s.S, a = q - r * s.S;
  const bool face = STAGE && treated_face(s, r);
  const double dtv = STAGE ? dtp[s.instance] : 0.0;
  const long long ub = 50LL * s.pt_off + q;                       // field f at ub + f*P
  const long long ab = 100LL * s.pt_off + (long long)r * 2 * s.S + a;   // d_theta of f at ab + f*n_r*2S
  const long long astride = (long long)s.n_r * 2 * s.S;
  const double g0 = gamma[3 * s.instance + 0];
  const double g1 = gamma[3 * s.instance + 1];
  const double g2 = gamma[3 * s.instance + 2];
  const Jac J = jacobian(angtab + 5LL * (s.ang_off + a), radtab[2 * (s.rad_off + r)]);

  double psi[10], Pi[10], Phi[30];
#pragma unroll
  for (int n = 0; n < 10; ++n) psi[n] = u[ub + (long long)n * P];
#pragma unroll
  for (int n = 0; n < 10; ++n) Pi[n] = u[ub + (long long)(10 + n) * P];
#pragma unroll
  for (int n = 0; n < 30; ++n) Phi[n] = u[ub + (long long)(20 + n) * P];
  Geo G;
  geometry(psi, G);
  const double N = G.N;

  // --- d_t psi and d_t Phi: principal part + algebraic part, stored at once;
  //     principal part of d_t Pi kept for later.
  double dtPi[10];
  // t^c t^d Phi_icd and G_ik = g^jk t^c Phi_ijc
  double ttPhi[3], tPhi[3][3], Gt[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double s2 = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int d = 0; d < 4; ++d) s2 += G.tu[c] * G.tu[d] * Phi[i * 10 + SYM(c, d)];
    ttPhi[i] = s2;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double s1 = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) s1 += G.tu[c] * Phi[i * 10 + SYM(j + 1, c)];
      tPhi[i][j] = s1;
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double s1 = 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j) s1 += G.gi[SYM3(j, k)] * tPhi[i][j];
      Gt[i][k] = s1;
    }

  const long long ob = ub;
  // d_t u of field f (its state value us, its stage-base value u0v)
  auto put = [&](int f, double val, double usv, double u0v) {
    const long long e = ob + (long long)f * P;
    if (STAGE == 0) {
      rhs[e] = val;
    } else if (face) {
      rhs[e] = val;
    } else {
      double v = c1 * (usv + dtv * val);
      if (STAGE == 2) v += c0 * u0v;
      out[e] = v;
    }
  };
  // The 15 spherical derivatives of pair n + 1 (dR, dA_theta, dA_phi of psi,
  // Pi and the three Phi) are loaded before pair n is computed, and the
  // scheduling barrier keeps the compiler from sinking them to their use: at
  // one wave per SIMD nothing else would hide their latency.
  // (with a stage base, its u0 of psi_n and the three Phi_in come along)
  auto load_pair = [&](int n, double (&raw)[15], double (&b0)[4]) {
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const int f = c < 2 ? 10 * c + n : 20 + 10 * (c - 2) + n;
      const long long fo = (long long)f * P, fa = (long long)f * astride;
      raw[3 * c] = dR[ub + fo];
      raw[3 * c + 1] = dA[ab + fa];
      raw[3 * c + 2] = dA[ab + fa + s.S];
    }
    if (STAGE == 2) {
      b0[0] = u0[ub + (long long)n * P];
#pragma unroll
      for (int i = 0; i < 3; ++i) b0[1 + i] = u0[ub + (long long)(20 + 10 * i + n) * P];
    }
  };
  double raw[2][15], b0[2][4];
  double H[4], dHr[16];   // the background's gauge source terms, loaded with the last pair
  load_pair(0, raw[0], b0[0]);
#pragma unroll
  for (int n = 0; n < 10; ++n) {
    if (n + 1 < 10) {
      load_pair(n + 1, raw[(n + 1) & 1], b0[(n + 1) & 1]);
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) H[c] = Hin[4LL * s.pt_off + (long long)c * P + q];
#pragma unroll
      for (int c = 0; c < 16; ++c) dHr[c] = dHin[16LL * s.pt_off + (long long)c * P + q];
    }
    __builtin_amdgcn_sched_barrier(0);
    const double* rw = raw[n & 1];
    double dpsi[3], dPi[3], dPhi[3][3];   // dPhi[k][i] = d_k Phi_i
    cart(J, rw[0], rw[1], rw[2], dpsi);
    cart(J, rw[3], rw[4], rw[5], dPi);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double d[3];
      cart(J, rw[6 + 3 * i], rw[7 + 3 * i], rw[8 + 3 * i], d);
      dPhi[0][i] = d[0]; dPhi[1][i] = d[1]; dPhi[2][i] = d[2];
    }
    const double adv_psi = G.Nu[0] * dpsi[0] + G.Nu[1] * dpsi[1] + G.Nu[2] * dpsi[2];
    const double adv_Pi = G.Nu[0] * dPi[0] + G.Nu[1] * dPi[1] + G.Nu[2] * dPi[2];
    double divPhi = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int i = 0; i < 3; ++i) divPhi += G.gi[SYM3(k, i)] * dPhi[k][i];
    const double NPhi = G.Nu[0] * Phi[n] + G.Nu[1] * Phi[10 + n] + G.Nu[2] * Phi[20 + n];

    put(n, (1.0 + g1) * adv_psi - N * Pi[n] - g1 * NPhi, psi[n], b0[n & 1][0]);
    dtPi[n] = adv_Pi - N * divPhi + g1 * g2 * adv_psi - g1 * g2 * NPhi;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double adv = G.Nu[0] * dPhi[0][i] + G.Nu[1] * dPhi[1][i] + G.Nu[2] * dPhi[2][i];
      double alg = 0.5 * N * ttPhi[i] * Pi[n] - g2 * N * Phi[i * 10 + n];
      alg += N * (Gt[i][0] * Phi[n] + Gt[i][1] * Phi[10 + n] + Gt[i][2] * Phi[20 + n]);
      put(20 + 10 * i + n, adv - N * dPi[i] + g2 * N * dpsi[i] + alg, Phi[i * 10 + n], b0[n & 1][1 + i]);
    }
  }

  // --- algebraic part of d_t Pi
  double Gm[4][10];
  christoffel(G, Pi, Phi, Gm);
  double Hup[4], C[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    double s1 = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) s1 += G.pinv[SYM(d, c)] * H[c];
    Hup[d] = s1;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) C[c] = H[c] + sym_dot(G.pinv, Gm[c]);
  const double tC = G.tu[0] * C[0] + G.tu[1] * C[1] + G.tu[2] * C[2] + G.tu[3] * C[3];

  // quad_ab = psi^cd (g^ij Phi_ica Phi_jdb - Pi_ca Pi_db - psi^ef Gamma_ace Gamma_bdf)
  double quad[10];
#pragma unroll
  for (int n = 0; n < 10; ++n) quad[n] = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    double Rj[10];    // Phi^j_ab = g^ji Phi_iab
#pragma unroll
    for (int n = 0; n < 10; ++n)
      Rj[n] = G.gi[SYM3(j, 0)] * Phi[n] + G.gi[SYM3(j, 1)] * Phi[10 + n] + G.gi[SYM3(j, 2)] * Phi[20 + n];
    add_xpy(Rj, G.pinv, Phi + 10 * j, 1.0, quad);
  }
  add_xpy(Pi, G.pinv, Pi, -1.0, quad);
#pragma unroll
  for (int bb = 0; bb < 4; ++bb) {
    double Gh[10];
    raise2(G.pinv, Gm[bb], Gh);
#pragma unroll
    for (int aa = 0; aa <= bb; ++aa) quad[SYM(aa, bb)] -= sym_dot(Gm[aa], Gh);
  }

  double ttPi = 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int d = 0; d < 4; ++d) ttPi += G.tu[c] * G.tu[d] * Pi[SYM(c, d)];
  double v[3];    // v_j = (t^c Pi_ci) g^ij
  {
    double tPi[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double s1 = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) s1 += G.tu[c] * Pi[SYM(c, i + 1)];
      tPi[i] = s1;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j)
      v[j] = tPi[0] * G.gi[SYM3(0, j)] + tPi[1] * G.gi[SYM3(1, j)] + tPi[2] * G.gi[SYM3(2, j)];
  }
  // (the stage base of the Pi fields is loaded only here: hoisted into the
  // algebra above, its ten values would not fit in the registers)
  if (STAGE) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int aa = 0; aa < 4; ++aa)
#pragma unroll
    for (int bb = aa; bb < 4; ++bb) {
      const int n = SYM(aa, bb);
      const double dHs = dHr[aa * 4 + bb] + dHr[bb * 4 + aa];
      const double GH = Hup[0] * Gm[0][n] + Hup[1] * Gm[1][n] + Hup[2] * Gm[2][n] + Hup[3] * Gm[3][n];
      const double vPhi = v[0] * Phi[n] + v[1] * Phi[10 + n] + v[2] * Phi[20 + n];
      // t_a = (-N, 0, 0, 0)
      const double tCsym = -N * ((aa == 0 ? C[bb] : 0.0) + (bb == 0 ? C[aa] : 0.0));
      const double damp = tCsym - psi[n] * tC;
      const double val = dtPi[n] + 2.0 * N * quad[n] - N * dHs + 2.0 * N * GH
                         - 0.5 * N * ttPi * Pi[n] - N * vPhi + g0 * N * damp;
      put(10 + n, val, Pi[n], STAGE == 2 ? u0[ub + (long long)(10 + n) * P] : 0.0);
    }
}

// ---------------------------------------------------------------------------
// Characteristic upwinding of one symmetric pair at an interface point.
// A, B: the five components (psi, Pi, Phi_x, Phi_y, Phi_z) of d_t u of that
// pair on the inner and the outer shell; T: the point's frozen record (s_i,
// s^i, upwind weights of u^0, u^+, u^-).  out: the value both shells take.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void interface_pair(const double A[5], const double B[5],
                                               const double* __restrict__ T, double g2,
                                               double out[5]) {
  const double sl[3] = {T[0], T[1], T[2]}, su[3] = {T[3], T[4], T[5]};
  const double w0 = T[6], wp = T[7], wm = T[8];
  const double sPa = su[0] * A[2] + su[1] * A[3] + su[2] * A[4];
  const double sPb = su[0] * B[2] + su[1] * B[3] + su[2] * B[4];
  const double upsi = 0.5 * (A[0] + B[0]);
  const double up = wp * (A[1] + sPa - g2 * A[0]) + (1.0 - wp) * (B[1] + sPb - g2 * B[0]);
  const double um = wm * (A[1] - sPa - g2 * A[0]) + (1.0 - wm) * (B[1] - sPb - g2 * B[0]);
  out[0] = upsi;
  out[1] = 0.5 * (up + um) + g2 * upsi;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double u0 = w0 * (A[2 + i] - sl[i] * sPa) + (1.0 - w0) * (B[2 + i] - sl[i] * sPb);
    out[2 + i] = u0 + 0.5 * sl[i] * (up - um);
  }
}

// ---------------------------------------------------------------------------
// Boundary treatment in place on d_t u: characteristic upwinding at
// interfaces, Dirichlet at the outer boundary.  blockIdx.y = shell; threads
// over angular points.  (Used by gh_rhs; a time step uses k_stage_faces.)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_boundary(const ShellDev* __restrict__ sh,
                                                  const double* __restrict__ bctab,
                                                  const double* __restrict__ gamma,
                                                  double* __restrict__ rhs, int outer_mode) {
  const int k = blockIdx.y;
  const ShellDev s = sh[k];
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= s.S) return;
  const int P = s.n_r * s.S;
  const long long ia = 50LL * s.pt_off + (long long)(s.n_r - 1) * s.S + a;
  if (s.outer) {
    // outer_mode 1: k_outer_cpbc has already treated the outer face in place
    if (!outer_mode) {
#pragma unroll 10
      for (int f = 0; f < 50; ++f) rhs[ia + (long long)f * P] = 0.0;
    }
    return;
  }
  if (s.bc_off < 0) return;
  const ShellDev t = sh[k + 1];
  const int Pt = t.n_r * t.S;
  const long long ib = 50LL * t.pt_off + a;
  const double* T = bctab + s.bc_off + 9LL * a;
  const double g2 = gamma[3 * s.instance + 2];
#pragma unroll 2
  for (int n = 0; n < 10; ++n) {
    double A[5], B[5], out[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      A[c] = rhs[ia + (long long)(10 * c + n) * P];
      B[c] = rhs[ib + (long long)(10 * c + n) * Pt];
    }
    interface_pair(A, B, T, g2, out);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      rhs[ia + (long long)(10 * c + n) * P] = out[c];
      rhs[ib + (long long)(10 * c + n) * Pt] = out[c];
    }
  }
}

// ---------------------------------------------------------------------------
// The faces of an SSP-RK3 stage whose other points k_pointwise_rhs<1 or 2>
// has finished: on every face the boundary treatment changes, the treated
// d_t u L' (from the raw one in L, read only) and out = c0 u0 + c1 (us + dt
// L'), with the arithmetic of the pointwise kernel's stage value: zero d_t u
// on the outer boundary (outer_mode 0; with outer_mode 1 k_outer_cpbc has
// treated the outer face of L in place, and it is used as it is), the
// upwinded interface value on both faces of an interface.  dt per instance.
// blockIdx.x: angular points, y: shell,
// z = 10 face + n: symmetric pair n (the five fields 10 c + n) of face 0, the
// inner face (an interface with shell y - 1 unless it is an excision face),
// or face 1, the outer face (the outer boundary, or an interface with shell
// y + 1).  Both shells of an interface recompute the pair's projection, so
// both get bitwise the same value.  out may alias u0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_stage_faces(const ShellDev* __restrict__ sh,
                                                     const double* __restrict__ bctab,
                                                     const double* __restrict__ gamma,
                                                     const double* __restrict__ dt, double c0,
                                                     const double* u0, double c1,
                                                     const double* __restrict__ us,
                                                     const double* __restrict__ L, double* out,
                                                     int outer_mode) {
  const int k = blockIdx.y;
  const ShellDev s = sh[k];
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= s.S) return;
  const int P = s.n_r * s.S;
  const int outer_face = blockIdx.z >= 10, n = blockIdx.z % 10;
  const int r = outer_face ? s.n_r - 1 : 0;
  const long long e0 = 50LL * s.pt_off + (long long)r * s.S + a;
  const double dtv = dt[s.instance];
  auto stage = [&](long long e, double val) {
    double v = c1 * (us[e] + dtv * val);
    if (c0 != 0.0) v += c0 * u0[e];
    out[e] = v;
  };
  if (outer_face && s.outer) {
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const long long e = e0 + (long long)(10 * c + n) * P;
      stage(e, outer_mode ? L[e] : 0.0);
    }
    return;
  }
  if (outer_face ? s.bc_off < 0 : s.inner) return;
  // the interface between shell ki (inner side) and ki + 1
  const int ki = outer_face ? k : k - 1;
  const ShellDev si = sh[ki], so = sh[ki + 1];
  const int Pi = si.n_r * si.S, Po = so.n_r * so.S;
  const long long ia = 50LL * si.pt_off + (long long)(si.n_r - 1) * si.S + a;
  const long long ib = 50LL * so.pt_off + a;
  const double* T = bctab + si.bc_off + 9LL * a;
  const double g2 = gamma[3 * si.instance + 2];
  double A[5], B[5], o[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    A[c] = L[ia + (long long)(10 * c + n) * Pi];
    B[c] = L[ib + (long long)(10 * c + n) * Po];
  }
  interface_pair(A, B, T, g2, o);
#pragma unroll
  for (int c = 0; c < 5; ++c) stage(e0 + (long long)(10 * c + n) * P, o[c]);
}

// ---------------------------------------------------------------------------
// Constraints: 64 components per point and the weighted sum of squares per block.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_constraints(
    const ShellDev* __restrict__ sh, const PtBlock* __restrict__ blk,
    const double* __restrict__ angtab, const double* __restrict__ radtab,
    const double* __restrict__ u, const double* __restrict__ dR, const double* __restrict__ dA,
    const double* __restrict__ Hin, double* __restrict__ Cout, double* __restrict__ partial) {
  __shared__ double red[256];
  const PtBlock b = blk[blockIdx.x];
  const ShellDev s = sh[b.shell];
  const int P = s.n_r * s.S;
  const int q = b.q0 + threadIdx.x;
  double ssq = 0.0;
  if (q < P) {
    const int r = q / s.S, a = q - r * s.S;
    const long long ub = 50LL * s.pt_off + q;
    const long long ab = 100LL * s.pt_off + (long long)r * 2 * s.S + a;
    const long long astride = (long long)s.n_r * 2 * s.S;
    const double* ang = angtab + 5LL * (s.ang_off + a);
    const Jac J = jacobian(ang, radtab[2 * (s.rad_off + r)]);
    const double w = ang[4] * radtab[2 * (s.rad_off + r) + 1];
    const long long cb = 64LL * s.pt_off + q;
    double psi[10], Pi[10], Phi[30];
#pragma unroll
    for (int n = 0; n < 10; ++n) psi[n] = u[ub + (long long)n * P];
#pragma unroll
    for (int n = 0; n < 10; ++n) Pi[n] = u[ub + (long long)(10 + n) * P];
#pragma unroll
    for (int n = 0; n < 30; ++n) Phi[n] = u[ub + (long long)(20 + n) * P];
    Geo G;
    geometry(psi, G);
    double Gm[4][10];
    christoffel(G, Pi, Phi, Gm);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double Ca = Hin[4LL * s.pt_off + (long long)c * P + q] + sym_dot(G.pinv, Gm[c]);
      ssq += Ca * Ca;
      if (Cout) Cout[cb + (long long)c * P] = Ca;
    }
    // C_iab = d_i psi_ab - Phi_iab
#pragma unroll 2
    for (int n = 0; n < 10; ++n) {
      const long long fo = (long long)n * P, fa = (long long)n * astride;
      double d[3];
      cart(J, dR[ub + fo], dA[ab + fa], dA[ab + fa + s.S], d);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double c3 = d[i] - Phi[10 * i + n];
        ssq += c3 * c3;
        if (Cout) Cout[cb + (long long)(4 + 10 * i + n) * P] = c3;
      }
    }
    // C_ijab = d_i Phi_jab - d_j Phi_iab, (i,j) = (x,y), (x,z), (y,z)
#pragma unroll 2
    for (int n = 0; n < 10; ++n) {
      double dPhi[3][3];   // dPhi[k][i] = d_k Phi_i
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const long long fo = (long long)(20 + 10 * i + n) * P;
        const long long fa = (long long)(20 + 10 * i + n) * astride;
        double d[3];
        cart(J, dR[ub + fo], dA[ab + fa], dA[ab + fa + s.S], d);
        dPhi[0][i] = d[0]; dPhi[1][i] = d[1]; dPhi[2][i] = d[2];
      }
      const double c01 = dPhi[0][1] - dPhi[1][0];
      const double c02 = dPhi[0][2] - dPhi[2][0];
      const double c12 = dPhi[1][2] - dPhi[2][1];
      ssq += c01 * c01 + c02 * c02 + c12 * c12;
      if (Cout) {
        Cout[cb + (long long)(34 + n) * P] = c01;
        Cout[cb + (long long)(44 + n) * P] = c02;
        Cout[cb + (long long)(54 + n) * P] = c12;
      }
    }
    ssq *= w;
  }
  red[threadIdx.x] = ssq;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// norm[i] = sqrt(sum_{blocks of instance i} partial / wsum[i]); one block per instance.
__global__ __launch_bounds__(256) void k_reduce_norm(const int* __restrict__ range,
                                                     const double* __restrict__ partial,
                                                     const double* __restrict__ wsum,
                                                     double* __restrict__ norm) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  const int b0 = range[2 * i], b1 = range[2 * i + 1];
  double s = 0.0;
  for (int b = b0 + threadIdx.x; b < b1; b += 256) s += partial[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) norm[i] = sqrt(red[0] / wsum[i]);
}

// ---------------------------------------------------------------------------
// Adjoint kernels.
// ---------------------------------------------------------------------------

// Reverse of the pointwise GH algebra and of the Cartesian Jacobian, in two
// register-light passes (one fused pass held 512 registers per lane and
// spilled 2.8 kB of it to scratch memory).
//
// k_pointwise_vjp_principal: from the cotangent lam of the raw (pre-boundary)
// d_t u, the cotangents of the spherical derivatives (dRb, dAb, laid out like
// dR and dA) pair by pair, and the partial cotangents of the geometry and of
// gamma1, gamma2 of these derivative terms into acc [12][P_total].
__global__ __launch_bounds__(256) void k_pointwise_vjp_principal(
    const ShellDev* __restrict__ sh, const PtBlock* __restrict__ blk,
    const double* __restrict__ angtab, const double* __restrict__ radtab,
    const double* __restrict__ u, const double* __restrict__ dR, const double* __restrict__ dA,
    const double* __restrict__ gamma, const double* __restrict__ mu, const double* __restrict__ lamf_,
    double* __restrict__ dRb, double* __restrict__ dAb, double* __restrict__ acc, long long p_total) {
  const PtBlock b = blk[blockIdx.x];
  const ShellDev s = sh[b.shell];
  const int P = s.n_r * s.S;
  const int q = b.q0 + threadIdx.x;
  if (q >= P) return;
  const int r = q / s.S, a = q - r * s.S;
  // the cotangent of the raw d_t u: mu itself, or on a treated face the
  // transposed boundary treatment's value
  const double* __restrict__ lam = treated_face(s, r) ? lamf_ : mu;
  const long long ub = 50LL * s.pt_off + q;
  const long long ab = 100LL * s.pt_off + (long long)r * 2 * s.S + a;
  const long long astride = (long long)s.n_r * 2 * s.S;
  const Jac J = jacobian(angtab + 5LL * (s.ang_off + a), radtab[2 * (s.rad_off + r)]);
  double psi[10];
#pragma unroll
  for (int f = 0; f < 10; ++f) psi[f] = u[ub + (long long)f * P];
  auto lamf = [&](int f) { return lam[ub + (long long)f * P]; };
  // derivatives of the five fields of pair n, streamed from dR / dA
  auto load = [&](int n, double* dpsi, double* dPi, double (*dPhi)[3]) {
    cart(J, dR[ub + (long long)n * P], dA[ab + (long long)n * astride], dA[ab + (long long)n * astride + s.S], dpsi);
    const int fp = 10 + n;
    cart(J, dR[ub + (long long)fp * P], dA[ab + (long long)fp * astride], dA[ab + (long long)fp * astride + s.S], dPi);
    for (int i = 0; i < 3; ++i) {
      const int ff = 20 + 10 * i + n;
      double d[3];
      cart(J, dR[ub + (long long)ff * P], dA[ab + (long long)ff * astride], dA[ab + (long long)ff * astride + s.S], d);
      dPhi[0][i] = d[0]; dPhi[1][i] = d[1]; dPhi[2][i] = d[2];
    }
  };
  // Cartesian cotangents -> spherical cotangents (transpose of the Jacobian)
  auto put = [&](int f, double x, double y, double z) {
    dRb[ub + (long long)f * P] = J.xr * x + J.yr * y + J.zr * z;
    dAb[ab + (long long)f * astride] = J.xt * x + J.yt * y + J.zt * z;
    dAb[ab + (long long)f * astride + s.S] = J.xp * x + J.yp * y;
  };
  auto store = [&](int n, const double* dpsi_b, const double* dPi_b, const double (*dPhi_b)[3]) {
    put(n, dpsi_b[0], dpsi_b[1], dpsi_b[2]);
    put(10 + n, dPi_b[0], dPi_b[1], dPi_b[2]);
    for (int i = 0; i < 3; ++i) put(20 + 10 * i + n, dPhi_b[0][i], dPhi_b[1][i], dPhi_b[2][i]);
  };
  double pa[GHP_VJP_ACC];
  ghp::rhs_vjp_principal(psi, gamma[3 * s.instance + 1], gamma[3 * s.instance + 2], lamf, load, store, pa);
  const long long pg = s.pt_off + q;
#pragma unroll
  for (int c = 0; c < GHP_VJP_ACC; ++c) acc[c * p_total + pg] = pa[c];
}

// A per-point field of a [component][point] array: v[i] is component i.
struct Strided {
  const double* p;
  long long stride;
  __device__ Strided operator+(int k) const { return Strided{p + k * stride, stride}; }
  __device__ double operator[](int i) const { return p[i * stride]; }
};

// k_pointwise_vjp_algebraic: the algebraic terms and the reverse of the
// geometry, continuing from acc: the direct cotangent of u (overwriting
// ubar) and per-block sums of the gamma cotangents.
__global__ __launch_bounds__(256) void k_pointwise_vjp_algebraic(
    const ShellDev* __restrict__ sh, const PtBlock* __restrict__ blk, const double* __restrict__ u,
    const double* __restrict__ Hin, const double* __restrict__ dHin, const double* __restrict__ gamma,
    const double* __restrict__ mu, const double* __restrict__ lamf_, const double* __restrict__ acc,
    double* __restrict__ ubar, double* __restrict__ gpart, long long p_total) {
  __shared__ double red[3][256];
  const PtBlock b = blk[blockIdx.x];
  const ShellDev s = sh[b.shell];
  const int P = s.n_r * s.S;
  const int q = b.q0 + threadIdx.x;
  double gb[3] = {0.0, 0.0, 0.0};
  if (q < P) {
    const long long ub = 50LL * s.pt_off + q;
    double H[4], dH[16], uo[50], pa[GHP_VJP_ACC];
    for (int c = 0; c < 4; ++c) H[c] = Hin[4LL * s.pt_off + (long long)c * P + q];
    for (int c = 0; c < 16; ++c) dH[c] = dHin[16LL * s.pt_off + (long long)c * P + q];
    const long long pg = s.pt_off + q;
    for (int c = 0; c < GHP_VJP_ACC; ++c) pa[c] = acc[c * p_total + pg];
    // the fields and the cotangent are read where they are used (from the
    // caches) rather than held in registers
    const double* lam = treated_face(s, q / s.S) ? lamf_ : mu;   // as in the principal pass
    ghp::rhs_vjp_algebraic(Strided{u + ub, P}, H, dH, gamma[3 * s.instance], gamma[3 * s.instance + 1],
                           gamma[3 * s.instance + 2], Strided{lam + ub, P}, pa, uo, gb);
    for (int f = 0; f < 50; ++f) ubar[ub + (long long)f * P] = uo[f];
  }
  for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = gb[c];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 3) gpart[3LL * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// Transpose of the boundary treatment: from the cotangent mu of the treated
// d_t u, the cotangent of the raw d_t u on the treated faces goes to Lb (only
// there; elsewhere it is mu itself, which the reverse pointwise passes read).
// The interface map writes the same value into both shells, so its transpose
// takes the summed cotangent back through reconstruction, upwind selection and
// projection; the outer Dirichlet rows have zero transpose.  The gamma2
// dependence of the exchange needs the raw d_t u (W); each point's gamma2
// cotangent goes to bcg[shell * max_S + a] (zero where there is no interface).
__global__ __launch_bounds__(256) void k_boundary_vjp(const ShellDev* __restrict__ sh, int max_S,
                                                      const double* __restrict__ bctab,
                                                      const double* __restrict__ gamma,
                                                      const double* __restrict__ W,
                                                      const double* __restrict__ mu, double* __restrict__ Lb,
                                                      double* __restrict__ bcg) {
  const int k = blockIdx.y;
  const ShellDev s = sh[k];
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= max_S) return;
  double contrib = 0.0;
  if (a < s.S) {
    const int P = s.n_r * s.S;
    const long long ia = 50LL * s.pt_off + (long long)(s.n_r - 1) * s.S + a;
    if (s.outer) {
      for (int f = 0; f < 50; ++f) Lb[ia + (long long)f * P] = 0.0;
    } else if (s.bc_off >= 0) {
      const ShellDev t = sh[k + 1];
      const int Pt = t.n_r * t.S;
      const long long ib = 50LL * t.pt_off + a;
      const double* T = bctab + s.bc_off + 9LL * a;
      const double sl[3] = {T[0], T[1], T[2]}, su[3] = {T[3], T[4], T[5]};
      const double w0 = T[6], wp = T[7], wm = T[8];
      const double g2 = gamma[3 * s.instance + 2];
      for (int n = 0; n < 10; ++n) {
        double l[5];
        for (int c = 0; c < 5; ++c)
          l[c] = mu[ia + (long long)(10 * c + n) * P] + mu[ib + (long long)(10 * c + n) * Pt];
        const double slL = sl[0] * l[2] + sl[1] * l[3] + sl[2] * l[4];
        const double ups_b = l[0] + g2 * l[1];
        const double up_b = 0.5 * l[1] + 0.5 * slL;
        const double um_b = 0.5 * l[1] - 0.5 * slL;
        const double A0 = W[ia + (long long)n * P], B0 = W[ib + (long long)n * Pt];
        contrib += l[1] * 0.5 * (A0 + B0) - up_b * (wp * A0 + (1.0 - wp) * B0) -
                   um_b * (wm * A0 + (1.0 - wm) * B0);
        const double sLu0 = sl[0] * l[2] + sl[1] * l[3] + sl[2] * l[4];   // sum_i s_i u0_b[i]
        for (int side = 0; side < 2; ++side) {
          const double xp = side ? 1.0 - wp : wp, xm = side ? 1.0 - wm : wm, x0 = side ? 1.0 - w0 : w0;
          const double sP_b = xp * up_b - xm * um_b - x0 * sLu0;
          double o[5];
          o[0] = 0.5 * ups_b - g2 * (xp * up_b + xm * um_b);
          o[1] = xp * up_b + xm * um_b;
          for (int i = 0; i < 3; ++i) o[2 + i] = x0 * l[2 + i] + su[i] * sP_b;
          for (int c = 0; c < 5; ++c) {
            if (side) Lb[ib + (long long)(10 * c + n) * Pt] = o[c];
            else Lb[ia + (long long)(10 * c + n) * P] = o[c];
          }
        }
      }
    }
  }
  bcg[(long long)k * max_S + a] = contrib;
}

// Reverse of the constraint norm: for loss sum_i lam_norm[i] ||C||_i the
// cotangent of C_c(p) is lam_norm w_p C_c / (||C|| sum w); it is taken back
// through C_a (gauge constraint), C_iab = d_i psi_ab - Phi_iab and
// C_ijab = d_i Phi_jab - d_j Phi_iab to u (overwriting ubar) and to the
// spherical derivatives (dRb, dAb).
__global__ __launch_bounds__(256) void k_constraints_vjp(
    const ShellDev* __restrict__ sh, const PtBlock* __restrict__ blk,
    const double* __restrict__ angtab, const double* __restrict__ radtab,
    const double* __restrict__ u, const double* __restrict__ Hin, const double* __restrict__ Cv,
    const double* __restrict__ norm, const double* __restrict__ wsum, const double* __restrict__ lam_norm,
    double* __restrict__ ubar, double* __restrict__ dRb, double* __restrict__ dAb) {
  const PtBlock b = blk[blockIdx.x];
  const ShellDev s = sh[b.shell];
  const int P = s.n_r * s.S;
  const int q = b.q0 + threadIdx.x;
  if (q >= P) return;
  const int r = q / s.S, a = q - r * s.S;
  const long long ub = 50LL * s.pt_off + q;
  const long long cb = 64LL * s.pt_off + q;
  const long long ab = 100LL * s.pt_off + (long long)r * 2 * s.S + a;
  const long long astride = (long long)s.n_r * 2 * s.S;
  const double* ang = angtab + 5LL * (s.ang_off + a);
  const Jac J = jacobian(ang, radtab[2 * (s.rad_off + r)]);
  const double w = ang[4] * radtab[2 * (s.rad_off + r) + 1];
  const double nrm = norm[s.instance];
  const double f = (nrm > 0.0) ? lam_norm[s.instance] * w / (nrm * wsum[s.instance]) : 0.0;
  double uu[50], H[4], uo[50], duo[3][50];
  for (int c = 0; c < 50; ++c) {
    uu[c] = u[ub + (long long)c * P];
    uo[c] = 0.0;
    duo[0][c] = duo[1][c] = duo[2][c] = 0.0;
  }
  for (int c = 0; c < 4; ++c) H[c] = Hin[4LL * s.pt_off + (long long)c * P + q];
  double Cb[4];
  for (int c = 0; c < 4; ++c) Cb[c] = f * Cv[cb + (long long)c * P];
  ghp::gauge_constraint_vjp(uu, H, Cb, uo);
  for (int i = 0; i < 3; ++i)
    for (int n = 0; n < 10; ++n) {
      const double g = f * Cv[cb + (long long)(4 + 10 * i + n) * P];
      duo[i][n] += g;
      uo[20 + 10 * i + n] -= g;
    }
  const int pi[3] = {0, 0, 1}, pj[3] = {1, 2, 2};
  for (int m = 0; m < 3; ++m)
    for (int n = 0; n < 10; ++n) {
      const double g = f * Cv[cb + (long long)(34 + 10 * m + n) * P];
      duo[pi[m]][20 + 10 * pj[m] + n] += g;
      duo[pj[m]][20 + 10 * pi[m] + n] -= g;
    }
  for (int c = 0; c < 50; ++c) {
    ubar[ub + (long long)c * P] = uo[c];
    const double x = duo[0][c], y = duo[1][c], z = duo[2][c];
    dRb[ub + (long long)c * P] = J.xr * x + J.yr * y + J.zr * z;
    dAb[ab + (long long)c * astride] = J.xt * x + J.yt * y + J.zt * z;
    dAb[ab + (long long)c * astride + s.S] = J.xp * x + J.yp * y;
  }
}

// g[i] += coef * (use_dt ? dt[i] : 1) * (gamma cotangents of instance i), summed
// in a fixed order over its point blocks and its interface points.
__global__ __launch_bounds__(256) void k_gamma_reduce(const int* __restrict__ blk_range,
                                                      const int* __restrict__ shell_range, int max_S,
                                                      const double* __restrict__ gpart,
                                                      const double* __restrict__ bcg,
                                                      const double* __restrict__ dt, double coef, int use_dt,
                                                      double* __restrict__ g) {
  __shared__ double red[3][256];
  const int i = blockIdx.x;
  double s[3] = {0.0, 0.0, 0.0};
  for (int b = blk_range[2 * i] + threadIdx.x; b < blk_range[2 * i + 1]; b += 256)
    for (int c = 0; c < 3; ++c) s[c] += gpart[3LL * b + c];
  const long long e0 = (long long)shell_range[2 * i] * max_S, e1 = (long long)shell_range[2 * i + 1] * max_S;
  for (long long e = e0 + threadIdx.x; e < e1; e += 256) s[2] += bcg[e];
  for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = s[c];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 3) g[3 * i + threadIdx.x] += coef * (use_dt ? dt[i] : 1.0) * red[threadIdx.x][0];
}

// out = a x + b y + c h z elementwise over the 50 fields (h = dt of the
// instance if use_dt, else 1); null x, y or z is skipped.  out may alias x, y or z.
__global__ __launch_bounds__(256) void k_lincomb(const ShellDev* __restrict__ sh, const PtBlock* __restrict__ blk,
                                                 const double* __restrict__ dt, int use_dt, double ca,
                                                 const double* x, double cb, const double* y, double cc,
                                                 const double* z, double* out) {
  const PtBlock b = blk[blockIdx.x];
  const ShellDev s = sh[b.shell];
  const int P = s.n_r * s.S;
  const int q = b.q0 + threadIdx.x;
  if (q >= P) return;
  const long long e = 50LL * s.pt_off + (long long)blockIdx.y * P + q;
  double v = 0.0;
  if (x) v += ca * x[e];
  if (y) v += cb * y[e];
  if (z) v += cc * (use_dt ? dt[s.instance] : 1.0) * z[e];
  out[e] = v;
}

// ---------------------------------------------------------------------------
// Setup: frozen interface projections from u_bg, and excision outflow speeds.
// bctab record per interface point: s_i (3), s^i (3), upwind weights of the
// inner side for u^0, u^+, u^- (1, 0 or 1/2 by the sign of the speed).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void face_normal(const double* u_bg, long long ib, int P, const double* ang,
                                            double sign, double* sl, double* su, double* v0,
                                            double* vp, double* vm) {
  double psi[10];
#pragma unroll
  for (int n = 0; n < 10; ++n) psi[n] = u_bg[ib + (long long)n * P];
  Geo G;
  geometry(psi, G);
  const double nh[3] = {sign * ang[0] * ang[3], sign * ang[0] * ang[2], sign * ang[1]};
  double nrm2 = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) nrm2 += G.gi[SYM3(i, j)] * nh[i] * nh[j];
  const double inrm = 1.0 / sqrt(nrm2);
#pragma unroll
  for (int i = 0; i < 3; ++i) sl[i] = nh[i] * inrm;
#pragma unroll
  for (int i = 0; i < 3; ++i)
    su[i] = G.gi[SYM3(i, 0)] * sl[0] + G.gi[SYM3(i, 1)] * sl[1] + G.gi[SYM3(i, 2)] * sl[2];
  const double sN = sl[0] * G.Nu[0] + sl[1] * G.Nu[1] + sl[2] * G.Nu[2];
  *v0 = -sN;
  *vp = -sN + G.N;
  *vm = -sN - G.N;
}

__device__ __forceinline__ double upwind_weight(double v) { return v > 0.0 ? 1.0 : (v < 0.0 ? 0.0 : 0.5); }

__global__ __launch_bounds__(256) void k_bc_setup(const ShellDev* __restrict__ sh, int max_S,
                                                  const double* __restrict__ angtab,
                                                  const double* __restrict__ u_bg,
                                                  double* __restrict__ bctab,
                                                  double* __restrict__ exmin) {
  const int k = blockIdx.y;
  const ShellDev s = sh[k];
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= max_S) return;
  if (a >= s.S) {                     // every entry of the shell's row is written
    exmin[(long long)k * max_S + a] = INFINITY;
    return;
  }
  const int P = s.n_r * s.S;
  const double* ang = angtab + 5LL * (s.ang_off + a);
  double sl[3], su[3], v0, vp, vm;
  if (s.bc_off >= 0) {
    const long long ib = 50LL * s.pt_off + (long long)(s.n_r - 1) * s.S + a;
    face_normal(u_bg, ib, P, ang, 1.0, sl, su, &v0, &vp, &vm);
    double* T = bctab + s.bc_off + 9LL * a;
    T[0] = sl[0]; T[1] = sl[1]; T[2] = sl[2];
    T[3] = su[0]; T[4] = su[1]; T[5] = su[2];
    T[6] = upwind_weight(v0); T[7] = upwind_weight(vp); T[8] = upwind_weight(vm);
  }
  double mn = INFINITY;
  if (s.inner) {
    const long long ib = 50LL * s.pt_off + a;
    face_normal(u_bg, ib, P, ang, -1.0, sl, su, &v0, &vp, &vm);
    mn = fmin(v0, fmin(vp, vm));
    if (mn != mn) mn = -INFINITY;   // NaN speed: report as inflow
  }
  exmin[(long long)k * max_S + a] = mn;
}

// Constraint-preserving treatment of d_t u at the outer boundary (the
// paper's ApplyBCs case (ii), Conclusions), in place on the raw RHS at every
// outer-face point; blockIdx.y = shell, threads over angular points.  With the
// unit normal s (+r_hat normalised with the state's metric at the face) and
// N.s = s_k N^k, per symmetric pair:
//   u^psi incoming (speed -(1+g1) N.s < 0): minus (1+g1)(N.s) s^k C_kab, the
//     normal part of the three-index constraint C_kab = d_k psi_ab - Phi_kab;
//   u^0 incoming (speed -N.s < 0): minus (N.s) P_i^l s^k C_klab, the normal
//     part of the four-index constraint C_klab = d_k Phi_lab - d_l Phi_kab
//     (P_i^l = delta_i^l - s_i s^l);
//   u^+, u^- incoming: frozen (zero); outgoing fields untouched.
// The Cartesian derivatives come from the derivative pass (dR, dA) through the
// same Jacobian as the pointwise kernel.
__global__ __launch_bounds__(256) void k_outer_cpbc(const ShellDev* __restrict__ sh,
                                                    const double* __restrict__ angtab,
                                                    const double* __restrict__ radtab,
                                                    const double* __restrict__ u,
                                                    const double* __restrict__ dR,
                                                    const double* __restrict__ dA,
                                                    const double* __restrict__ gamma,
                                                    double* __restrict__ rhs) {
  const int k = blockIdx.y;
  const ShellDev s = sh[k];
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (!s.outer || a >= s.S) return;
  const int P = s.n_r * s.S;
  const int r = s.n_r - 1;
  const long long ib = 50LL * s.pt_off + (long long)r * s.S + a;
  const long long ab = 100LL * s.pt_off + (long long)r * 2 * s.S + a;
  const long long astride = (long long)s.n_r * 2 * s.S;
  const double* ang = angtab + 5LL * (s.ang_off + a);
  double sl[3], su[3], v0, vp, vm;
  face_normal(u, ib, P, ang, 1.0, sl, su, &v0, &vp, &vm);
  const double g1 = gamma[3 * s.instance + 1], g2 = gamma[3 * s.instance + 2];
  const double sN = -v0;
  const double vpsi = -(1.0 + g1) * sN;
  const Jac J = jacobian(ang, radtab[2 * (s.rad_off + r)]);
  for (int n = 0; n < 10; ++n) {
    double L[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) L[c] = rhs[ib + (long long)(10 * c + n) * P];
    const double sPhi = su[0] * L[2] + su[1] * L[3] + su[2] * L[4];
    double upsi = L[0];
    double u0[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) u0[i] = L[2 + i] - sl[i] * sPhi;
    double up = L[1] + sPhi - g2 * L[0];
    double um = L[1] - sPhi - g2 * L[0];
    if (vpsi < 0.0) {
      double dpsi[3];
      cart(J, dR[ib + (long long)n * P], dA[ab + (long long)n * astride], dA[ab + (long long)n * astride + s.S],
           dpsi);
      double sC3 = 0.0;
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) sC3 += su[kk] * (dpsi[kk] - u[ib + (long long)(20 + 10 * kk + n) * P]);
      upsi -= (1.0 + g1) * sN * sC3;
    }
    if (v0 < 0.0) {
      double dPhi[3][3];   // dPhi[l][k] = d_k Phi_l
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        const int f = 20 + 10 * l + n;
        cart(J, dR[ib + (long long)f * P], dA[ab + (long long)f * astride], dA[ab + (long long)f * astride + s.S],
             dPhi[l]);
      }
      double sC4[3];
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        double t = 0.0;
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) t += su[kk] * (dPhi[l][kk] - dPhi[kk][l]);
        sC4[l] = t;
      }
      const double ss = su[0] * sC4[0] + su[1] * sC4[1] + su[2] * sC4[2];
#pragma unroll
      for (int i = 0; i < 3; ++i) u0[i] -= sN * (sC4[i] - sl[i] * ss);
    }
    if (vp < 0.0) up = 0.0;
    if (vm < 0.0) um = 0.0;
    rhs[ib + (long long)n * P] = upsi;
    rhs[ib + (long long)(10 + n) * P] = 0.5 * (up + um) + g2 * upsi;
#pragma unroll
    for (int i = 0; i < 3; ++i) rhs[ib + (long long)(20 + 10 * i + n) * P] = u0[i] + 0.5 * sl[i] * (up - um);
  }
}

__global__ __launch_bounds__(256) void k_nonfinite(const double* __restrict__ x, long long n,
                                                   int* __restrict__ count) {
  int c = 0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    c += isfinite(x[i]) ? 0 : 1;
  if (c) atomicAdd(count, c);
}

// ---------------------------------------------------------------------------
// Dormand-Prince 5(4) stepping: stage combinations, scaled error, per-instance
// step control, masked acceptance.  blockIdx.y = field where present.
// ---------------------------------------------------------------------------
struct DpTerms {
  const double* k[7];
  double c[7];
};

__global__ __launch_bounds__(256) void k_dp_combine(const ShellDev* __restrict__ sh,
                                                    const PtBlock* __restrict__ blk,
                                                    const double* __restrict__ dt,
                                                    const double* __restrict__ u, DpTerms T, int nk,
                                                    double* __restrict__ out) {
  const PtBlock b = blk[blockIdx.x];
  const ShellDev s = sh[b.shell];
  const int P = s.n_r * s.S;
  const int q = b.q0 + threadIdx.x;
  if (q >= P) return;
  const long long e = 50LL * s.pt_off + (long long)blockIdx.y * P + q;
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < 7; ++j)
    if (j < nk && T.c[j] != 0.0) acc += T.c[j] * T.k[j][e];
  out[e] = u[e] + dt[s.instance] * acc;
}

// Sum over the 50 values of each point of the block of (err / sk)^2, with
// err = dt sum_j e_j k_j and sk = atol + rtol max(|u|, |u5|).
__global__ __launch_bounds__(256) void k_dp_error(const ShellDev* __restrict__ sh,
                                                  const PtBlock* __restrict__ blk,
                                                  const double* __restrict__ dt,
                                                  const double* __restrict__ u,
                                                  const double* __restrict__ u5, DpTerms T, double atol,
                                                  double rtol, double* __restrict__ partial) {
  __shared__ double red[256];
  const PtBlock b = blk[blockIdx.x];
  const ShellDev s = sh[b.shell];
  const int P = s.n_r * s.S;
  const int q = b.q0 + threadIdx.x;
  double sum = 0.0;
  if (q < P) {
    const double h = dt[s.instance];
    const long long e0 = 50LL * s.pt_off + q;
    for (int f = 0; f < 50; ++f) {
      const long long e = e0 + (long long)f * P;
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < 7; ++j)
        if (T.c[j] != 0.0) acc += T.c[j] * T.k[j][e];
      const double err = h * acc;
      const double sk = atol + rtol * fmax(fabs(u[e]), fabs(u5[e]));
      const double r = err / sk;
      sum += r * r;
    }
  }
  red[threadIdx.x] = sum;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// One block per instance: RMS scaled error over its values, accept when <= 1,
// next step h min(10, max(0.2, 0.9 err^-1/5)) (10 for err = 0), not growing
// after a rejection; t advances by the step taken.
__global__ __launch_bounds__(256) void k_dp_control(const int* __restrict__ range,
                                                    const double* __restrict__ nval,
                                                    const double* __restrict__ partial, double* dt, double* t,
                                                    int* rejected, int* accepted, int* n_accepted,
                                                    double* err_out) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int b = range[2 * i] + threadIdx.x; b < range[2 * i + 1]; b += 256) s += partial[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double err = sqrt(red[0] / nval[i]);
  const double h = dt[i];
  double scale;
  int acc;
  if (err <= 1.0) {
    acc = 1;
    scale = (err == 0.0) ? 10.0 : fmin(10.0, fmax(0.2, 0.9 * pow(err, -0.2)));
    if (rejected[i]) scale = fmin(scale, 1.0);
    t[i] += h;
    if (n_accepted) n_accepted[i] += 1;
  } else {
    acc = 0;
    scale = fmax(0.2, 0.9 * pow(err, -0.2));
  }
  rejected[i] = 1 - acc;
  accepted[i] = acc;
  dt[i] = h * scale;
  if (err_out) err_out[i] = err;
}

__global__ __launch_bounds__(256) void k_dp_accept(const ShellDev* __restrict__ sh,
                                                   const PtBlock* __restrict__ blk,
                                                   const int* __restrict__ accepted,
                                                   const double* __restrict__ src, double* __restrict__ dst,
                                                   const double* __restrict__ src2, double* __restrict__ dst2) {
  const PtBlock b = blk[blockIdx.x];
  const ShellDev s = sh[b.shell];
  const int P = s.n_r * s.S;
  const int q = b.q0 + threadIdx.x;
  if (q >= P || !accepted[s.instance]) return;
  const long long e = 50LL * s.pt_off + (long long)blockIdx.y * P + q;
  dst[e] = src[e];
  if (dst2) dst2[e] = src2[e];
}

// Split-K tail of a GEMM plan: C[r][c] = (or +=) the sum over chunks q of
// W[q][r][c], added in chunk order (so the result is the same on every run).
// W holds nchunk row-major blocks of rows x cols.
template <bool ACC>
__global__ __launch_bounds__(256) void k_sum_chunks(const double* __restrict__ W, int nchunk, int rows, int cols,
                                                   double* __restrict__ C, int ldc) {
  const long long n = (long long)rows * cols;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = W[i];
  for (int q = 1; q < nchunk; ++q) s += W[(long long)q * n + i];
  const long long r = i / cols, col = i - r * cols;
  double* o = C + r * ldc + col;
  if (ACC) *o += s;
  else *o = s;
}

__global__ __launch_bounds__(256) void k_fill_int(int* __restrict__ x, int n, int v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] = v;
}

// ---------------------------------------------------------------------------
// Transform path of the angular operators: the theta step.  Per (field,
// radius) row the Fourier coefficients AB[i'][m'] (n = L+1 theta nodes i',
// columns m' < n the cos(m phi) coefficients, m' >= n the sin(m phi) ones,
// m = m' mod n) are mapped by the per-order theta kernels K_m[i][i'].  One
// thread owns a (theta node i, column m') pair: it keeps the kernel rows it
// needs in registers and sweeps a chunk of ROWS rows, so the kernel table is
// read once per thread and the coefficient loads are coalesced over m'.
// Block (shell, q0 = r0 * S + a0): rows r0.., pairs a0 .. a0 + 255.
// ktab (per L at kt_off): [3][n][n][n] = d/dtheta, d/dphi, filter kernels.
// ---------------------------------------------------------------------------
template <int NMAX, int MODE>
__global__ __launch_bounds__(256) void k_ang_theta(const ShellDev* __restrict__ sh,
                                                   const PtBlock* __restrict__ tblk,
                                                   const double* __restrict__ ktab,
                                                   const double* __restrict__ AB, double* __restrict__ X) {
  constexpr int ROWS = 16;
  const PtBlock b = tblk[blockIdx.x];
  const ShellDev s = sh[b.shell];
  const int n = s.L + 1, nc = 2 * n;
  const int r0 = b.q0 / s.S;
  const int a = b.q0 - r0 * s.S + threadIdx.x;
  if (a >= s.S) return;
  const int i = a / nc, mp = a - i * nc, m = mp % n;
  const int nrows = 50 * s.n_r;
  const long long nn = (long long)n * n;
  double k0[NMAX], k1[NMAX];
  const double* __restrict__ K0 = ktab + s.kt_off + (MODE == 0 ? 0 : 2 * (long long)n * nn) + m * nn +
                                  (long long)i * n;
#pragma unroll
  for (int ip = 0; ip < NMAX; ++ip) {
    k0[ip] = (ip < n) ? K0[ip] : 0.0;
    k1[ip] = (MODE == 0 && ip < n) ? K0[(long long)n * nn + ip] : 0.0;
  }
  const int r1 = min(nrows, r0 + ROWS);
  for (int r = r0; r < r1; ++r) {
    const double* __restrict__ col = AB + 50LL * s.pt_off + (long long)r * s.S + mp;
    // every load is issued unconditionally (index clamped to the last node;
    // the kernel entries past n are zero) so that they can all be in flight
    double v[NMAX];
#pragma unroll
    for (int ip = 0; ip < NMAX; ++ip) v[ip] = col[(long long)min(ip, n - 1) * nc];
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int ip = 0; ip < NMAX; ++ip) {
      a0 += k0[ip] * v[ip];
      if (MODE == 0) a1 += k1[ip] * v[ip];
    }
    if (MODE == 0) {
      double* __restrict__ out = X + 100LL * s.pt_off + (long long)r * 2 * s.S;
      out[i * nc + mp] = a0;
      // d/dphi: the cos(m phi) coefficient (m' < n) multiplies sin(m phi) in
      // the synthesis and the sin one multiplies -cos(m phi)
      if (mp < n) out[s.S + i * nc + mp + n] = a1;
      else out[s.S + i * nc + mp - n] = -a1;
    } else {
      X[50LL * s.pt_off + (long long)r * s.S + i * nc + mp] = a0;
    }
  }
}


// ---------------------------------------------------------------------------
// The theta step on the matrix cores, for shells with n = L + 1 a multiple of
// 16 (v_mfma_f64_16x16x4_f64).  A work item is 8 rows x MB orders m0 ..
// m0+MB-1 (MB = 16 for n <= 32: every access a whole 128-byte line; 8 for
// n = 48, 64, where 16 orders would leave one workgroup per CU's LDS).
// For one order m the step is a product
//   C[i][(r, c)] = sum_i' K_m[i][i'] W_m[i'][(r, c)],
// with the 16 columns (r, c) = (row r0 + r, c = 0 cos / 1 sin) of the item.
// The item's coefficient columns are staged in LDS as [i'][m][c][r], 16
// doubles per (i', m), each i' row padded by 16 doubles: consecutive i' then
// fall in opposite halves of the banks, so the B operands of a half-wave hit
// every bank once.  The kernel rows come from the transposed table
// ktabT[kind][m][i'][i] as MFMA A operands (16 consecutive i per
// quarter-wave).  MB / 2 waves take two orders each.  Each workgroup reads
// and writes whole 8 MB-byte segments (the MB orders of one (row, node, c));
// with MB = 8 the host orders the items so that the other half of each line
// is handled on the same XCD.  Items with r0 < 0 are padding.  The results
// are stored through LDS in whole runs (see below).
// ---------------------------------------------------------------------------
// (16-order items: two workgroups of 8 waves per CU, so at least four waves
// per SIMD, at most 128 registers)
template <int N, int MODE, int MB>
__global__ __launch_bounds__(32 * MB, MB == 16 ? 4 : 1) void k_ang_theta_mfma(const ShellDev* __restrict__ sh,
                                                            const ThetaItem* __restrict__ items,
                                                            const double* __restrict__ ktabT,
                                                            const double* __restrict__ AB, double* __restrict__ X) {
  constexpr int R = 8, NB = N / 16, KS = N / 4;
  constexpr int NW = MB / 2, NT = 64 * NW;   // waves of two orders each
  constexpr int ROWLEN = MB * 2 * R + 16;
  static_assert(N % 16 == 0, "n must be a multiple of 16");
  static_assert(MB == 8 || MB == 16, "items of 8 or 16 orders");
  __shared__ double Ws[N * ROWLEN];
  const ThetaItem it = items[blockIdx.x];
  if (it.r0 < 0) return;   // padding of the XCD grouping
  const ShellDev s = sh[it.shell];
  const int nc = 2 * N, S = s.S;
  const int nrows = 50 * s.n_r;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* __restrict__ Wg = AB + 50LL * s.pt_off;
  // stage the item's columns: 16-byte loads of two consecutive orders
  for (int idx = tid; idx < R * N * 2 * (MB / 2); idx += NT) {
    const int mp2 = idx % (MB / 2);
    int t = idx / (MB / 2);
    const int c = t & 1;
    t >>= 1;
    const int ip = t % N, r = t / N;
    const int row = min(it.r0 + r, nrows - 1);
    const double2 v =
        *reinterpret_cast<const double2*>(Wg + (long long)row * S + ip * nc + c * N + it.m0 + 2 * mp2);
    Ws[ip * ROWLEN + (4 * mp2 + c) * R + r] = v.x;
    Ws[ip * ROWLEN + (4 * mp2 + 2 + c) * R + r] = v.y;
  }
  __syncthreads();
  const double* __restrict__ Kt = ktabT + s.kt_off;
  const long long n3 = (long long)N * N * N, n2 = (long long)N * N;
  const int col = lane & 15, q = lane >> 4;
  d4 rA[2][NB], rB[2][NB];
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    const int m = it.m0 + wave + NW * w;
    const double* __restrict__ KA = Kt + (MODE == 0 ? 0 : 2 * n3) + m * n2;   // d/dtheta or filter
    const double* __restrict__ KB = Kt + n3 + m * n2;                         // d/dphi
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) {
      rA[w][bi] = d4{0.0, 0.0, 0.0, 0.0};
      rB[w][bi] = d4{0.0, 0.0, 0.0, 0.0};
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int ip = ks * 4 + q;
      const double b = Ws[ip * ROWLEN + (wave + NW * w) * 16 + col];
#pragma unroll
      for (int bi = 0; bi < NB; ++bi) {
        const int i = bi * 16 + col;
        rA[w][bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(KA[ip * N + i], b, rA[w][bi], 0, 0, 0);
        if (MODE == 0) rB[w][bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(KB[ip * N + i], b, rB[w][bi], 0, 0, 0);
      }
    }
    if (MB == 16) __builtin_amdgcn_sched_barrier(0);
  }
  // The results go out through LDS (the staging buffer, free again), one
  // part at a time (d/dtheta or the filter; then d/dphi with its cos and sin
  // slots exchanged and the sin one negated), as runs of the item's MB
  // orders: 8 MB bytes per (row, node, slot), written by MB / 2 lanes at once.
  // In LDS a run of row r, node i, slot c sits at r * OST + i * IST + c * MB;
  // the strides put the 32 stores of a half-wave, and its reads of the runs,
  // in distinct banks.
  constexpr int IST = MB == 8 ? 16 : 2 * MB + 1;
  constexpr int OST = MB == 8 ? N * 16 + 1 : N * IST + 2;
  constexpr int HL = MB / 2;   // lanes per run
  static_assert(R * OST <= N * ROWLEN, "the output runs fit in the staging buffer");
  const int rr = col & 7, c = col >> 3;
  const int nrun = R * N * 2;
#pragma unroll
  for (int part = 0; part < (MODE == 0 ? 2 : 1); ++part) {
    __syncthreads();
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
      for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = bi * 16 + q + 4 * v;
          const int slot = part == 0 ? c : 1 - c;
          const double val = part == 0 ? rA[w][bi][v] : (c == 0 ? rB[w][bi][v] : -rB[w][bi][v]);
          Ws[rr * OST + i * IST + slot * MB + wave + NW * w] = val;
        }
    __syncthreads();
    for (int idx = tid; idx < nrun * HL; idx += NT) {
      const int run = idx / HL, h = idx % HL;
      const int r = run / (2 * N), rem = run - r * 2 * N, i = rem >> 1, sl = rem & 1;
      const int row = it.r0 + r;
      if (row >= nrows) continue;
      const double* o = Ws + r * OST + i * IST + sl * MB + 2 * h;
      double2 val;
      val.x = o[0];
      val.y = o[1];
      double* dst = MODE == 0 ? X + 100LL * s.pt_off + (long long)row * 2 * S + part * S
                              : X + 50LL * s.pt_off + (long long)row * S;
      *reinterpret_cast<double2*>(dst + i * nc + sl * N + it.m0 + 2 * h) = val;
    }
  }
}


// ---------------------------------------------------------------------------
// Tensor-coupled filter: the coupling step Y = F X on the angular
// coefficients.  One workgroup (16 waves) per work item (segment, NC columns
// (shell, radius), a range of slices): the segment's inputs are staged in
// LDS, NC doubles per input row (runs of nsg consecutive coefficients per
// field from HBM); then every wave takes a 64-row slice: lane = row, the k-th
// couplings of the 64 rows are one contiguous load of values and one of input
// rows, and each coupling is applied to the staged columns of its input (NC/2
// 16-byte LDS reads).  Column pair p of input row r sits at pair slot
// (p + r/4) mod (NC/2), so the reads of 64 random rows spread over the LDS
// banks.
// ---------------------------------------------------------------------------
constexpr int TF_THREADS = 1024;

template <int NP>
__device__ __forceinline__ int tf_slot(int row, int pair) {
  return row * NP + ((pair + (row >> 2)) & (NP - 1));
}

template <int NC>
__global__ __launch_bounds__(TF_THREADS) void k_tensor_couple(const TfItem* __restrict__ items,
                                                              const TfSeg* __restrict__ segs,
                                                              const TfCol* __restrict__ cols,
                                                              const long long* __restrict__ soff,
                                                              const int* __restrict__ swidth,
                                                              const int* __restrict__ perm,
                                                              const int* __restrict__ lidx,
                                                              const double* __restrict__ val,
                                                              const double* __restrict__ X, double* __restrict__ Y) {
  constexpr int NP = NC / 2;
  static_assert(NP == 1 || NP == 2 || NP == 4, "column pairs must be a power of two");
  __shared__ double2 lds[TF_LDS_DOUBLES / 2];
  const TfItem it = items[blockIdx.x];
  const TfSeg sg = segs[it.seg];
  const int n = sg.ne * sg.nsg;
  const int nc = it.ncol;
  long long cbase[NC], cstr[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const TfCol cc = cols[it.col0 + (c < nc ? c : 0)];
    cbase[c] = cc.base;
    cstr[c] = cc.fstride;
  }
  for (int i = threadIdx.x; i < n; i += TF_THREADS) {
    const int e = i / sg.nsg, s = i - e * sg.nsg;
    double x[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c)
      x[c] = (c < nc) ? X[cbase[c] + (long long)(sg.e0 + e) * cstr[c] + sg.s0 + s] : 0.0;
#pragma unroll
    for (int p = 0; p < NP; ++p) lds[tf_slot<NP>(i, p)] = double2{x[2 * p], x[2 * p + 1]};
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int q = it.q0 + wave; q < it.q1; q += TF_THREADS / 64) {
    const long long off = soff[sg.slice0 + q];
    const int w = swidth[sg.slice0 + q];
    const int row = perm[(long long)(sg.slice0 + q) * 64 + lane];
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    const double* __restrict__ vq = val + off + lane;
    const int* __restrict__ iq = lidx + off + lane;
    // groups of 16 couplings: all 32 loads issued before the first is used
    constexpr int U = 16;
    int k = 0;
    for (; k + U <= w; k += U) {
      double v[U];
      int li[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        v[u] = vq[64 * (k + u)];
        li[u] = iq[64 * (k + u)];
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          const double2 x = lds[tf_slot<NP>(li[u], p)];
          acc[2 * p] += v[u] * x.x;
          acc[2 * p + 1] += v[u] * x.y;
        }
    }
    for (; k < w; ++k) {
      const double v = vq[64 * k];
      const int li = iq[64 * k];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const double2 x = lds[tf_slot<NP>(li, p)];
        acc[2 * p] += v * x.x;
        acc[2 * p + 1] += v * x.y;
      }
    }
    if (row >= 0) {
      const int e = row / sg.nsg, s = row - e * sg.nsg;
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (c < nc) Y[cbase[c] + (long long)(sg.e0 + e) * cstr[c] + sg.s0 + s] = acc[c];
    }
  }
}


// ---------------------------------------------------------------------------
// Tensor-coupled filter by transforms: the per-order Legendre steps between
// the Fourier GEMMs and the coupling.  Analysis: one thread per (row, s),
// s fastest:
//   X[s] = sum_i TA[i][s] F[i][m'(s)],  TA[i][s] = f_m (2 pi / N_phi) w_i P_l^|m|(x_i)
// (f_0 = 1, f_m = sqrt2; m'(s) = m for m >= 0, n + |m| for m < 0): the table
// loads of a wave are contiguous, its F loads fall in one 2n-row of the block.
// Each thread takes LG_ROWS consecutive rows, so every table value it loads
// serves LG_ROWS rows.  Synthesis: one thread per (row, m', i), i fastest:
//   G[i][m'] = sum_{l >= m} TS[s(l, +-m)][i] Y[s],  TS[s][i] = f_m P_l^|m|(x_i)
// (zero for the sin column of m = 0): the table loads of a wave are
// contiguous and its coefficient loads take a few values (4 columns m').
// ---------------------------------------------------------------------------
constexpr int LG_ROWS = 10;   // rows per thread (divides the 50 n_r rows of every shell)

__global__ __launch_bounds__(256) void k_leg_analysis(const ShellDev* __restrict__ sh,
                                                      const PtBlock* __restrict__ blk,
                                                      const double* __restrict__ legtab,
                                                      const double* __restrict__ F, double* __restrict__ X) {
  const PtBlock b = blk[blockIdx.x];
  const ShellDev d = sh[b.shell];
  const int n = d.L + 1, ns = n * n, S = 2 * n * n;
  const int q = b.q0 + threadIdx.x;
  if (q >= 5 * d.n_r * ns) return;
  const int g = q / ns, sidx = q - g * ns;
  int l = int(sqrt(double(sidx)));      // degree of s = l l + l + m
  if (l * l > sidx) --l;
  if ((l + 1) * (l + 1) <= sidx) ++l;
  const int m = sidx - l * l - l;
  const int col = m >= 0 ? m : n - m;
  const double* __restrict__ TA = legtab + d.lg_off + sidx;
  const double* __restrict__ f = F + 50LL * d.pt_off + (long long)g * LG_ROWS * S + col;
  double acc[LG_ROWS];
#pragma unroll
  for (int r = 0; r < LG_ROWS; ++r) acc[r] = 0.0;
  for (int i = 0; i < n; ++i) {
    const double t = TA[(long long)i * ns];
#pragma unroll
    for (int r = 0; r < LG_ROWS; ++r) acc[r] += t * f[(long long)r * S + (long long)i * 2 * n];
  }
  double* __restrict__ x = X + d.tf_off + (long long)g * LG_ROWS * d.nsp + sidx;
#pragma unroll
  for (int r = 0; r < LG_ROWS; ++r) x[(long long)r * d.nsp] = acc[r];
}

__global__ __launch_bounds__(256) void k_leg_synthesis(const ShellDev* __restrict__ sh,
                                                       const PtBlock* __restrict__ blk,
                                                       const double* __restrict__ legtab,
                                                       const double* __restrict__ Y, double* __restrict__ G) {
  const PtBlock b = blk[blockIdx.x];
  const ShellDev d = sh[b.shell];
  const int n = d.L + 1, ns = n * n, S = 2 * n * n;
  const int q = b.q0 + threadIdx.x;
  if (q >= 5 * d.n_r * S) return;
  const int g = q / S, rem = q - g * S, col = rem / n, i = rem - col * n;
  const bool sinpart = col >= n;
  const int m = sinpart ? col - n : col;
  double acc[LG_ROWS];
#pragma unroll
  for (int r = 0; r < LG_ROWS; ++r) acc[r] = 0.0;
  if (!(sinpart && m == 0)) {
    const double* __restrict__ TS = legtab + d.lg_off + (long long)ns * n + i;
    const double* __restrict__ y = Y + d.tf_off + (long long)g * LG_ROWS * d.nsp;
    for (int l = m; l < n; ++l) {
      const int sidx = l * l + l + (sinpart ? -m : m);
      const double t = TS[(long long)sidx * n];
#pragma unroll
      for (int r = 0; r < LG_ROWS; ++r) acc[r] += t * y[(long long)r * d.nsp + sidx];
    }
  }
  double* __restrict__ out = G + 50LL * d.pt_off + (long long)g * LG_ROWS * S + (long long)i * 2 * n + col;
#pragma unroll
  for (int r = 0; r < LG_ROWS; ++r) out[(long long)r * S] = acc[r];
}

}  // namespace

namespace ghk {


// Deterministic non-zero fill (bounded values in [-0.5, 0.5)), used so that the
// autotuner times the matrix cores on data of realistic activity.
__global__ __launch_bounds__(256) void k_fill_pattern(double* __restrict__ x, long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    unsigned long long h = (unsigned long long)i * 0x9E3779B97F4A7C15ull;
    h ^= h >> 29;
    x[i] = double(h & 0xFFFFF) / double(0x100000) - 0.5;
  }
}

hipError_t fill_pattern(double* x, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  long long nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_fill_pattern, dim3((unsigned)(nb < 8192 ? nb : 8192)), dim3(256), 0, st, x, n);
  return hipGetLastError();
}

hipError_t leg_analysis(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* legtab, const double* F,
                        double* X, hipStream_t st) {
  if (n_blk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_leg_analysis, dim3(n_blk), dim3(256), 0, st, sh, blk, legtab, F, X);
  return hipGetLastError();
}

hipError_t leg_synthesis(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* legtab, const double* Y,
                         double* G, hipStream_t st) {
  if (n_blk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_leg_synthesis, dim3(n_blk), dim3(256), 0, st, sh, blk, legtab, Y, G);
  return hipGetLastError();
}

hipError_t tensor_couple(const TfItem* items, const int n_items[3], const TfSeg* segs, const TfCol* cols,
                         const long long* soff, const int* swidth, const int* perm, const int* lidx,
                         const double* val, const double* X, double* Y, hipStream_t st) {
  const TfItem* it = items;
  if (n_items[0] > 0)
    hipLaunchKernelGGL(k_tensor_couple<8>, dim3(n_items[0]), dim3(TF_THREADS), 0, st, it, segs, cols, soff, swidth,
                       perm, lidx, val, X, Y);
  it += n_items[0];
  if (n_items[1] > 0)
    hipLaunchKernelGGL(k_tensor_couple<4>, dim3(n_items[1]), dim3(TF_THREADS), 0, st, it, segs, cols, soff, swidth,
                       perm, lidx, val, X, Y);
  it += n_items[1];
  if (n_items[2] > 0)
    hipLaunchKernelGGL(k_tensor_couple<2>, dim3(n_items[2]), dim3(TF_THREADS), 0, st, it, segs, cols, soff, swidth,
                       perm, lidx, val, X, Y);
  return hipGetLastError();
}

hipError_t radial(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* dtab,
                  const double* u, double* dR, int ncomp_lo, int ncomp_hi, bool transpose, bool accumulate,
                  hipStream_t st) {
  dim3 grid(n_blk, ncomp_hi - ncomp_lo), block(256);
  if (!transpose && !accumulate)
    hipLaunchKernelGGL((k_radial<false, false>), grid, block, 0, st, sh, blk, dtab, u, dR, ncomp_lo);
  else if (!transpose)
    hipLaunchKernelGGL((k_radial<false, true>), grid, block, 0, st, sh, blk, dtab, u, dR, ncomp_lo);
  else if (!accumulate)
    hipLaunchKernelGGL((k_radial<true, false>), grid, block, 0, st, sh, blk, dtab, u, dR, ncomp_lo);
  else
    hipLaunchKernelGGL((k_radial<true, true>), grid, block, 0, st, sh, blk, dtab, u, dR, ncomp_lo);
  return hipGetLastError();
}

hipError_t sum_chunks(const double* W, int nchunk, int rows, int cols, double* C, int ldc, bool accumulate,
                      hipStream_t st) {
  const long long n = (long long)rows * cols;
  if (n <= 0) return hipSuccess;
  dim3 grid(unsigned((n + 255) / 256));
  if (accumulate) hipLaunchKernelGGL(k_sum_chunks<true>, grid, dim3(256), 0, st, W, nchunk, rows, cols, C, ldc);
  else hipLaunchKernelGGL(k_sum_chunks<false>, grid, dim3(256), 0, st, W, nchunk, rows, cols, C, ldc);
  return hipGetLastError();
}

int radial_col_maxr(int max_nr) {
  if (max_nr <= 16) return 16;
  if (max_nr <= 24) return 24;
  if (max_nr <= 36) return 36;
  if (max_nr <= 64) return 64;
  return 0;
}

template <int MAXR>
static void launch_col(dim3 grid, hipStream_t st, bool trans, bool acc, const ShellDev* sh,
                       const PtBlock* cblk, const double* dtab, const double* u, double* dR, int f0) {
  if (!trans && !acc)
    hipLaunchKernelGGL((k_radial_col<MAXR, false, false>), grid, dim3(256), 0, st, sh, cblk, dtab, u, dR, f0);
  else if (!trans && acc)
    hipLaunchKernelGGL((k_radial_col<MAXR, false, true>), grid, dim3(256), 0, st, sh, cblk, dtab, u, dR, f0);
  else if (trans && !acc)
    hipLaunchKernelGGL((k_radial_col<MAXR, true, false>), grid, dim3(256), 0, st, sh, cblk, dtab, u, dR, f0);
  else
    hipLaunchKernelGGL((k_radial_col<MAXR, true, true>), grid, dim3(256), 0, st, sh, cblk, dtab, u, dR, f0);
}

hipError_t radial_col(int maxr, const ShellDev* sh, const PtBlock* cblk, int n_cblk, const double* dtab,
                      const double* u, double* dR, int ncomp_lo, int ncomp_hi, bool transpose, bool accumulate,
                      hipStream_t st) {
  dim3 grid(n_cblk, ncomp_hi - ncomp_lo);
  switch (maxr) {
    case 16: launch_col<16>(grid, st, transpose, accumulate, sh, cblk, dtab, u, dR, ncomp_lo); break;
    case 24: launch_col<24>(grid, st, transpose, accumulate, sh, cblk, dtab, u, dR, ncomp_lo); break;
    case 36: launch_col<36>(grid, st, transpose, accumulate, sh, cblk, dtab, u, dR, ncomp_lo); break;
    case 64: launch_col<64>(grid, st, transpose, accumulate, sh, cblk, dtab, u, dR, ncomp_lo); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t pointwise_rhs(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* angtab,
                         const double* radtab, const double* u, const double* dR, const double* dA,
                         const double* H, const double* dH, const double* gamma, double* rhs,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_pointwise_rhs<0>, dim3(n_blk), dim3(256), 0, st, sh, blk, angtab, radtab, u, dR,
                     dA, H, dH, gamma, rhs, nullptr, 0.0, nullptr, 0.0, nullptr);
  return hipGetLastError();
}

hipError_t pointwise_stage(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* angtab,
                           const double* radtab, const double* us, const double* dR, const double* dA,
                           const double* H, const double* dH, const double* gamma, double* L, const double* dt,
                           double c0, const double* u0, double c1, double* out, hipStream_t st) {
  if (c0 != 0.0 && !u0) return hipErrorInvalidValue;
  if (c0 != 0.0)
    hipLaunchKernelGGL(k_pointwise_rhs<2>, dim3(n_blk), dim3(256), 0, st, sh, blk, angtab, radtab, us, dR,
                       dA, H, dH, gamma, L, dt, c0, u0, c1, out);
  else
    hipLaunchKernelGGL(k_pointwise_rhs<1>, dim3(n_blk), dim3(256), 0, st, sh, blk, angtab, radtab, us, dR,
                       dA, H, dH, gamma, L, dt, c0, u0, c1, out);
  return hipGetLastError();
}

hipError_t stage_faces(const ShellDev* sh, int n_shells, int max_S, const double* bctab, const double* gamma,
                       const double* dt, double c0, const double* u0, double c1, const double* us, const double* L,
                       double* out, int outer_mode, hipStream_t st) {
  dim3 grid((max_S + 255) / 256, n_shells, 20), block(256);
  hipLaunchKernelGGL(k_stage_faces, grid, block, 0, st, sh, bctab, gamma, dt, c0, u0, c1, us, L, out, outer_mode);
  return hipGetLastError();
}

hipError_t boundary(const ShellDev* sh, int n_shells, int max_S, const double* bctab,
                    const double* gamma, double* rhs, int outer_mode, hipStream_t st) {
  dim3 grid((max_S + 255) / 256, n_shells), block(256);
  hipLaunchKernelGGL(k_boundary, grid, block, 0, st, sh, bctab, gamma, rhs, outer_mode);
  return hipGetLastError();
}

hipError_t outer_cpbc(const ShellDev* sh, int n_shells, int max_S, const double* angtab, const double* radtab,
                      const double* u, const double* dR, const double* dA, const double* gamma, double* rhs,
                      hipStream_t st) {
  dim3 grid((max_S + 255) / 256, n_shells), block(256);
  hipLaunchKernelGGL(k_outer_cpbc, grid, block, 0, st, sh, angtab, radtab, u, dR, dA, gamma, rhs);
  return hipGetLastError();
}

hipError_t constraints(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* angtab,
                       const double* radtab, const double* u, const double* dR, const double* dA,
                       const double* H, double* C, double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_constraints, dim3(n_blk), dim3(256), 0, st, sh, blk, angtab, radtab, u, dR,
                     dA, H, C, partial);
  return hipGetLastError();
}

hipError_t reduce_norm(const int* range, int n_inst, const double* partial, const double* wsum,
                       double* norm, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_norm, dim3(n_inst), dim3(256), 0, st, range, partial, wsum, norm);
  return hipGetLastError();
}

hipError_t bc_setup(const ShellDev* sh, int n_shells, int max_S, const double* angtab,
                    const double* u_bg, double* bctab, double* exmin, hipStream_t st) {
  dim3 grid((max_S + 255) / 256, n_shells), block(256);
  hipLaunchKernelGGL(k_bc_setup, grid, block, 0, st, sh, max_S, angtab, u_bg, bctab, exmin);
  return hipGetLastError();
}

hipError_t pointwise_vjp(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* angtab,
                         const double* radtab, const double* u, const double* dR, const double* dA,
                         const double* H, const double* dH, const double* gamma, const double* mu,
                         const double* lamf, double* ubar, double* dRb, double* dAb, double* gpart, double* acc,
                         long long p_total, hipStream_t st) {
  hipLaunchKernelGGL(k_pointwise_vjp_principal, dim3(n_blk), dim3(256), 0, st, sh, blk, angtab, radtab, u, dR, dA,
                     gamma, mu, lamf, dRb, dAb, acc, p_total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pointwise_vjp_algebraic, dim3(n_blk), dim3(256), 0, st, sh, blk, u, H, dH, gamma, mu, lamf,
                     acc, ubar, gpart, p_total);
  return hipGetLastError();
}

hipError_t constraints_vjp(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* angtab,
                           const double* radtab, const double* u, const double* H, const double* C,
                           const double* norm, const double* wsum, const double* lam_norm, double* ubar,
                           double* dRb, double* dAb, hipStream_t st) {
  hipLaunchKernelGGL(k_constraints_vjp, dim3(n_blk), dim3(256), 0, st, sh, blk, angtab, radtab, u, H, C, norm, wsum,
                     lam_norm, ubar, dRb, dAb);
  return hipGetLastError();
}

hipError_t boundary_vjp(const ShellDev* sh, int n_shells, int max_S, const double* bctab, const double* gamma,
                        const double* W, const double* mu, double* Lb, double* bcg, hipStream_t st) {
  dim3 grid((max_S + 255) / 256, n_shells), block(256);
  hipLaunchKernelGGL(k_boundary_vjp, grid, block, 0, st, sh, max_S, bctab, gamma, W, mu, Lb, bcg);
  return hipGetLastError();
}

hipError_t gamma_reduce(const int* blk_range, const int* shell_range, int n_inst, int max_S,
                        const double* gpart, const double* bcg, const double* dt, double coef, int use_dt,
                        double* g, hipStream_t st) {
  hipLaunchKernelGGL(k_gamma_reduce, dim3(n_inst), dim3(256), 0, st, blk_range, shell_range, max_S, gpart, bcg,
                     dt, coef, use_dt, g);
  return hipGetLastError();
}

hipError_t lincomb(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* dt, int use_dt, double ca,
                   const double* x, double cb, const double* y, double cc, const double* z, double* out,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_lincomb, dim3(n_blk, 50), dim3(256), 0, st, sh, blk, dt, use_dt, ca, x, cb, y, cc, z, out);
  return hipGetLastError();
}

hipError_t nonfinite_count(const double* x, long long n, int* count, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  long long nb = (n + 255) / 256;
  int grid = (int)(nb < 4096 ? nb : 4096);
  hipLaunchKernelGGL(k_nonfinite, dim3(grid), dim3(256), 0, st, x, n, count);
  return hipGetLastError();
}

hipError_t dp_combine(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* dt, const double* u,
                      double* const k[7], const double c[7], int nk, double* out, hipStream_t st) {
  DpTerms T;
  for (int j = 0; j < 7; ++j) {
    T.k[j] = k[j];
    T.c[j] = (j < nk) ? c[j] : 0.0;
  }
  hipLaunchKernelGGL(k_dp_combine, dim3(n_blk, 50), dim3(256), 0, st, sh, blk, dt, u, T, nk, out);
  return hipGetLastError();
}

hipError_t dp_error(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* dt, const double* u,
                    const double* u5, double* const k[7], const double e[7], double atol, double rtol,
                    double* partial, hipStream_t st) {
  DpTerms T;
  for (int j = 0; j < 7; ++j) {
    T.k[j] = k[j];
    T.c[j] = e[j];
  }
  hipLaunchKernelGGL(k_dp_error, dim3(n_blk), dim3(256), 0, st, sh, blk, dt, u, u5, T, atol, rtol, partial);
  return hipGetLastError();
}

hipError_t dp_control(const int* blk_range, int n_inst, const double* nval, const double* partial, double* dt,
                      double* t, int* rejected, int* accepted, int* n_accepted, double* err, hipStream_t st) {
  hipLaunchKernelGGL(k_dp_control, dim3(n_inst), dim3(256), 0, st, blk_range, nval, partial, dt, t, rejected,
                     accepted, n_accepted, err);
  return hipGetLastError();
}

hipError_t dp_accept(const ShellDev* sh, const PtBlock* blk, int n_blk, const int* accepted, const double* src,
                     double* dst, const double* src2, double* dst2, hipStream_t st) {
  hipLaunchKernelGGL(k_dp_accept, dim3(n_blk, 50), dim3(256), 0, st, sh, blk, accepted, src, dst, src2, dst2);
  return hipGetLastError();
}

hipError_t fill_int(int* x, int n, int value, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, st, x, n, value);
  return hipGetLastError();
}

int theta_item_orders(int n) { return n <= 32 ? 16 : 8; }

hipError_t ang_theta_mfma(int n, const ShellDev* sh, const ThetaItem* items, int n_items, const double* ktabT,
                          const double* AB, double* X, int mode, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  dim3 grid(n_items);
#define GH_ANGM(NN)                                                                                             \
  {                                                                                                             \
    constexpr int MB = NN <= 32 ? 16 : 8;                                                                       \
    const dim3 block(32 * MB);                                                                                  \
    if (mode == 0) hipLaunchKernelGGL((k_ang_theta_mfma<NN, 0, MB>), grid, block, 0, st, sh, items, ktabT, AB, X); \
    else hipLaunchKernelGGL((k_ang_theta_mfma<NN, 1, MB>), grid, block, 0, st, sh, items, ktabT, AB, X);         \
  }
  switch (n) {
    case 16: GH_ANGM(16) break;
    case 32: GH_ANGM(32) break;
    case 48: GH_ANGM(48) break;
    case 64: GH_ANGM(64) break;
    default: return hipErrorInvalidValue;
  }
#undef GH_ANGM
  return hipGetLastError();
}

hipError_t ang_theta(int nmax, const ShellDev* sh, const PtBlock* tblk, int n_tblk, const double* ktab,
                     const double* AB, double* X, int mode, hipStream_t st) {
  if (n_tblk <= 0) return hipSuccess;
  dim3 grid(n_tblk), block(256);
#define GH_ANG(NM)                                                                                        \
  if (mode == 0) hipLaunchKernelGGL((k_ang_theta<NM, 0>), grid, block, 0, st, sh, tblk, ktab, AB, X);   \
  else hipLaunchKernelGGL((k_ang_theta<NM, 1>), grid, block, 0, st, sh, tblk, ktab, AB, X);
  switch (nmax) {
    case 16: GH_ANG(16) break;
    case 32: GH_ANG(32) break;
    case 64: GH_ANG(64) break;
    default: return hipErrorInvalidValue;
  }
#undef GH_ANG
  return hipGetLastError();
}

}  // namespace ghk

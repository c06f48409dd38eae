// Device-side data structures shared by the kernels and the C interface.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "ghmi_gemm.h"

// One shell as the kernels see it.
struct ShellDev {
  long long pt_off;   // first collocation point of the shell
  int n_r, L, S, n_ph;
  int instance;
  int d_off;          // offset of this n_r's CGL d/dxi matrix in the radial table
  int ang_off;        // offset (in 5-double records) of this L's angular table
  int rad_off;        // offset of this shell's radial records (r_j, quadrature weight) x n_r
  int bc_off;         // interface at the outer face: offset of its records (9 doubles x S), else -1
  int outer;          // 1: outer face is the outer boundary of its instance
  int inner;          // 1: inner face is an excision boundary
  double dscale;      // d/dr = dscale * d/dxi, dscale = 2/(r_out - r_in)
  long long kt_off;   // offset of this L's per-order theta kernels in the transform table (-1: none)
  long long tf_off;   // tensor filter: first coefficient of the shell in the coefficient arrays
  long long lg_off;   // tensor filter: offset of this L's Legendre tables (analysis [ns][n], synthesis [n][ns])
  int nsp;            // tensor filter: coefficients per (field, radius) row, (L+1)^2 rounded up to even
  int pad_;
};

// A block of up to 256 consecutive points inside one shell.
struct PtBlock {
  int shell;
  int q0;             // first local point index (r*S + a)
};

// Work item of the matrix-core theta step: 8 rows from r0, orders m0 .. m0+7.
struct ThetaItem {
  int shell;
  int r0;
  int m0;
  int pad;
};

// Tensor-coupled filter, the coupling step on the coefficient array X (per
// shell [field][radius][nsp]): Y = F X for every column (shell, radius).
// The rows of F come in segments: rows (e, s) with e0 <= e < e0 + ne and
// s0 <= s < s0 + nsg (segment row i = (e - e0) * nsg + (s - s0)), whose
// couplings all stay in the segment.  A segment's rows, sorted by their number
// of couplings, are cut into slices of 64 (one per wave) stored sliced-ELL:
// slice q holds width[q] couplings per row, the k-th of every row contiguous
// (val/lidx[off[q] + 64 k + lane], zero-padded), perm[64 q + lane] is the
// segment row of the lane (-1: padding); lidx is the input's segment row.  A
// work item stages its segment's inputs for ncol columns in LDS (64 KB: up to
// 8 columns for segments of at most 1024 rows, 4 up to 2048, 2 up to 4096) and
// computes the slices [q0, q1) for them.
enum { TF_LDS_DOUBLES = 8192, TF_MAX_ROWS = 4096 };
inline int tf_cols_for_rows(int n) { return n <= 1024 ? 8 : (n <= 2048 ? 4 : 2); }
struct TfSeg {
  int e0, ne, s0, nsg;
  int slice0, pad;     // first slice of the segment in the slice tables
};
struct TfCol {
  long long base;     // X offset of (shell, radius, field 0, s = 0)
  long long fstride;  // distance between fields: n_r nsp
};
struct TfItem {
  int seg, col0, ncol, q0, q1, pad0, pad1, pad2;
};

// Kernel launchers (ghmi_kernels.hip).  All are asynchronous on `st`.
namespace ghk {

// Dormand-Prince pieces.  dp_combine: out = u + dt (sum_{j<nk} c_j k_j);
// dp_error: per point block, sum over values of (dt sum_j e_j k_j / (atol +
// rtol max(|u|, |u5|)))^2 into partial[block]; dp_control: per instance the
// RMS error, accept flag, t and dt update (Numerical Recipes' controller);
// dp_accept: dst = src (and dst2 = src2) on the values of accepted instances.
hipError_t dp_combine(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* dt, const double* u,
                      double* const k[7], const double c[7], int nk, double* out, hipStream_t st);
hipError_t dp_error(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* dt, const double* u,
                    const double* u5, double* const k[7], const double e[7], double atol, double rtol,
                    double* partial, hipStream_t st);
hipError_t dp_control(const int* blk_range, int n_inst, const double* nval, const double* partial, double* dt,
                      double* t, int* rejected, int* accepted, int* n_accepted, double* err, hipStream_t st);
hipError_t dp_accept(const ShellDev* sh, const PtBlock* blk, int n_blk, const int* accepted, const double* src,
                     double* dst, const double* src2, double* dst2, hipStream_t st);
hipError_t fill_int(int* x, int n, int value, hipStream_t st);

// Per-order theta kernels of the transform path of the angular operators.
// AB: Fourier coefficients of every row ([50] layout, per (field, radius)
// row the [n][2n] array of cos | sin coefficients).  mode 0: X ([100] layout)
// receives per row the d/dtheta coefficients and the d/dphi ones with the
// cos and sin halves exchanged and negated as the synthesis needs;
// mode 1: X ([50] layout) receives the filtered coefficients.  tblk: blocks
// (shell, q0 = first row * S + first (theta node, column) pair) of 16 rows x
// 256 pairs; nmax: 16, 32 or 64 >= L + 1 of every shell.
hipError_t ang_theta(int nmax, const ShellDev* sh, const PtBlock* tblk, int n_tblk, const double* ktab,
                     const double* AB, double* X, int mode, hipStream_t st);
// The same step on the matrix cores for the shells with n = L + 1 (16, 32,
// 48 or 64; one launch per n): items of 8 rows x theta_item_orders(n) orders
// (m0 a multiple of it); ktabT: the kernel table transposed per order
// ([3][n][i'][i], same offsets as ktab).
int theta_item_orders(int n);
hipError_t ang_theta_mfma(int n, const ShellDev* sh, const ThetaItem* items, int n_items, const double* ktabT,
                          const double* AB, double* X, int mode, hipStream_t st);

hipError_t fill_pattern(double* x, long long n, hipStream_t st);

// Tensor-coupled filter by transforms.  leg_analysis: Fourier coefficients
// F (per shell at 50 pt_off, [field, radius][theta node i][m'], m' < n: cos m,
// m' >= n: sin (m' - n)) -> real Y_lm coefficients X[tf_off + row nsp + s],
// s = l l + l + m, with the analysis table (weights, sqrt2 folded in);
// leg_synthesis: coefficients Y -> the same Fourier layout G for the synthesis
// GEMM.  Blocks: (shell, first (group of 10 rows, s) or (group, m', i) index),
// 256 threads.
hipError_t leg_analysis(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* legtab, const double* F,
                        double* X, hipStream_t st);
hipError_t leg_synthesis(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* legtab, const double* Y,
                         double* G, hipStream_t st);

// n_items[3]: the items come grouped by their column class (8, 4, 2 columns).
hipError_t tensor_couple(const TfItem* items, const int n_items[3], const TfSeg* segs, const TfCol* cols,
                         const long long* soff, const int* swidth, const int* perm, const int* lidx,
                         const double* val, const double* X, double* Y, hipStream_t st);

hipError_t radial(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* dtab,
                  const double* u, double* dR, int ncomp_lo, int ncomp_hi, bool transpose, bool accumulate,
                  hipStream_t st);

// Column form of the radial derivative (one thread per field x angular point);
// maxr = radial_col_maxr(largest n_r) selects the register-array size (0: unsupported).
int radial_col_maxr(int max_nr);
hipError_t radial_col(int maxr, const ShellDev* sh, const PtBlock* cblk, int n_cblk, const double* dtab,
                      const double* u, double* dR, int ncomp_lo, int ncomp_hi, bool transpose, bool accumulate,
                      hipStream_t st);

hipError_t pointwise_rhs(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* angtab,
                         const double* radtab, const double* u, const double* dR, const double* dA,
                         const double* H, const double* dH, const double* gamma, double* rhs,
                         hipStream_t st);

// d_t u of the stage state us and the SSP-RK3 stage out = c0 u0 + c1 (us + dt
// L) in one pass: out gets every point off the treated faces, L (raw d_t u)
// the points on them, for stage_faces.  out may alias u0.
hipError_t pointwise_stage(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* angtab,
                           const double* radtab, const double* us, const double* dR, const double* dA,
                           const double* H, const double* dH, const double* gamma, double* L, const double* dt,
                           double c0, const double* u0, double c1, double* out, hipStream_t st);

// The treated faces of that stage: boundary treatment of L there (read only)
// and the stage update.  out may alias u0.
hipError_t stage_faces(const ShellDev* sh, int n_shells, int max_S, const double* bctab, const double* gamma,
                       const double* dt, double c0, const double* u0, double c1, const double* us, const double* L,
                       double* out, int outer_mode, hipStream_t st);

// outer_mode 0: Dirichlet d_t u = 0 on outer faces; 1: outer faces left as
// they are (already treated in place by outer_cpbc).
hipError_t boundary(const ShellDev* sh, int n_shells, int max_S, const double* bctab,
                    const double* gamma, double* rhs, int outer_mode, hipStream_t st);

// Constraint-preserving treatment of the outer faces of rhs in place, from the
// state u and its radial (dR) and angular (dA) derivatives.
hipError_t outer_cpbc(const ShellDev* sh, int n_shells, int max_S, const double* angtab, const double* radtab,
                      const double* u, const double* dR, const double* dA, const double* gamma, double* rhs,
                      hipStream_t st);

hipError_t constraints(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* angtab,
                       const double* radtab, const double* u, const double* dR, const double* dA,
                       const double* H, double* C, double* partial, hipStream_t st);

hipError_t reduce_norm(const int* inst_blk_range, int n_inst, const double* partial,
                       const double* wsum, double* norm, hipStream_t st);

hipError_t bc_setup(const ShellDev* sh, int n_shells, int max_S, const double* angtab,
                    const double* u_bg, double* bctab, double* excision_min, hipStream_t st);

hipError_t nonfinite_count(const double* x, long long n, int* count, hipStream_t st);

// adjoint
// Reverse of the pointwise algebra in two passes; acc: work space of
// 12 x p_total doubles (p_total = all points of the domain).  The cotangent
// of the raw d_t u is lamf on the faces the boundary treatment changes (from
// boundary_vjp) and mu everywhere else.
hipError_t pointwise_vjp(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* angtab,
                         const double* radtab, const double* u, const double* dR, const double* dA,
                         const double* H, const double* dH, const double* gamma, const double* mu,
                         const double* lamf, double* ubar, double* dRb, double* dAb, double* gpart, double* acc,
                         long long p_total, hipStream_t st);
hipError_t constraints_vjp(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* angtab,
                           const double* radtab, const double* u, const double* H, const double* C,
                           const double* norm, const double* wsum, const double* lam_norm, double* ubar,
                           double* dRb, double* dAb, hipStream_t st);
// Transposed boundary treatment: from mu (cotangent of the treated d_t u,
// read only) the raw cotangent of every treated face into Lb (nothing else).
hipError_t boundary_vjp(const ShellDev* sh, int n_shells, int max_S, const double* bctab, const double* gamma,
                        const double* W, const double* mu, double* Lb, double* bcg, hipStream_t st);
hipError_t gamma_reduce(const int* blk_range, const int* shell_range, int n_inst, int max_S,
                        const double* gpart, const double* bcg, const double* dt, double coef, int use_dt,
                        double* g, hipStream_t st);
// C (rows x cols, leading dimension ldc) = (accumulate: +=) the chunk-ordered
// sum of the nchunk row-major partial blocks in W (split-K tail of a GEMM plan).
hipError_t sum_chunks(const double* W, int nchunk, int rows, int cols, double* C, int ldc, bool accumulate,
                      hipStream_t st);
hipError_t lincomb(const ShellDev* sh, const PtBlock* blk, int n_blk, const double* dt, int use_dt, double ca,
                   const double* x, double cb, const double* y, double cc, const double* z, double* out,
                   hipStream_t st);

}  // namespace ghk

/*
 * ghmi.h -- C interface of the MI355X generalized-harmonic shell evolution.
 *
 * Evolves the 50 first-order generalized-harmonic (GH) fields psi_ab, Pi_ab,
 * Phi_iab of an isolated black hole on stacks of spherical shells (topology
 * I1 x S2), as in Lewis & Pfeiffer, arXiv:1804.09101 ("Details of our port":
 * modules Deriv, Trans/DiffJac, GHEqns, ApplyBCs, Filter).  One right-hand-side
 * (RHS) evaluation is
 *   1. spectral derivatives of every field along r (Chebyshev) and theta, phi
 *      (Y_lm), applied as cached dense matrices traced from the transforms
 *      (section "Spectral Operations", eqs. Differentiation and
 *      DifferentiatorI1S2);
 *   2. the Jacobian to Cartesian derivatives (section "Jacobian
 *      multiplication", eq. DiffJac);
 *   3. the pointwise GH algebra ("GHEqns"; equations of the first-order GH
 *      system of Lindblom et al. 2006, which the paper does not print);
 *   4. boundary treatment ("Apply BCs"): characteristic upwinding at shell
 *      interfaces, Dirichlet d_t u = 0 at the outer boundary, nothing at the
 *      excision (inner) boundary.
 * A step is one SSP-RK3 step (three RHS evaluations) followed, if enabled, by
 * an angular filter ("Filter" module): the exponential filter of every
 * component, or the tensor-coupled filter of the section on spectral filtering
 * on I1 x S2 (PhysToSpec, a sparse matrix coupling the tensor components,
 * SpecToPhys).
 *
 * Conventions for every function:
 *  - Return value: GH_OK (0) or a negative GH_ERR_* code; gh_last_error()
 *    then holds a message.  No C++ exception crosses this interface.
 *  - Field buffers are DEVICE pointers owned by the caller: FP64, contiguous,
 *    in the layout below.  The library owns operators, tables and work space,
 *    allocated in gh_set_domain and freed by gh_destroy / the next
 *    gh_set_domain.
 *  - Setup calls (gh_set_domain, gh_set_background, gh_set_params) are
 *    synchronous: they return when the new values are in place, after the
 *    work already queued on the context has used the old ones.  Compute
 *    calls (gh_rhs, gh_step, gh_constraints, ...) are queued on the
 *    context's HIP stream and return before the work completes.
 *  - Calls on one context must not overlap (one host thread at a time).
 *
 * Layout: shells are concatenated in the order given to gh_set_domain
 * (grouped by instance, inner to outer).  Shell k holds n_r * S points,
 * S = N_theta * N_phi = (L+1) * 2(L+1), and a per-point quantity with C
 * components occupies C * n_r * S doubles starting at C * offset_k, ordered
 * [component][r][theta][phi] (phi fastest).  Radial points are
 * Chebyshev-Gauss-Lobatto, r_j = (r_in+r_out)/2 - cos(pi j/(n_r-1))(r_out-r_in)/2;
 * theta_i = arccos(x_i) with x_i the L+1 Gauss-Legendre nodes in increasing
 * order; phi_k = 2 pi k / N_phi.
 * Field components (50): psi_ab, Pi_ab, Phi_xab, Phi_yab, Phi_zab, each over
 * the symmetric pairs 00,01,02,03,11,12,13,22,23,33.
 */
#ifndef GHMI_H
#define GHMI_H

#ifdef __cplusplus
extern "C" {
#endif

#define GH_OK 0
#define GH_ERR_ARG (-1)          /* null pointer, bad count or value            */
#define GH_ERR_SHAPE (-2)        /* inconsistent shells (see gh_set_domain)      */
#define GH_ERR_ORDER (-3)        /* call made before the setup it needs          */
#define GH_ERR_OOM (-4)          /* device allocation failed                     */
#define GH_ERR_NOT_OUTFLOW (-5)  /* an excision boundary point has inflow        */
#define GH_ERR_NONFINITE (-6)    /* NaN/Inf found in an input or result          */
#define GH_ERR_DEVICE (-7)       /* HIP runtime error                            */

typedef struct gh_ctx gh_ctx;

/* One spherical shell.  n_r >= 3 radial points, 1 <= L <= 63. */
typedef struct {
  int instance;   /* index of the black hole (0 .. n_inst-1) it belongs to */
  int n_r;        /* radial (Chebyshev-Gauss-Lobatto) points               */
  int L;          /* highest Y_lm degree; N_theta = L+1, N_phi = 2(L+1)     */
  double r_in;    /* inner radius (> 0)                                     */
  double r_out;   /* outer radius (> r_in)                                  */
} gh_shell;

/* Create a context on HIP device `device` that queues work on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  *out receives the handle. */
int gh_create(gh_ctx** out, int device, void* hip_stream);
int gh_destroy(gh_ctx* ctx);
/* Change the HIP stream used by later compute calls. */
int gh_set_stream(gh_ctx* ctx, void* hip_stream);

/* Describe the domain: n_shells shells of n_inst independent instances.
 * Shells must be grouped by instance (instances in increasing order) and
 * ordered inner to outer; consecutive shells of one instance must share L and
 * satisfy r_out(k) == r_in(k+1) exactly (GH_ERR_SHAPE otherwise).
 * filter_kind 0: no filter; 1: angular exponential filter of every component
 * after every step, sigma_l = 1 for l/L <= eta_c else
 * exp(-alpha ((l/L - eta_c)/(1 - eta_c))^order), filter_params = {eta_c,
 * alpha, order}; 2, 3: the tensor-coupled filter (see gh_tensor_filter_matrix)
 * after every step with the ExpCheb factors of kind 1 in j instead of l
 * (kind 2, filter_params = {eta_c, alpha, order}) or the Heaviside factors
 * sigma(j) = 1 for j <= eta_c L, else 0 (kind 3, filter_params = {eta_c}).
 * filter_params is a host pointer, ignored for kind 0.
 * Builds and uploads the derivative and filter operators (cached per L and
 * per n_r) and allocates all work space.  Invalidates background and params. */
int gh_set_domain(gh_ctx* ctx, int n_inst, int n_shells, const gh_shell* shells,
                  int filter_kind, const double* filter_params);

/* Total number of collocation points, and (if shell_offsets != NULL) the
 * first point of every shell, n_shells+1 entries (host pointers). */
int gh_num_points(const gh_ctx* ctx, long long* total_points, long long* shell_offsets);

/* Background data, DEVICE pointers in the shell layout (copied; the caller
 * may free them afterwards).  The paper's test problem is an isolated
 * Kerr-Schild black hole (port overview, eq. dimensionlessspin); the gauge
 * source of the GH system is an input here, frozen in time (for a stationary
 * hole H_a = -psi^bc Gamma_abc of the exact metric, which makes the hole an
 * exact solution).  Of the paper's three ApplyBCs cases (Conclusions) this
 * call prepares the internal-boundary exchange (through u_bg) and checks the
 * excision case, which needs no condition when all characteristics leave the
 * domain:
 *   H    [4 components]  gauge source H_a;
 *   dH   [16 components] d_a H_b at component a*4+b (a = 0: time derivative);
 *   u_bg [50 components] background state.  At shell interfaces it fixes the
 *        unit normal and the characteristic speeds used for upwinding.  At
 *        excision boundaries every speed of u^0, u^+ and u^- along the inward
 *        normal must be >= 0 (pure outflow), else GH_ERR_NOT_OUTFLOW.
 * Non-finite values give GH_ERR_NONFINITE. */
int gh_set_background(gh_ctx* ctx, const double* H, const double* dH, const double* u_bg);

/* Constraint-damping parameters gamma [n_inst][3] = (gamma0, gamma1, gamma2)
 * of the first-order GH system (Lindblom et al. 2006, eqs. 35-37; the paper
 * names the system in its port overview but prints neither the equations nor
 * the parameter values) and time steps dt [n_inst] of the method-of-lines
 * evolution (section "The Spectral Einstein Code") (HOST pointers; dt may be
 * NULL if only gh_rhs and gh_constraints are used).  Waits for the work
 * already queued on the context's stream (and for graph replays) before the
 * new values replace the old ones, since that work reads them from device
 * memory. */
int gh_set_params(gh_ctx* ctx, const double* gamma, const double* dt);

/* dudt = d_t u including boundary treatment.  u, dudt: device [50] layout;
 * they must not overlap. */
int gh_rhs(gh_ctx* ctx, const double* u, double* dudt);

/* n_steps SSP-RK3 steps in place on u (device [50] layout):
 *   u1 = u + dt L(u); u2 = 3/4 u + 1/4 (u1 + dt L(u1));
 *   u <- 1/3 u + 2/3 (u2 + dt L(u2)), then the filter if enabled. */
int gh_step(gh_ctx* ctx, double* u, int n_steps);

/* Adaptive Dormand-Prince 5(4) stepping (the paper evolves with a
 * Dormand-Prince stepper, section "The Spectral Einstein Code"): n_attempts
 * step attempts in place on u (device [50] layout).  Every instance takes its
 * own step dt[i] (device [n_inst], in/out) from t[i] (device [n_inst],
 * in/out).  An attempt forms the seven stages of the Dormand & Prince (1980)
 * RK5(4) pair (each stage a full RHS with boundary treatment) and per
 * instance the RMS over its values of err / (atol + rtol max(|u_old|, |u_new|)),
 * err the difference of the fifth- and fourth-order solutions.  At most 1:
 * the instance takes the fifth-order solution (then the filter, if enabled)
 * and t[i] += dt[i]; otherwise its values are kept.  Either way dt[i] is
 * multiplied by min(10, max(0.2, 0.9 err^-1/5)) (10 for err = 0), capped at 1
 * right after a rejection (Numerical Recipes' controller).  rejected (device
 * int [n_inst], in/out, may be NULL) holds whether each instance's last
 * attempt was rejected, so that consecutive calls continue one integration
 * (NULL: all zero at the start of the call).  n_accepted (device int
 * [n_inst], may be NULL) is incremented per accepted step; err (device
 * [n_inst], may be NULL) receives the last attempt's error norms.
 * Needs gh_set_params (gamma; its dt is not used).  The first call allocates
 * about 10 further [50] arrays.  GH_ERR_ARG for n_attempts < 0, negative or
 * non-finite tolerances, or atol + rtol == 0. */
int gh_step_dp5(gh_ctx* ctx, double* u, int n_attempts, double atol, double rtol, double* t, double* dt,
                int* rejected, int* n_accepted, double* err);

/* How the angular derivatives and the angular filter are applied.
 * method 0 (default): the dense S x S operators as one grouped FP64-MFMA GEMM
 * (eq. DifferentiatorI1S2).  method 1: the same operators factorised by
 * azimuthal order (the paper's transform route: PhysToSpec, coefficient
 * operation, SpecToPhys): a Fourier analysis along phi (GEMM with a
 * [2n x 2n] table, n = L+1), per order m the n x n theta kernels of
 * d/dtheta, d/dphi or the filter, and a Fourier synthesis (GEMM), about
 * 4 (L+1)^3 instead of 4 (L+1)^4 multiply-adds per field and radius.  Both
 * give the same values up to rounding.  method 2: for the derivative pass and
 * for the filter separately, whichever of the two forms is faster on this
 * domain (both timed on the GPU during the call).  The reverse pass (the *_vjp
 * calls) uses the dense transposed operators in every method.  The first call
 * with method 1 or 2 builds the transform tables and tunes their GEMMs
 * (synchronous); a step graph is recaptured after a change. */
int gh_set_angular(gh_ctx* ctx, int method);

/* Graph mode for gh_step (default off).  When on, the first gh_step on a
 * state pointer captures one whole SSP-RK3 step (every kernel of the three
 * stages and the filter, for all shells of all instances) into a HIP graph on
 * a stream owned by the context, and every gh_step replays it n_steps times,
 * ordered after earlier work on the context's stream and before later work
 * by events.  A new state pointer or domain recaptures; gh_set_params values
 * are read from device memory at run time, so they need no recapture.
 * Bypassed while kernel timing is on. */
int gh_set_graph(gh_ctx* ctx, int enable);

/* Constraints of u.  The paper evolves the GH system without printing its
 * constraints; these are the constraints of the first-order system
 * (Lindblom et al. 2006: the gauge constraint, their eq. 40, and the three-
 * and four-index constraints of the first-order reduction), and the norm is
 * this library's monitor, a volume average with the grid's own quadrature.
 * C (device [64] layout, may be NULL) receives per point
 * C_a (4), C_iab = d_i psi_ab - Phi_iab (30, i = x,y,z) and
 * C_ijab = d_i Phi_jab - d_j Phi_iab (30, ij = xy, xz, yz).
 * norm (device [n_inst], may be NULL) receives per instance
 * sqrt(sum_p w_p sum_c C_c^2 / sum_p w_p) with w_p the volume quadrature
 * weight (Clenshaw-Curtis x r^2 (r_out-r_in)/2 x Gauss-Legendre x 2pi/N_phi). */
int gh_constraints(gh_ctx* ctx, const double* u, double* C, double* norm);

/* gh_constraints for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * kernels and the same results (bitwise), with the per-block partial sums of
 * the norm kept in a file-scope device array of GH_STATIC_SCRATCH_DOUBLES
 * doubles (8 MiB) instead of the context's work space.  The call itself
 * allocates nothing: no hipMalloc, hipFree or event (kernel timing is not
 * recorded for it); the derivative work space is the context's, allocated by
 * gh_set_domain.  Limit: at most GH_STATIC_SCRATCH_DOUBLES blocks of 256
 * points (domains up to 268 435 456 points), else GH_ERR_ARG.  The array is
 * shared by every context on the same GPU and keeps the last call's partial
 * sums: calls that overlap on one GPU (two streams, two host threads) race,
 * so callers must order them. */
#define GH_STATIC_SCRATCH_DOUBLES (1 << 20)
int gh_constraints_static(gh_ctx* ctx, const double* u, double* C, double* norm);

/* ---- adjoint (reverse mode) ---------------------------------------------
 * The paper has no adjoint; these are the transposes of the linearised
 * operations above, for gradients of a loss of the final state with respect
 * to the initial state and the damping parameters.  The background (H, dH,
 * frozen boundary projections) and dt are constants.  Every domain that
 * gh_set_domain accepts (n_r up to 256, L up to 63) has a reverse pass.  The
 * first call of
 * either function allocates ~9 further [50] work arrays and tunes the
 * transposed GEMMs (synchronous); later calls are queued on the stream. */

/* lam_u = (d rhs(u)/d u)^T lam, i.e. the transpose of the linearised gh_rhs
 * (boundary treatment included) at state u.  g_gamma (device [n_inst][3], may
 * be NULL) is INCREMENTED by (d rhs/d gamma)^T lam.  lam_u must not alias u or lam. */
int gh_rhs_vjp(gh_ctx* ctx, const double* u, const double* lam, double* lam_u, double* g_gamma);

/* Transpose of one gh_step (SSP-RK3 + filter) linearised at u_n:
 * lam_n = (d u_{n+1}/d u_n)^T lam_np1, and g_gamma (device, may be NULL) is
 * INCREMENTED by (d u_{n+1}/d gamma)^T lam_np1.  The stages are recomputed
 * from u_n.  lam_n may alias lam_np1 but not u_n. */
int gh_step_vjp(gh_ctx* ctx, const double* u_n, const double* lam_np1, double* lam_n, double* g_gamma);

/* One gh_step (same arithmetic) that also stores the two SSP-RK3 stage states
 * u1 = u + dt L(u) and u2 = 3/4 u + 1/4 (u1 + dt L(u1)) into u1, u2 (device
 * [50], distinct from u), for a later gh_step_vjp_stages.  derivs (device,
 * may be NULL) receives the spatial derivatives the three RHS evaluations
 * computed, of u, u1 and u2 in that order, each as the radial derivative
 * d/dxi ([50] layout) followed by the angular ones (per shell a row-major
 * [50 n_r][2S] block starting at 100 * offset_k: d_theta of the row's S
 * points, then d_phi): 3 x 150 P doubles, owned by the caller. */
int gh_step_stages(gh_ctx* ctx, double* u, double* u1, double* u2, double* derivs);

/* gh_step_vjp with the stage states supplied (from gh_step_stages on u_n), so
 * they are not recomputed; with derivs (from the same gh_step_stages call,
 * may be NULL) the derivatives of the three states are not recomputed either.
 * Same outputs and aliasing rules as gh_step_vjp (lam_n must also not alias
 * u1, u2 or derivs).  The results do not depend on whether derivs is given. */
int gh_step_vjp_stages(gh_ctx* ctx, const double* u_n, const double* u1, const double* u2, const double* derivs,
                       const double* lam_np1, double* lam_n, double* g_gamma);

/* Transpose of the constraint norm: lam_u = sum_i lam_norm[i] d||C||_i / d u
 * at state u (lam_norm: device [n_inst]; lam_u: device [50], overwritten,
 * not aliasing u).  A zero norm contributes nothing. */
int gh_constraints_vjp(gh_ctx* ctx, const double* u, const double* lam_norm, double* lam_u);

/* Kernel timing.  enable 1: every launch of the kernels named below is
 * bracketed by HIP events on the context's stream (about 4 us per launch on
 * the 8-shell workload's RK3 step); 2: only the angular derivative GEMM
 * (kind 0), the least overhead for timing the dominant kernel inside a timed
 * run; 0: off.  GH_ERR_ARG for other values.
 * gh_kernel_stats waits for the recorded work, returns the number of launches
 * and their summed duration in milliseconds since timing was enabled or last
 * queried, and clears that kind's record.
 * kind 0: angular derivative GEMM; 1: filter GEMM; 2: radial derivative;
 *      3: pointwise GH RHS (in gh_step together with the RK3 stage update of
 *      every point off the faces the boundary treatment changes); 4: boundary
 *      treatment (in gh_step: those faces, with their stage update); 5: RK3
 *      stage combinations of the reverse pass;
 *      6: pointwise reverse pass; 7: transposed angular derivative GEMM;
 *      8: angular derivatives by transforms (gh_set_angular 1: the three
 *      launches of one derivative pass counted as one); 9: the coupling
 *      kernel of the tensor-coupled filter (also inside kind 1). */
#define GH_NUM_KERNEL_KINDS 10
int gh_set_timing(gh_ctx* ctx, int enable);
int gh_kernel_stats(gh_ctx* ctx, int kind, long long* launches, double* total_ms);

/* Facts about the configured context: what 0: tile shape of the angular
 * derivative GEMM chosen by the autotuner, as BM*1000 + BN; 1: the same for the
 * filter GEMM (0 without filter); 2: number of tiles of one derivative GEMM
 * launch; 3: total collocation points; 4: tile order of the derivative GEMM
 * (0: each XCD takes whole column blocks, 1: whole row blocks, 2: blocks of
 * 8 x 8 tiles); 5: the same
 * for the filter GEMM; 6: kernel variant of the derivative GEMM (index into
 * the library's list of tile shape, wave layout and LDS layout); 7: the same
 * for the filter GEMM (-1 without filter); 8: the angular method (gh_set_angular);
 * 9, 10: whether the derivative pass / the filter use the transform form. */
int gh_query(const gh_ctx* ctx, int what, long long* value);
/* (continued) 11: number of stored couplings of the tensor-coupled filter
 * (kinds 2, 3; summed over the distinct L of the domain, else 0); 12: work
 * items of one launch of its coupling kernel; 13: the interface mode
 * (gh_set_interface); 14: kernel variant of the tail launch of the
 * derivative GEMM, -1 when it is one launch; 15: the same for the filter GEMM;
 * 16: number of K chunks of the derivative GEMM's tail (0 without); 17: the
 * outer boundary mode (gh_set_outer_bc).
 *
 * Split plans.  Workgroups of a GEMM launch finish in rounds of one tile per
 * compute unit, so a tile count just above a multiple of the CU count costs a
 * whole extra round.  After timing every variant and order the autotuner also
 * times the fastest one on the leading rows that fill whole rounds (whole row
 * tiles peeled from the end of the last group), followed by the peeled rows
 * in smaller tiles over 2, 4 or 8 chunks of K (partial products in a work
 * space the plan owns) and a kernel that adds the chunks into C in chunk
 * order, and keeps the split when it is faster.  The split changes the order
 * of the K sums of the peeled rows (results differ from one launch by
 * rounding; every run gives the same values).  Query 2 then counts the main
 * launch's tiles. */

/* Pin the kernel variant and tile order of a GEMM plan instead of the
 * autotuner's choice (for reproducible timing, and to check every variant):
 * plan 0: the angular derivative GEMM, 1: the filter GEMM (filter_kind 1);
 * shape: variant index 0 .. 17 (tile, wave layout, LDS layout, k-slice depth;
 * gh_query 6/7 report the current one); order 0: column blocks per XCD, 1:
 * row blocks, 2: blocks of 8 x 8 tiles.  A pinned plan is one launch (no
 * tail).  GH_ERR_ARG otherwise.
 * Drops a captured step graph. */
int gh_set_gemm_variant(gh_ctx* ctx, int plan, int shape, int order);

/* Pin any GEMM plan of the context, including a split plan (for reproducible
 * timing and to check every plan form).  plan 0: angular derivative, 1:
 * filter, 2: transposed derivative (adjoint), 3: transposed filter, 4:
 * Fourier analysis, 5: Fourier synthesis of the derivatives, 6: Fourier
 * synthesis of the filter (4-6 exist after gh_set_angular 1 or 2), 7, 8:
 * PhysToSpec and SpecToPhys of the tensor-coupled filter, 9, 10: their
 * transposes (2, 3, 9, 10 set up the reverse pass on first use).  shape and
 * order as in gh_set_gemm_variant.  tail_shape -1: one launch.  Otherwise a
 * split plan: the leading rows that fill whole rounds of `round` tiles (0:
 * one round = the number of compute units) in one launch of `shape`, the
 * remaining rows (one group) in tiles of `tail_shape` over tail_chunks (1 .. 8)
 * chunks of K with partial products in the plan's work space, then their sum
 * in chunk order.  GH_ERR_ARG if the plan does not exist for this domain,
 * its tiles do not split that way, or the tail's K is under 16 per chunk.
 * Drops a captured step graph. */
int gh_set_gemm_plan(gh_ctx* ctx, int plan, int shape, int order, int tail_shape, int tail_chunks, int round);

/* Where the characteristic projection at shell interfaces comes from.
 * mode 0 (default): the unit normal's metric normalisation and the upwind
 * choice (signs of the characteristic speeds) are taken from u_bg at
 * gh_set_background and frozen, so the boundary treatment is a fixed linear
 * map.  mode 1: they are recomputed from the state whose d_t u is being
 * treated (the paper's internal boundaries compute the characteristic
 * variables from the evolved fields; section on benchmarks of the overall
 * code, the ApplyBCs cases), before every boundary treatment of gh_rhs,
 * gh_step, gh_step_stages and gh_step_dp5.  The reverse-pass entry points
 * (gh_rhs_vjp, gh_step_vjp, gh_step_vjp_stages) need mode 0 and return
 * GH_ERR_ARG in mode 1.  Drops a captured step graph when the mode changes. */
int gh_set_interface(gh_ctx* ctx, int mode);

/* Boundary condition at the outer boundary of every instance.
 * mode 0 (default): Dirichlet, d_t u = 0 for all 50 fields.  mode 1: the
 * paper's constraint-preserving outer condition (Conclusions, ApplyBCs case
 * (ii)), read for the constraints of the first-order GH system: with the unit
 * normal s (+r_hat normalised with the state's metric at the face) and the
 * characteristic fields of the state,
 *   incoming u^psi: minus (1+gamma1)(s.N) s^k C_kab (three-index constraint
 *     C_kab = d_k psi_ab - Phi_kab, the part that needs d_s psi);
 *   incoming u^0:  minus (s.N) (delta_i^l - s_i s^l) s^k C_klab (four-index
 *     constraint C_klab = d_k Phi_lab - d_l Phi_kab, the part that needs
 *     d_s Phi);
 *   incoming u^- (and u^+ if incoming): frozen, d_t = 0;
 *   outgoing fields untouched.
 * So the incoming fields no longer depend on normal derivatives (which carry
 * constraint violations into the domain), and on data that satisfy the
 * constraints nothing changes but the incoming u^-.  Applied in gh_rhs,
 * gh_step, gh_step_stages, gh_step_dp5 and captured graphs.  The reverse-pass
 * entry points need mode 0 and return GH_ERR_ARG in mode 1.  Drops a captured
 * step graph when the mode changes.  gh_query 17 reports the mode. */
int gh_set_outer_bc(gh_ctx* ctx, int mode);

/* Apply the domain's angular filter (filter_kind 1-3) once: out = F u.
 * Device pointers, [50 P] each, distinct (GH_ERR_ARG if out == u, or if the
 * domain has no filter).  Asynchronous; uses the RHS work space. */
int gh_filter(gh_ctx* ctx, const double* u, double* out);

/* The coupling matrix of the tensor-coupled angular filter on one sphere of
 * degree L (section on spectral filtering on I1 x S2: the (N_e N_s) x
 * (N_e N_s) matrix between PhysToSpec and SpecToPhys, N_e = 50 stored fields,
 * N_s = (L+1)^2), in CSR form.  Rows and columns are e (L+1)^2 + s with e the
 * stored field and s = l*l + l + m the real orthonormal Y_lm (m > 0:
 * sqrt2 P_l^m cos(m phi), m < 0: sqrt2 P_l^|m| sin(|m| phi), m = 0: P_l, no
 * Condon-Shortley phase).  The paper does not say what the coupling is; here
 * it is the filter in total angular momentum: psi_ab, Pi_ab and Phi_iab rotate
 * as tensors (positions and spatial indices together), J^2 = -sum_k G_k^2 with
 * G_k = -(r x grad)_k + (e_k x) on every spatial index, and
 * F = sum_j sigma(j) P_j, P_j the projector onto J^2 = j(j+1); F keeps the
 * degree l and mixes components and orders within it.  kind 2 (ExpCheb) and 3
 * (Heaviside) as in gh_set_domain; transpose != 0 gives F^T.
 * Host memory, no GPU needed.  Call with row_ptr = col = val = NULL to get
 * *nnz; then with row_ptr[50 (L+1)^2 + 1], col[*nnz], val[*nnz] (*nnz at
 * least the count).  GH_ERR_ARG for L outside 1..63 or invalid params. */
int gh_tensor_filter_matrix(int L, int kind, const double* params, int transpose, long long* nnz,
                            long long* row_ptr, int* col, double* val);

/* Message of the last error on this context (never NULL). */
const char* gh_last_error(const gh_ctx* ctx);

/* ---- host-only helpers (no device needed) ------------------------------- */

/* Cartesian coordinates of every collocation point, HOST xyz[3][P]. */
int gh_grid_coords(int n_shells, const gh_shell* shells, double* xyz);

/* The dense operators exactly as uploaded to the device (HOST out, row-major,
 * acting on column vectors of collocation values):
 *  kind 0: Chebyshev-Gauss-Lobatto d/dxi, n x n (n = n_r);
 *  kind 1: d/dtheta on the sphere, S x S (n = L);
 *  kind 2: d/dphi on the sphere, S x S (n = L);
 *  kind 3: angular filter, S x S (n = L, params = {eta_c, alpha, order});
 *  kind 4: Clenshaw-Curtis weights on [-1,1], n (n = n_r);
 *  kind 5: Gauss-Legendre nodes then weights, 2(L+1) (n = L);
 *  kind 6: the derivative GEMM's B operand (Theta^T | Phi^T), S x 2S (n = L);
 *  kind 7: the filter GEMM's B operand F^T, S x S (n = L, params as kind 3).
 * GH_ERR_ARG for an unknown kind, n out of range (L above 63) or missing
 * params. */
int gh_host_operator(int kind, int n, const double* params, double* out);

#ifdef __cplusplus
}
#endif

#endif /* GHMI_H */

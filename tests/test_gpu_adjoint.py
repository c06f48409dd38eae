"""Adjoint of the GPU path: dot-product tests against the oracle's
complex-step directional derivatives, and central finite differences of a
multi-step constraint-norm loss.

<lam, J v> (oracle, complex step, exact to rounding) must equal
<J^T lam, v> (GPU reverse mode) for random lam, v and damping directions."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import domain  # noqa: E402
from paper_1804_09101_amd import autograd as gha  # noqa: E402
from paper_1804_09101_amd import configs, ghmi, inputs  # noqa: E402

pytestmark = pytest.mark.gpu
H_CS = 1e-30


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def _setup(shells, holes, gamma, dt, filt, pert=1e-3, seed=1):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = configs.Workload("adjoint", shells, holes, gamma, dt, filt, 1, None)
    d = domain.Domain([domain.Shell(*s) for s in shells], filter_params=filt)
    xyz = d.xyz()
    u0, ubg, H, dH = wl.initial_data(xyz, d.offsets)
    u0 = u0 + d.to_layout(inputs.smooth_random_field(xyz, pert, seed, 3, 2.0))
    s = ghmi.GHSolver(shells, wl.n_inst, filt)
    s.set_background(dev(H), dev(dH), dev(ubg))
    s.set_params(wl.gamma, wl.dt)
    return wl, d, s, u0, ubg, H, dH


SHELLS = [(0, 7, 5, 1.8, 2.8), (0, 7, 5, 2.8, 4.5), (1, 6, 3, 1.3, 2.4), (1, 5, 3, 2.4, 3.1)]
HOLES = [(1.0, 0.0, (0, 0, 1)), (0.8, 0.6, (0.3, -0.5, 0.8))]
GAM = [(0.7, -0.6, 1.3), (1.0, 0.3, 0.6)]


def test_rhs_vjp_dot_product():
    wl, d, s, u0, ubg, H, dH = _setup(SHELLS, HOLES, GAM, [0.004, 0.003], None)
    rng = np.random.default_rng(0)
    lam = rng.standard_normal(u0.shape)
    v = rng.standard_normal(u0.shape)
    vg = rng.standard_normal((2, 3))
    jv = d.rhs(u0 + 1j * H_CS * v, H, dH, ubg, wl.gamma + 1j * H_CS * vg).imag / H_CS
    lhs = np.sum(lam * jv)
    g = torch.zeros(6, dtype=torch.float64, device="cuda:0")
    lu = s.rhs_vjp(dev(u0), dev(lam), g_gamma=g).cpu().numpy()
    rhs = np.sum(lu * v) + np.sum(g.cpu().numpy().reshape(2, 3) * vg)
    err = abs(lhs - rhs) / np.sum(np.abs(lam * jv))
    print(f"  rhs vjp: <lam,Jv> {lhs:.12e} vs {rhs:.12e}, rel {err:.2e}", flush=True)
    assert err < 1e-12
    # the gamma part alone
    jg = d.rhs(u0.astype(complex), H, dH, ubg, wl.gamma + 1j * H_CS * vg).imag / H_CS
    lg, rg = np.sum(lam * jg), np.sum(g.cpu().numpy().reshape(2, 3) * vg)
    assert abs(lg - rg) < 1e-11 * np.sum(np.abs(lam * jg))


def test_vjp_dot_products_beyond_column_radial_form():
    """n_r = 70 is above what the register-column radial kernel holds (64), so
    the reverse pass takes the point form of the transposed radial derivative;
    the RHS and constraint-norm transposes must still pass the dot test."""
    shells = [(0, 70, 3, 1.8, 4.0), (0, 9, 3, 4.0, 5.0)]
    wl, d, s, u0, ubg, H, dH = _setup(shells, [(1.0, 0.2, (0, 1, 1))], [(0.8, -0.4, 1.2)], [0.001], None,
                                      pert=1e-2)
    rng = np.random.default_rng(5)
    lam = rng.standard_normal(u0.shape)
    v = rng.standard_normal(u0.shape)
    vg = rng.standard_normal((1, 3))
    jv = d.rhs(u0 + 1j * H_CS * v, H, dH, ubg, wl.gamma + 1j * H_CS * vg).imag / H_CS
    lhs = np.sum(lam * jv)
    g = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    lu = s.rhs_vjp(dev(u0), dev(lam), g_gamma=g).cpu().numpy()
    rhs = np.sum(lu * v) + np.sum(g.cpu().numpy() * vg.ravel())
    err = abs(lhs - rhs) / np.sum(np.abs(lam * jv))
    print(f"  rhs vjp at n_r = 70: rel {err:.2e}", flush=True)
    assert err < 1e-12
    # The norm's gradient is C-weighted, so unlike the RHS transpose it
    # inherits the forward rounding of C: at n_r = 70 the radial derivative
    # matrix has entries of ~n_r^2 / (r_out - r_in), and the two sides' C differ
    # by ~1e-10 of C.  The bar is that forward difference (times 10), measured
    # here, not 1e-12.
    lam_n = np.array([0.9])
    jn = d.constraint_norm(u0 + 1j * H_CS * v, H).imag / H_CS
    ln = s.constraints_vjp(dev(u0), dev(lam_n)).cpu().numpy()
    err = abs(np.sum(lam_n * jn) - np.sum(ln * v)) / np.sum(np.abs(lam_n * jn))
    C_gpu = s.constraints(dev(u0))[0].cpu().numpy()
    C_or = d.constraints(u0, H)
    e_C = np.max(np.abs(C_gpu - C_or)) / np.max(np.abs(C_or))
    print(f"  constraints vjp at n_r = 70: rel {err:.2e} (forward C differs by {e_C:.2e})", flush=True)
    assert err < max(1e-12, 10.0 * e_C)


def test_step_vjp_dot_product_with_filter():
    rs = configs.geometric_radii(1.8, 9.0, 2)
    shells = [(0, 9, 7, rs[0], rs[1]), (0, 9, 7, rs[1], rs[2])]
    wl, d, s, u0, ubg, H, dH = _setup(shells, [(1.0, 0.4, (0.1, 0.2, 1.0))], [(0.9, -0.2, 1.1)], [0.005],
                                      configs.FILTER_DEFAULT)
    rng = np.random.default_rng(1)
    lam = rng.standard_normal(u0.shape)
    v = rng.standard_normal(u0.shape)
    vg = rng.standard_normal((1, 3))
    jv = d.rk3_step(u0 + 1j * H_CS * v, H, dH, ubg, wl.gamma + 1j * H_CS * vg, wl.dt).imag / H_CS
    lhs = np.sum(lam * jv)
    g = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    ln = s.step_vjp(dev(u0), dev(lam), g_gamma=g).cpu().numpy()
    rhs = np.sum(ln * v) + np.sum(g.cpu().numpy() * vg.ravel())
    err = abs(lhs - rhs) / np.sum(np.abs(lam * jv))
    print(f"  step vjp: rel {err:.2e}", flush=True)
    assert err < 1e-12


def test_constraints_vjp_dot_product():
    wl, d, s, u0, ubg, H, dH = _setup(SHELLS, HOLES, GAM, [0.004, 0.003], None, pert=1e-2)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(u0.shape)
    lam_n = np.array([0.7, -1.3])
    jv = d.constraint_norm(u0 + 1j * H_CS * v, H).imag / H_CS
    lhs = np.sum(lam_n * jv)
    lu = s.constraints_vjp(dev(u0), dev(lam_n)).cpu().numpy()
    rhs = np.sum(lu * v)
    err = abs(lhs - rhs) / np.sum(np.abs(lam_n * jv))
    print(f"  constraints vjp: rel {err:.2e}", flush=True)
    assert err < 1e-12


def test_evolve_gradient_matches_central_differences_and_oracle():
    """Loss = ||C(u_n)|| after 12 RK3 steps (checkpoint every 5).  The gradient
    with respect to (gamma0, gamma1, gamma2) and the log-amplitude of the initial
    Pi perturbation is compared with (a) central differences, h = 1e-6, run
    through the same GPU forward path, to 1e-6 of the gradient norm, and (b) the
    oracle's complex-step derivatives through 12 oracle steps, to 1e-9."""
    wl, d, s, u0, ubg, H, dH = _setup([(0, 9, 5, 1.8, 4.0)], [(1.0, 0.0, (0, 0, 1))], [(1.0, -1.0, 1.0)], [0.01],
                                      None, pert=0.0)
    dpi = d.to_layout(inputs.gaussian_pulse_Pi(d.xyz(), 1.0, 2.8, 0.4, 3))
    amp = 1e-3
    n = 12

    def loss(gamma_np, a):
        s.set_params(gamma_np, wl.dt)
        u = dev(u0 + a * dpi)
        s.step(u, n)
        return float(s.constraints(u, want_C=False)[1].cpu().numpy()[0])

    gamma = torch.tensor(wl.gamma, dtype=torch.float64, requires_grad=True)
    a = torch.tensor(amp, dtype=torch.float64, device="cuda:0", requires_grad=True)
    u_init = dev(u0) + a * dev(dpi)
    un = gha.evolve(u_init, gamma, s, wl.dt, n, checkpoint_every=5, save_derivatives=True)
    L = gha.constraint_norm(un, s).sum()
    L.backward()
    g_adj = np.concatenate([gamma.grad.numpy().ravel(), [float(a.grad.cpu()) * amp]])
    h = 1e-6
    g_fd = []
    for c in range(3):
        gp = wl.gamma.copy()
        gm = wl.gamma.copy()
        gp[0, c] += h
        gm[0, c] -= h
        g_fd.append((loss(gp, amp) - loss(gm, amp)) / (2 * h))
    g_fd.append((loss(wl.gamma, amp * (1 + h)) - loss(wl.gamma, amp * (1 - h))) / (2 * h))
    g_fd = np.array(g_fd)
    # oracle reference: complex step through the oracle's own RK3 evolution
    g_or = []
    hc = 1e-30
    for c in range(4):
        gam = wl.gamma.astype(complex)
        uc = (u0 + amp * dpi).astype(complex)
        if c < 3:
            gam[0, c] += 1j * hc
        else:
            uc = uc + 1j * hc * amp * dpi
        for _ in range(n):
            uc = d.rk3_step(uc, H, dH, ubg, gam, wl.dt)
        g_or.append(d.constraint_norm(uc, H)[0].imag / hc)
    g_or = np.array(g_or)
    gn = np.linalg.norm(g_or)
    print(f"  adjoint {g_adj}\n  FD      {g_fd}\n  oracle  {g_or}", flush=True)
    print(f"  max |adj-FD|/|g| {np.max(np.abs(g_adj - g_fd)) / gn:.2e}, "
          f"max |adj-oracle|/|g| {np.max(np.abs(g_adj - g_or)) / gn:.2e}", flush=True)
    assert np.max(np.abs(g_adj - g_fd)) <= 1e-6 * gn
    assert np.max(np.abs(g_adj - g_or)) <= 1e-9 * gn


def test_stage_saving_step_and_vjp_match_plain_ones():
    """gh_step_stages == gh_step and gh_step_vjp_stages == gh_step_vjp, bitwise,
    with and without the saved stage derivatives."""
    rs = configs.geometric_radii(1.8, 9.0, 2)
    shells = [(0, 9, 7, rs[0], rs[1]), (0, 9, 7, rs[1], rs[2])]
    wl, d, s, u0, ubg, H, dH = _setup(shells, [(1.0, 0.4, (0.1, 0.2, 1.0))], [(0.9, -0.2, 1.1)], [0.005],
                                      configs.FILTER_DEFAULT)
    lam = dev(np.random.default_rng(4).standard_normal(u0.shape))
    a, b = dev(u0), dev(u0)
    u1, u2 = torch.empty_like(a), torch.empty_like(a)
    s.step(a, 1)
    s.step_stages(b, u1, u2)
    assert torch.equal(a, b)
    g1 = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    g2 = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    l1 = s.step_vjp(dev(u0), lam, g_gamma=g1)
    l2 = s.step_vjp_stages(dev(u0), u1, u2, lam, g_gamma=g2)
    assert torch.equal(l1, l2) and torch.equal(g1, g2)
    c = dev(u0)
    d = torch.full((450 * s.P,), float("nan"), dtype=torch.float64, device="cuda:0")
    v1, v2 = torch.empty_like(c), torch.empty_like(c)
    s.step_stages(c, v1, v2, derivs=d)
    assert torch.equal(a, c) and torch.equal(u1, v1) and torch.equal(u2, v2)
    assert bool(torch.isfinite(d).all())
    g3 = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    l3 = s.step_vjp_stages(dev(u0), v1, v2, lam, g_gamma=g3, derivs=d)
    assert torch.equal(l1, l3) and torch.equal(g1, g3)


def test_pulse_8shell_200_step_gradient_matches_central_differences():
    """The adjoint workload at full size: the 8-shell pulse domain (filter on),
    200 RK3 steps, checkpoint every 20, loss = final constraint norm.  The
    derivatives with respect to gamma0, gamma1, gamma2 and along two initial
    Pi directions (the seeded pulse itself and a smooth random Pi field) are
    compared with central differences, h = 1e-6, through the same GPU forward
    path, to 1e-6 of the norm of the five."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = configs.pulse_8shell()
    print(f"\n[case] pulse_8shell adjoint: {len(wl.shells)} shells, P={wl.npoints}, 200 steps", flush=True)
    xyz = ghmi.grid_coords(wl.shells)
    offs = np.concatenate([[0], np.cumsum([s[1] * 2 * (s[2] + 1) ** 2 for s in wl.shells])])
    u0, ubg, H, dH = wl.initial_data(xyz, offs, device="cuda:0")
    pulse = configs.to_layout(inputs.gaussian_pulse_Pi(xyz, 1e-3, 10.0, 2.0, 0), wl.shells, offs)
    rnd = inputs.smooth_random_field(xyz, 1e-3, 11, 4, 3.0)
    rnd[:10] = 0.0
    rnd[20:] = 0.0
    rnd = configs.to_layout(rnd, wl.shells, offs)
    s = ghmi.GHSolver(wl.shells, wl.n_inst, wl.filter_params)
    s.set_background(dev(H), dev(dH), dev(ubg))
    n = 200
    dirs = [dev(pulse), dev(rnd)]

    def loss(gamma_np, d=None, h=0.0):
        s.set_params(gamma_np, wl.dt)
        u = dev(u0)
        if d is not None:
            u += h * d
        s.step(u, n)
        return float(s.constraints(u, want_C=False)[1].cpu().numpy()[0])

    gamma = torch.tensor(wl.gamma, dtype=torch.float64, requires_grad=True)
    ua = dev(u0).requires_grad_(True)
    un = gha.evolve(ua, gamma, s, wl.dt, n, checkpoint_every=20)
    gha.constraint_norm(un, s).sum().backward()
    g_adj = np.concatenate([gamma.grad.numpy().ravel(), [float((ua.grad * d).sum()) for d in dirs]])
    h = 1e-6
    g_fd = []
    for c in range(3):
        gp, gm = wl.gamma.copy(), wl.gamma.copy()
        gp[0, c] += h
        gm[0, c] -= h
        g_fd.append((loss(gp) - loss(gm)) / (2 * h))
    for d in dirs:
        g_fd.append((loss(wl.gamma, d, h) - loss(wl.gamma, d, -h)) / (2 * h))
    g_fd = np.array(g_fd)
    gn = np.linalg.norm(g_fd)
    err = np.max(np.abs(g_adj - g_fd)) / gn
    print(f"  adjoint {g_adj}\n  FD      {g_fd}\n  max |adj-FD|/|g| {err:.2e}", flush=True)
    assert err <= 1e-6

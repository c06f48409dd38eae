"""The tensor-coupled angular filter on the GPU (filter_kind 2 ExpCheb, 3
Heaviside) against the oracle, element by element, through the C interface.

The GPU path applies PhysToSpec and SpecToPhys as grouped MFMA GEMMs and the
coupling as a segmented sparse product; the oracle transforms by quadrature
and couples with dense Lagrange projectors.  Both apply the same discrete
operator, so the filtered state must agree to 1e-12 of its size and RK3
evolutions with the filter to 1e-10 of the change (as for the other parity
tests).  Column counts are chosen ragged (not multiples of the kernel's column
chunk) and the L = 31 case has the largest segments.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import domain  # noqa: E402
from paper_1804_09101_amd import configs, ghmi, inputs  # noqa: E402

pytestmark = pytest.mark.gpu
H_CS = 1e-30
EXPCHEB = (2.0 / 3.0, 36.0, 8.0)
STRONG = (0.0, 3.0, 2.0)          # every degree damped, so every coupling matters


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def _setup(shells, holes, kind, params, pert=1e-3, seed=1, dt=None, gamma=None):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n = len(holes)
    gamma = gamma if gamma is not None else [configs.GAMMA_DEFAULT] * n
    dt = dt if dt is not None else [0.005] * n
    wl = configs.Workload("tensor_filter", shells, holes, gamma, dt, params, 1, None)
    print(f"\n[case] tensor filter kind {kind} {params}: {len(shells)} shells, P={wl.npoints}", flush=True)
    d = domain.Domain([domain.Shell(*s) for s in shells], filter_params=params, filter_kind=kind)
    xyz = d.xyz()
    u0, ubg, H, dH = wl.initial_data(xyz, d.offsets)
    if pert:
        u0 = u0 + d.to_layout(inputs.smooth_random_field(xyz, pert, seed, 3, 2.0))
    s = ghmi.GHSolver(shells, n, params, filter_kind=kind)
    assert s.P == d.P
    s.set_background(dev(H), dev(dH), dev(ubg))
    s.set_params(wl.gamma, wl.dt)
    return wl, d, s, u0, ubg, H, dH


# per L: 9 + 10 = 19 and 7 + 6 = 13 columns (shell, radius): ragged chunks
MIXED = [(0, 9, 7, 1.8, 3.0), (0, 10, 7, 3.0, 5.5), (1, 7, 11, 1.7, 2.9), (1, 6, 11, 2.9, 6.0)]
HOLES2 = [(1.0, 0.0, (0, 0, 1)), (1.0, 0.5, (0.3, -0.2, 0.9))]


@pytest.mark.parametrize("kind,params", [(2, EXPCHEB), (2, STRONG), (3, (0.6,))])
def test_filter_matches_oracle_mixed_L(kind, params):
    wl, d, s, u0, ubg, H, dH = _setup(MIXED, HOLES2, kind, params)
    rng = np.random.default_rng(5)
    u = u0 + 1e-3 * rng.standard_normal(u0.shape)     # not band-limited: the projection counts too
    got = s.filter(dev(u)).cpu().numpy()
    ref = d.apply_filter(u)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    change = np.max(np.abs(ref - u)) / np.max(np.abs(u))
    print(f"  filter rel err {err:.3e} (filter changes the state by {change:.2e})", flush=True)
    assert err < 1e-12 and change > 1e-6


def test_heaviside_filter_is_a_projector_on_the_gpu():
    wl, d, s, u0, ubg, H, dH = _setup(MIXED, HOLES2, 3, (0.5,))
    u = dev(u0 + 1e-2 * np.random.default_rng(6).standard_normal(u0.shape))
    once = s.filter(u)
    twice = s.filter(once)
    err = float((twice - once).abs().max() / once.abs().max())
    print(f"  F F u - F u: {err:.3e}", flush=True)
    assert err < 1e-13


def test_steps_with_tensor_filter_match_oracle():
    """The tensor-coupled filter leaves the Kerr-Schild background nearly
    unchanged (about 5e-5 per application here, against 9e-4 for the filter of
    every component), so the state moves little in a few steps; a 1e-2
    perturbation keeps the change of the evolution well above rounding.  Bars:
    1e-10 of the change, 1e-13 of the state."""
    rs = configs.geometric_radii(1.8, 12.0, 3)
    shells = [(0, 9, 7, rs[i], rs[i + 1]) for i in range(3)]
    wl, d, s, u0, ubg, H, dH = _setup(shells, [(1.0, 0.3, (0.2, 0.3, 0.4))], 2, EXPCHEB, pert=1e-2, dt=[0.004])
    u = dev(u0)
    s.step(u, 5)
    got = u.cpu().numpy()
    ref = u0.copy()
    for _ in range(5):
        ref = d.rk3_step(ref, H, dH, ubg, wl.gamma, wl.dt)
    diff = np.max(np.abs(got - ref))
    err = diff / np.max(np.abs(ref - u0))
    e_state = diff / np.max(np.abs(ref))
    print(f"  5 steps with the tensor filter: err/change {err:.3e}, err/state {e_state:.3e}", flush=True)
    assert err < 1e-10 and e_state < 1e-13


def test_pulse_8shell_full_size_filter():
    wl0 = configs.pulse_8shell()
    wl, d, s, u0, ubg, H, dH = _setup(wl0.shells, wl0.holes, 2, EXPCHEB, pert=1e-3, seed=0)
    got = s.filter(dev(u0)).cpu().numpy()
    ref = d.apply_filter(u0)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"  pulse_8shell tensor filter rel err {err:.3e}; couplings {s.query(11)}, "
          f"work items {s.query(12)}", flush=True)
    assert err < 1e-12


def test_L31_shell_largest_segments():
    wl, d, s, u0, ubg, H, dH = _setup([(0, 5, 31, 1.8, 3.0)], [(1.0, 0.2, (0, 0, 1))], 2, STRONG)
    got = s.filter(dev(u0)).cpu().numpy()
    ref = d.apply_filter(u0)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"  L = 31 tensor filter rel err {err:.3e}", flush=True)
    assert err < 1e-12


def test_step_vjp_dot_product_with_tensor_filter():
    rs = configs.geometric_radii(1.8, 9.0, 2)
    shells = [(0, 9, 7, rs[0], rs[1]), (0, 9, 7, rs[1], rs[2])]
    wl, d, s, u0, ubg, H, dH = _setup(shells, [(1.0, 0.4, (0.1, 0.2, 1.0))], 2, STRONG,
                                      gamma=[(0.9, -0.2, 1.1)], dt=[0.005])
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
    print(f"  step vjp with tensor filter: rel {err:.2e}", flush=True)
    assert err < 1e-12


def test_graph_replays_with_tensor_filter_equal_eager_steps():
    rs = configs.geometric_radii(1.8, 9.0, 2)
    shells = [(0, 9, 7, rs[0], rs[1]), (0, 10, 7, rs[1], rs[2])]
    wl, d, s, u0, ubg, H, dH = _setup(shells, [(1.0, 0.4, (0.1, 0.2, 1.0))], 3, (0.7,), dt=[0.005])
    a, b = dev(u0), dev(u0)
    s.step(a, 3)
    s.set_graph(True)
    for _ in range(3):
        s.step(b, 1)
        torch.cuda.synchronize()
    s.set_graph(False)
    assert torch.equal(a, b)


def test_dp5_attempt_with_tensor_filter_matches_oracle():
    shells = [(0, 7, 5, 1.8, 3.0), (0, 7, 5, 3.0, 4.5), (1, 7, 3, 1.7, 3.2)]
    holes = [(1.0, 0.0, (0, 0, 1)), (1.0, 0.5, (0, 0, 1))]
    wl, d, s, u0, ubg, H, dH = _setup(shells, holes, 2, STRONG, pert=1e-4, dt=[0.01, 0.01],
                                      gamma=[(1.0, -1.0, 1.0)] * 2)
    u = dev(u0)
    t = torch.zeros(2, dtype=torch.float64, device="cuda:0")
    dtv = dev(np.array([0.004, 0.004]))
    rej = torch.zeros(2, dtype=torch.int32, device="cuda:0")
    na = torch.zeros(2, dtype=torch.int32, device="cuda:0")
    s.step_dp5(u, 1, 1e-6, 1e-6, t, dtv, rejected=rej, n_accepted=na)
    uo, acc_o, dt_o, err_o = d.dp5_attempt(u0, H, dH, ubg, wl.gamma, np.array([0.004, 0.004]), 1e-6, 1e-6,
                                           [False, False])
    assert np.array_equal(na.cpu().numpy() > 0, acc_o)
    diff = np.max(np.abs(u.cpu().numpy() - uo)) / np.max(np.abs(uo - u0))
    print(f"  dp5 attempt with tensor filter: err/change {diff:.3e}", flush=True)
    assert diff < 1e-10


def test_tensor_filter_queries_and_errors():
    wl, d, s, u0, ubg, H, dH = _setup(MIXED, HOLES2, 2, EXPCHEB)
    nnz = sum(len(ghmi.tensor_filter_matrix(L, 2, EXPCHEB)[2]) for L in (7, 11))
    assert s.query(11) == nnz and s.query(12) > 0
    u = dev(u0)
    with pytest.raises(ghmi.GHError) as ei:
        s.filter(u, out=u)
    assert ei.value.code == -1
    plain = ghmi.GHSolver(MIXED, 2, None)
    with pytest.raises(ghmi.GHError) as ei:
        plain.filter(u)
    assert ei.value.code == -1
    for kind, params in ((2, (1.0, 36.0, 8.0)), (3, (-0.5,)), (4, EXPCHEB)):
        with pytest.raises(ghmi.GHError) as ei:
            ghmi.GHSolver(MIXED, 2, params, filter_kind=kind)
        assert ei.value.code == -1


def test_transform_form_matches_oracle_and_dense_form():
    """gh_set_angular 1: PhysToSpec and SpecToPhys by Fourier GEMMs and
    per-order Legendre steps; the same discrete filter as the dense form (to
    rounding), in single applications, filtered steps and (the reverse pass
    keeping the dense transposes) the step transpose."""
    wl, d, s, u0, ubg, H, dH = _setup(MIXED, HOLES2, 2, STRONG)
    rng = np.random.default_rng(8)
    u = u0 + 1e-3 * rng.standard_normal(u0.shape)
    dense = s.filter(dev(u)).cpu().numpy()
    s.set_angular(1)
    assert s.query(10) == 1
    got = s.filter(dev(u)).cpu().numpy()
    ref = d.apply_filter(u)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    diff = np.max(np.abs(got - dense)) / np.max(np.abs(ref))
    print(f"  transform-form tensor filter: rel err {err:.3e}, vs dense {diff:.3e}", flush=True)
    assert err < 1e-12 and diff < 1e-12
    a = dev(u0)
    s.step(a, 3)
    ref = u0.copy()
    for _ in range(3):
        ref = d.rk3_step(ref, H, dH, ubg, wl.gamma, wl.dt)
    e3 = np.max(np.abs(a.cpu().numpy() - ref)) / np.max(np.abs(ref - u0))
    print(f"  3 steps, transform form: err/change {e3:.3e}", flush=True)
    assert e3 < 1e-10
    lam = rng.standard_normal(u0.shape)
    v = rng.standard_normal(u0.shape)
    jv = d.rk3_step(u0 + 1j * H_CS * v, H, dH, ubg, wl.gamma, wl.dt).imag / H_CS
    ln = s.step_vjp(dev(u0), dev(lam)).cpu().numpy()
    ed = abs(np.sum(lam * jv) - np.sum(ln * v)) / np.sum(np.abs(lam * jv))
    print(f"  step vjp (transform forward, dense reverse): rel {ed:.2e}", flush=True)
    assert ed < 1e-12
    s.set_angular(2)
    assert s.query(10) in (0, 1)
    got2 = s.filter(dev(u)).cpu().numpy()
    ref2 = d.apply_filter(u)
    assert np.max(np.abs(got2 - ref2)) / np.max(np.abs(ref2)) < 1e-12

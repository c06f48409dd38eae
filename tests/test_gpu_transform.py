"""The transform method of the angular operators (gh_set_angular 1) against
the oracle, at the same bars as the dense method's parity tests, and against
the dense method at full size.

The transform method applies the same discrete operators as the dense GEMM
(factorised by azimuthal order), so both must agree with the oracle to
rounding: the RHS to 1e-12 of the term scale, RK3 evolutions to 1e-10 of the
change; on the 20-shell L = 31 domain sampled shells are compared with the
derivative term scale kappa at 1e-14 (see test_gpu_large).  The reverse pass
keeps the dense transposed operators, so its dot-product test checks that the
two methods are transposes of each other to rounding."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import domain  # noqa: E402
from paper_1804_09101_amd import configs, ghmi  # noqa: E402
from parity_util import rounding_scale  # noqa: E402
from test_gpu_parity import Case, _wl, dev  # noqa: E402

pytestmark = pytest.mark.gpu
H_CS = 1e-30


def _transform(case):
    case.s.set_angular(1)
    assert case.s.query(8) == 1
    return case


def test_transform_rhs_two_instances_mixed_L():
    shells = [(0, 9, 7, 1.8, 3.0), (0, 11, 7, 3.0, 5.5), (1, 7, 11, 1.7, 2.9), (1, 9, 11, 2.9, 6.0)]
    wl = _wl("mixed_L", shells, [(1.0, 0.0, (0, 0, 1)), (1.0, 0.5, (0.3, -0.2, 0.9))],
             gamma=[(0.4, 0.3, 1.7), (1.0, -1.0, 1.0)])
    c = _transform(Case(wl, pert_amp=1e-3, seed=7))
    got = c.s.rhs(dev(c.u0)).cpu().numpy()
    ref = c.oracle_rhs(c.u0)
    err = np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), c.term_scale(c.u0))
    print(f"  transform rhs rel err {err:.3e}", flush=True)
    assert err < 1e-12


def test_transform_100_steps_single_shell():
    c = _transform(Case(configs.single_shell(), pert_amp=1e-3, seed=2))
    u = dev(c.u0)
    c.s.step(u, 100)
    got = u.cpu().numpy()
    ref = c.u0.copy()
    for _ in range(100):
        ref = c.d.rk3_step(ref, c.H, c.dH, c.ubg, c.wl.gamma, c.wl.dt)
    change = np.max(np.abs(ref - c.u0))
    e_change = np.max(np.abs(got - ref)) / change
    e_state = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"  transform 100 steps: err/change {e_change:.3e}, err/state {e_state:.3e}", flush=True)
    assert e_change < 1e-10 and e_state < 1e-12


@pytest.mark.parametrize("mixed", [False, True])
def test_transform_filtered_steps_multishell(mixed):
    """Five filtered steps by transforms against the oracle.  Shells with
    L + 1 = 16 take the matrix-core theta step (derivatives and filter), the
    others the register kernel; the mixed case (a hole of two L = 15 shells
    next to one of an L = 11 shell) runs both in one pass."""
    rs = configs.geometric_radii(1.8, 12.0, 3)
    if mixed:
        shells = [(0, 9, 15, rs[0], rs[1]), (0, 9, 15, rs[1], rs[2]), (1, 9, 11, 1.7, 4.0)]
        holes = [(1.0, 0.3, (0.2, 0.3, 0.4)), (1.0, 0.5, (0.3, -0.2, 0.9))]
        dt = [0.004, 0.004]
    else:
        shells = [(0, 9, 7, rs[i], rs[i + 1]) for i in range(3)]
        holes = [(1.0, 0.3, (0.2, 0.3, 0.4))]
        dt = [0.004]
    wl = _wl("filtered_3shell", shells, holes, dt=dt, filt=configs.FILTER_DEFAULT)
    # the L = 15 shells resolve the stationary hole well, so their state moves
    # little in five steps: a larger perturbation keeps the change well above
    # the rounding of the O(1) state that the bar is measured against
    c = _transform(Case(wl, pert_amp=1e-2 if mixed else 1e-3, seed=3))
    u = dev(c.u0)
    c.s.step(u, 5)
    got = u.cpu().numpy()
    ref = c.u0.copy()
    for _ in range(5):
        ref = c.d.rk3_step(ref, c.H, c.dH, c.ubg, c.wl.gamma, c.wl.dt)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref - c.u0))
    e_state = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"  transform 5 filtered steps: err/change {err:.3e}, err/state {e_state:.3e}", flush=True)
    assert err < 1e-10 and e_state < 1e-13


def test_transform_pulse_8shell_full_size_matches_oracle_and_dense():
    c = Case(configs.pulse_8shell())
    u = dev(c.u0)
    dense = c.s.rhs(u).cpu().numpy()
    _transform(c)
    got = c.s.rhs(u).cpu().numpy()
    ref = c.oracle_rhs(c.u0)
    scale = max(np.max(np.abs(ref)), c.term_scale(c.u0))
    err = np.max(np.abs(got - ref)) / scale
    diff = np.max(np.abs(got - dense)) / scale
    print(f"  transform full-size rhs rel err {err:.3e}, vs dense {diff:.3e}", flush=True)
    assert err < 1e-12 and diff < 1e-12


def test_transform_graph_replays_equal_eager_steps():
    rs = configs.geometric_radii(1.8, 9.0, 2)
    shells = [(0, 9, 7, rs[0], rs[1]), (0, 9, 7, rs[1], rs[2])]
    wl = _wl("graph_transform", shells, [(1.0, 0.4, (0.1, 0.2, 1.0))], dt=[0.005], filt=configs.FILTER_DEFAULT)
    c = _transform(Case(wl, pert_amp=1e-3, seed=4))
    a, b = dev(c.u0), dev(c.u0)
    c.s.step(a, 3)
    c.s.set_graph(True)
    for _ in range(3):
        c.s.step(b, 1)
        torch.cuda.synchronize()
    c.s.set_graph(False)
    assert torch.equal(a, b)


def test_transform_forward_and_dense_reverse_are_transposes():
    shells = [(0, 7, 5, 1.8, 2.8), (0, 7, 5, 2.8, 4.5), (1, 6, 3, 1.3, 2.4)]
    wl = _wl("adjoint_transform", shells, [(1.0, 0.0, (0, 0, 1)), (0.8, 0.6, (0.3, -0.5, 0.8))],
             gamma=[(0.7, -0.6, 1.3), (1.0, 0.3, 0.6)], dt=[0.004, 0.003])
    c = _transform(Case(wl, pert_amp=1e-3, seed=1))
    rng = np.random.default_rng(0)
    lam = rng.standard_normal(c.u0.shape)
    v = rng.standard_normal(c.u0.shape)
    jv = c.d.rhs(c.u0 + 1j * H_CS * v, c.H, c.dH, c.ubg, wl.gamma).imag / H_CS
    lhs = np.sum(lam * jv)
    lu = c.s.rhs_vjp(dev(c.u0), dev(lam)).cpu().numpy()
    rhs = np.sum(lu * v)
    err = abs(lhs - rhs) / np.sum(np.abs(lam * jv))
    print(f"  transform rhs vjp dot: rel {err:.2e}", flush=True)
    assert err < 1e-12


@pytest.fixture(scope="module")
def large_transform():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = configs.large_20shell()
    print(f"\n[case] large_20shell transform: P={wl.npoints}", flush=True)
    xyz = ghmi.grid_coords(wl.shells)
    offs = np.concatenate([[0], np.cumsum([s[1] * 2 * (s[2] + 1) ** 2 for s in wl.shells])])
    u0, ubg, H, dH = wl.initial_data(xyz, offs, device="cuda:0")
    s = ghmi.GHSolver(wl.shells, wl.n_inst, wl.filter_params)
    s.set_background(dev(H), dev(dH), dev(ubg))
    s.set_params(wl.gamma, wl.dt)
    s.set_angular(1)
    rhs = s.rhs(dev(u0)).cpu().numpy()
    return wl, offs, u0, ubg, H, dH, rhs


@pytest.mark.parametrize("k", [0, 19])
def test_transform_large_sampled_shells(large_transform, k):
    wl, offs, u0, ubg, H, dH, rhs = large_transform
    d = domain.Domain([domain.Shell(*wl.shells[k])])
    sl = lambda a, c: a[c * offs[k]: c * offs[k + 1]]
    ref = d.rhs(sl(u0, 50), sl(H, 4), sl(dH, 16), sl(ubg, 50), wl.gamma, apply_bc=False)
    g = d.split(sl(rhs, 50), 50)[0][:, 1:-1]
    r = d.split(ref, 50)[0][:, 1:-1]
    ublk = d.split(sl(u0, 50), 50)[0]
    kappa = rounding_scale(d, 0, ublk)
    diff = np.max(np.abs(g - r))
    print(f"  transform shell {k}: max diff {diff:.3e} / term scale {kappa:.3e} = {diff / kappa:.3e}", flush=True)
    assert diff < 1e-14 * kappa


def test_fastest_method_matches_dense_and_rejects_unknown_methods():
    """Method 2 picks each operation's form by timing; whatever it picks, a
    filtered multi-shell step equals the dense one to rounding."""
    rs = configs.geometric_radii(1.8, 12.0, 3)
    shells = [(0, 9, 7, rs[i], rs[i + 1]) for i in range(3)]
    wl = _wl("auto_3shell", shells, [(1.0, 0.3, (0.2, 0.3, 0.4))], dt=[0.004], filt=configs.FILTER_DEFAULT)
    c = Case(wl, pert_amp=1e-3, seed=3)
    a = dev(c.u0)
    c.s.step(a, 3)
    c.s.set_angular(2)
    assert c.s.query(8) == 2 and c.s.query(9) in (0, 1) and c.s.query(10) in (0, 1)
    b = dev(c.u0)
    c.s.step(b, 3)
    err = float((a - b).abs().max()) / float((a - dev(c.u0)).abs().max())
    print(f"  method 2 (deriv {c.s.query(9)}, filter {c.s.query(10)}): 3 steps vs dense, err/change {err:.3e}",
          flush=True)
    assert err < 1e-10
    for bad in (-1, 3):
        with pytest.raises(ghmi.GHError) as ei:
            c.s.set_angular(bad)
        assert ei.value.code == -1

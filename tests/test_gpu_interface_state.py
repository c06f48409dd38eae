"""Interfaces with the characteristic projection taken from the state
(gh_set_interface 1) against the oracle (interface_from_state=True), through
the C interface, at the bars of the other parity tests: the RHS to 1e-12 of
the term scale, evolutions to 1e-10 of the change.  The perturbation is large
enough (5e-2) that the state's metric at the interfaces differs from the
background's, so the two modes give different d_t u there."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import domain  # noqa: E402
from paper_1804_09101_amd import configs, ghmi, inputs  # noqa: E402

pytestmark = pytest.mark.gpu

SHELLS = [(0, 9, 7, 1.8, 2.8), (0, 8, 7, 2.8, 4.2), (0, 7, 7, 4.2, 6.0), (1, 7, 5, 1.4, 2.9), (1, 6, 5, 2.9, 4.5)]
HOLES = [(1.0, 0.4, (0.1, 0.2, 1.0)), (0.8, 0.0, (0, 0, 1))]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def _setup(shells=SHELLS, holes=HOLES, pert=5e-2, dt=None, filt=None):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n = len(holes)
    dt = dt if dt is not None else [0.004] * n
    wl = configs.Workload("iface_state", shells, holes, [configs.GAMMA_DEFAULT] * n, dt, filt, 1, None)
    print(f"\n[case] interface from state: {len(shells)} shells, P={wl.npoints}", flush=True)
    d = domain.Domain([domain.Shell(*s) for s in shells], filter_params=filt, interface_from_state=True)
    d0 = domain.Domain([domain.Shell(*s) for s in shells], filter_params=filt)
    xyz = d.xyz()
    u0, ubg, H, dH = wl.initial_data(xyz, d.offsets)
    u0 = u0 + d.to_layout(inputs.smooth_random_field(xyz, pert, 4, 3, 2.0))
    s = ghmi.GHSolver(shells, n, filt)
    s.set_background(dev(H), dev(dH), dev(ubg))
    s.set_params(wl.gamma, wl.dt)
    s.set_interface(1)
    assert s.query(13) == 1
    return wl, d, d0, s, u0, ubg, H, dH


def _term_scale(d, u):
    return max(np.max(np.abs(d.cartesian_derivs(k, b))) for k, b in enumerate(d.split(u, 50)))


def test_rhs_matches_oracle_and_differs_from_frozen_mode():
    wl, d, d0, s, u0, ubg, H, dH = _setup()
    got = s.rhs(dev(u0)).cpu().numpy()
    ref = d.rhs(u0, H, dH, ubg, wl.gamma)
    frozen = d0.rhs(u0, H, dH, ubg, wl.gamma)
    scale = max(np.max(np.abs(ref)), _term_scale(d, u0))
    err = np.max(np.abs(got - ref)) / scale
    moved = np.max(np.abs(ref - frozen)) / scale
    print(f"  rhs rel err {err:.3e}; the modes differ by {moved:.3e}", flush=True)
    assert err < 1e-12 and moved > 1e-8
    s.set_interface(0)
    got0 = s.rhs(dev(u0)).cpu().numpy()
    assert np.max(np.abs(got0 - frozen)) / scale < 1e-12


def test_steps_match_oracle():
    wl, d, d0, s, u0, ubg, H, dH = _setup()
    u = dev(u0)
    s.step(u, 20)
    got = u.cpu().numpy()
    ref = u0.copy()
    for _ in range(20):
        ref = d.rk3_step(ref, H, dH, ubg, wl.gamma, wl.dt)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref - u0))
    print(f"  20 steps, interface from state: err/change {err:.3e}", flush=True)
    assert err < 1e-10


def test_filtered_steps_graph_and_dp5():
    rs = configs.geometric_radii(1.8, 9.0, 2)
    shells = [(0, 9, 7, rs[0], rs[1]), (0, 9, 7, rs[1], rs[2])]
    wl, d, d0, s, u0, ubg, H, dH = _setup(shells, [(1.0, 0.4, (0.1, 0.2, 1.0))], filt=configs.FILTER_DEFAULT)
    a, b = dev(u0), dev(u0)
    s.step(a, 3)
    s.set_graph(True)
    for _ in range(3):
        s.step(b, 1)
        torch.cuda.synchronize()
    s.set_graph(False)
    assert torch.equal(a, b)
    ref = u0.copy()
    for _ in range(3):
        ref = d.rk3_step(ref, H, dH, ubg, wl.gamma, wl.dt)
    err = np.max(np.abs(a.cpu().numpy() - ref)) / np.max(np.abs(ref - u0))
    print(f"  3 filtered steps: err/change {err:.3e}", flush=True)
    assert err < 1e-10
    # one Dormand-Prince attempt from the same state
    u = dev(u0)
    t = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    dtv = dev(np.array([0.004]))
    na = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    rej = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    s.step_dp5(u, 1, 1e-6, 1e-6, t, dtv, rejected=rej, n_accepted=na)
    uo, acc_o, _, _ = d.dp5_attempt(u0, H, dH, ubg, wl.gamma, np.array([0.004]), 1e-6, 1e-6, [False])
    assert np.array_equal(na.cpu().numpy() > 0, acc_o)
    e5 = np.max(np.abs(u.cpu().numpy() - uo)) / np.max(np.abs(uo - u0))
    print(f"  dp5 attempt: err/change {e5:.3e}", flush=True)
    assert e5 < 1e-10


def test_reverse_pass_needs_the_frozen_projection():
    wl, d, d0, s, u0, ubg, H, dH = _setup()
    u = dev(u0)
    lam = dev(np.ones_like(u0))
    for call in (lambda: s.rhs_vjp(u, lam), lambda: s.step_vjp(u, lam)):
        with pytest.raises(ghmi.GHError) as ei:
            call()
        assert ei.value.code == -1
    for bad in (-1, 2):
        with pytest.raises(ghmi.GHError):
            s.set_interface(bad)
    s.set_interface(0)
    assert s.query(13) == 0
    s.rhs_vjp(u, lam)

"""The constraint-preserving outer boundary (gh_set_outer_bc 1) on the GPU
against the oracle (outer_bc "constraint_preserving"), through the C interface.

Bars as for the other parity tests: the RHS to 1e-12 of the term scale,
evolutions to 1e-10 of the change of the state, graph replays bitwise equal to
eager steps, one Dormand-Prince attempt to 1e-12 of the state's change.
One instance has gamma1 = 0.5, so its u^psi is incoming at the outer boundary
and the three-index correction is exercised; the other has gamma1 = -1.
The property the condition is for is checked on the GPU alone: a pulse that
leaves through the outer boundary leaves the constraint norm decaying, while
with the Dirichlet condition it grows.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import domain  # noqa: E402
from paper_1804_09101_amd import configs, ghmi, inputs  # noqa: E402

pytestmark = pytest.mark.gpu

SHELLS = [(0, 9, 7, 1.8, 3.0), (0, 9, 7, 3.0, 4.6), (0, 8, 7, 4.6, 6.0),
          (1, 7, 5, 1.5, 2.9), (1, 9, 5, 2.9, 5.0)]
HOLES = [(1.0, 0.0, (0.0, 0.0, 1.0)), (0.9, 0.5, (0.3, -0.2, 0.9))]
GAMMA = [(1.0, 0.5, 1.0), (0.7, -1.0, 1.3)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def _setup(filt=None, pert=1e-3, seed=7):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dt = [configs.COURANT * min(configs.min_radial_spacing(s[1], s[3], s[4]) for s in SHELLS if s[0] == i)
          for i in range(2)]
    wl = configs.Workload("outer_cpbc", SHELLS, HOLES, GAMMA, dt, filt, 1, None)
    d = domain.Domain([domain.Shell(*s) for s in SHELLS], filter_params=filt, outer_bc="constraint_preserving")
    xyz = d.xyz()
    u0, ubg, H, dH = wl.initial_data(xyz, d.offsets)
    u0 = u0 + d.to_layout(inputs.smooth_random_field(xyz, pert, seed, 3, 2.0))
    s = ghmi.GHSolver(SHELLS, 2, filt)
    s.set_background(dev(H), dev(dH), dev(ubg))
    s.set_params(wl.gamma, wl.dt)
    s.set_outer_bc(1)
    assert s.query(17) == 1
    return wl, d, s, u0, ubg, H, dH


def _term_scale(d, u):
    return max(np.max(np.abs(d.cartesian_derivs(k, b))) for k, b in enumerate(d.split(u, 50)))


def test_rhs_matches_oracle():
    wl, d, s, u0, ubg, H, dH = _setup(pert=1e-2)
    print("\n[case] outer constraint-preserving rhs", flush=True)
    got = s.rhs(dev(u0)).cpu().numpy()
    ref = d.rhs(u0, H, dH, ubg, wl.gamma)
    err = np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), _term_scale(d, u0))
    # the treatment is not vacuous: it differs from Dirichlet on the outer faces
    b = d.split(got, 50)
    print(f"  rel err {err:.3e}; outer faces max |d_t u| {np.max(np.abs(b[2][:, -1])):.3e}", flush=True)
    assert err < 1e-12
    assert np.max(np.abs(b[2][:, -1])) > 1e-4 and np.max(np.abs(b[4][:, -1])) > 1e-4
    s.close()


@pytest.mark.parametrize("method", [0, 1])
def test_steps_match_oracle(method):
    wl, d, s, u0, ubg, H, dH = _setup(filt=configs.FILTER_DEFAULT)
    print(f"\n[case] outer constraint-preserving, 30 filtered steps, angular method {method}", flush=True)
    if method:
        s.set_angular(1)
    u = dev(u0)
    s.step(u, 30)
    got = u.cpu().numpy()
    s.close()
    ref = u0.copy()
    for _ in range(30):
        ref = d.rk3_step(ref, H, dH, ubg, wl.gamma, wl.dt)
    e_change = np.max(np.abs(got - ref)) / np.max(np.abs(ref - u0))
    e_state = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"  err/change {e_change:.3e}, err/state {e_state:.3e}", flush=True)
    assert e_change < 1e-10 and e_state < 1e-12


def test_graph_replay_and_dp5_attempt():
    wl, d, s, u0, ubg, H, dH = _setup()
    print("\n[case] outer constraint-preserving: graph replay and one Dormand-Prince attempt", flush=True)
    ue = dev(u0)
    s.step(ue, 4)
    s.set_graph(True)
    ug = dev(u0)
    s.step(ug, 2)
    s.step(ug, 2)
    assert torch.equal(ue, ug)
    s.set_graph(False)
    u = dev(u0)
    t = torch.zeros(2, dtype=torch.float64, device="cuda:0")
    dt = dev(np.array(wl.dt) * 4.0)
    acc = torch.zeros(2, dtype=torch.int32, device="cuda:0")
    s.step_dp5(u, 1, 1e-6, 1e-6, t, dt, n_accepted=acc)
    got = u.cpu().numpy()
    ref, acc_ref, _, _ = d.dp5_attempt(u0, H, dH, ubg, wl.gamma, np.array(wl.dt) * 4.0, 1e-6, 1e-6,
                                       np.zeros(2, dtype=bool))
    assert np.array_equal(acc.cpu().numpy() > 0, acc_ref)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref - u0))
    print(f"  dp5 accepted {acc_ref}, err/change {err:.3e}", flush=True)
    assert err < 1e-10
    s.close()


def test_reverse_pass_is_refused():
    wl, d, s, u0, ubg, H, dH = _setup()
    with pytest.raises(ghmi.GHError) as ei:
        s.rhs_vjp(dev(u0), dev(np.ones_like(u0)))
    assert ei.value.code == -1
    s.set_outer_bc(0)
    s.rhs_vjp(dev(u0), dev(np.ones_like(u0)))
    s.close()


def test_constraint_norm_decays_when_a_pulse_leaves():
    """Four shells in [1.8, 10], a pulse at r = 7.5 that reaches the outer
    boundary; 1600 RK3 steps (t = 5.2) with each outer condition."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rs = configs.geometric_radii(1.8, 10.0, 4)
    shells = [(0, 15, 11, rs[i], rs[i + 1]) for i in range(4)]
    dt = configs.COURANT * min(configs.min_radial_spacing(s[1], s[3], s[4]) for s in shells)
    wl = configs.Workload("pulse_out", shells, [(1.0, 0.0, (0, 0, 1))], [configs.GAMMA_DEFAULT], [dt],
                          configs.FILTER_DEFAULT, 1, None)
    xyz = ghmi.grid_coords(shells)
    offs = np.concatenate([[0], np.cumsum([s[1] * 2 * (s[2] + 1) ** 2 for s in shells])])
    u0, ubg, H, dH = wl.initial_data(xyz, offs)
    u0 = u0 + configs.to_layout(inputs.gaussian_pulse_Pi(xyz, 1e-3, 7.5, 1.0, 0), shells, offs)
    n_steps = int(round(5.2 / dt))
    res = {}
    for mode in (0, 1):
        s = ghmi.GHSolver(shells, 1, configs.FILTER_DEFAULT)
        s.set_background(dev(H), dev(dH), dev(ubg))
        s.set_params(wl.gamma, wl.dt)
        s.set_outer_bc(mode)
        u = dev(u0)
        n0 = float(s.constraints(u, want_C=False)[1].cpu()[0])
        norms = []
        for _ in range(4):
            s.step(u, n_steps // 4)
            norms.append(float(s.constraints(u, want_C=False)[1].cpu()[0]))
        assert bool(torch.isfinite(u).all())
        res[mode] = (n0, norms)
        print(f"  outer mode {mode}: constraint norm {n0:.3e} -> " + ", ".join(f"{x:.3e}" for x in norms),
              flush=True)
        s.close()
    (n0, dirichlet), (_, cp) = res[0], res[1]
    assert cp[-1] < n0 and cp[-1] < 0.5 * dirichlet[-1]
